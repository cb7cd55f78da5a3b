// Host-side trie structures: the CRS trie and the device image derived from it.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace pfac {

constexpr uint32_t kNone = 0xffffffffu;
constexpr uint32_t kTermFlag = 1u << 16;   // node record .z: terminal node
constexpr uint32_t kNcMask = 0xffffu;      // node record .z: number of children
constexpr uint32_t kSkipFlag = 1u << 17;   // node record .z: compressed single-child run
constexpr uint32_t kSkipShift = 18;        // node record .z: run length above this bit
constexpr uint32_t kLeafEnd = 1u << 15;    // skip node .z: the run ends at a leaf
constexpr uint32_t kSkipMax = (1u << 14) - 1;
constexpr uint32_t kCountShift = 18;       // terminal record .z: pattern-list length above this bit
constexpr uint32_t kCountEsc = (1u << 14) - 1;  // length stored before the list

// The CRS trie of Design and Implementation.  Nodes are numbered breadth first
// (step I), level by level, with children by ascending unsigned label, so the
// row-major array of step II is simply node order and edge e leads to node e+1.
struct CrsTrie {
    uint32_t k = 0;                    // number of patterns
    std::vector<uint8_t> pat_data;     // patterns back to back (copied in)
    std::vector<uint64_t> pat_off;     // k + 1
    uint64_t min_len = 0, max_len = 0;

    std::vector<uint32_t> row_ptr;     // N + 1: edges of node v = [row_ptr[v], row_ptr[v+1])
    std::vector<uint8_t> labels;       // N - 1: label of edge e (= of node e + 1)
    std::vector<uint32_t> term_ptr;    // N + 1
    std::vector<uint32_t> term_ids;    // k, ascending within a node
    std::vector<uint32_t> level_start; // depth d nodes: [level_start[d], level_start[d+1])
    std::vector<uint32_t> rep;         // N: one pattern id whose prefix is node v (root: kNone)

    uint32_t n_nodes() const { return (uint32_t)(row_ptr.size() - 1); }
    uint32_t n_edges() const { return (uint32_t)labels.size(); }
};

// Builds the trie level by level from the lexicographically sorted patterns
// (step I).  Returns false on an empty pattern.
bool build_crs(const uint8_t *data, const uint64_t *off, uint32_t k, CrsTrie &out,
               std::string &err);

// Everything the scan kernel reads, laid out for the device.
struct DeviceImageHost {
    // Per node, 16 bytes: x = labels of the first four children (byte j =
    // label j), y = first child node id (children are y .. y+nc-1),
    // z = nc | kTermFlag | list length << kCountShift, w = offset of the
    // node's pattern list in pout_ids (terminal nodes).  Skip nodes use
    // x = chain offset, z = 1 | kSkipFlag | run length << kSkipShift,
    // w = node reached after the run; when that node is a leaf whose list
    // length is below 255 and the chain offset below 2^24, z also has
    // kLeafEnd, x bits 24..31 hold the leaf's list length and w its list
    // offset.
    std::vector<uint32_t> node;        // 4 * N
    std::vector<uint8_t> label;        // N - 1 (a copy of the CRS labels, padded)
    std::vector<uint8_t> chain;        // labels of single-child runs (skip nodes)
    std::vector<uint32_t> pout_ptr;    // unused (kept empty)
    std::vector<uint32_t> pout_ids;
    // Level index: the depth-K nodes as a bitmap over K-symbol codes, with
    // the number of set bits before each 32-bit word.  Breadth-first order
    // with ascending labels is ascending code order within a level, so the
    // rank of a code is the node's offset in its level.
    uint32_t K = 0;                    // index depth (0 = no index)
    uint32_t b = 8;                    // bits per symbol
    uint32_t identity = 1;             // 1: symbol = byte (b = 8)
    uint32_t lvl_words = 0;            // 32-bit words of the bitmap
    uint32_t lvl_start = 0;            // first node id of depth K
    std::vector<uint32_t> lvl;         // 2 * lvl_words: {bits, rank before}
    std::vector<uint8_t> sym;          // 256: symbol code, 0xff = byte unused
    // The same K levels as bitmapped nodes (the node format of Design and
    // Implementation, with the bitmap narrowed to the 2^b symbols): node
    // v < lvl_start has top_rw words, the bitmap of its children's symbols
    // (at least one word) and then the id of its first child; the child on
    // symbol s is the first child + the set bits below s.
    uint32_t top_rw = 0;
    uint32_t top_nodes = 0;            // nodes of depths 0 .. K-1
    std::vector<uint32_t> top;
    // Truncated image (trunc_depth D > 0): only nodes of depths 0..D; a
    // depth-D node with children has x = 1 + its first tail entry, y = the
    // number of entries, no children.  Entry (4 words): offset of the bytes
    // after depth D in tail_bytes, their count, the root-path pattern list of
    // the terminal node they reach (offset, stored length); longest first.
    uint32_t trunc_depth = 0;
    std::vector<uint32_t> tail;
    std::vector<uint8_t> tail_bytes;
    // Merged image (dag = 1): the trie's equal subtries shared as one DAG
    // node.  dnode per node: labels of the first four edges, first edge,
    // nc | kTermFlag, 0; per edge: label, child DAG node, rank added.
    // rank_list[2r], [2r+1]: root-path pattern list (offset, stored length) of
    // the r-th distinct pattern string in sorted order; lvl_dag[2i], [2i+1]:
    // DAG node and rank so far of the level index's i-th depth-K node.
    uint32_t dag = 0;
    std::vector<uint32_t> dnode;
    std::vector<uint8_t> dlabel;
    std::vector<uint32_t> dchild, dradd, rank_list, lvl_dag;
    uint32_t alphabet = 0;
    uint32_t n_term = 0;
    // Prefix filter of the wave kernel.  With K >= 1 it is a table of E-bit
    // entries indexed by the K-symbol code of a depth-K node: bit
    // (code of the next m symbols) & (E - 1) is set for each of its
    // depth-(K+m) descendants, i.e. a child bitmap of the node folded to E
    // bits (exact when b * m <= log2 E).  A start position whose first K + m
    // symbols miss it cannot match (K + m <= shortest pattern).  With K = 0
    // the filter is the root's child bitmap over the first symbol.
    uint32_t fold_bits = 0;            // E: 8 or 16 (0 = no table)
    uint32_t fold_syms = 0;            // m
    std::vector<uint8_t> ftab;         // 2^(b K) entries of E bits
    std::vector<uint32_t> root_bits;   // 2^b bits: codes of the root's children
    // Child labels of every depth-K node in breadth-first order: bytes 0..2
    // hold up to three labels, byte 3 the count (0xff when there are more).
    std::vector<uint32_t> krec;
    // Prefix-4 filter (byte alphabets, every pattern of 4 bytes or more): a
    // blocked Bloom filter of 2^(pfx4_log2 - 5) words.  Each pattern's first
    // four bytes x = B0 | B1 << 8 | B2 << 16 | B3 << 24 give
    // h1 = (x mod 2^24) * kPfx4M1 + (x >> 8) and h2 = (x >> 8) * kPfx4M2 + x
    // (mod 2^32, two 24 x 24-bit multiplies); word h1 >> (37 - pfx4_log2)
    // has bits (h1 >> (32 - pfx4_log2)) & 31 and h2 >> 27 set.  A start
    // position with either bit clear matches no pattern.
    uint32_t pfx4_log2 = 0;            // 0 = no filter
    std::vector<uint32_t> pfx4;
    // Four-symbol filter (alphabets of at most four bytes whose sorted bytes
    // c_i satisfy ((c_i >> qa) ^ (c_i >> qb)) & 3 == i, every pattern of 16
    // bytes or more).  key = the first 16 symbols, 2 bits each, symbol 0
    // lowest; h = (key mod 2^24) * kQ16Mul + (key >> 8) mod 2^32.
    //  - q16: 2^q16_lw words; word h >> (32 - q16_lw) has bits h & 31 and
    //    (h >> 5) & 31 set for every distinct 16-symbol prefix;
    //  - qfp: 2^qfp_lb buckets of 8 nonzero 16-bit fingerprints
    //    (key * kPfx4Mul) & 0xffff | 1 in bucket (key * kPfx4Mul) >> (32 -
    //    qfp_lb) or the next one (qfp_lb = 0: no fingerprints);
    //  - qalph: byte i = c_i (an unused symbol holds a byte of another one).
    uint32_t q16_lw = 0;               // 0 = no four-symbol filter
    uint32_t qfp_lb = 0;
    uint32_t qa = 0, qb = 0, qalph = 0;
    std::vector<uint32_t> q16;
    std::vector<uint16_t> qfp;
};

// Multiplicative (Fibonacci) hashing, Knuth TAOCP vol. 3, 6.4: odd
// multipliers near 2^w / golden ratio, the hash taken from the top bits.
constexpr uint32_t kQ16Mul = 0x9E3779u;     // 24-bit multiplier (one 24 x 24-bit multiply)
constexpr uint32_t kPfx4Mul = 0x9E3779B1u;  // 32-bit multiplier
constexpr uint32_t kPfx4M1 = 0x9E3779u;     // 24-bit multipliers of the prefix-4 filter
constexpr uint32_t kPfx4M2 = 0x7F4A7Du;

// Derives the device image from the CRS trie for a level index of at most
// `index_bits` bits and a prefix filter of `fold_bits` (0, 8 or 16) bits per
// entry.
void pack_image(const CrsTrie &t, uint32_t index_bits, uint32_t fold_bits, uint32_t trunc_depth,
                uint32_t dag, DeviceImageHost &img);
// Nodes and edges of the trie with equal subtries merged (the DAG of pack_image's dag = 1).
void dag_size(const CrsTrie &t, uint64_t &nodes, uint64_t &edges);

}  // namespace pfac
