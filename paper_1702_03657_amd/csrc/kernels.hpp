// Device-side structures and launchers of the scan kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/pfac.h"

namespace pfac {

constexpr uint32_t kWG = 256;            // threads per workgroup (4 waves of 64)
constexpr uint32_t kMatchCap = 256;      // matched positions a tile sorts in LDS
constexpr uint32_t kSumShift = 5;        // units per block-sum entry and finisher workgroup = 32
constexpr uint32_t kHaloCap = 1024;      // most halo bytes staged in LDS
constexpr uint32_t kInlineCap = 8;       // records a wave unit stages without an atomic (at least)
constexpr uint32_t kInlinePerChunk = 2;  // ... and per 1 KiB chunk of the unit

// Device image as the kernels see it (pointers into one device allocation).
struct ImageView {
    const uint4 *node;        // per node: labels4, first child, nc | term flag, terminal ordinal
    const uint8_t *label;     // per edge
    const uint32_t *pout_ptr; // per terminal ordinal + 1
    const uint32_t *pout_ids;
    const uint32_t *lvl;      // 2 per word: bits, rank before
    const uint8_t *sym;       // 256
    const uint8_t *ftab;      // prefix filter: folded child bitmaps of depth-K nodes
    const uint32_t *root_bits;  // codes of the root's children
    const uint8_t *chain;     // labels of compressed single-child runs
    const uint32_t *krec;     // per depth-K node: up to three child labels, count in the top byte
    const uint32_t *pfx4;     // prefix-4 filter bitmap (2^pfx4_log2 bits)
    const uint32_t *q16;      // four-symbol filter: bitmap words (2^q16_lw)
    const uint4 *qfp;         // four-symbol filter: buckets of 8 x 16-bit fingerprints
    const uint32_t *top;      // bitmapped nodes of depths 0 .. K-1: top_rw words each
    const uint4 *tail;        // truncated image: tail entries (byte offset, length, list)
    const uint8_t *tail_bytes;
    const uint4 *dnode;       // merged image: DAG nodes (labels4, first edge, nc | term, 0)
    const uint8_t *dlabel;    // per DAG edge: label, child, rank added
    const uint32_t *dchild;
    const uint32_t *dradd;
    const uint2 *rank_list;   // per distinct pattern string: root-path pattern list
    const uint2 *lvl_dag;     // per depth-K node of the level index: DAG node, rank so far
    uint32_t dag;
    uint32_t K, b, identity, lvl_words;
    uint32_t lvl_start, max_len, n_nodes, fold_syms;
    uint32_t pfx4_log2, pfx4_mul;     // prefix-4 filter: 2^pfx4_log2 bits; 32-bit hash multiplier
    uint32_t pfx4_m1, pfx4_m2;        // the prefix-4 filter's 24-bit hash multipliers
    uint32_t q16_lw, qfp_lb;          // four-symbol filter sizes (0 = none)
    uint32_t qa, qb, qalph, q16_mul;  // its symbol map, alphabet bytes and hash multiplier
    uint32_t top_nodes, top_rw;       // bitmapped top nodes: count, words per node
};

struct ScanArgs {
    ImageView im;
    const uint8_t *base;              // text frame: 16-byte aligned address
    uint64_t shift;                   // frame position of the first text byte (0..15)
    uint64_t total;                   // bytes of all texts
    const uint64_t *offsets;          // n_texts + 1 text starts, or NULL for one text
    const uint32_t *tile_first_text;  // per plan unit: text holding its first byte (batch only)
    const uint2 *chunk_info;          // wave kernels, batch only: text boundaries per 1 KiB chunk
    uint64_t n_plan;                  // plan units of 1 << plan_shift bytes
    uint32_t plan_shift, pad3;
    uint64_t n_tiles;
    uint32_t n_texts;
    uint32_t text_id0;                // added to every reported text id
    uint32_t halo;                    // bytes staged past each tile (multiple of 16)
    uint32_t pad0;
    // dynamic LDS layout (byte offsets)
    uint32_t off_bits, off_rank, off_sym, off_text, off_bnd, off_queue, off_match, lds_total;
    // wave kernel: shared tables, then one area per wave
    uint32_t fold;                    // prefix-filter bits per entry (0, 8, 16)
    uint32_t ftab_bytes, off_ftab, root_words, off_root;
    uint32_t off_wave, wave_bytes, woff_bnd, woff_queue, woff_cand, woff_match, ccap, mcap;
    uint32_t krec_words, off_krec, group, pad1;   // LDS child records, chunks per unit
    uint32_t pfx4_words, off_pfx4;    // LDS prefix-4 filter (instead of the child records)
    uint32_t q16_words;               // four-symbol filter words in LDS (mode 3; 0 = other modes)
    uint32_t lvl_lds;                 // level-index words kept in LDS (0 in mode 3)
    uint32_t top_words, off_top;      // tile kernel: bitmapped top nodes in LDS (0 = level index)
    // outputs
    pfac_match *stage;
    uint64_t stage_cap;
    unsigned long long *stage_cursor;
    uint32_t *unit_count;             // per tile
    unsigned long long *unit_off;     // per tile
    unsigned long long *blocksum;     // per 1 << kSumShift units
    uint32_t *counts;                 // optional per-position counts
    pfac_match *inline_stage;         // wave kernel: inline_cap records per chunk
    uint64_t inline_cap;
    // split wave kernels: walk candidates of unit u at cand[u * cand_cap ..)
    // as {unit position | limit << 16, depth-K node, 8 text bytes after the
    // index}, their number in cand_count[u] (above cand_cap: overflowed)
    uint4 *cand;
    uint32_t *cand_count;
    uint32_t cand_cap;
    uint32_t n_sums;                  // split filter kernel: clears blocksum[0 .. n_sums) and the cursor
};

struct FinishArgs {
    const uint32_t *unit_count;
    const unsigned long long *unit_off;
    const unsigned long long *blocksum;
    const pfac_match *stage;
    uint64_t stage_cap;
    uint64_t n_tiles;
    uint32_t n_sums;                  // block-sum entries = finisher workgroups: 1 << kSumShift units each
    pfac_match *out;
    uint64_t capacity;
    uint64_t *n_matches;              // receives this launch's match count
    const unsigned long long *base_dev;  // optional device value added to every output index
    const pfac_match *inline_stage;   // units with unit_off == ~0 keep their records here
    uint64_t inline_cap;
};

// LDS bytes and section offsets for a tile of `bpl` bytes per lane.
void lds_layout(ScanArgs &a, uint32_t bpl);

hipError_t launch_reset(unsigned long long *stage_cursor, unsigned long long *blocksum,
                        uint32_t n_sums, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s);
hipError_t launch_plan(const uint64_t *offsets, uint32_t n_texts, uint64_t shift,
                       uint64_t n_tiles, uint32_t tile, uint32_t *tile_first_text,
                       uint2 *chunk_info, hipStream_t s);
hipError_t launch_scan(const ScanArgs &a, uint32_t bpl, uint32_t grid, hipStream_t s);
hipError_t launch_finish(const FinishArgs &f, hipStream_t s);
hipError_t launch_add_running(unsigned long long *running, const uint64_t *n, hipStream_t s);
hipError_t launch_copy_u64(uint64_t *dst, const unsigned long long *src, hipStream_t s);

// Wave kernel: LDS layout for `waves` waves within `lds_limit` bytes, launch,
// and occupancy.
constexpr uint32_t kWaveChunk = 1024;
constexpr uint32_t kCandPerChunk = 32;   // split kernels: candidate slots per 1 KiB chunk
constexpr uint32_t kWalkWaves = 4;       // waves per workgroup of the walk kernel
void wave_lds_layout(ScanArgs &a, uint32_t waves, uint32_t lds_limit, bool split);
int wave_mode(const ScanArgs &a);
hipError_t prepare_wave_kernel(int mode, uint32_t lds_bytes);
hipError_t launch_scan_waves(const ScanArgs &a, uint32_t waves, uint32_t grid, hipStream_t s);
hipError_t launch_walk_units(const ScanArgs &a, hipStream_t s);
int max_wave_wg_per_cu(const ScanArgs &a, uint32_t waves);

// Largest resident workgroups per CU for this layout.
int max_wg_per_cu(uint32_t bpl, uint32_t lds_bytes, int var);  // var: 0 level index, 1 top nodes, 2 DAG
hipError_t prepare_kernels(uint32_t bpl, uint32_t lds_bytes);

}  // namespace pfac
