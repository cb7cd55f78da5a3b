// Host-side CRS trie builder and device-image packer.
//
// Design and Implementation builds the trie breadth first, level by level
// (step I), keeps it as a row-major ordered array (step II), views it as a
// node x symbol sparse matrix (step VI) and compresses that matrix with
// compressed row storage: row_ptr per node, the symbol (edge label) as the
// column index and the child node as the value.  Steps III-V (truncation and
// suffix / end-node merging) are built only in exact forms, as optional
// device images: a truncated image keeps the pattern tails below the cut for
// verification (pack_image, tails), and the merged DAG keeps the pattern
// identities as ranks carried on its edges (build_dag).  The default image is
// the whole CRS trie, since every (position, pattern id) match is reported.
#include <algorithm>
#include <cstring>
#include <numeric>
#include <string>
#include <unordered_map>

#include "trie.hpp"

namespace pfac {

bool build_crs(const uint8_t *data, const uint64_t *off, uint32_t k, CrsTrie &T,
               std::string &err) {
    T = CrsTrie{};
    T.k = k;
    T.pat_off.assign(k + 1, 0);
    uint64_t base = k ? off[0] : 0;
    for (uint32_t j = 0; j < k; j++) {
        if (off[j + 1] < off[j]) { err = "pattern offsets decrease"; return false; }
        if (off[j + 1] == off[j]) { err = "empty pattern"; return false; }
        T.pat_off[j + 1] = off[j + 1] - base;
    }
    uint64_t total = T.pat_off[k];
    T.pat_data.assign(data ? data + base : nullptr, data ? data + base + total : nullptr);
    T.min_len = k ? UINT64_MAX : 0;
    for (uint32_t j = 0; j < k; j++) {
        uint64_t L = T.pat_off[j + 1] - T.pat_off[j];
        T.min_len = std::min(T.min_len, L);
        T.max_len = std::max(T.max_len, L);
    }
    const uint8_t *P = T.pat_data.data();
    auto len = [&](uint32_t j) { return T.pat_off[j + 1] - T.pat_off[j]; };
    auto at = [&](uint32_t j, uint64_t d) { return P[T.pat_off[j] + d]; };

    // Lexicographic order (unsigned bytes); a proper prefix sorts before its
    // extensions; equal patterns by id.  Every trie node is then a contiguous
    // run of this order, and its children are consecutive sub-runs.
    std::vector<uint32_t> ord(k);
    std::iota(ord.begin(), ord.end(), 0u);
    std::sort(ord.begin(), ord.end(), [&](uint32_t a, uint32_t b) {
        uint64_t la = len(a), lb = len(b);
        int c = std::memcmp(P + T.pat_off[a], P + T.pat_off[b], std::min(la, lb));
        if (c != 0) return c < 0;
        if (la != lb) return la < lb;
        return a < b;
    });

    struct Run { uint32_t a, b; };
    std::vector<Run> cur{{0, k}}, nxt;
    T.row_ptr.push_back(0);
    T.term_ptr.push_back(0);
    T.level_start.push_back(0);
    T.rep.push_back(kNone);
    uint64_t depth = 0;
    while (!cur.empty()) {
        nxt.clear();
        for (const Run &r : cur) {
            uint32_t a = r.a;
            // patterns that end here come first in the run
            while (a < r.b && len(ord[a]) == depth) T.term_ids.push_back(ord[a++]);
            T.term_ptr.push_back((uint32_t)T.term_ids.size());
            while (a < r.b) {
                uint8_t c = at(ord[a], depth);
                uint32_t e = a + 1;
                while (e < r.b && at(ord[e], depth) == c) e++;
                T.labels.push_back(c);
                T.rep.push_back(ord[a]);
                nxt.push_back({a, e});
                a = e;
            }
            T.row_ptr.push_back((uint32_t)T.labels.size());
        }
        T.level_start.push_back(T.level_start.back() + (uint32_t)cur.size());
        cur.swap(nxt);
        depth++;
    }
    return true;
}

static uint32_t ceil_log2(uint32_t x) {
    uint32_t b = 0;
    while ((1u << b) < x) b++;
    return b;
}

static void pack_core(const CrsTrie &T, uint32_t index_bits, uint32_t fold_bits, uint32_t trunc_depth,
                      DeviceImageHost &I) {
    I = DeviceImageHost{};
    const uint32_t N = T.n_nodes();
    const uint32_t E = T.n_edges();
    // truncation applies when some node lies deeper than trunc_depth
    const uint32_t D = (trunc_depth >= 1 && T.level_start.size() > (size_t)trunc_depth + 2) ? trunc_depth : 0u;

    // node records and terminal ordinals
    I.node.assign(4ull * N, 0);
    std::vector<uint32_t> ord_of(N, kNone);
    for (uint32_t v = 0; v < N; v++)
        if (T.term_ptr[v + 1] > T.term_ptr[v]) ord_of[v] = I.n_term++;
    for (uint32_t v = 0; v < N; v++) {
        uint32_t e0 = T.row_ptr[v], nc = T.row_ptr[v + 1] - e0;
        uint32_t x = 0;
        for (uint32_t j = 0; j < 4; j++) {
            // unused bytes repeat the last label; the kernel ignores j >= nc
            uint32_t lab = nc ? T.labels[e0 + std::min(j, nc - 1)] : 0;
            x |= lab << (8 * j);
        }
        I.node[4 * v + 0] = x;
        I.node[4 * v + 1] = e0 + 1;
        I.node[4 * v + 2] = nc | (ord_of[v] != kNone ? kTermFlag : 0);
        I.node[4 * v + 3] = kNone;
    }
    I.label = T.labels;
    if (I.label.empty()) I.label.push_back(0);

    // Path compression for the walk: a maximal run u_0 -> u_1 -> ... -> u_s
    // of non-terminal single-child nodes ending at w = u_s stores its labels
    // once in `chain`; every u_i with at least two labels left becomes a skip
    // node (x = offset of its remaining labels, z = 1 | kSkipFlag | len << 18,
    // w = the node reached after len labels).  No pattern ends strictly
    // inside the run, so comparing the text with the stored labels in bulk
    // reaches the same node as walking them one by one, and a mismatch ends
    // the walk with nothing reported.  (A truncated image walks node by
    // node: no run may cross the truncation depth.)
    if (D) I.chain.assign(40, 0);
    if (!D) {
        std::vector<uint32_t> parent0(N, kNone);
        for (uint32_t v = 0; v < N; v++)
            for (uint32_t e = T.row_ptr[v]; e < T.row_ptr[v + 1]; e++) parent0[e + 1] = v;
        auto chain_node = [&](uint32_t v) {
            return T.row_ptr[v + 1] - T.row_ptr[v] == 1 && T.term_ptr[v + 1] == T.term_ptr[v];
        };
        std::vector<uint32_t> run;
        for (uint32_t v = 0; v < N; v++) {
            if (!chain_node(v)) continue;
            if (v != 0 && chain_node(parent0[v])) continue;  // not the top of its run
            run.assign(1, v);
            const uint32_t off0 = (uint32_t)I.chain.size();
            uint32_t u = v;
            while (chain_node(u)) {
                const uint32_t e = T.row_ptr[u];
                I.chain.push_back(T.labels[e]);
                u = e + 1;
                run.push_back(u);
            }
            const uint32_t s = (uint32_t)run.size() - 1;
            for (uint32_t i = 0; i + 2 <= s; i++) {
                const uint32_t len = std::min(s - i, kSkipMax);
                uint32_t *rec = &I.node[4ull * run[i]];
                rec[0] = off0 + i;
                rec[2] = 1u | kSkipFlag | (len << kSkipShift);
                rec[3] = run[i + len];
            }
        }
        I.chain.resize(I.chain.size() + 40, 0);  // the kernels read whole words past the end
    }

    // Root-path pattern lists of terminal nodes: for a terminal node t, the
    // ascending ids of every pattern that ends on the path from the root to t
    // (t's own ids merged with the list of its nearest terminal ancestor).  A
    // walk reports the list of the deepest terminal node it passed.  The
    // record of t holds the list's offset (w) and length (z bits 18..31); a
    // length of kCountEsc or more is stored as kCountEsc and the true length
    // precedes the ids.
    std::vector<uint32_t> parent(N, kNone), near_term(N, kNone);
    for (uint32_t v = 0; v < N; v++)
        for (uint32_t e = T.row_ptr[v]; e < T.row_ptr[v + 1]; e++) parent[e + 1] = v;
    std::vector<uint32_t> list_at(N, kNone), list_len(N, 0);
    std::vector<uint32_t> tmp;
    for (uint32_t v = 1; v < N; v++) {
        const uint32_t up = near_term[parent[v]];
        if (ord_of[v] == kNone) { near_term[v] = up; continue; }
        near_term[v] = v;
        const uint32_t *own = T.term_ids.data() + T.term_ptr[v];
        const uint32_t n_own = T.term_ptr[v + 1] - T.term_ptr[v];
        tmp.clear();
        if (up != kNone) {
            const uint32_t *anc = I.pout_ids.data() + list_at[up];
            const uint32_t n_anc = list_len[up];
            tmp.resize(n_own + n_anc);
            std::merge(own, own + n_own, anc, anc + n_anc, tmp.begin());
        } else {
            tmp.assign(own, own + n_own);
        }
        const uint32_t n = (uint32_t)tmp.size();
        uint32_t *rec = &I.node[4ull * v];
        rec[3] = (uint32_t)I.pout_ids.size();
        if (n >= kCountEsc) {
            I.pout_ids.push_back(n);
            rec[2] |= kCountEsc << kCountShift;
        } else {
            rec[2] |= n << kCountShift;
        }
        list_at[v] = (uint32_t)I.pout_ids.size();
        list_len[v] = n;
        I.pout_ids.insert(I.pout_ids.end(), tmp.begin(), tmp.end());
    }
    I.pout_ptr.assign(1, 0);
    if (I.pout_ids.empty()) I.pout_ids.push_back(0);

    // A run that ends at a leaf: its skip nodes carry the leaf's pattern list
    // instead of the leaf's id (x bits 24..31 its length, w its offset, z
    // kLeafEnd), so a walk that matches the run ends without reading the
    // leaf's record.
    if (!D) {
        for (uint32_t v = 0; v < N; v++) {
            uint32_t *rec = &I.node[4ull * v];
            if (!(rec[2] & kSkipFlag)) continue;
            const uint32_t *end = &I.node[4ull * rec[3]];
            const uint32_t n = end[2] >> kCountShift;
            if ((end[2] & kNcMask) != 0 || !(end[2] & kTermFlag) || n >= 255 || rec[0] >= (1u << 24))
                continue;
            rec[0] |= n << 24;
            rec[2] |= kLeafEnd;
            rec[3] = end[3];
        }
    }

    // Truncation (Design and Implementation, step III) kept exact: only the
    // nodes of depths 0..D stay; a depth-D node with children becomes a tail
    // node whose record lists every terminal node below it (its pattern's
    // bytes after depth D, their count, and the node's root-path pattern
    // list), longest first.  The walk compares the text with each in turn;
    // the first one equal gives the list of every pattern matching there.
    if (D) {
        I.trunc_depth = D;
        const uint32_t t0 = T.level_start[D], t1 = T.level_start[D + 1];
        std::vector<uint32_t> anc(N, kNone);  // depth-D ancestor of deeper nodes
        std::vector<std::vector<std::pair<uint32_t, uint32_t>>> under(t1 - t0);  // (depth, node)
        for (size_t d = D + 1; d + 1 < T.level_start.size(); d++) {
            for (uint32_t v = T.level_start[d]; v < T.level_start[d + 1]; v++) {
                const uint32_t p = parent[v];
                anc[v] = d == D + 1 ? p : anc[p];
                if (ord_of[v] != kNone) under[anc[v] - t0].push_back({(uint32_t)d, v});
            }
        }
        for (uint32_t t = t0; t < t1; t++) {
            if (T.row_ptr[t + 1] == T.row_ptr[t]) continue;  // a leaf: nothing below
            auto &L = under[t - t0];
            std::sort(L.begin(), L.end(), [](const std::pair<uint32_t, uint32_t> &x,
                                             const std::pair<uint32_t, uint32_t> &y) {
                return x.first != y.first ? x.first > y.first : x.second < y.second;
            });
            uint32_t *rec = &I.node[4ull * t];
            rec[0] = 1u + (uint32_t)(I.tail.size() / 4);
            rec[1] = (uint32_t)L.size();
            rec[2] &= ~kNcMask;
            for (const auto &dv : L) {
                const uint32_t v = dv.second, len = dv.first - D;
                const uint8_t *pb = T.pat_data.data() + T.pat_off[T.rep[v]];
                I.tail.push_back((uint32_t)I.tail_bytes.size());
                I.tail.push_back(len);
                I.tail.push_back(I.node[4ull * v + 3]);
                I.tail.push_back(I.node[4ull * v + 2] >> kCountShift);
                I.tail_bytes.insert(I.tail_bytes.end(), pb + D, pb + dv.first);
            }
        }
        I.node.resize(4ull * t1);
        I.label.resize(std::max<size_t>(1, t1 - 1));
    }
    I.tail_bytes.resize(I.tail_bytes.size() + 40, 0);  // the kernels read whole words past the end

    // alphabet and level index
    bool used[256] = {false};
    for (uint32_t e = 0; e < E; e++) used[T.labels[e]] = true;
    for (int c = 0; c < 256; c++) I.alphabet += used[c];
    index_bits = std::max(1u, std::min(index_bits, 18u));
    uint32_t b_comp = std::max(1u, ceil_log2(std::max(I.alphabet, 1u)));
    uint32_t depth = (uint32_t)T.max_len;
    uint32_t k_cap = T.k ? (uint32_t)std::min<uint64_t>(T.min_len - 1, depth) : 0;
    k_cap = std::min(k_cap, 12u);
    if (D) k_cap = std::min(k_cap, D);  // the index's nodes must stay in the image
    uint32_t K8 = std::min(index_bits / 8, k_cap);
    uint32_t Kc = std::min(index_bits / b_comp, k_cap);
    I.sym.assign(256, 0xff);
    if (Kc > K8 && b_comp < 8) {
        I.identity = 0;
        I.b = b_comp;
        I.K = Kc;
        uint32_t s = 0;
        for (int c = 0; c < 256; c++)
            if (used[c]) I.sym[c] = (uint8_t)s++;
    } else {
        I.identity = 1;
        I.b = 8;
        I.K = K8;
        for (int c = 0; c < 256; c++) I.sym[c] = (uint8_t)c;
    }
    // codes of the root's children (the filter when K = 0)
    I.root_bits.assign(std::max(1u, (1u << I.b) / 32), 0);
    for (uint32_t e = T.row_ptr[0]; e < T.row_ptr[1]; e++) {
        const uint32_t s = I.sym[T.labels[e]];
        I.root_bits[s >> 5] |= 1u << (s & 31);
    }
    if (I.K == 0) {
        I.lvl_words = 0;
        I.lvl_start = 0;
        return;
    }
    uint32_t code_bits = I.b * I.K;
    uint64_t n_codes = 1ull << code_bits;
    I.lvl_words = (uint32_t)std::max<uint64_t>(1, n_codes / 32);
    I.lvl.assign(2ull * I.lvl_words, 0);
    I.lvl_start = T.level_start[I.K];
    const uint32_t v0 = T.level_start[I.K], v1 = T.level_start[I.K + 1];
    for (uint32_t v = v0; v < v1; v++) {
        const uint8_t *p = T.pat_data.data() + T.pat_off[T.rep[v]];
        uint32_t code = 0;
        for (uint32_t d = 0; d < I.K; d++) code = (code << I.b) | I.sym[p[d]];
        I.lvl[2 * (code >> 5)] |= 1u << (code & 31);
    }
    uint32_t run = 0;
    for (uint32_t w = 0; w < I.lvl_words; w++) {
        I.lvl[2 * w + 1] = run;
        run += (uint32_t)__builtin_popcount(I.lvl[2 * w]);
    }
    // the same K levels as bitmapped nodes: node v < lvl_start holds the
    // bitmap of its children's symbols and the id of its first child
    I.top_rw = std::max(1u, (1u << I.b) / 32) + 1;
    I.top_nodes = I.lvl_start;
    I.top.assign((size_t)I.top_nodes * I.top_rw, 0);
    for (uint32_t v = 0; v < I.top_nodes; v++) {
        uint32_t *rec = &I.top[(size_t)v * I.top_rw];
        for (uint32_t e = T.row_ptr[v]; e < T.row_ptr[v + 1]; e++) {
            const uint32_t s = I.sym[T.labels[e]];
            rec[s >> 5] |= 1u << (s & 31);
        }
        rec[I.top_rw - 1] = T.row_ptr[v] + 1;
    }
    I.krec.assign(v1 - v0, 0);
    for (uint32_t v = v0; v < v1; v++) {
        const uint32_t e0 = T.row_ptr[v], nc = T.row_ptr[v + 1] - e0;
        uint32_t rec = (nc <= 3 ? nc : 0xffu) << 24;
        for (uint32_t j = 0; j < 3; j++) {
            // unused slots repeat the last label; the kernel ignores j >= count
            const uint32_t lab = nc ? T.labels[e0 + std::min(j, nc - 1)] : 0;
            rec |= lab << (8 * j);
        }
        I.krec[v - v0] = rec;
    }

    // prefix-4 filter: about 16 bits per distinct 4-byte prefix, 2^10..2^18
    I.pfx4_log2 = 0;
    I.pfx4.clear();
    if (I.identity && T.k && T.min_len >= 4 && T.level_start.size() > 5) {
        const uint32_t n4 = T.level_start[5] - T.level_start[4];  // depth-4 nodes
        uint32_t lg = 10;
        while (lg < 18 && (1ull << lg) < 16ull * n4) lg++;
        I.pfx4_log2 = lg;
        I.pfx4.assign((1u << lg) / 32, 0);
        for (uint32_t v = T.level_start[4]; v < T.level_start[5]; v++) {
            const uint8_t *p = T.pat_data.data() + T.pat_off[T.rep[v]];
            const uint32_t x = (uint32_t)p[0] | (uint32_t)p[1] << 8 | (uint32_t)p[2] << 16 |
                               (uint32_t)p[3] << 24;
            const uint32_t h1 = (x & 0xffffffu) * kPfx4M1 + (x >> 8);
            const uint32_t h2 = (x >> 8) * kPfx4M2 + x;
            I.pfx4[h1 >> (37 - lg)] |= (1u << ((h1 >> (32 - lg)) & 31)) | (1u << (h2 >> 27));
        }
    }

    // four-symbol filter over the 16-symbol prefixes
    I.q16_lw = I.qfp_lb = 0;
    I.q16.clear();
    I.qfp.clear();
    if (!I.identity && I.b == 2 && T.k && T.min_len >= 16 && T.level_start.size() > 17) {
        std::vector<uint8_t> alph;
        for (int c = 0; c < 256; c++)
            if (used[c]) alph.push_back((uint8_t)c);
        bool found = false;
        for (uint32_t qa = 0; qa <= 6 && !found; qa++)
            for (uint32_t qb = qa + 1; qb <= 6 && !found; qb++) {
                bool ok = true;
                for (size_t i = 0; i < alph.size() && ok; i++)
                    ok = (((alph[i] >> qa) ^ (alph[i] >> qb)) & 3u) == i;
                if (ok) {
                    found = true;
                    I.qa = qa;
                    I.qb = qb;
                }
            }
        if (found) {
            // unused symbols get a byte that maps to another symbol
            I.qalph = 0;
            for (uint32_t i = 0; i < 4; i++) {
                const uint32_t c = i < alph.size() ? alph[i] : alph[0];
                I.qalph |= c << (8 * i);
            }
            const uint32_t v0 = T.level_start[16], v1 = T.level_start[17];
            const uint64_t n16 = v1 - v0;
            uint32_t lg = 10;  // bits of the bitmap: about 10.5 per key, at most 2^20
            while (lg < 20 && (1ull << lg) < 10ull * n16 + n16 / 2) lg++;
            I.q16_lw = lg - 5;
            I.q16.assign(1u << I.q16_lw, 0);
            uint32_t lb = 0;  // buckets of 8: about two keys each
            while ((1ull << lb) * 2 < n16) lb++;
            I.qfp_lb = std::max(lb, 1u);
            const uint32_t nb = 1u << I.qfp_lb;
            I.qfp.assign((size_t)nb * 8, 0);
            bool fp_ok = true;
            for (uint32_t v = v0; v < v1; v++) {
                const uint8_t *p = T.pat_data.data() + T.pat_off[T.rep[v]];
                uint32_t key = 0;
                for (uint32_t i = 0; i < 16; i++) key |= (uint32_t)I.sym[p[i]] << (2 * i);
                const uint32_t h = (uint32_t)((uint64_t)(key & 0xffffffu) * kQ16Mul + (key >> 8));
                const uint32_t wd = h >> (32 - I.q16_lw);
                I.q16[wd] |= (1u << (h & 31)) | (1u << ((h >> 5) & 31));
                const uint32_t h2 = key * kPfx4Mul;
                const uint32_t b = h2 >> (32 - I.qfp_lb);
                const uint16_t fp = (uint16_t)((h2 & 0xffffu) | 1u);
                bool put = false;
                for (uint32_t q = 0; q < 2 && !put; q++) {
                    uint16_t *bk = I.qfp.data() + (size_t)((b + q) & (nb - 1)) * 8;
                    for (uint32_t s = 0; s < 8 && !put; s++)
                        if (bk[s] == 0 || bk[s] == fp) {
                            bk[s] = fp;
                            put = true;
                        }
                }
                fp_ok = fp_ok && put;
            }
            if (!fp_ok) {  // two full buckets: no fingerprint stage
                I.qfp_lb = 0;
                I.qfp.clear();
            }
        }
    }

    // prefix filter over the depth-(K+m) nodes
    if (fold_bits != 8 && fold_bits != 16) return;
    const uint32_t log2e = fold_bits == 8 ? 3 : 4;
    uint32_t m = std::max(1u, log2e / I.b);
    m = (uint32_t)std::min<uint64_t>(std::min(m, 4u), T.min_len - I.K);
    if (I.K + m + 1 > T.level_start.size()) return;
    I.fold_bits = fold_bits;
    I.fold_syms = m;
    I.ftab.assign((size_t)n_codes * (fold_bits / 8), 0);
    const uint32_t d = I.K + m;
    const uint32_t w0 = T.level_start[d], w1 = T.level_start[d + 1];
    for (uint32_t w = w0; w < w1; w++) {
        const uint8_t *p = T.pat_data.data() + T.pat_off[T.rep[w]];
        uint32_t code = 0, next = 0;
        for (uint32_t q = 0; q < I.K; q++) code = (code << I.b) | I.sym[p[q]];
        for (uint32_t q = I.K; q < d; q++) next = (next << I.b) | I.sym[p[q]];
        const uint32_t bit = next & (fold_bits - 1);
        if (fold_bits == 8)
            I.ftab[code] |= (uint8_t)(1u << bit);
        else
            reinterpret_cast<uint16_t *>(I.ftab.data())[code] |= (uint16_t)(1u << bit);
    }
}

// Suffix and end-node merging (Design and Implementation, steps IV and V):
// trie nodes whose subtries are equal (same terminal flag, same labels to
// equal subtries) become one DAG node, so all leaves become a single end node
// and equal suffixes are stored once.  Pattern identities survive on the
// edges: each edge adds the number of distinct pattern strings that sort
// before its subtrie among its parent's (the parent's own string, then the
// subtries of smaller labels), so a walk sums to the rank of the string it
// spells, and rank_list[rank] gives that string's root-path pattern list.
// Equivalence classes of trie nodes (equal subtries), children first
// (breadth-first ids: children are larger); per class a trie node of it and
// the number of distinct pattern strings in its subtrie.
static void dag_classes(const CrsTrie &T, std::vector<uint32_t> &cls, std::vector<uint32_t> &cls_rep,
                        std::vector<uint32_t> &cls_strings) {
    const uint32_t N = T.n_nodes();
    auto term = [&](uint32_t v) -> uint32_t { return T.term_ptr[v + 1] > T.term_ptr[v] ? 1u : 0u; };
    cls.assign(N, 0);
    cls_rep.clear();
    cls_strings.clear();
    std::unordered_map<std::string, uint32_t> seen;
    seen.reserve(N);
    std::string key;
    for (uint32_t v = N; v-- > 0;) {
        key.assign(1, (char)term(v));
        uint32_t strings = term(v);
        for (uint32_t e = T.row_ptr[v]; e < T.row_ptr[v + 1]; e++) {
            const uint32_t c = cls[e + 1];
            key.push_back((char)T.labels[e]);
            key.append((const char *)&c, 4);
            strings += cls_strings[c];
        }
        auto it = seen.find(key);
        if (it == seen.end()) {
            const uint32_t id = (uint32_t)cls_rep.size();
            seen.emplace(key, id);
            cls_rep.push_back(v);
            cls_strings.push_back(strings);
            cls[v] = id;
        } else {
            cls[v] = it->second;
        }
    }
}

void dag_size(const CrsTrie &T, uint64_t &nodes, uint64_t &edges) {
    std::vector<uint32_t> cls, rep, strings;
    dag_classes(T, cls, rep, strings);
    nodes = rep.size();
    edges = 0;
    for (uint32_t v : rep) edges += T.row_ptr[v + 1] - T.row_ptr[v];
}

static void build_dag(const CrsTrie &T, DeviceImageHost &I) {
    const uint32_t N = T.n_nodes();
    auto term = [&](uint32_t v) -> uint32_t { return T.term_ptr[v + 1] > T.term_ptr[v] ? 1u : 0u; };
    std::vector<uint32_t> cls, cls_rep, cls_strings;
    dag_classes(T, cls, cls_rep, cls_strings);
    // DAG nodes numbered breadth first from the root's class
    std::vector<uint32_t> newid(cls_rep.size(), kNone), order;
    newid[cls[0]] = 0;
    order.push_back(cls[0]);
    for (size_t i = 0; i < order.size(); i++) {
        const uint32_t v = cls_rep[order[i]];
        for (uint32_t e = T.row_ptr[v]; e < T.row_ptr[v + 1]; e++) {
            const uint32_t c = cls[e + 1];
            if (newid[c] == kNone) {
                newid[c] = (uint32_t)order.size();
                order.push_back(c);
            }
        }
    }
    I.dag = 1;
    I.dnode.assign(4 * order.size(), 0);
    I.dlabel.clear();
    I.dchild.clear();
    I.dradd.clear();
    for (size_t i = 0; i < order.size(); i++) {
        const uint32_t v = cls_rep[order[i]];
        const uint32_t e0 = T.row_ptr[v], nc = T.row_ptr[v + 1] - e0;
        uint32_t x = 0;
        for (uint32_t j = 0; j < 4; j++) x |= (uint32_t)(nc ? T.labels[e0 + std::min(j, nc - 1)] : 0) << (8 * j);
        I.dnode[4 * i + 0] = x;
        I.dnode[4 * i + 1] = (uint32_t)I.dlabel.size();
        I.dnode[4 * i + 2] = nc | (term(v) ? kTermFlag : 0u);
        uint32_t run = term(v);
        for (uint32_t e = e0; e < e0 + nc; e++) {
            I.dlabel.push_back(T.labels[e]);
            I.dchild.push_back(newid[cls[e + 1]]);
            I.dradd.push_back(run);
            run += cls_strings[cls[e + 1]];
        }
    }
    // rank of every trie node's string (parents before children)
    std::vector<uint32_t> R(N, 0);
    for (uint32_t v = 0; v < N; v++) {
        uint32_t run = R[v] + term(v);
        for (uint32_t e = T.row_ptr[v]; e < T.row_ptr[v + 1]; e++) {
            R[e + 1] = run;
            run += cls_strings[cls[e + 1]];
        }
    }
    const uint32_t S = N ? cls_strings[cls[0]] : 0;
    I.rank_list.assign(2ull * std::max(S, 1u), 0);
    for (uint32_t v = 0; v < N; v++) {
        if (!term(v)) continue;
        I.rank_list[2ull * R[v]] = I.node[4ull * v + 3];
        I.rank_list[2ull * R[v] + 1] = I.node[4ull * v + 2] >> kCountShift;
    }
    // the level index's depth-K nodes as (DAG node, rank so far)
    I.lvl_dag.clear();
    if (I.K) {
        for (uint32_t v = T.level_start[I.K]; v < T.level_start[I.K + 1]; v++) {
            I.lvl_dag.push_back(newid[cls[v]]);
            I.lvl_dag.push_back(R[v]);
        }
    }
    if (I.dlabel.empty()) {
        I.dlabel.push_back(0);
        I.dchild.push_back(0);
        I.dradd.push_back(0);
    }
    // the trie's own node records are not read by the DAG walk
    I.node.assign(4, 0);
    I.label.assign(1, 0);
    I.chain.assign(40, 0);
}

void pack_image(const CrsTrie &T, uint32_t index_bits, uint32_t fold_bits, uint32_t trunc_depth,
                uint32_t dag, DeviceImageHost &I) {
    pack_core(T, index_bits, fold_bits, dag ? 0u : trunc_depth, I);
    if (dag) build_dag(T, I);
}

}  // namespace pfac
