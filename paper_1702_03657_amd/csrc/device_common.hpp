// Device helpers shared by the scan kernels: wave scans, the trie walk and
// match emission.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace pfac {

constexpr uint32_t kNoneD = 0xffffffffu;
constexpr uint32_t kTermFlagD = 1u << 16;
constexpr uint32_t kSkipFlagD = 1u << 17;
constexpr uint32_t kSkipShiftD = 18;
constexpr uint32_t kLeafEndD = 1u << 15;
constexpr uint32_t kCountShiftD = 18;
constexpr uint32_t kCountEscD = (1u << 14) - 1;

// ------------------------------------------------------------- wave helpers

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63; }

// x moved by a DPP control: lanes with no source lane, or masked off by
// row_mask / bank_mask, read 0.
template <int CTRL, int ROW_MASK, int BANK_MASK>
__device__ __forceinline__ uint32_t dpp_or0(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROW_MASK, BANK_MASK, false);
}

// Inclusive prefix sum over the 64 lanes with DPP moves only (no LDS):
// shifts by 1, 2, 3 inside each row of 16 lanes, then 4 and 8 over banks of
// 4 lanes, then the last lane of rows 0 and 2 into rows 1 and 3
// (row_bcast:15) and lane 31 into rows 2 and 3 (row_bcast:31).  Every lane
// of the wave must be active.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    uint32_t v = x;
    v += dpp_or0<0x111, 0xf, 0xf>(x);
    v += dpp_or0<0x112, 0xf, 0xf>(x);
    v += dpp_or0<0x113, 0xf, 0xf>(x);
    v += dpp_or0<0x114, 0xf, 0xe>(v);
    v += dpp_or0<0x118, 0xf, 0xc>(v);
    v += dpp_or0<0x142, 0xa, 0xf>(v);
    v += dpp_or0<0x143, 0xc, 0xf>(v);
    return v;
}

// Value of lane 63 in every lane (a scalar read).
__device__ __forceinline__ uint32_t wave_last(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

__device__ __forceinline__ unsigned long long wave_reduce_u64(unsigned long long x) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// Exclusive scan over the workgroup in thread order; `tmp` holds kWG/64 words.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t *tmp, uint32_t &total) {
    const uint32_t w = threadIdx.x >> 6;
    uint32_t incl = wave_incl_scan(x);
    if (lane_id() == 63) tmp[w] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (uint32_t i = 0; i < kWG / 64; i++) {
        uint32_t s = tmp[i];
        before += (i < w) ? s : 0;
        all += s;
    }
    __syncthreads();
    total = all;
    return before + incl - x;
}

// ------------------------------------------------------------------ the walk

struct Tile {
    const uint8_t *text;      // LDS copy of the window
    const uint32_t *bnd;      // LDS boundary bits of the window
    uint64_t lo;              // frame position of window byte 0
    uint32_t win;             // window bytes in LDS
    bool dirty;               // some boundary lies in the window
    uint64_t next_bnd;        // first boundary at or after the window end
};

// True when text[q .. q+len) (LDS window) equals chain[o .. o+len) (global).
// Both sides are read as aligned words and realigned with alignbyte; eight
// chain words are requested before any is compared, so a run costs about one
// memory round trip per 32 bytes.
__device__ __forceinline__ bool chain_equal(const uint8_t *text, uint32_t q, const uint8_t *chain,
                                            uint32_t o, uint32_t len) {
    const uint32_t *t32 = (const uint32_t *)text;
    const uint32_t *c32 = (const uint32_t *)chain;
    uint32_t diff = 0;
    for (uint32_t i = 0; i < len; i += 32) {
        uint32_t cw[9], tw[9];
        const uint32_t cb = (o + i) >> 2, tb = (q + i) >> 2;
#pragma unroll
        for (int k = 0; k < 9; k++) cw[k] = c32[cb + k];
#pragma unroll
        for (int k = 0; k < 9; k++) tw[k] = t32[tb + k];
        const uint32_t cs = (o + i) & 3, ts = (q + i) & 3;
#pragma unroll
        for (int k = 0; k < 8; k++) {
            const uint32_t rem = len - i - 4 * k;  // may wrap: masked below
            const int32_t r = (int32_t)(len - i) - 4 * k;
            const uint32_t mask = r >= 4 ? 0xffffffffu : (r <= 0 ? 0u : ((1u << (8 * rem)) - 1u));
            const uint32_t c = __builtin_amdgcn_alignbyte(cw[k + 1], cw[k], cs);
            const uint32_t t = __builtin_amdgcn_alignbyte(tw[k + 1], tw[k], ts);
            diff |= (c ^ t) & mask;
        }
    }
    return diff == 0;
}

// True when no boundary bit is set in [a, b) of the window bit map.
__device__ __forceinline__ bool range_clear(const uint32_t *bnd, uint32_t a, uint32_t b) {
    uint32_t any = 0;
    for (uint32_t w = a >> 5; w <= ((b - 1) >> 5) && a < b; w++) {
        uint32_t m = 0xffffffffu;
        if (w == (a >> 5)) m &= 0xffffffffu << (a & 31);
        if (w == ((b - 1) >> 5)) m &= 0xffffffffu >> (31 - ((b - 1) & 31));
        any |= bnd[w] & m;
    }
    return any == 0;
}

// Tail node of a truncated image: the text from window offset q on against
// the node's entries, longest first; the first equal one gives the pattern
// list of the walk, else `hit` (the deepest terminal node above) stands.
__device__ __forceinline__ uint2 verify_tails(const ImageView &im, const uint8_t *gbase,
                                              const Tile &T, uint32_t q, uint32_t first,
                                              uint32_t count, uint2 hit) {
    for (uint32_t i = 0; i < count; i++) {
        const uint4 e = im.tail[first + i];
        const uint32_t len = e.y;
        bool eq;
        if (q + len <= T.win) {
            // in the window, with no text boundary inside
            eq = (!T.dirty || range_clear(T.bnd, q, q + len)) &&
                 chain_equal(T.text, q, im.tail_bytes, e.x, len);
        } else {
            // past the window: the next boundary must not fall inside
            eq = (q >= T.win || !T.dirty || range_clear(T.bnd, q, T.win)) &&
                 T.lo + q + len <= T.next_bnd;
            for (uint32_t b = 0; b < len && eq; b++) {
                const uint32_t c = q + b < T.win ? (uint32_t)T.text[q + b] : (uint32_t)gbase[T.lo + q + b];
                eq = c == im.tail_bytes[e.x + b];
            }
        }
        if (eq) return make_uint2(e.z, e.w);
    }
    return hit;
}

// Walk from node v at depth d for the start position at window offset pl.
// Returns the pattern list of the deepest terminal node passed as
// (offset, stored length); length 0 means no pattern ends on the walk.
__device__ __forceinline__ uint2 walk(const ImageView &im, const uint8_t *gbase,
                                      const Tile &T, uint32_t pl, uint32_t v, uint32_t d) {
    uint2 hit = make_uint2(0, 0);
    for (;;) {
        const uint4 r = im.node[v];
        if (r.z & kTermFlagD) hit = make_uint2(r.w, r.z >> kCountShiftD);
        const uint32_t nc = r.z & 0xffffu;
        if (nc == 0) {
            if (r.x) hit = verify_tails(im, gbase, T, pl + d, r.x - 1, r.y, hit);
            break;
        }
        const uint32_t q = pl + d;
        const bool skip = (r.z & kSkipFlagD) != 0;
        if (skip) {
            // compressed run: compare its labels with the text in bulk when
            // they lie in the window and no text boundary falls inside them
            const uint32_t len = r.z >> kSkipShiftD;
            if (q + len <= T.win && (!T.dirty || range_clear(T.bnd, q + (d == 0), q + len))) {
                const bool leaf = (r.z & kLeafEndD) != 0;
                if (!chain_equal(T.text, q, im.chain, leaf ? r.x & 0xffffffu : r.x, len)) break;
                if (leaf) {
                    // the run ends at a leaf: its pattern list is in the record
                    hit = make_uint2(r.w, r.x >> 24);
                    break;
                }
                v = r.w;
                d += len;
                continue;
            }
        }
        uint32_t c;
        if (q < T.win) {
            // a boundary at q > pl starts the next text; at q == pl it starts this one
            if (T.dirty && d != 0 && ((T.bnd[q >> 5] >> (q & 31)) & 1u)) break;
            c = T.text[q];
        } else {
            const uint64_t g = T.lo + q;
            if (g >= T.next_bnd) break;
            c = gbase[g];
        }
        uint32_t j;
        if (skip) {
            if (c != im.label[r.y - 1]) break;
            j = 0;
        } else if (nc <= 4) {
            const uint32_t x = r.x ^ (c * 0x01010101u);
            const uint32_t m = (x - 0x01010101u) & ~x & 0x80808080u;  // lowest flag = first zero byte
            if (m == 0) break;
            j = (uint32_t)__builtin_ctz(m) >> 3;
            if (j >= nc) break;
        } else {
            const uint8_t *lab = im.label + (r.y - 1);
            uint32_t lo = 0, hi = nc;
            while (lo < hi) {
                uint32_t mid = (lo + hi) >> 1;
                if (lab[mid] < c) lo = mid + 1; else hi = mid;
            }
            if (lo == nc || lab[lo] != c) break;
            j = lo;
        }
        v = r.y + j;
        d++;
    }
    return hit;
}

// Walk of the merged DAG from DAG node v at depth d with rank R so far: each
// edge taken adds its rank, and the rank at the deepest terminal node passed
// names the pattern string whose root-path pattern list is returned (length
// 0: no pattern ends on the walk).
__device__ __forceinline__ uint2 walk_dag(const ImageView &im, const uint8_t *gbase,
                                          const Tile &T, uint32_t pl, uint32_t v, uint32_t R,
                                          uint32_t d) {
    uint32_t last = kNoneD;
    for (;;) {
        const uint4 r = im.dnode[v];
        if (r.z & kTermFlagD) last = R;
        const uint32_t nc = r.z & 0xffffu;
        if (nc == 0) break;
        const uint32_t q = pl + d;
        uint32_t c;
        if (q < T.win) {
            // a boundary at q > pl starts the next text; at q == pl it starts this one
            if (T.dirty && d != 0 && ((T.bnd[q >> 5] >> (q & 31)) & 1u)) break;
            c = T.text[q];
        } else {
            const uint64_t g = T.lo + q;
            if (g >= T.next_bnd) break;
            c = gbase[g];
        }
        uint32_t j;
        if (nc <= 4) {
            const uint32_t x = r.x ^ (c * 0x01010101u);
            const uint32_t m = (x - 0x01010101u) & ~x & 0x80808080u;  // lowest flag = first zero byte
            if (m == 0) break;
            j = (uint32_t)__builtin_ctz(m) >> 3;
            if (j >= nc) break;
        } else {
            const uint8_t *lab = im.dlabel + r.y;
            uint32_t lo = 0, hi = nc;
            while (lo < hi) {
                uint32_t mid = (lo + hi) >> 1;
                if (lab[mid] < c) lo = mid + 1; else hi = mid;
            }
            if (lo == nc || lab[lo] != c) break;
            j = lo;
        }
        R += im.dradd[r.y + j];
        v = im.dchild[r.y + j];
        d++;
    }
    return last == kNoneD ? make_uint2(0, 0) : im.rank_list[last];
}

// Text holding frame position g (batch): the last text starting at or before
// g, by binary search over the starts with the answer known to be in
// [lo, hi).
__device__ __forceinline__ uint32_t text_of(const uint64_t *offsets, uint32_t lo, uint32_t hi,
                                            uint64_t shift, uint64_t g) {
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (offsets[mid] + shift <= g) lo = mid; else hi = mid;
    }
    return lo;
}

// (first id offset, number of ids) of a walk's pattern list.
__device__ __forceinline__ uint2 hit_list(const ImageView &im, uint2 h) {
    if (h.y == kCountEscD) return make_uint2(h.x + 1, im.pout_ids[h.x]);
    return h;
}

// The text of a whole output unit of a batch, when one text holds it: its
// index and frame start.
struct UnitText {
    bool known = false;
    uint32_t tid = 0;
    uint64_t start = 0;
};

// Write the matches of one start position (frame position `frame_pos`, the
// pattern list `ids` = (offset, count)) to dst[idx ..], dropping records at
// or beyond `cap`; also its per-position count when requested.
__device__ __forceinline__ void emit(const ScanArgs &a, uint64_t frame_pos, uint2 ids,
                                     pfac_match *dst, uint64_t idx, uint64_t cap,
                                     const UnitText &ut = UnitText{}) {
    const ImageView &im = a.im;
    uint32_t tid = 0;
    uint64_t start = a.shift;
    if (a.offsets && ut.known) {
        tid = ut.tid;
        start = ut.start;
    } else if (a.offsets) {
        // the batch plan bounds the search: the texts holding the first
        // bytes of this plan unit and of the next one
        const uint64_t c = frame_pos >> a.plan_shift;
        const uint32_t lo = a.tile_first_text[c];
        const uint32_t hi = (c + 1 < a.n_plan ? a.tile_first_text[c + 1] : a.n_texts - 1) + 1;
        tid = text_of(a.offsets, lo, hi, a.shift, frame_pos);
        start = a.offsets[tid] + a.shift;
    }
    tid += a.text_id0;
    const uint64_t pos = frame_pos - start;
    for (uint32_t k = 0; k < ids.y; k++, idx++) {
        if (idx < cap) {
            pfac_match m;
            m.pos = pos;
            m.pattern_id = im.pout_ids[ids.x + k];
            m.text_id = tid;
            dst[idx] = m;
        }
    }
    if (a.counts) a.counts[frame_pos - a.shift] = ids.y;
}

}  // namespace pfac
