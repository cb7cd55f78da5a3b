// Device helpers shared by the scan kernels: wave scans, the trie walk and
// match emission.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace pfac {

constexpr uint32_t kNoneD = 0xffffffffu;
constexpr uint32_t kTermFlagD = 1u << 16;

// ------------------------------------------------------------- wave helpers

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t y = __shfl_up(x, off, 64);
        if (lane >= (uint32_t)off) x += y;
    }
    return x;
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

// Walk from node v at depth d for the start position at window offset pl;
// returns the deepest terminal node passed (kNoneD if none).
__device__ __forceinline__ uint32_t walk(const ImageView &im, const uint8_t *gbase,
                                         const Tile &T, uint32_t pl, uint32_t v, uint32_t d) {
    uint32_t vt = kNoneD;
    for (;;) {
        const uint4 r = im.node[v];
        if (r.z & kTermFlagD) vt = v;
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
    return vt;
}

// Text holding frame position g (batch), by binary search over the starts.
__device__ __forceinline__ uint32_t text_of(const uint64_t *offsets, uint32_t n_texts,
                                            uint64_t shift, uint64_t g) {
    uint32_t lo = 0, hi = n_texts;  // answer in [0, n_texts)
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (offsets[mid] + shift <= g) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ uint32_t pout_count(const ImageView &im, uint32_t vt) {
    const uint32_t o = im.node[vt].w;
    return im.pout_ptr[o + 1] - im.pout_ptr[o];
}

__device__ __forceinline__ void emit(const ScanArgs &a, uint64_t frame_pos, uint32_t vt,
                                     uint64_t dst) {
    const ImageView &im = a.im;
    const uint32_t o = im.node[vt].w;
    const uint32_t p0 = im.pout_ptr[o], p1 = im.pout_ptr[o + 1];
    uint32_t tid = 0;
    uint64_t start = a.shift;
    if (a.offsets) {
        tid = text_of(a.offsets, a.n_texts, a.shift, frame_pos);
        start = a.offsets[tid] + a.shift;
    }
    tid += a.text_id0;
    const uint64_t pos = frame_pos - start;
    for (uint32_t k = p0; k < p1; k++, dst++) {
        if (dst < a.stage_cap) {
            pfac_match m;
            m.pos = pos;
            m.pattern_id = im.pout_ids[k];
            m.text_id = tid;
            a.stage[dst] = m;
        }
    }
    if (a.counts) a.counts[frame_pos - a.shift] = p1 - p0;
}

}  // namespace pfac
