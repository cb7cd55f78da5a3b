// Scan kernels for gfx950: the failure-less Aho-Corasick walk of Background,
// "Parallel Failure-Less Aho-Corasick" over the CRS trie of Design and
// Implementation.
//
// Work decomposition.  The texts form one byte frame starting at a 16-byte
// aligned address.  A tile is kWG * BPL consecutive start positions; a
// persistent workgroup takes tiles round robin and, for each tile,
//   1. stages the tile plus a halo of >= (longest pattern - 1) bytes into LDS
//      with 16-byte loads (the overlap rule of Background, "Multi-Pattern
//      Matching"), and marks every text boundary in the window in an LDS bit
//      map so that no walk crosses into the next text;
//   2. filters: each lane holds BPL consecutive start positions and looks
//      their first K symbols up in the level index (a bitmap over K-symbol
//      codes of the depth-K nodes, kept in LDS).  A position whose first K
//      bytes are not a trie prefix cannot match (K < shortest pattern), so it
//      ends here; survivors are compacted per wave with ballots;
//   3. walks each survivor from its depth-K node down the CRS trie in global
//      memory (L2 resident) until a byte has no edge, remembering the deepest
//      terminal node passed;
//   4. emits: matched positions are sorted in LDS, their pattern lists counted
//      and prefix-summed, space is reserved in the staging buffer with one
//      atomic, and (pos, id) records are written in (pos, id) order.
// A finisher kernel then orders the tiles: block sums give each tile its
// output offset and the staged records are copied there.
#include <hip/hip_runtime.h>

#include "device_common.hpp"

namespace pfac {

// ------------------------------------------------------------------- scan

template <int BPL, bool IDENT, bool TOP, bool DAG>
__global__ __launch_bounds__(kWG) void scan_tiles(const ScanArgs a) {
    constexpr uint32_t TILE = kWG * BPL;
    extern __shared__ __align__(16) uint8_t lds[];
    uint32_t *s_bits = (uint32_t *)(lds + a.off_bits);
    uint32_t *s_rank = (uint32_t *)(lds + a.off_rank);
    uint8_t *s_sym = lds + a.off_sym;
    uint8_t *s_text = lds + a.off_text;
    uint32_t *s_bnd = (uint32_t *)(lds + a.off_bnd);
    uint32_t *s_queue = (uint32_t *)(lds + a.off_queue);
    uint2 *s_match = (uint2 *)(lds + a.off_match);
    __shared__ uint32_t s_qn[kWG / 64];
    __shared__ uint32_t s_mn, s_dirty, s_tmp[kWG / 64];
    __shared__ unsigned long long s_next, s_base;

    const ImageView &im = a.im;
    const uint32_t tid = threadIdx.x;
    const uint32_t wave = tid >> 6, lane = tid & 63;

    uint32_t *s_top = (uint32_t *)(lds + a.off_top);
    const uint32_t top_rw = im.top_rw;
    const bool top = TOP;  // the first K levels through the bitmapped nodes
    for (uint32_t i = tid; i < (top ? 0u : im.lvl_words); i += kWG) {
        const uint2 e = ((const uint2 *)im.lvl)[i];
        s_bits[i] = e.x;
        s_rank[i] = e.y;
    }
    for (uint32_t i = tid; i < (TOP ? a.top_words : 0u); i += kWG) s_top[i] = im.top[i];
    if (!IDENT)
        for (uint32_t i = tid; i < 256; i += kWG) s_sym[i] = im.sym[i];

    const uint32_t win = TILE + a.halo;
    const uint32_t bnd_words = win / 32 + 2;
    const uint64_t lo_valid = a.shift, hi_valid = a.shift + a.total;
    const uint32_t K = im.K;
    const uint32_t code_mask = (K == 0) ? 0u : ((1u << (im.b * K)) - 1u);

    for (uint64_t t = blockIdx.x; t < a.n_tiles; t += gridDim.x) {
        const uint64_t tile_lo = t * TILE;
        const uint64_t win_end = tile_lo + win;
        __syncthreads();  // the previous tile is done with LDS

        // ---- 1. stage the window and its boundaries
        for (uint32_t v = tid; v < win / 16; v += kWG) {
            const uint64_t g = tile_lo + 16ull * v;
            uint4 val = make_uint4(0, 0, 0, 0);
            if (g + 16 > lo_valid && g < hi_valid) {
                // an aligned 16-byte block holding a text byte lies in a mapped page
                val = *(const uint4 *)(a.base + g);
                if (g < lo_valid || g + 16 > hi_valid) {
                    uint32_t w[4] = {val.x, val.y, val.z, val.w};
#pragma unroll
                    for (int q = 0; q < 16; q++) {
                        const uint64_t p = g + q;
                        if (p < lo_valid || p >= hi_valid) w[q >> 2] &= ~(0xffu << (8 * (q & 3)));
                    }
                    val = make_uint4(w[0], w[1], w[2], w[3]);
                }
            }
            *(uint4 *)(s_text + 16 * v) = val;
        }
        for (uint32_t i = tid; i < bnd_words; i += kWG) s_bnd[i] = 0;
        if (tid == 0) {
            s_mn = 0;
            s_dirty = 0;
            s_next = ~0ull;
        }
        __syncthreads();
        {
            auto mark = [&](uint64_t bp) -> bool {
                if (bp >= win_end) {
                    atomicMin(&s_next, (unsigned long long)bp);
                    return false;
                }
                if (bp >= tile_lo) {
                    const uint32_t q = (uint32_t)(bp - tile_lo);
                    atomicOr(&s_bnd[q >> 5], 1u << (q & 31));
                    s_dirty = 1;
                }
                return true;
            };
            if (a.offsets == nullptr) {
                if (tid < 2) mark(tid ? hi_valid : lo_valid);
            } else {
                const uint32_t first = a.tile_first_text ? a.tile_first_text[t] : 0u;
                for (uint32_t r = first;; r += kWG) {
                    const uint32_t i = r + tid;
                    bool more = false;
                    if (i <= a.n_texts) more = mark(a.offsets[i] + a.shift);
                    if (!__syncthreads_or(more)) break;
                }
            }
        }
        __syncthreads();
        Tile T;
        T.text = s_text;
        T.bnd = s_bnd;
        T.lo = tile_lo;
        T.win = win;
        T.dirty = s_dirty != 0;
        T.next_bnd = s_next;

        // ---- 2. filter through the level index; compact survivors per wave
        uint32_t *wq = s_queue + wave * (64 * BPL);
        uint32_t qn = 0;  // wave-uniform
        const uint32_t lb = tid * BPL;
        if (K == 0) {
#pragma unroll
            for (int j = 0; j < BPL; j++) {
                const uint64_t p = tile_lo + lb + j;
                const bool ok = p >= lo_valid && p < hi_valid;
                const unsigned long long m = __ballot(ok);
                if (ok) {
                    const uint32_t r = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                       __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                    wq[qn + r] = (lb + j) << 18;
                }
                qn += (uint32_t)__popcll(m);
            }
        } else if (top) {
            // the first K symbols through the bitmapped nodes of depths
            // 0 .. K-1: at each node the symbol's bit must be set, and the
            // child is the first child + the set bits below it
            for (int j = 0; j < BPL; j++) {
                const uint32_t pl = lb + j;
                const uint64_t p = tile_lo + pl;
                // the K bytes lie in one text
                bool ok = p >= lo_valid && p + K <= hi_valid &&
                          (!T.dirty || range_clear(s_bnd, pl + 1, pl + K));
                uint32_t v = 0;
                for (uint32_t d = 0; d < K && ok; d++) {
                    const uint32_t byte = s_text[pl + d];
                    const uint32_t sy = IDENT ? byte : s_sym[byte];
                    const uint32_t *rec = s_top + v * top_rw;
                    const uint32_t wi = min(sy >> 5, top_rw - 2);  // in the node's bitmap
                    const uint32_t word = rec[wi];
                    // (0xff marks a byte outside a compressed alphabet)
                    ok = (IDENT || sy != 0xffu) && ((word >> (sy & 31)) & 1u);
                    uint32_t below = (uint32_t)__builtin_popcount(word & ((1u << (sy & 31)) - 1u));
                    for (uint32_t q = 0; q < wi; q++) below += (uint32_t)__builtin_popcount(rec[q]);
                    v = rec[top_rw - 1] + below;
                }
                const unsigned long long m = __ballot(ok);
                if (ok) {
                    const uint32_t r = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                       __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                    wq[qn + r] = (pl << 18) | (v - im.lvl_start);
                }
                qn += (uint32_t)__popcll(m);
            }
        } else {
            uint32_t w[BPL / 4 + 4];
#pragma unroll
            for (int q = 0; q < BPL / 4 + 4; q++) w[q] = *(const uint32_t *)(s_text + lb + 4 * q);
            unsigned long long brk = 0, inv = 0;
            if (T.dirty) {
                const uint32_t b0 = lb >> 5;
                const unsigned long long bw =
                    (unsigned long long)s_bnd[b0] | ((unsigned long long)s_bnd[b0 + 1] << 32);
                brk = bw >> (lb & 31);
                const uint64_t p0 = tile_lo + lb;
                if (lo_valid > p0) {
                    const uint64_t nb = lo_valid - p0;
                    inv |= nb >= 64 ? ~0ull : ((1ull << nb) - 1);
                }
                if (hi_valid < p0 + 64) {
                    const uint64_t na = hi_valid > p0 ? hi_valid - p0 : 0;
                    inv |= ~0ull << na;
                }
            }
            const bool plain = IDENT && !T.dirty;
            const uint32_t b = IDENT ? 8u : im.b;
            const uint32_t pbase = lb - (K - 1);
            uint32_t code = 0, run = 0;
#pragma unroll
            for (int j = 0; j < BPL + 15; j++) {
                if ((uint32_t)j >= BPL + K - 1) continue;  // wave-uniform
                const uint32_t byte = (w[j >> 2] >> (8 * (j & 3))) & 0xffu;
                uint32_t s = byte;
                bool ok = true;
                if (!IDENT) {
                    s = s_sym[byte];
                    ok = s != 0xffu;
                }
                if (!plain) {
                    if ((brk >> j) & 1ull) run = 0;
                    if ((inv >> j) & 1ull) ok = false;
                    run = ok ? run + 1 : 0;
                }
                code = ((code << b) | (s & 0xffu)) & code_mask;
                if ((uint32_t)j >= K - 1) {
                    const bool valid = plain || run >= K;
                    const uint32_t bits = s_bits[code >> 5];
                    const bool hit = valid && ((bits >> (code & 31)) & 1u);
                    const unsigned long long m = __ballot(hit);
                    if (hit) {
                        const uint32_t r = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                           __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                        wq[qn + r] = ((pbase + j) << 18) | code;
                    }
                    qn += (uint32_t)__popcll(m);
                }
            }
        }

        // ---- 3. walk the survivors of this wave
        for (uint32_t e = lane; e < qn; e += 64) {
            const uint32_t ent = wq[e];
            const uint32_t pl = ent >> 18;
            uint32_t v = 0, d = 0, R = 0;
            if (K && top) {
                v = im.lvl_start + (ent & 0x3ffffu);
                d = K;
            } else if (K) {
                const uint32_t code = ent & 0x3ffffu;
                const uint32_t bits = s_bits[code >> 5];
                const uint32_t below = bits & ((1u << (code & 31)) - 1u);
                const uint32_t rank = s_rank[code >> 5] + (uint32_t)__builtin_popcount(below);
                if (DAG) {
                    // the DAG node and the rank so far of this depth-K node
                    const uint2 vr = im.lvl_dag[rank];
                    v = vr.x;
                    R = vr.y;
                } else {
                    v = im.lvl_start + rank;
                }
                d = K;
            }
            const uint2 h = DAG ? walk_dag(im, a.base, T, pl, v, R, d) : walk(im, a.base, T, pl, v, d);
            if (h.y) {
                const uint32_t slot = atomicAdd(&s_mn, 1u);
                if (slot < kMatchCap) s_match[slot] = make_uint2(pl | (h.y << 16), h.x);
            }
        }
        __syncthreads();

        // ---- 4. emit this tile's matches in (pos, id) order
        const uint32_t mn = s_mn;
        if (mn == 0) {
            if (tid == 0) {
                a.unit_count[t] = 0;
                a.unit_off[t] = 0;
            }
            continue;
        }
        if (mn <= kMatchCap) {
            uint2 *sorted = (uint2 *)s_queue;  // the survivor queues are spent
            for (uint32_t i = tid; i < mn; i += kWG) {
                const uint2 e = s_match[i];
                uint32_t rk = 0;
                for (uint32_t q = 0; q < mn; q++) rk += (s_match[q].x & 0xffffu) < (e.x & 0xffffu);
                sorted[rk] = e;
            }
            __syncthreads();
            const uint32_t per = (mn + kWG - 1) / kWG;
            const uint32_t i0 = min(tid * per, mn), i1 = min(i0 + per, mn);
            uint32_t mine = 0;
            for (uint32_t i = i0; i < i1; i++)
                mine += hit_list(im, make_uint2(sorted[i].y, sorted[i].x >> 16)).y;
            uint32_t total;
            const uint32_t before = block_excl_scan(mine, s_tmp, total);
            if (tid == 0) {
                const unsigned long long base = atomicAdd(a.stage_cursor, (unsigned long long)total);
                a.unit_count[t] = total;
                a.unit_off[t] = base;
                atomicAdd(&a.blocksum[t >> kSumShift], (unsigned long long)total);
                s_base = base;
            }
            __syncthreads();
            uint64_t dst = s_base + before;
            for (uint32_t i = i0; i < i1; i++) {
                const uint2 e = sorted[i];
                const uint2 ids = hit_list(im, make_uint2(e.y, e.x >> 16));
                emit(a, tile_lo + (e.x & 0xffffu), ids, a.stage, dst, a.stage_cap);
                dst += ids.y;
            }
        } else {
            // Too many matched positions to sort in LDS: walk the tile again
            // from the root, one position per thread, in position order.
            uint32_t mine = 0;
            for (uint32_t r = 0; r < BPL; r++) {
                const uint32_t pl = r * kWG + tid;
                const uint64_t p = tile_lo + pl;
                if (p < lo_valid || p >= hi_valid) continue;
                const uint2 h = DAG ? walk_dag(im, a.base, T, pl, 0, 0, 0) : walk(im, a.base, T, pl, 0, 0);
                if (h.y) mine += hit_list(im, h).y;
            }
            uint32_t total;
            block_excl_scan(mine, s_tmp, total);
            if (tid == 0) {
                const unsigned long long base = atomicAdd(a.stage_cursor, (unsigned long long)total);
                a.unit_count[t] = total;
                a.unit_off[t] = base;
                atomicAdd(&a.blocksum[t >> kSumShift], (unsigned long long)total);
                s_base = base;
            }
            __syncthreads();
            uint64_t run_off = s_base;
            for (uint32_t r = 0; r < BPL; r++) {
                const uint32_t pl = r * kWG + tid;
                const uint64_t p = tile_lo + pl;
                uint2 ids = make_uint2(0, 0);
                if (p >= lo_valid && p < hi_valid) {
                    const uint2 h = DAG ? walk_dag(im, a.base, T, pl, 0, 0, 0) : walk(im, a.base, T, pl, 0, 0);
                    if (h.y) ids = hit_list(im, h);
                }
                const uint32_t c = ids.y;
                uint32_t round_total;
                const uint32_t before = block_excl_scan(c, s_tmp, round_total);
                if (c) emit(a, p, ids, a.stage, run_off + before, a.stage_cap);
                run_off += round_total;
            }
        }
    }
}

// ---------------------------------------------------------------- finisher

// One workgroup per block-sum entry (1 << kSumShift units): the units'
// records go to out[] in unit order.  The workgroup's first output slot is
// the sum of the block sums before it; its first wave scans the units'
// counts, then every thread copies records, each finding its unit by binary
// search over the unit starts.
__global__ __launch_bounds__(kWG) void finish_tiles(const FinishArgs f) {
    constexpr uint32_t kUnits = 1u << kSumShift;
    static_assert(kUnits <= 64, "one wave scans the units");
    __shared__ unsigned long long s_red[2][kWG / 64];
    __shared__ uint32_t s_start[kUnits + 1];
    __shared__ const pfac_match *s_from[kUnits];
    const uint32_t tid = threadIdx.x, b = blockIdx.x;
    unsigned long long pre = 0, all = 0;
    for (uint32_t i = tid; i < f.n_sums; i += kWG) {
        const unsigned long long s = f.blocksum[i];
        all += s;
        if (i < b) pre += s;
    }
    pre = wave_reduce_u64(pre);
    all = wave_reduce_u64(all);
    if ((tid & 63) == 0) {
        s_red[0][tid >> 6] = pre;
        s_red[1][tid >> 6] = all;
    }
    if (tid < 64) {
        const uint64_t t = ((uint64_t)b << kSumShift) + tid;
        const uint32_t cnt = (tid < kUnits && t < f.n_tiles) ? f.unit_count[t] : 0u;
        const pfac_match *from = nullptr;
        if (cnt) {
            const uint64_t src = f.unit_off[t];
            if (src == ~0ull)
                from = f.inline_stage + t * f.inline_cap;
            else if (src + cnt <= f.stage_cap)
                from = f.stage + src;  // else the staging area overflowed: nothing to copy
        }
        const uint32_t incl = wave_incl_scan(cnt);
        if (tid < kUnits) {
            s_start[tid] = incl - cnt;
            s_from[tid] = from;
        }
        if (tid == kUnits - 1) s_start[kUnits] = incl;
    }
    __syncthreads();
    pre = 0;
    all = 0;
    for (uint32_t i = 0; i < kWG / 64; i++) {
        pre += s_red[0][i];
        all += s_red[1][i];
    }
    if (b == 0 && tid == 0) *f.n_matches = all;
    const uint64_t base = pre + (f.base_dev ? *f.base_dev : 0ull);
    const uint32_t total = s_start[kUnits];
    for (uint32_t r = tid; r < total; r += kWG) {
        // last unit whose start is <= r: s_start[lo] <= r < s_start[hi]
        uint32_t lo = 0, hi = kUnits;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (s_start[mid] <= r) lo = mid; else hi = mid;
        }
        const pfac_match *src = s_from[lo];
        const uint64_t dst = base + r;
        if (src && dst < f.capacity) f.out[dst] = src[r - s_start[lo]];
    }
}

// ------------------------------------------------------------ small kernels

__global__ void reset_kernel(unsigned long long *cursor, unsigned long long *blocksum,
                             uint32_t n_sums) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *cursor = 0;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n_sums;
         i += gridDim.x * blockDim.x)
        blocksum[i] = 0;
}

__global__ void fill_u32_kernel(uint32_t *p, uint64_t n, uint32_t v) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// Largest i in [lo, hi) whose text starts at or before frame position G
// (wave-uniform), or lo when there is none: each round the wave's 64 lanes
// probe 64 evenly spaced starts (a 64-ary search, three rounds for 65,600
// texts).
__device__ __forceinline__ uint32_t wave_last_start(const uint64_t *offsets, uint64_t shift,
                                                    uint32_t lo, uint32_t hi, uint64_t G,
                                                    uint32_t lane) {
    while (hi - lo > 1) {
        const uint32_t step = (hi - lo + 63) / 64;
        const uint32_t i = lo + lane * step;
        const bool ok = i < hi && offsets[i] + shift <= G;
        const uint32_t c = (uint32_t)__popcll(__ballot(ok));  // starts are ascending: lanes 0 .. c-1
        if (c == 0) break;
        lo += (c - 1) * step;
        hi = min(hi, lo + step);
    }
    return lo;
}

// tile_first_text[t] = last text i whose start (in frame coordinates) is at or
// before the first byte of tile t.  With chunk_info (1 KiB plan units of the
// wave kernels) also the text boundaries of each chunk, packed as
//   x: bits 0..16  distance from the chunk start to the first boundary at or
//                  past its end (capped at 0x1ffff, the cap when none),
//      bits 17..19 boundaries inside the chunk, 0..4 (7: more than four),
//      bits 20..29 the first one (chunk position);
//   y: the second, third and fourth, 10 bits each (0 when absent),
// in ascending order, so that the filter kernel finds the distance from any
// start position to the end of its text without searching the offsets.
// One wave per 64 consecutive tiles: two wave searches bound the texts of
// its tiles, whose starts the lanes then hold two each; every lane finds its
// tile's text among them (or, past 128 texts, in global memory).
__global__ void plan_kernel(const uint64_t *offsets, uint32_t n_texts, uint64_t shift,
                            uint64_t n_tiles, uint32_t tile, uint32_t *tile_first_text,
                            uint2 *chunk_info) {
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t n_groups = (n_tiles + 63) / 64;
    const uint64_t wpb = blockDim.x / 64;
    const uint64_t waves = (uint64_t)gridDim.x * wpb;
    for (uint64_t w = (uint64_t)blockIdx.x * wpb + (threadIdx.x >> 6); w < n_groups; w += waves) {
        const uint64_t t0 = w * 64, t = t0 + lane;
        const uint64_t tl = min(t0 + 63, n_tiles - 1);
        const uint64_t g = t * tile;
        const uint32_t lo_w = wave_last_start(offsets, shift, 0, n_texts, t0 * tile, lane);
        // starts of texts lo_w .. lo_w + 127, two per lane (~0 past the end)
        const uint32_t wi = lo_w + lane;
        const unsigned long long wv0 = wi <= n_texts ? offsets[wi] + shift : ~0ull;
        const unsigned long long wv1 = wi + 64 <= n_texts ? offsets[wi + 64] + shift : ~0ull;
        // the last text starting at or before the last tile's first byte:
        // counted in the window when the window holds a start past that byte
        // (or the last text), else a second wave search
        const uint64_t gl = tl * tile;
        const uint32_t in_w = (uint32_t)__popcll(__ballot(wi < n_texts && wv0 <= gl)) +
                              (uint32_t)__popcll(__ballot(wi + 64 < n_texts && wv1 <= gl));
        const uint32_t hi_w = in_w < 128 ? lo_w + (in_w > 0 ? in_w - 1 : 0u)
                                         : wave_last_start(offsets, shift, lo_w, n_texts, gl, lane);
        auto window = [&](uint32_t r) -> uint64_t {  // r < 128; every lane calls it at once
            const uint64_t a = __shfl(wv0, (int)(r & 63u), 64);
            const uint64_t b = __shfl(wv1, (int)(r & 63u), 64);
            return r < 64 ? a : b;
        };
        // start of text i >= lo_w; every lane calls it at the same time
        auto start_of = [&](uint32_t i) -> uint64_t {
            const uint32_t r = i - lo_w;
            const uint64_t v = window(r & 127u);
            if (r < 128) return v;
            return i <= n_texts ? offsets[i] + shift : ~0ull;
        };
        uint32_t lo;
        if (hi_w - lo_w < 128) {
            // largest r < span with start_of(lo_w + r) <= g (r = 0 when none)
            const uint32_t span = hi_w - lo_w + 1;
            uint32_t r = 0;
            for (uint32_t step = 64; step > 0; step >>= 1) {
                const uint32_t c = r + step;
                const uint64_t v = window(c & 127u);
                if (c < span && v <= g) r = c;
            }
            lo = lo_w + r;
        } else {
            lo = lo_w;
            uint32_t hi = hi_w + 1;
            while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) >> 1;
                if (offsets[mid] + shift <= g) lo = mid; else hi = mid;
            }
        }
        if (t < n_tiles) tile_first_text[t] = lo;
        if (chunk_info) {
            // boundaries start_of(lo), start_of(lo + 1), ...: the first is at
            // or before g, so only it can equal g; the rest lie after g.  Six
            // are enough: one before g, four inside, then the next one past
            // the chunk or a fifth inside it.
            uint32_t cnt = 0, w0 = 0, w1 = 0, w2 = 0, w3 = 0;
            uint64_t next = ~0ull;
            bool done = false;
            for (uint32_t k = 0; k < 6; k++) {
                const uint64_t b = start_of(lo + k);
                if (done || b < g) continue;
                if (b >= g + tile) {
                    next = b;
                    done = true;
                } else if (cnt == 4) {
                    cnt = 7;
                    done = true;
                } else {
                    const uint32_t rel = (uint32_t)(b - g);
                    if (cnt == 0) w0 = rel; else if (cnt == 1) w1 = rel; else if (cnt == 2) w2 = rel; else w3 = rel;
                    cnt++;
                }
            }
            const uint32_t nrel = next - g > 0x1ffffull ? 0x1ffffu : (uint32_t)(next - g);
            if (t < n_tiles)
                chunk_info[t] = make_uint2(nrel | (cnt << 17) | (w0 << 20), w1 | (w2 << 10) | (w3 << 20));
        }
    }
}

__global__ void copy_u64_kernel(uint64_t *dst, const unsigned long long *src) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = *src;
}

__global__ void add_u64_kernel(unsigned long long *acc, const uint64_t *x) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *acc += *x;
}

// ------------------------------------------------------------------ launchers

void lds_layout(ScanArgs &a, uint32_t bpl) {
    const uint32_t tile = kWG * bpl;
    uint32_t off = 0;
    auto take = [&](uint32_t bytes) {
        const uint32_t o = off;
        off += (bytes + 15u) & ~15u;
        return o;
    };
    // the first K levels: the level index, or the bitmapped top nodes
    const uint32_t lw = a.top_words ? 0u : a.im.lvl_words;
    a.off_bits = take(4 * lw);
    a.off_rank = take(4 * lw);
    a.off_top = take(4 * a.top_words);
    a.off_sym = take(a.im.identity ? 0 : 256);
    a.off_text = take(tile + a.halo + 16);
    a.off_bnd = take(4 * ((tile + a.halo) / 32 + 2));
    a.off_queue = take(4 * tile);
    a.off_match = take(8 * kMatchCap);
    a.lds_total = off;
}

template <int BPL, bool IDENT>
static hipError_t launch_scan_t(const ScanArgs &a, uint32_t grid, hipStream_t s) {
    if (a.top_words)
        hipLaunchKernelGGL((scan_tiles<BPL, IDENT, true, false>), dim3(grid), dim3(kWG), a.lds_total, s, a);
    else if (a.im.dag)
        hipLaunchKernelGGL((scan_tiles<BPL, IDENT, false, true>), dim3(grid), dim3(kWG), a.lds_total, s, a);
    else
        hipLaunchKernelGGL((scan_tiles<BPL, IDENT, false, false>), dim3(grid), dim3(kWG), a.lds_total, s, a);
    return hipGetLastError();
}

hipError_t launch_scan(const ScanArgs &a, uint32_t bpl, uint32_t grid, hipStream_t s) {
    const bool id = a.im.identity != 0;
    switch (bpl) {
        case 4: return id ? launch_scan_t<4, true>(a, grid, s) : launch_scan_t<4, false>(a, grid, s);
        case 8: return id ? launch_scan_t<8, true>(a, grid, s) : launch_scan_t<8, false>(a, grid, s);
        case 16: return id ? launch_scan_t<16, true>(a, grid, s) : launch_scan_t<16, false>(a, grid, s);
        default: return hipErrorInvalidValue;
    }
}

// variant 0: level index, 1: bitmapped top nodes, 2: level index + DAG walk
template <int BPL, bool IDENT>
static const void *scan_fn(int var) {
    return var == 1 ? (const void *)scan_tiles<BPL, IDENT, true, false>
         : var == 2 ? (const void *)scan_tiles<BPL, IDENT, false, true>
                    : (const void *)scan_tiles<BPL, IDENT, false, false>;
}

static const void *scan_fn_for(uint32_t bpl, bool id, int var) {
    switch (bpl) {
        case 4: return id ? scan_fn<4, true>(var) : scan_fn<4, false>(var);
        case 8: return id ? scan_fn<8, true>(var) : scan_fn<8, false>(var);
        case 16: return id ? scan_fn<16, true>(var) : scan_fn<16, false>(var);
        default: return nullptr;
    }
}

hipError_t prepare_kernels(uint32_t bpl, uint32_t lds_bytes) {
    for (int v = 0; v < 6; v++) {
        const void *fn = scan_fn_for(bpl, (v & 1) != 0, v >> 1);
        if (!fn) return hipErrorInvalidValue;
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds_bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

int max_wg_per_cu(uint32_t bpl, uint32_t lds_bytes, int var) {
    int n = 0;
    const void *fn = scan_fn_for(bpl, true, var);
    if (!fn) return 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, kWG, lds_bytes) != hipSuccess || n < 1)
        n = 1;
    return n;
}

hipError_t launch_finish(const FinishArgs &f, hipStream_t s) {
    hipLaunchKernelGGL(finish_tiles, dim3(f.n_sums), dim3(kWG), 0, s, f);
    return hipGetLastError();
}

hipError_t launch_reset(unsigned long long *cursor, unsigned long long *blocksum,
                        uint32_t n_sums, hipStream_t s) {
    const uint32_t grid = (n_sums + 255) / 256 + 1;
    hipLaunchKernelGGL(reset_kernel, dim3(grid), dim3(256), 0, s, cursor, blocksum, n_sums);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    uint64_t g = (n + 255) / 256;
    const uint32_t grid = (uint32_t)(g < 65536 ? g : 65536);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_plan(const uint64_t *offsets, uint32_t n_texts, uint64_t shift,
                       uint64_t n_tiles, uint32_t tile, uint32_t *tile_first_text,
                       uint2 *chunk_info, hipStream_t s) {
    if (n_tiles == 0) return hipSuccess;
    if (chunk_info && tile != kWaveChunk) return hipErrorInvalidValue;
    // one wave per 64 tiles, four waves per workgroup
    uint64_t g = (n_tiles + 255) / 256;
    const uint32_t grid = (uint32_t)(g < 65536 ? g : 65536);
    hipLaunchKernelGGL(plan_kernel, dim3(grid), dim3(256), 0, s, offsets, n_texts, shift,
                       n_tiles, tile, tile_first_text, chunk_info);
    return hipGetLastError();
}

hipError_t launch_copy_u64(uint64_t *dst, const unsigned long long *src, hipStream_t s) {
    hipLaunchKernelGGL(copy_u64_kernel, dim3(1), dim3(64), 0, s, dst, src);
    return hipGetLastError();
}

hipError_t launch_add_running(unsigned long long *running, const uint64_t *n, hipStream_t s) {
    hipLaunchKernelGGL(add_u64_kernel, dim3(1), dim3(64), 0, s, running, n);
    return hipGetLastError();
}

}  // namespace pfac
