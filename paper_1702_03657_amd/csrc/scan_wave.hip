// Wave-independent scan kernel for gfx950.
//
// The same failure-less walk as the tile kernel (one start position per
// lane-slot, walk from the root until the first byte without an edge, report
// every pattern ending on the way), organised so that no step waits for the
// whole workgroup:
//
//   * a workgroup only cooperates to load the shared tables into LDS once;
//   * each wave then owns chunks of 1024 consecutive start positions (16 per
//     lane), round robin over the grid, and loads the next chunk's 16-byte
//     vectors while it processes the current one;
//   * a prefix filter rejects most positions with one LDS lookup: the table is
//     indexed by the first K symbols (the code of a depth-K trie node) and
//     holds that node's child bitmap folded to 8 or 16 bits, tested with the
//     next symbol, so K + 1 symbols are checked at once (the bitmapped node of
//     Design and Implementation, with the bitmap narrowed as that section
//     allows);
//   * survivors are compacted with ballots into a per-wave queue and walked
//     from their depth-K node (found by rank in the level bitmap) through the
//     CRS records in global memory (L2 resident);
//   * matches of a chunk are sorted by position in the wave's LDS area and
//     staged with one atomic per chunk; the shared finisher orders chunks.
// A chunk whose survivors or matches overflow the per-wave buffers is redone
// from the root, 64 positions at a time, in position order.
#include <hip/hip_runtime.h>

#include "device_common.hpp"

namespace pfac {

constexpr uint32_t kChunk = 1024;   // start positions per wave chunk (16 per lane)

__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t x, uint32_t &total) {
    const uint32_t incl = wave_incl_scan(x);
    total = __shfl(incl, 63, 64);
    return incl - x;
}

__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long x) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long y = __shfl_xor(x, off, 64);
        x = y < x ? y : x;
    }
    return x;
}

__device__ __forceinline__ uint32_t mbcnt(unsigned long long m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Byte j (0..31) of the 32-byte lane window w[0..7].
__device__ __forceinline__ uint32_t wbyte(const uint32_t *w, int j) {
    return (w[j >> 2] >> (8 * (j & 3))) & 0xffu;
}

// Stage the matches of one chunk in (pos, id) order.  wm[i] = (window
// position | stored list length << 16, list offset).  A chunk with at most
// inline_cap records writes them to its own inline slots (no atomic with a
// return value); larger ones reserve staging space with one atomic.
__device__ __forceinline__ void emit_chunk(const ScanArgs &a, uint64_t c, uint64_t chunk_lo,
                                           uint2 *wm, uint32_t mn, uint2 *sorted) {
    const ImageView &im = a.im;
    const uint32_t lane = lane_id();
    if (mn == 0) {
        if (lane == 0) a.unit_count[c] = 0;
        return;
    }
    for (uint32_t i = lane; i < mn; i += 64) {
        const uint2 e = wm[i];
        uint32_t rk = 0;
        for (uint32_t q = 0; q < mn; q++) rk += (wm[q].x & 0xffffu) < (e.x & 0xffffu);
        sorted[rk] = e;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    uint2 ids[2];
    uint32_t off[2], total = 0;
#pragma unroll
    for (int r = 0; r < 2; r++) {
        const uint32_t i = lane + 64u * r;
        ids[r] = make_uint2(0, 0);
        if (i < mn) ids[r] = hit_list(im, make_uint2(sorted[i].y, sorted[i].x >> 16));
        uint32_t t;
        off[r] = total + wave_excl_scan(ids[r].y, t);
        total += t;
    }
    pfac_match *dst;
    uint64_t base, cap;
    if (total <= a.inline_cap) {
        dst = a.inline_stage + c * a.inline_cap;
        base = 0;
        cap = a.inline_cap;
        if (lane == 0) {
            a.unit_count[c] = total;
            a.unit_off[c] = ~0ull;
            atomicAdd(&a.blocksum[c >> kTpbShift], (unsigned long long)total);
        }
    } else {
        unsigned long long b = 0;
        if (lane == 0) {
            b = atomicAdd(a.stage_cursor, (unsigned long long)total);
            a.unit_count[c] = total;
            a.unit_off[c] = b;
            atomicAdd(&a.blocksum[c >> kTpbShift], (unsigned long long)total);
        }
        base = __shfl(b, 0, 64);
        dst = a.stage;
        cap = a.stage_cap;
    }
#pragma unroll
    for (int r = 0; r < 2; r++) {
        const uint32_t i = lane + 64u * r;
        if (i < mn) emit(a, chunk_lo + (sorted[i].x & 0xffffu), ids[r], dst, base + off[r], cap);
    }
}

// Redo a chunk from the root, in position order, when its buffers overflow.
__device__ __forceinline__ void chunk_from_root(const ScanArgs &a, const Tile &T, uint64_t c) {
    const ImageView &im = a.im;
    const uint32_t lane = lane_id();
    const uint64_t lo_valid = a.shift, hi_valid = a.shift + a.total;
    uint32_t total = 0;
    for (uint32_t r = 0; r < kChunk / 64; r++) {
        const uint32_t pl = r * 64 + lane;
        const uint64_t p = T.lo + pl;
        uint32_t cnt = 0;
        if (p >= lo_valid && p < hi_valid) {
            const uint2 h = walk(im, a.base, T, pl, 0, 0);
            if (h.y) cnt = hit_list(im, h).y;
        }
        uint32_t t;
        wave_excl_scan(cnt, t);
        total += t;
    }
    unsigned long long base = 0;
    if (lane == 0) {
        base = atomicAdd(a.stage_cursor, (unsigned long long)total);
        a.unit_count[c] = total;
        a.unit_off[c] = base;
        if (total) atomicAdd(&a.blocksum[c >> kTpbShift], (unsigned long long)total);
    }
    base = __shfl(base, 0, 64);
    for (uint32_t r = 0; r < kChunk / 64; r++) {
        const uint32_t pl = r * 64 + lane;
        const uint64_t p = T.lo + pl;
        uint2 ids = make_uint2(0, 0);
        if (p >= lo_valid && p < hi_valid) {
            const uint2 h = walk(im, a.base, T, pl, 0, 0);
            if (h.y) ids = hit_list(im, h);
        }
        uint32_t t;
        const uint32_t before = wave_excl_scan(ids.y, t);
        if (ids.y) emit(a, p, ids, a.stage, base + before, a.stage_cap);
        base += t;
    }
}

// MODE 1: byte symbols, K = 2, 8-bit folded table.  MODE 2: same, 16-bit.
// MODE 0: any image (symbol table, any K, table or plain level bitmap, or
// the root bitmap when K = 0).
template <int MODE>
__global__ __launch_bounds__(1024) void scan_waves(const ScanArgs a) {
    extern __shared__ __align__(16) uint8_t lds[];
    const ImageView &im = a.im;
    const uint32_t tid = threadIdx.x;
    const uint32_t nthreads = blockDim.x;
    const uint32_t waves = nthreads >> 6;
    const uint32_t wave = tid >> 6, lane = tid & 63;

    uint8_t *s_ftab = lds + a.off_ftab;
    uint32_t *s_bits = (uint32_t *)(lds + a.off_bits);
    uint32_t *s_rank = (uint32_t *)(lds + a.off_rank);
    uint32_t *s_root = (uint32_t *)(lds + a.off_root);
    uint8_t *s_sym = lds + a.off_sym;

    // ---- shared tables, once per workgroup
    {
        const uint32_t fbytes = a.ftab_bytes;
        for (uint32_t i = tid; i < fbytes / 16; i += nthreads)
            ((uint4 *)s_ftab)[i] = ((const uint4 *)im.ftab)[i];
        for (uint32_t i = tid; i < im.lvl_words; i += nthreads) {
            const uint2 e = ((const uint2 *)im.lvl)[i];
            s_bits[i] = e.x;
            s_rank[i] = e.y;
        }
        for (uint32_t i = tid; i < a.root_words; i += nthreads) s_root[i] = im.root_bits[i];
        if (MODE == 0 && !im.identity)
            for (uint32_t i = tid; i < 256; i += nthreads) s_sym[i] = im.sym[i];
    }
    __syncthreads();

    uint8_t *wbase = lds + a.off_wave + wave * a.wave_bytes;
    uint8_t *wtext = wbase;                                         // kChunk + halo + 16
    uint32_t *wbnd = (uint32_t *)(wbase + a.woff_bnd);
    uint32_t *wq = (uint32_t *)(wbase + a.woff_queue);
    uint2 *wm = (uint2 *)(wbase + a.woff_match);

    const uint64_t lo_valid = a.shift, hi_valid = a.shift + a.total;
    const uint32_t halo = a.halo;
    const uint32_t win = kChunk + halo;
    const uint32_t nbw = win / 32 + 2;
    const uint64_t stride = (uint64_t)gridDim.x * waves;
    const uint32_t K = im.K;
    const uint32_t qcap = a.qcap, mcap = a.mcap;

    auto load_vec = [&](uint64_t g) -> uint4 {
        uint4 v = make_uint4(0, 0, 0, 0);
        // an aligned 16-byte block holding a text byte lies in a mapped page
        if (g + 16 > lo_valid && g < hi_valid) v = *(const uint4 *)(a.base + g);
        return v;
    };

    uint64_t c = (uint64_t)blockIdx.x * waves + wave;
    uint4 cur = make_uint4(0, 0, 0, 0), cur_h = make_uint4(0, 0, 0, 0);
    if (c < a.n_tiles) {
        cur = load_vec(c * kChunk + 16ull * lane);
        if (lane < halo / 16) cur_h = load_vec(c * kChunk + kChunk + 16ull * lane);
    }
    for (; c < a.n_tiles; c += stride) {
        const uint64_t chunk_lo = c * kChunk;
        const uint64_t win_end = chunk_lo + win;
        // next chunk's text, in flight while this one is processed
        uint4 nxt = make_uint4(0, 0, 0, 0), nxt_h = make_uint4(0, 0, 0, 0);
        const uint64_t cn = c + stride;
        if (cn < a.n_tiles) {
            nxt = load_vec(cn * kChunk + 16ull * lane);
            if (lane < halo / 16) nxt_h = load_vec(cn * kChunk + kChunk + 16ull * lane);
        }

        // ---- 1. window into the wave's LDS area
        *(uint4 *)(wtext + 16 * lane) = cur;
        if (lane < halo / 16) *(uint4 *)(wtext + kChunk + 16 * lane) = cur_h;

        // ---- 2. text boundaries in the window
        bool dirty;
        unsigned long long next_bnd;
        if (a.offsets == nullptr) {
            const bool lo_in = lo_valid >= chunk_lo && lo_valid < win_end;
            const bool hi_in = hi_valid >= chunk_lo && hi_valid < win_end;
            dirty = lo_in || hi_in;
            next_bnd = hi_valid >= win_end ? hi_valid : ~0ull;
            if (dirty) {
                for (uint32_t i = lane; i < nbw; i += 64) wbnd[i] = 0;
                __builtin_amdgcn_wave_barrier();
                if (lane == 0 && lo_in) atomicOr(&wbnd[(lo_valid - chunk_lo) >> 5], 1u << ((lo_valid - chunk_lo) & 31));
                if (lane == 1 && hi_in) atomicOr(&wbnd[(hi_valid - chunk_lo) >> 5], 1u << ((hi_valid - chunk_lo) & 31));
            }
        } else {
            for (uint32_t i = lane; i < nbw; i += 64) wbnd[i] = 0;
            __builtin_amdgcn_wave_barrier();
            dirty = false;
            next_bnd = ~0ull;
            for (uint32_t i = a.tile_first_text[c] + lane;; i += 64) {
                const unsigned long long bp = i <= a.n_texts ? a.offsets[i] + a.shift : ~0ull;
                const bool in = bp >= chunk_lo && bp < win_end;
                if (in) atomicOr(&wbnd[(bp - chunk_lo) >> 5], 1u << ((bp - chunk_lo) & 31));
                dirty = dirty || __ballot(in) != 0;
                next_bnd = wave_min_u64(bp >= win_end ? bp : next_bnd);
                if (__ballot(bp >= win_end) != 0) break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

        Tile T;
        T.text = wtext;
        T.bnd = wbnd;
        T.lo = chunk_lo;
        T.win = win;
        T.dirty = dirty;
        T.next_bnd = next_bnd;

        // ---- 3. prefix filter over this lane's 16 start positions
        uint32_t w[8];
        {
            w[0] = cur.x; w[1] = cur.y; w[2] = cur.z; w[3] = cur.w;
            const uint4 x = *(const uint4 *)(wtext + 16 * lane + 16);
            w[4] = x.x; w[5] = x.y; w[6] = x.z; w[7] = x.w;
        }
        uint32_t qn = 0;
        bool overflow = false;
        auto push = [&](bool hit, uint32_t entry) {
            const unsigned long long m = __ballot(hit);
            if (hit) {
                const uint32_t slot = qn + mbcnt(m);
                if (slot < qcap) wq[slot] = entry;
            }
            qn += (uint32_t)__popcll(m);
        };
        if (MODE == 1 || MODE == 2) {
#pragma unroll
            for (int j = 0; j < 16; j++) {
                // code = (B[j] << 8) | B[j+1]; next = B[j+2]
                const uint32_t lo = w[j >> 2], hi = w[(j >> 2) + 1];
                const uint32_t r = j & 3;
                const uint32_t sel = 0x0c0c0000u | (r << 8) | (r + 1);
                const uint32_t code = __builtin_amdgcn_perm(hi, lo, sel);
                const uint32_t nx = wbyte(w, j + 2);
                uint32_t hit;
                if (MODE == 1)
                    hit = (s_ftab[code] >> (nx & 7)) & 1u;
                else
                    hit = (((const uint16_t *)s_ftab)[code] >> (nx & 15)) & 1u;
                push(hit != 0, ((16 * lane + j) << 20) | code);
            }
        } else {
            const uint32_t b = im.b;
            const uint32_t m = (K >= 1 && a.fold) ? im.fold_syms : 0u;
            const uint32_t L = K >= 1 ? K + m : 1u;
            const uint32_t full_mask = (b * L >= 32) ? 0xffffffffu : ((1u << (b * L)) - 1u);
            // the folded bit reads only the last m symbols of the window
            const uint32_t fmask = (a.fold - 1u) & ((b * m >= 32) ? 0xffffffffu : ((1u << (b * m)) - 1u));
            uint32_t full = 0, run = 0;
#pragma unroll
            for (int j = 0; j < 31; j++) {
                if ((uint32_t)j >= 15 + L) continue;  // wave-uniform
                const uint32_t byte = wbyte(w, j);
                uint32_t s = byte;
                bool ok = true;
                if (!im.identity) {
                    s = s_sym[byte];
                    ok = s != 0xffu;
                }
                run = ok ? run + 1 : 0u;
                full = ((full << b) | (s & 0xffu)) & full_mask;
                if ((uint32_t)j + 1 >= L) {
                    const uint32_t pos = j + 1 - L;
                    uint32_t hit = 0, code = 0;
                    if (run >= L) {
                        if (K == 0) {
                            hit = (s_root[full >> 5] >> (full & 31)) & 1u;
                        } else if (a.fold) {
                            code = full >> (b * m);
                            const uint32_t bit = full & fmask;
                            hit = a.fold == 8 ? (s_ftab[code] >> bit) & 1u
                                              : (((const uint16_t *)s_ftab)[code] >> bit) & 1u;
                        } else {
                            code = full;
                            hit = (s_bits[code >> 5] >> (code & 31)) & 1u;
                        }
                    }
                    push(hit != 0, ((16 * lane + pos) << 20) | code);
                }
            }
        }
        overflow = qn > qcap;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

        // ---- 4. walk the survivors
        uint32_t mn = 0;
        if (!overflow) {
            for (uint32_t r0 = 0; r0 < qn; r0 += 64) {
                const uint32_t e = r0 + lane;
                uint2 h = make_uint2(0, 0);
                uint32_t pl = 0;
                if (e < qn) {
                    const uint32_t ent = wq[e];
                    pl = ent >> 20;
                    const uint64_t p = chunk_lo + pl;
                    // the filter read K symbols without looking at text
                    // boundaries: none may start inside them
                    bool crosses = false;
                    if (dirty)
                        for (uint32_t q = pl + 1; q < pl + K; q++)
                            crosses = crosses || ((wbnd[q >> 5] >> (q & 31)) & 1u);
                    if (p >= lo_valid && p < hi_valid && !crosses) {
                        uint32_t v = 0, d = 0;
                        if (K) {
                            const uint32_t code = ent & 0xfffffu;
                            const uint32_t bits = s_bits[code >> 5];
                            const uint32_t below = bits & ((1u << (code & 31)) - 1u);
                            v = im.lvl_start + s_rank[code >> 5] + (uint32_t)__builtin_popcount(below);
                            d = K;
                        }
                        h = walk(im, a.base, T, pl, v, d);
                    }
                }
                const bool got = h.y != 0;
                const unsigned long long mk = __ballot(got);
                if (got) {
                    const uint32_t slot = mn + mbcnt(mk);
                    if (slot < mcap) wm[slot] = make_uint2(pl | (h.y << 16), h.x);
                }
                mn += (uint32_t)__popcll(mk);
            }
            overflow = mn > mcap;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

        // ---- 5. stage this chunk's matches in (pos, id) order
        if (!overflow)
            emit_chunk(a, c, chunk_lo, wm, mn, (uint2 *)wq);
        else
            chunk_from_root(a, T, c);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

        cur = nxt;
        cur_h = nxt_h;
    }
}

// ------------------------------------------------------------------ launchers

void wave_lds_layout(ScanArgs &a, uint32_t waves, uint32_t lds_limit) {
    uint32_t off = 0;
    auto take = [&](uint32_t bytes) {
        const uint32_t o = off;
        off += (bytes + 15u) & ~15u;
        return o;
    };
    a.ftab_bytes = (uint32_t)((a.fold && a.im.K) ? ((1ull << (a.im.b * a.im.K)) * (a.fold / 8)) : 0);
    a.ftab_bytes = (a.ftab_bytes + 15u) & ~15u;
    a.off_ftab = take(a.ftab_bytes);
    a.off_bits = take(4 * a.im.lvl_words);
    a.off_rank = take(4 * a.im.lvl_words);
    a.root_words = a.im.K == 0 ? std::max(1u, (1u << a.im.b) / 32) : 0u;
    a.off_root = take(4 * a.root_words);
    a.off_sym = take(a.im.identity ? 0 : 256);
    a.off_wave = off;
    const uint32_t win = kChunk + a.halo;
    a.mcap = 128;
    const uint32_t fixed = ((win + 16 + 15) & ~15u) + ((4 * (win / 32 + 2) + 15) & ~15u) + 8 * a.mcap;
    // the survivor queue takes what is left, up to one entry per position
    uint32_t left = lds_limit > off ? (lds_limit - off) / waves : 0;
    uint32_t q = left > fixed ? (left - fixed) / 4 : 0;
    q = std::min<uint32_t>(q & ~63u, kChunk);
    a.qcap = std::max<uint32_t>(q, 2 * a.mcap);
    a.woff_bnd = (win + 16 + 15) & ~15u;
    a.woff_queue = a.woff_bnd + ((4 * (win / 32 + 2) + 15) & ~15u);
    a.woff_match = a.woff_queue + 4 * a.qcap;
    a.wave_bytes = a.woff_match + 8 * a.mcap;
    a.lds_total = off + waves * a.wave_bytes;
}

int wave_mode(const ScanArgs &a) {
    if (a.im.identity && a.im.K == 2 && a.fold == 8 && a.im.fold_syms == 1) return 1;
    if (a.im.identity && a.im.K == 2 && a.fold == 16 && a.im.fold_syms == 1) return 2;
    return 0;
}

template <int MODE>
static const void *wave_fn() {
    return (const void *)scan_waves<MODE>;
}

static const void *wave_fn_for(int mode) {
    switch (mode) {
        case 1: return wave_fn<1>();
        case 2: return wave_fn<2>();
        default: return wave_fn<0>();
    }
}

hipError_t prepare_wave_kernel(int mode, uint32_t lds_bytes) {
    return hipFuncSetAttribute(wave_fn_for(mode), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds_bytes);
}

hipError_t launch_scan_waves(const ScanArgs &a, uint32_t waves, uint32_t grid, hipStream_t s) {
    const int mode = wave_mode(a);
    const dim3 block(64 * waves);
    switch (mode) {
        case 1: hipLaunchKernelGGL(scan_waves<1>, dim3(grid), block, a.lds_total, s, a); break;
        case 2: hipLaunchKernelGGL(scan_waves<2>, dim3(grid), block, a.lds_total, s, a); break;
        default: hipLaunchKernelGGL(scan_waves<0>, dim3(grid), block, a.lds_total, s, a); break;
    }
    return hipGetLastError();
}

int max_wave_wg_per_cu(const ScanArgs &a, uint32_t waves) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, wave_fn_for(wave_mode(a)), 64 * waves,
                                                     a.lds_total) != hipSuccess || n < 1)
        n = 1;
    return n;
}

}  // namespace pfac
