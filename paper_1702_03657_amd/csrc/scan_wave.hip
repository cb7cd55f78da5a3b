// Wave-independent scan kernels for gfx950.
//
// The failure-less walk of the paper (one start position per lane slot, walk
// the trie from the root until the first byte without an edge, report every
// pattern that ends on the way), organised so that no step waits for the
// whole workgroup, so that positions no pattern can start at cost one LDS
// lookup, and so that walks do not hold up the filtering:
//
//   * a workgroup cooperates only to load the shared tables into LDS;
//   * each wave owns units of G consecutive 1 KiB chunks (round robin over
//     the grid) and loads chunks two ahead of the one it filters;
//   * stage 1 tests all 16 start positions of a lane against a table at LDS
//     address 0 and builds a hit mask: for byte alphabets the table is
//     indexed by the first two bytes (the code of a depth-2 trie node) and
//     holds that node's child bitmap folded to 8 or 16 bits, tested with the
//     third byte (the bitmapped node of Design and Implementation, narrowed
//     as that section allows); for alphabets of at most four bytes (mode 3)
//     it is a hashed bitmap over 16-symbol prefixes; other images use a
//     rolling code over K symbols (mode 0);
//   * stage 2 takes the compacted hits: the text end, the prefix-4 filter or
//     the depth-K node's child labels (byte alphabets), the alphabet bytes
//     and a fingerprint (mode 3), and the depth-K node from the level index;
//   * survivors become walk candidates (start, depth-K node, distance to the
//     end of their text).  The split kernel writes them, with the 8 text
//     bytes after the index, for walk_units; the fused kernel walks a unit's
//     candidates itself, reading the text and the CRS records from global
//     memory, with single-child runs compared in bulk;
//   * matches of a unit are sorted by position in LDS and staged in the
//     unit's inline slots (or with one atomic when there are more); the
//     shared finisher orders units.
// A unit whose candidates or matches overflow their lists is redone from the
// root, 64 positions at a time, in position order.
#include <hip/hip_runtime.h>

#include <utility>

#include "device_common.hpp"

namespace pfac {

constexpr uint32_t kChunk = 1024;   // start positions per chunk (16 per lane)
constexpr uint32_t kWin = kChunk + 16;  // chunk bytes staged in LDS (+ one vector)
constexpr uint32_t kPPL = 4;        // start positions per lane per filter pass
constexpr uint32_t kQ1 = 64 * kPPL; // stage-1 survivors of one pass (32-bit entries)
constexpr uint32_t kQ16 = 2 * kQ1;  // the same area as 16-bit entries

// The prefix-filter table at LDS address 0 (the first section of the dynamic
// LDS of a kernel without static LDS; checked on the host at launch set-up).
typedef __attribute__((address_space(3))) const uint8_t lds_u8_t;
typedef __attribute__((address_space(3))) const uint16_t lds_u16_t;
__device__ __forceinline__ const lds_u8_t *lds_tab8() { return (const lds_u8_t *)(uintptr_t)0; }
__device__ __forceinline__ const lds_u16_t *lds_tab16() { return (const lds_u16_t *)(uintptr_t)0; }
typedef __attribute__((address_space(3))) const uint32_t lds_u32_t;
__device__ __forceinline__ const lds_u32_t *lds_tab32() { return (const lds_u32_t *)(uintptr_t)0; }

__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t x, uint32_t &total) {
    const uint32_t incl = wave_incl_scan(x);
    total = wave_last(incl);
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

__device__ __forceinline__ uint64_t umin64(uint64_t x, uint64_t y) { return x < y ? x : y; }

// The lane index, tied to a value that changes from chunk to chunk: a
// comparison of it inside the chunk loop stays there (one compare) instead
// of being hoisted into a lane mask that occupies two scalar registers for
// the whole kernel.
__device__ __forceinline__ uint32_t lane_at(uint32_t salt) {
    uint32_t l;
    asm("; lane %1" : "=v"(l) : "s"(salt), "0"(threadIdx.x & 63u));
    return l;
}

// (x << J) | y in one instruction (the compiler would build a tree of
// separate shifts and three-input ORs)
template <int J>
__device__ __forceinline__ uint32_t lshl_or(uint32_t x, uint32_t y) {
    uint32_t r;
    asm("v_lshl_or_b32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "i"(J), "v"(y));
    return r;
}

// sum of bit[j] << j over j = 0 .. sizeof...(J) (each bit[j] is 0 or 1);
// J runs over 0 .. n - 1 for bits 1 .. n
template <int... J>
__device__ __forceinline__ uint32_t gather_bits(const uint32_t *bit, std::integer_sequence<int, J...>) {
    uint32_t hm = bit[0];
    ((hm = lshl_or<J + 1>(bit[J + 1], hm)), ...);
    return hm;
}

__device__ __forceinline__ uint32_t mbcnt(unsigned long long m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Byte j (0..31) of the 32-byte lane window w[0..7].
__device__ __forceinline__ uint32_t wbyte(const uint32_t *w, int j) {
    return (w[j >> 2] >> (8 * (j & 3))) & 0xffu;
}

// True when text[g .. g+len) (global) equals chain[o .. o+len); the caller
// guarantees g + len + 36 <= the end of the valid text.
__device__ __forceinline__ bool chain_equal_g(const uint8_t *base, uint64_t g, const uint8_t *chain,
                                              uint32_t o, uint32_t len) {
    const uint32_t *c32 = (const uint32_t *)chain;
    uint32_t diff = 0;
    for (uint32_t i = 0; i < len; i += 32) {
        uint32_t cw[9], tw[9];
        const uint32_t cb = (o + i) >> 2;
        const uint32_t *t32 = (const uint32_t *)(base + ((g + i) & ~3ull));
#pragma unroll
        for (int k = 0; k < 9; k++) cw[k] = c32[cb + k];
#pragma unroll
        for (int k = 0; k < 9; k++) tw[k] = t32[k];
        const uint32_t cs = (o + i) & 3, ts = (uint32_t)((g + i) & 3);
#pragma unroll
        for (int k = 0; k < 8; k++) {
            const int32_t r = (int32_t)(len - i) - 4 * k;
            const uint32_t mask = r >= 4 ? 0xffffffffu : (r <= 0 ? 0u : ((1u << (8 * r)) - 1u));
            const uint32_t c = __builtin_amdgcn_alignbyte(cw[k + 1], cw[k], cs);
            const uint32_t t = __builtin_amdgcn_alignbyte(tw[k + 1], tw[k], ts);
            diff |= (c ^ t) & mask;
        }
    }
    return diff == 0;
}

// Walk for the start position at frame position p from node v at depth d,
// reading the text from global memory; the text ends lim bytes after p.
// Returns the pattern list of the deepest terminal node passed.
__device__ __forceinline__ uint2 walk_g(const ImageView &im, const uint8_t *base, uint64_t p,
                                        uint32_t lim, uint32_t v, uint32_t d, uint64_t hi_valid) {
    uint2 hit = make_uint2(0, 0);
    for (;;) {
        const uint4 r = im.node[v];
        if (r.z & kTermFlagD) hit = make_uint2(r.w, r.z >> kCountShiftD);
        const uint32_t nc = r.z & 0xffffu;
        if (nc == 0 || d >= lim) break;
        const bool skip = (r.z & kSkipFlagD) != 0;
        if (skip) {
            // no pattern ends inside a single-child run: it matches whole or
            // the walk ends with nothing more to report
            const uint32_t len = r.z >> kSkipShiftD;
            if (d + len > lim) break;
            if (p + d + len + 36 <= hi_valid) {
                const bool leaf = (r.z & kLeafEndD) != 0;
                if (!chain_equal_g(base, p + d, im.chain, leaf ? r.x & 0xffffffu : r.x, len)) break;
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
        const uint32_t c = base[p + d];
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
                const uint32_t mid = (lo + hi) >> 1;
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

// Text boundaries of the chunk window [lo, lo + kWin): bits in `bnd`,
// `dirty` when any lies in it, and the first boundary at or past its end.
__device__ __forceinline__ void chunk_bounds(const ScanArgs &a, uint64_t chunk, uint64_t lo,
                                             uint32_t *bnd, bool &dirty,
                                             unsigned long long &next_bnd) {
    const uint32_t lane = lane_at((uint32_t)chunk);
    const uint64_t lo_valid = a.shift, hi_valid = a.shift + a.total;
    const uint64_t end = lo + kWin;
    constexpr uint32_t nbw = kWin / 32 + 2;
    if (a.offsets == nullptr) {
        const bool lo_in = lo_valid >= lo && lo_valid < end;
        const bool hi_in = hi_valid >= lo && hi_valid < end;
        dirty = lo_in || hi_in;
        next_bnd = hi_valid >= end ? hi_valid : ~0ull;
        if (dirty) {
            if (lane < nbw) bnd[lane] = 0;
            wave_sync();
            if (lane == 0 && lo_in) atomicOr(&bnd[(lo_valid - lo) >> 5], 1u << ((lo_valid - lo) & 31));
            if (lane == 1 && hi_in) atomicOr(&bnd[(hi_valid - lo) >> 5], 1u << ((hi_valid - lo) & 31));
        }
    } else {
        if (lane < nbw) bnd[lane] = 0;
        wave_sync();
        dirty = false;
        next_bnd = ~0ull;
        for (uint32_t i = a.tile_first_text[chunk] + lane;; i += 64) {
            const unsigned long long bp = i <= a.n_texts ? a.offsets[i] + a.shift : ~0ull;
            const bool in = bp >= lo && bp < end;
            if (in) atomicOr(&bnd[(bp - lo) >> 5], 1u << ((bp - lo) & 31));
            dirty = dirty || __ballot(in) != 0;
            next_bnd = wave_min_u64(bp >= end ? bp : next_bnd);
            if (__ballot(bp >= end) != 0) break;
        }
    }
    wave_sync();
}

// Distance from window position pl to the next text boundary after it.
__device__ __forceinline__ uint32_t limit_after(const uint32_t *bnd, bool dirty, uint64_t lo,
                                                uint32_t pl, unsigned long long next_bnd) {
    unsigned long long nb = next_bnd;
    if (dirty) {
        constexpr uint32_t nbw = kWin / 32 + 2;
        const uint32_t q = pl + 1;
        uint32_t w = q >> 5;
        uint32_t bits = bnd[w] & (0xffffffffu << (q & 31));
        while (bits == 0 && ++w < nbw) bits = bnd[w];
        if (bits) nb = lo + (w << 5) + (uint32_t)__builtin_ctz(bits);
    }
    const unsigned long long d = nb - (lo + pl);
    return d > 0xffffull ? 0xffffu : (uint32_t)d;
}

// Stage the matches of unit u in (pos, id) order.  wm[i] = (unit position |
// stored list length << 16, list offset).  At most inline_cap records go to
// the unit's inline slots; more reserve staging space with one atomic.
__device__ __forceinline__ void emit_unit(const ScanArgs &a, uint64_t u, uint64_t unit_lo,
                                          const uint2 *wm, uint32_t mn, uint2 *sorted,
                                          const UnitText &ut = UnitText{}) {
    const ImageView &im = a.im;
    const uint32_t lane = lane_id();
    if (mn == 0) {
        if (lane == 0) a.unit_count[u] = 0;
        return;
    }
    for (uint32_t i = lane; i < mn; i += 64) {
        const uint2 e = wm[i];
        uint32_t rk = 0;
        for (uint32_t q = 0; q < mn; q++) rk += (wm[q].x & 0xffffu) < (e.x & 0xffffu);
        sorted[rk] = e;
    }
    wave_sync();
    uint32_t total = 0;
    for (uint32_t r0 = 0; r0 < mn; r0 += 64) {
        const uint32_t i = r0 + lane;
        const uint32_t n = i < mn ? hit_list(im, make_uint2(sorted[i].y, sorted[i].x >> 16)).y : 0u;
        uint32_t t;
        wave_excl_scan(n, t);
        total += t;
    }
    pfac_match *dst;
    uint64_t base = 0, cap;
    if (total <= a.inline_cap) {
        dst = a.inline_stage + u * a.inline_cap;
        cap = a.inline_cap;
        if (lane == 0) {
            a.unit_count[u] = total;
            a.unit_off[u] = ~0ull;
            atomicAdd(&a.blocksum[u >> kSumShift], (unsigned long long)total);
        }
    } else {
        unsigned long long b = 0;
        if (lane == 0) {
            b = atomicAdd(a.stage_cursor, (unsigned long long)total);
            a.unit_count[u] = total;
            a.unit_off[u] = b;
            atomicAdd(&a.blocksum[u >> kSumShift], (unsigned long long)total);
        }
        base = __shfl(b, 0, 64);
        dst = a.stage;
        cap = a.stage_cap;
    }
    for (uint32_t r0 = 0; r0 < mn; r0 += 64) {
        const uint32_t i = r0 + lane;
        uint2 ids = make_uint2(0, 0);
        if (i < mn) ids = hit_list(im, make_uint2(sorted[i].y, sorted[i].x >> 16));
        uint32_t t;
        const uint32_t before = wave_excl_scan(ids.y, t);
        if (i < mn) emit(a, unit_lo + (sorted[i].x & 0xffffu), ids, dst, base + before, cap, ut);
        base += t;
    }
}

// Redo unit u from the root, in position order, when its match list overflows.
__device__ __forceinline__ void unit_from_root(const ScanArgs &a, uint64_t u, uint64_t unit_lo,
                                               uint32_t n_chunks, uint32_t *bnd) {
    const ImageView &im = a.im;
    const uint32_t lane = lane_id();
    const uint64_t lo_valid = a.shift, hi_valid = a.shift + a.total;
    uint32_t total = 0;
    unsigned long long base = 0;
    for (int pass = 0; pass < 2; pass++) {
        for (uint32_t g = 0; g < n_chunks; g++) {
            const uint64_t lo = unit_lo + (uint64_t)g * kChunk;
            bool dirty;
            unsigned long long next_bnd;
            chunk_bounds(a, lo / kChunk, lo, bnd, dirty, next_bnd);
            for (uint32_t r = 0; r < kChunk / 64; r++) {
                const uint32_t pl = r * 64 + lane;
                const uint64_t p = lo + pl;
                uint2 ids = make_uint2(0, 0);
                if (p >= lo_valid && p < hi_valid) {
                    const uint32_t lim = limit_after(bnd, dirty, lo, pl, next_bnd);
                    const uint2 h = walk_g(im, a.base, p, lim, 0, 0, hi_valid);
                    if (h.y) ids = hit_list(im, h);
                }
                uint32_t t;
                const uint32_t before = wave_excl_scan(ids.y, t);
                if (pass == 1 && ids.y) emit(a, p, ids, a.stage, base + before, a.stage_cap);
                if (pass == 0) total += t; else base += t;
            }
            wave_sync();
        }
        if (pass == 0) {
            unsigned long long b = 0;
            if (lane == 0) {
                b = atomicAdd(a.stage_cursor, (unsigned long long)total);
                a.unit_count[u] = total;
                a.unit_off[u] = b;
                if (total) atomicAdd(&a.blocksum[u >> kSumShift], (unsigned long long)total);
            }
            base = __shfl(b, 0, 64);
        }
    }
}

// MODE 1: byte symbols, K = 2, 8-bit folded table.  MODE 2: same, 16-bit.
// MODE 0: any image (symbol table, any K, table or plain level bitmap, or
// the root bitmap when K = 0).
// SPLIT: stop after stage 2 and write each unit's walk candidates to global
// memory for walk_units (the walks then run at the occupancy of a kernel
// without the LDS tables); otherwise walk and emit here.
// P4 (modes 1 and 2, split): stage 2 checks the prefix-4 filter, which the
// launch guarantees, and has no child-record path.
// TX: 1 for one text (every chunk's boundaries follow from the text's two
// ends; no boundary record is loaded), 2 for batches (the plan's record per
// chunk), 0 decided at run time; the split kernels of modes 1..3 come in
// forms 1 and 2, so that neither keeps the other's state in registers.
template <int MODE, bool SPLIT, bool P4 = false, int TX = 0>
__global__ __launch_bounds__(1024) void scan_waves(const ScanArgs a) {
    extern __shared__ __align__(16) uint8_t lds[];
    const ImageView &im = a.im;
    const uint32_t tid = threadIdx.x;
    const uint32_t nthreads = blockDim.x;
    const uint32_t waves = nthreads >> 6;
    // the wave index is wave-uniform: keep it (and all unit bookkeeping) scalar
    const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane((int)(tid >> 6));
    const uint32_t lane = tid & 63;

    uint8_t *s_ftab = lds + a.off_ftab;
    // level index in LDS: per 32 codes the bit map and the first node
    // (level start + rank) of the word
    uint2 *s_lvl = (uint2 *)(lds + a.off_bits);
    uint32_t *s_root = (uint32_t *)(lds + a.off_root);
    uint32_t *s_krec = (uint32_t *)(lds + a.off_krec);
    uint32_t *s_pfx4 = (uint32_t *)(lds + a.off_pfx4);
    const uint8_t *pfx4_base = lds + a.off_pfx4;
    uint8_t *s_sym = lds + a.off_sym;

    // the split path needs no reset kernel: the walk kernel, the first to
    // count into them, starts after this kernel ends
    if (SPLIT) {
        const uint32_t gt = blockIdx.x * nthreads + tid;
        if (gt == 0) *a.stage_cursor = 0;
        for (uint32_t i = gt; i < a.n_sums; i += gridDim.x * nthreads) a.blocksum[i] = 0;
    }

    // ---- shared tables, once per workgroup
    {
        // the filter table and the prefix-4 filter by direct global-to-LDS
        // loads: 1 KiB per wave instruction, no registers, one wait
        const uint4 *tab = (const uint4 *)(a.q16_words ? (const void *)im.q16 : (const void *)im.ftab);
        const uint32_t n_tab = a.ftab_bytes / 16, n_p4 = a.pfx4_words / 4;
        for (uint32_t b = wave * 64; b < n_tab; b += waves * 64)
            if (b + lane < n_tab)
                __builtin_amdgcn_global_load_lds((const void *)(tab + b + lane),
                                                 (__attribute__((address_space(3))) void *)(s_ftab + 16 * b), 16, 0, 0);
        for (uint32_t b = wave * 64; b < n_p4; b += waves * 64)
            if (b + lane < n_p4)
                __builtin_amdgcn_global_load_lds((const void *)((const uint4 *)im.pfx4 + b + lane),
                                                 (__attribute__((address_space(3))) void *)((uint8_t *)s_pfx4 + 16 * b), 16, 0, 0);
        for (uint32_t i = 4 * n_p4 + tid; i < a.pfx4_words; i += nthreads) s_pfx4[i] = im.pfx4[i];
    }
    for (uint32_t i = tid; i < a.lvl_lds; i += nthreads) {
        const uint2 e = ((const uint2 *)im.lvl)[i];
        s_lvl[i] = make_uint2(e.x, e.y + im.lvl_start);
    }
    for (uint32_t i = tid; i < a.root_words; i += nthreads) s_root[i] = im.root_bits[i];
    for (uint32_t i = tid; i < a.krec_words; i += nthreads) s_krec[i] = im.krec[i];
    __builtin_amdgcn_s_waitcnt(0);
    if (MODE == 0 && !im.identity)
        for (uint32_t i = tid; i < 256; i += nthreads) s_sym[i] = im.sym[i];
    __syncthreads();

    uint8_t *wbase = lds + a.off_wave + wave * a.wave_bytes;
    uint8_t *wtext = wbase;
    uint32_t *wbnd = (uint32_t *)(wbase + a.woff_bnd);
    uint32_t *wq = (uint32_t *)(wbase + a.woff_queue);
    uint2 *wc = (uint2 *)(wbase + a.woff_cand);
    uint2 *wm = (uint2 *)(wbase + a.woff_match);

    const uint64_t lo_valid = a.shift, hi_valid = a.shift + a.total;
    const uint64_t n_units = a.n_tiles;
    const uint32_t G = a.group;
    const uint64_t stride = (uint64_t)gridDim.x * waves;
    const uint32_t K = im.K;
    const uint32_t ccap = a.ccap, mcap = a.mcap;
    const bool krec = !P4 && a.krec_words != 0;
    const bool pfx4 = P4 || a.pfx4_words != 0;
    // text boundaries per chunk from the batch plan (TX 2), from the one
    // text's two ends (TX 1), or as chunk_info says (TX 0)
    const bool has_info = TX == 0 ? a.chunk_info != nullptr : TX == 2;

    // Chunk c covers frame bytes [c KiB, (c + 1) KiB); chunks 0 .. n_ch - 1
    // hold text.  Chunk and unit indices are 32-bit (the host refuses texts
    // of 2^31 chunks or more).
    const uint32_t n_ch = (uint32_t)a.n_plan;
    const uint32_t n_u = (uint32_t)n_units;
    const uint32_t ustride = (uint32_t)stride;
    // chunks 1 .. n_ch - 2: every 16-byte block of the chunk and the block
    // after it hold text, and neither end of the text lies inside it
    const uint32_t n_in = n_ch >= 2 ? n_ch - 2 : 0u;
    auto interior = [&](uint32_t c) -> bool { return c - 1u < n_in; };
    // chunks of unit u that hold text
    auto unit_chunks = [&](uint32_t u) -> uint32_t { return min(G, n_ch - u * G); };

    // The wave's chunks in order: units u0, u0 + stride, ...; chunks 0 .. n-1
    // of each.
    struct Cur {
        uint32_t u, g, n;
    };
    auto start_at = [&](uint32_t uu) -> Cur { return Cur{uu, 0u, uu < n_u ? unit_chunks(uu) : 0u}; };
    auto advance = [&](Cur &c) {
        if (++c.g >= c.n) {
            c.u += ustride;
            c.g = 0;
            c.n = c.u < n_u ? unit_chunks(c.u) : 0u;
        }
    };
    // One chunk's loads: its 1 KiB (16 bytes a lane), the next 16 bytes of
    // each lane (lane 63: the 16 bytes after the chunk) and its boundary
    // word.  They are issued
    // unconditionally (at the text's first or last block for the chunks at
    // its two ends and past the end of the wave's work), so that the wait for
    // a chunk's data counts only the loads issued after it, and the next
    // chunk's loads are in flight while it is filtered.  Bytes outside the
    // text are never reported: every start position is checked against the
    // text range and every walk stops at the end of its text.
    struct Slot {
        uint4 v, h;
        uint2 info;
    };
    const uint64_t blk_lo = lo_valid & ~15ull;
    const uint64_t blk_hi = (hi_valid - 1) & ~15ull;
    const uint32_t lane16 = 16u * lane;
    auto load_slot = [&](const Cur &cr) -> Slot {
        const uint32_t c = cr.u * G + cr.g;
        const uint64_t lo = (uint64_t)c * kChunk;
        Slot sl;
        // a wave-uniform base and 32-bit lane offsets; at the ends the
        // offsets are clamped to [blk_lo, blk_hi] - base
        uint64_t sb = lo;
        uint32_t ov = lane16, oh = lane16 + 16u;
        if (!interior(c)) {
            sb = lo < blk_hi ? lo : blk_hi;
            const uint32_t lo_off = blk_lo > sb ? (uint32_t)(blk_lo - sb) : 0u;
            const uint32_t hi_off = (uint32_t)umin64(blk_hi - sb, 0x7fffffffull);
            ov = min(max(ov, lo_off), hi_off);
            oh = min(max(oh, lo_off), hi_off);
        }
        sl.v = *(const uint4 *)(a.base + sb + ov);
        sl.h = *(const uint4 *)(a.base + sb + oh);
        if (TX == 1) {
            sl.info = make_uint2(0u, 0u);
        } else {
            const uint2 *ip = has_info ? a.chunk_info + min(c, n_ch - 1) : (const uint2 *)(a.base + blk_lo);
            sl.info = *ip;
        }
        return sl;
    };

    // The split kernels of modes 1 and 2 filter two chunks of a unit with one
    // compaction and one run of stage-2 rounds when neither holds a text
    // boundary (PAIR): their window is 2 KiB + 16 bytes, and the stage-1
    // queue holds QCAP positions per round (a round with more takes the hit
    // masks PB bits at a time).
    constexpr bool PAIR = SPLIT && (MODE == 1 || MODE == 2);
    constexpr uint32_t QCAP = PAIR ? kQ16 / 2 : kQ16;
    constexpr uint32_t PB = QCAP / 64;
    uint16_t *const wq16 = (uint16_t *)wq;

    // ---- stage 1 of modes 1 and 2 over a lane's 16 positions into a hit
    // mask: code = (B[j] << 8) | B[j+1] indexes the table, B[j+2] picks the
    // folded child bit.  The table is the first LDS section and the kernel
    // has no static LDS, so the code is the LDS address; all sixteen lookups
    // are issued before any is used.  w: the lane's 16 bytes and the next 4.
    auto stage1_mask = [&](const uint32_t *w) -> uint32_t {
        uint32_t ent[16];
#pragma unroll
        for (int j = 0; j < 16; j++) {
            const uint32_t r = j & 3;
            const uint32_t code = __builtin_amdgcn_perm(w[(j >> 2) + 1], w[j >> 2], 0x0c0c0000u | (r << 8) | (r + 1));
            ent[j] = MODE == 1 ? (uint32_t)lds_tab8()[code] : (uint32_t)lds_tab16()[code];
        }
        uint32_t bit[16];
#pragma unroll
        for (int j = 0; j < 16; j++) {
            const uint32_t nx = __builtin_amdgcn_ubfe(w[(j + 2) >> 2], 8 * ((j + 2) & 3), MODE == 1 ? 3 : 4);
            bit[j] = __builtin_amdgcn_ubfe(ent[j], nx, 1);
        }
        return gather_bits(bit, std::make_integer_sequence<int, 15>{});
    };
    // ---- stage 2 of modes 1 and 2 for a position whose first four bytes
    // are `by` and that passed the range checks: the prefix-4 filter or the
    // exact third byte against the depth-2 node's child labels; v = the
    // depth-2 node (from the level index)
    auto stage2_check = [&](uint32_t by, bool &pass2, uint32_t &v) {
        if (pass2 && pfx4) {
            // both bits of the first four bytes' hash must be set, in the
            // word that h1 names
            const uint32_t t8 = by >> 8;
            const uint32_t h1 = __umul24(by, im.pfx4_m1) + t8;
            const uint32_t h2 = __umul24(t8, im.pfx4_m2) + by;
            const uint32_t sh = 32u - im.pfx4_log2;
            const uint32_t wd = *(const uint32_t *)(pfx4_base + ((h1 >> (sh + 5u)) << 2));
            pass2 = ((wd >> ((h1 >> sh) & 31u)) & (wd >> (h2 >> 27)) & 1u) != 0;
        }
        if (pass2) {
            const uint32_t code = __builtin_amdgcn_perm(0u, by, 0x0c0c0001u);
            const uint2 lv = s_lvl[code >> 5];
            v = lv.y + (uint32_t)__builtin_popcount(__builtin_amdgcn_ubfe(lv.x, 0, code));
            if (krec) {
                // up to three child labels, or a count above 3
                const uint32_t rec = s_krec[v - im.lvl_start];
                const uint32_t ncc = rec >> 24;
                if (ncc <= 3) {
                    const uint32_t c = (by >> 16) & 0xffu;
                    const uint32_t x = rec ^ (c * 0x00010101u);
                    const uint32_t mm = (x - 0x00010101u) & ~x & 0x00808080u;
                    pass2 = mm != 0 && ((uint32_t)__builtin_ctz(mm) >> 3) < ncc;
                }
            }
        }
    };

    uint32_t cn = 0, mn = 0;  // candidates, matches of the current unit (wave-uniform)
    // split kernels: queue a candidate of unit u (ballot mask mk over the
    // wave) with the 8 text bytes after the level index, B[pl+K ..
    // pl+K+8), so that short walks read no text from global memory (bytes
    // past the window are not text of it; the walk knows how many are valid)
    auto push_cand = [&](uint32_t u, bool pass, unsigned long long mk, uint32_t entry, uint32_t v,
                         uint32_t pl) {
        const uint32_t idx = cn + mbcnt(mk);
        if (pass && idx < a.cand_cap) {
            const uint32_t q = pl + K, q4 = q & ~3u;
            const uint32_t e0 = *(const uint32_t *)(wtext + q4);
            const uint32_t e1 = *(const uint32_t *)(wtext + q4 + 4);
            const uint32_t e2 = *(const uint32_t *)(wtext + q4 + 8);
            a.cand[(uint64_t)u * a.cand_cap + idx] =
                make_uint4(entry, v, __builtin_amdgcn_alignbyte(e1, e0, q & 3u), __builtin_amdgcn_alignbyte(e2, e1, q & 3u));
        }
        cn += (uint32_t)__popcll(mk);
    };

    // Filter chunk cc with the data of slot sl, close its unit after its last
    // chunk, and step cc to the wave's next chunk (nothing past the wave's
    // last chunk).
    auto chunk = [&](const Slot &sl, Cur &cc) {
        if (cc.u >= n_u) return;
        const uint32_t u = cc.u, g = cc.g, nch = cc.n;
        const uint32_t c = u * G + g;
        const uint64_t unit_lo = (uint64_t)(u * G) * kChunk;
        const uint64_t chunk_lo = (uint64_t)c * kChunk;
        const bool inner = interior(c);
        if (g == 0) {
            cn = 0;
            mn = 0;
        }
        // queue a candidate (ballot mask mk over the wave)
        auto push = [&](bool pass, unsigned long long mk, uint32_t entry, uint32_t v, uint32_t pl) {
            if (SPLIT) {
                push_cand(u, pass, mk, entry, v, pl);
                return;
            }
            const uint32_t idx = cn + mbcnt(mk);
            if (pass) wc[idx] = make_uint2(entry, v);
            cn += (uint32_t)__popcll(mk);
        };

        // walk every queued candidate; matches go to wm
        auto flush = [&]() {
            if (SPLIT) return;
            for (uint32_t r0 = 0; r0 < cn; r0 += 64) {
                const uint32_t e = r0 + lane;
                uint2 h = make_uint2(0, 0);
                uint32_t pr = 0;
                if (e < cn) {
                    const uint2 c = wc[e];
                    pr = c.x & 0xffffu;
                    h = walk_g(im, a.base, unit_lo + pr, c.x >> 16, c.y, K, hi_valid);
                }
                const bool got = h.y != 0;
                const unsigned long long mk = __ballot(got);
                if (got) {
                    const uint32_t slot = mn + mbcnt(mk);
                    if (slot < mcap) wm[slot] = make_uint2(pr | (h.y << 16), h.x);
                }
                mn += (uint32_t)__popcll(mk);
            }
            cn = 0;
        };

        *(uint4 *)(wtext + 16 * lane) = sl.v;
        if (lane_at(c) == 63) *(uint4 *)(wtext + kChunk) = sl.h;
        wave_sync();

        // Text boundaries of the chunk: the distance from its start to the
        // first boundary at or past its end, and up to four inside it in
        // ascending order (from the batch plan, or from the text's two ends);
        // more than four: the bit map in LDS.
        // (read in every case: a load left unread would hold up the next
        // load into its registers)
        uint32_t bx = (uint32_t)__builtin_amdgcn_readfirstlane((int)sl.info.x);
        uint32_t by = (uint32_t)__builtin_amdgcn_readfirstlane((int)sl.info.y);
        if (!has_info && inner) {
            // no end of the text in the chunk; the next one is its end
            bx = n_ch - c > 128u ? 0x1ffffu : min((uint32_t)hi_valid - (uint32_t)chunk_lo, 0x1ffffu);
            by = 0;
        } else if (!has_info) {
            // the text's first byte and its end: ascending, at most one of
            // each in the chunk
            const bool lo_in = lo_valid >= chunk_lo && lo_valid < chunk_lo + kChunk;
            const bool hi_in = hi_valid >= chunk_lo && hi_valid < chunk_lo + kChunk;
            const uint32_t lo_rel = (uint32_t)(lo_valid - chunk_lo) & 0x3ffu;
            const uint32_t hi_rel = (uint32_t)(hi_valid - chunk_lo) & 0x3ffu;
            const uint64_t hi_dist = hi_valid - chunk_lo;
            const uint32_t nrel0 = hi_in || hi_dist > 0x1ffffull ? 0x1ffffu : (uint32_t)hi_dist;
            const uint32_t cnt = (uint32_t)lo_in + (uint32_t)hi_in;
            bx = nrel0 | (cnt << 17) | ((lo_in ? lo_rel : hi_rel) << 20);
            by = lo_in && hi_in ? hi_rel : 0u;
        }
        const uint32_t bcnt = (bx >> 17) & 7u;
        const uint32_t nrel = bx & 0x1ffffu;
        bool dirty = false;
        unsigned long long next_bnd = 0;
        if (bcnt > 4) chunk_bounds(a, c, chunk_lo, wbnd, dirty, next_bnd);
        // distance from chunk position pl to the end of its text, at most 0xffff
        auto lim_of = [&](uint32_t pl) -> uint32_t {
            if (bcnt > 4) return limit_after(wbnd, dirty, chunk_lo, pl, next_bnd);
            uint32_t nb = nrel;
            if (bcnt) {
                const uint32_t b0 = bx >> 20, b1 = by & 0x3ffu, b2 = (by >> 10) & 0x3ffu, b3 = by >> 20;
                // the list is ascending and unused entries are 0: the least
                // entry above pl is the first boundary after it
                nb = b3 > pl ? b3 : nb;
                nb = b2 > pl ? b2 : nb;
                nb = b1 > pl ? b1 : nb;
                nb = b0 > pl ? b0 : nb;
            }
            return min(nb - pl, 0xffffu);
        };
        // valid chunk positions (inside the batch's or the text's range)
        uint32_t vlo = 0, vhi = kWin;
        if (!inner) {
            vlo = lo_valid > chunk_lo ? (uint32_t)umin64(lo_valid - chunk_lo, kWin) : 0u;
            vhi = hi_valid > chunk_lo ? (uint32_t)umin64(hi_valid - chunk_lo, kWin) : 0u;
        }

        // the lane's 16 bytes and the 16 after them
        const uint32_t w[8] = {sl.v.x, sl.v.y, sl.v.z, sl.v.w, sl.h.x, sl.h.y, sl.h.z, sl.h.w};

        // ---- stage 2: the exact byte after the level index, the end of
        // the text, and the depth-K node; survivors become candidates.
        // decode(e) gives (window position, K-symbol code) of entry e.
        auto stage2 = [&](uint32_t qn, auto decode) {
            for (uint32_t r0 = 0; r0 < qn; r0 += 64) {
                if (!SPLIT && cn + 64 > ccap) flush();
                const uint32_t e = r0 + lane;
                bool pass2 = false;
                uint32_t entry = 0, v = 0;
                if (e < qn) {
                    const uint2 pc = decode(e);
                    const uint32_t pl = pc.x;
                    const uint64_t p = chunk_lo + pl;
                    const uint32_t lim = lim_of(pl);
                    // the filter read K + 1 bytes: all must be in this text
                    pass2 = p >= lo_valid && p < hi_valid && lim > K;
                    if (pass2 && K) {
                        const uint32_t code = pc.y;
                        const uint2 lv = s_lvl[code >> 5];
                        // (the field width is taken from the code's low five bits)
                        v = lv.y + (uint32_t)__builtin_popcount(__builtin_amdgcn_ubfe(lv.x, 0, code));
                        if (krec) {
                            const uint32_t rank = v - im.lvl_start;
                            // up to three child labels, or 0xff.. for more
                            const uint32_t rec = s_krec[rank];
                            const uint32_t ncc = rec >> 24;
                            if (ncc <= 3) {
                                const uint32_t c = wtext[pl + K];
                                const uint32_t x = rec ^ (c * 0x00010101u);
                                const uint32_t mm = (x - 0x00010101u) & ~x & 0x00808080u;
                                pass2 = mm != 0 && ((uint32_t)__builtin_ctz(mm) >> 3) < ncc;
                            }
                        }
                    }
                    entry = (uint32_t)(g * kChunk + pl) | (lim << 16);
                }
                push(pass2, __ballot(pass2), entry, v, entry & (kChunk - 1));
            }
            wave_sync();
        };

        if (MODE == 1 || MODE == 2) {
            const uint32_t hm = stage1_mask(w);
            __builtin_amdgcn_s_setprio(2);  // compaction and stage 2 (as in pair())
            // compact the hits of the wave, at most QCAP per round
            uint32_t tot;
            const uint32_t off_all = wave_excl_scan((uint32_t)__builtin_popcount(hm), tot);
            const int parts = tot > QCAP ? (int)(16 / PB) : 1;
            for (int part = 0; part < parts; part++) {
                uint32_t mset = hm, o = off_all, qn = tot, jb = 0;
                if (parts > 1) {
                    jb = (uint32_t)part * PB;
                    mset = (hm >> jb) & ((1u << PB) - 1u);
                    o = wave_excl_scan((uint32_t)__builtin_popcount(mset), qn);
                }
                while (mset) {
                    const uint32_t j = (uint32_t)__builtin_ctz(mset);
                    wq16[o++] = (uint16_t)(16 * lane + jb + j);
                    mset &= mset - 1;
                }
                wave_sync();
                // ---- stage 2 (K = 2): the text's end, then the prefix-4
                // filter or the child labels and the depth-2 node.  The
                // filters read 4 bytes (prefix-4 filter: every pattern is
                // that long) or 3 (child labels); in a chunk without
                // boundaries the positions [vlo, top) have them in the text
                const uint32_t need = pfx4 ? 4u : 3u;
                const uint32_t top = min(vhi, nrel + 1u - need);
                for (uint32_t r0 = 0; r0 < qn; r0 += 64) {
                    if (!SPLIT && cn + 64 > ccap) flush();
                    const uint32_t e = r0 + lane;
                    bool pass2 = false;
                    uint32_t entry = 0, v = 0;
                    if (e < qn) {
                        const uint32_t pl = wq16[e];
                        const uint32_t a4 = pl & ~3u;
                        const uint32_t d0 = *(const uint32_t *)(wtext + a4);
                        const uint32_t d1 = *(const uint32_t *)(wtext + a4 + 4);
                        const uint32_t by = __builtin_amdgcn_alignbyte(d1, d0, pl);  // B[pl..pl+3]
                        uint32_t lim;
                        if (bcnt == 0) {
                            lim = min(nrel - pl, 0xffffu);
                            pass2 = pl - vlo < top - vlo;
                        } else {
                            lim = lim_of(pl);
                            pass2 = pl >= vlo && pl < vhi && lim >= need;
                        }
                        stage2_check(by, pass2, v);
                        entry = (uint32_t)(g * kChunk + pl) | (lim << 16);
                    }
                    push(pass2, __ballot(pass2), entry, v, entry & (kChunk - 1));
                }
                wave_sync();
            }
            __builtin_amdgcn_s_setprio(0);
        } else if (MODE == 3) {
            // ---- four-symbol alphabets.  Stage 1: the lane's 32 bytes
            // as 2-bit symbols (symbol j at bits 2j of P), the 16-symbol
            // key of position j = bits [2j, 2j + 32), one LDS word of the
            // filter per position, two bits of it tested.
            const uint32_t qa = im.qa, qb = im.qb;
            // 2-bit symbols of the four bytes of x in one byte: a dot
            // product of the per-byte symbols with weights 1, 4, 16, 64
            auto pack4 = [&](uint32_t x) -> uint32_t {
                const uint32_t t = ((x >> qa) ^ (x >> qb)) & 0x03030303u;
                return __builtin_amdgcn_udot4(t, 0x40100401u, 0u, false);
            };
            const uint32_t P0 = pack4(w[0]) | pack4(w[1]) << 8 | pack4(w[2]) << 16 | pack4(w[3]) << 24;
            const uint32_t P1 = pack4(w[4]) | pack4(w[5]) << 8 | pack4(w[6]) << 16 | pack4(w[7]) << 24;
            const uint32_t qsh = 32u - im.q16_lw;
            uint32_t hh[16], ent[16];
#pragma unroll
            for (int j = 0; j < 16; j++) {
                const uint32_t key = j == 0 ? P0 : __builtin_amdgcn_alignbit(P1, P0, 2 * j);
                hh[j] = __umul24(key, im.q16_mul) + (key >> 8);  // 24 x 24-bit multiply
                ent[j] = lds_tab32()[hh[j] >> qsh];
            }
            uint32_t hm = 0;
#pragma unroll
            for (int j = 0; j < 16; j++)
                hm |= ((ent[j] >> hh[j]) & (ent[j] >> (hh[j] >> 5)) & 1u) << j;
            __builtin_amdgcn_s_setprio(2);  // compaction and stage 2 (as in pair())
            uint32_t tot;
            const uint32_t off_all = wave_excl_scan((uint32_t)__builtin_popcount(hm), tot);
            const int rounds = tot > kQ16 ? 2 : 1;
            for (int half = 0; half < rounds; half++) {
                uint32_t mset = hm, o = off_all, qn = tot, jb = 0;
                if (rounds == 2) {
                    mset = half == 0 ? (hm & 0xffu) : (hm >> 8);
                    jb = half == 0 ? 0u : 8u;
                    o = wave_excl_scan((uint32_t)__builtin_popcount(mset), qn);
                }
                while (mset) {
                    const uint32_t j = (uint32_t)__builtin_ctz(mset);
                    wq16[o++] = (uint16_t)(16 * lane + jb + j);
                    mset &= mset - 1;
                }
                wave_sync();
                // ---- stage 2: the 16 bytes all in this text and all of
                // the alphabet, the key's fingerprint in its buckets,
                // then the depth-K node from the level index
                for (uint32_t r0 = 0; r0 < qn; r0 += 64) {
                    const uint32_t e = r0 + lane;
                    bool pass2 = false;
                    uint32_t entry = 0, v = 0, pl = 0;
                    if (e < qn) {
                        pl = wq16[e];
                        const uint32_t lim = lim_of(pl);
                        pass2 = pl >= vlo && pl < vhi && lim >= 16u;
                        entry = (uint32_t)(g * kChunk + pl) | (lim << 16);
                        uint32_t key = 0;
                        if (pass2) {
                            const uint32_t *t32 = (const uint32_t *)(wtext + (pl & ~3u));
                            uint32_t d[5];
#pragma unroll
                            for (int k = 0; k < 5; k++) d[k] = t32[k];
                            bool valid = true;
#pragma unroll
                            for (int k = 0; k < 4; k++) {
                                const uint32_t x = __builtin_amdgcn_alignbyte(d[k + 1], d[k], pl & 3u);
                                const uint32_t t = ((x >> qa) ^ (x >> qb)) & 0x03030303u;
                                valid = valid && __builtin_amdgcn_perm(0u, im.qalph, t) == x;
                                key |= __builtin_amdgcn_udot4(t, 0x40100401u, 0u, false) << (8 * k);
                            }
                            pass2 = valid;
                        }
                        if (pass2 && im.qfp_lb) {
                            const uint32_t h2 = key * a.im.pfx4_mul;
                            const uint32_t fp = (h2 & 0xffffu) | 1u;
                            const uint32_t nb = 1u << im.qfp_lb;
                            const uint32_t bk = h2 >> (32u - im.qfp_lb);
                            const uint4 f[2] = {im.qfp[bk], im.qfp[(bk + 1) & (nb - 1)]};
                            const uint32_t fp2 = fp * 0x00010001u;
                            uint32_t hit = 0;
#pragma unroll
                            for (int k = 0; k < 2; k++) {
                                const uint32_t wv[4] = {f[k].x, f[k].y, f[k].z, f[k].w};
#pragma unroll
                                for (int q = 0; q < 4; q++) {
                                    const uint32_t x = wv[q] ^ fp2;  // a zero half = equal fingerprint
                                    hit |= (x - 0x00010001u) & ~x & 0x80008000u;
                                }
                            }
                            pass2 = hit != 0;
                        }
                        if (pass2) {
                            // depth-K code, first symbol highest: the low
                            // 2K bits of the key with the symbol order reversed
                            const uint32_t r = __builtin_bitreverse32(key);
                            uint32_t code = ((r >> 1) & 0x55555555u) | ((r & 0x55555555u) << 1);
                            code >>= 32u - 2u * K;
                            const uint2 lv = ((const uint2 *)im.lvl)[code >> 5];
                            v = im.lvl_start + lv.y +
                                (uint32_t)__builtin_popcount(lv.x & ((1u << (code & 31)) - 1u));
                            pass2 = (lv.x >> (code & 31)) & 1u;
                        }
                    }
                    push(pass2, __ballot(pass2), entry, v, pl);
                }
                wave_sync();
            }
            __builtin_amdgcn_s_setprio(0);
        } else {
            // generic filter: rolling code over L = K + m symbols
            const uint32_t b = im.b;
            const uint32_t m = (K >= 1 && a.fold) ? im.fold_syms : 0u;
            const uint32_t L = K >= 1 ? K + m : 1u;
            const uint32_t full_mask = (b * L >= 32) ? 0xffffffffu : ((1u << (b * L)) - 1u);
            const uint32_t fmask = (a.fold - 1u) & ((b * m >= 32) ? 0xffffffffu : ((1u << (b * m)) - 1u));
            uint32_t full = 0, run = 0;
            // the first L - 1 symbols of the lane window
#pragma unroll
            for (int j = 0; j < 15; j++) {
                if ((uint32_t)j + 1 >= L) continue;
                const uint32_t byte = wbyte(w, j);
                uint32_t s = byte;
                bool ok = true;
                if (!im.identity) { s = s_sym[byte]; ok = s != 0xffu; }
                run = ok ? run + 1 : 0u;
                full = ((full << b) | (s & 0xffu)) & full_mask;
            }
#pragma unroll
            for (int pass = 0; pass < 16 / (int)kPPL; pass++) {
                uint32_t qn = 0;
#pragma unroll
                for (int jj = 0; jj < (int)kPPL; jj++) {
                    const int j = pass * (int)kPPL + jj;
                    // the symbol at window byte j + L - 1 completes position j
                    const uint32_t byte = wtext[16 * lane + j + L - 1];
                    uint32_t s = byte;
                    bool ok = true;
                    if (!im.identity) { s = s_sym[byte]; ok = s != 0xffu; }
                    run = ok ? run + 1 : 0u;
                    full = ((full << b) | (s & 0xffu)) & full_mask;
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
                            hit = (s_lvl[code >> 5].x >> (code & 31)) & 1u;
                        }
                    }
                    const unsigned long long mk = __ballot(hit != 0);
                    if (hit) wq[qn + mbcnt(mk)] = ((16 * lane + j) << 20) | code;
                    qn += (uint32_t)__popcll(mk);
                }
                wave_sync();
                stage2(qn, [&](uint32_t e) {
                    const uint32_t ent = wq[e];
                    return make_uint2(ent >> 20, ent & 0xfffffu);
                });
            }
        }
        // the unit's last chunk: hand over or emit its results
        if (g + 1 == nch) {
            if (SPLIT) {
                if (lane_at(u) == 0) a.cand_count[u] = cn;
            } else {
                flush();
                wave_sync();
                // ---- this unit's matches, in (pos, id) order
                if (mn <= mcap)
                    emit_unit(a, u, unit_lo, wm, mn, (uint2 *)wq);
                else
                    unit_from_root(a, u, unit_lo, nch, wbnd);
                wave_sync();
            }
        }
        advance(cc);
    };

    // Chunks cc and cc + 1 from slots sa and sb: together when they are
    // chunks g and g + 1 of one unit, both inside the text (see interior)
    // and neither holding a text boundary; else one by one.  Together they
    // share one window (chunk g at 0, chunk g + 1 at kChunk), one
    // compaction of their 32 stage-1 bits per lane and one run of stage-2
    // rounds over positions 0 .. 2 kChunk - 1 relative to chunk g.
    auto pair = [&](const Slot &sa, const Slot &sb, Cur &cc) {
        if (cc.u >= n_u) return;
        const uint32_t u = cc.u, g = cc.g, nch = cc.n;
        const uint32_t c = u * G + g;
        const uint32_t bxa = (uint32_t)__builtin_amdgcn_readfirstlane((int)sa.info.x);
        const uint32_t bxb = (uint32_t)__builtin_amdgcn_readfirstlane((int)sb.info.x);
        bool together = g + 1 < nch && interior(c) && interior(c + 1);
        if (has_info) together = together && ((bxa | bxb) & (7u << 17)) == 0;
        if (!together) {
            chunk(sa, cc);
            chunk(sb, cc);
            return;
        }
        if (g == 0) cn = 0;
        const uint64_t chunk_lo = (uint64_t)c * kChunk;
        *(uint4 *)(wtext + 16 * lane) = sa.v;
        *(uint4 *)(wtext + kChunk + 16 * lane) = sb.v;
        if (lane_at(c) == 63) *(uint4 *)(wtext + 2 * kChunk) = sb.h;
        wave_sync();
        // distance from chunk g's start to the first text boundary at or
        // past its end, which lies at or past chunk g + 1's end
        const uint32_t nrel = has_info
                                  ? (bxa & 0x1ffffu)
                                  : (n_ch - c > 128u ? 0x1ffffu : min((uint32_t)hi_valid - (uint32_t)chunk_lo, 0x1ffffu));
        const uint32_t wa[5] = {sa.v.x, sa.v.y, sa.v.z, sa.v.w, sa.h.x};
        const uint32_t wb[5] = {sb.v.x, sb.v.y, sb.v.z, sb.v.w, sb.h.x};
        // bit j < 16: position 16 lane + j of chunk g; bit 16 + j: of chunk g + 1
        const uint32_t hm = stage1_mask(wa) | (stage1_mask(wb) << 16);
        // compaction and stage 2 at raised wave priority: their chains of
        // dependent scans and LDS reads issue ahead of other waves' stage 1
        __builtin_amdgcn_s_setprio(2);
        uint32_t tot;
        const uint32_t off_all = wave_excl_scan((uint32_t)__builtin_popcount(hm), tot);
        const int parts = tot > QCAP ? (int)(32 / PB) : 1;
        for (int part = 0; part < parts; part++) {
            uint32_t mset = hm, o = off_all, qn = tot, jb = 0;
            if (parts > 1) {
                jb = (uint32_t)part * PB;
                mset = (hm >> jb) & ((1u << PB) - 1u);
                o = wave_excl_scan((uint32_t)__builtin_popcount(mset), qn);
            }
            // bit j < 16: position 16 lane + j of chunk g, else 16 lane + j - 16
            // of chunk g + 1 (one compare and select per survivor)
            const uint32_t pa = 16 * lane, pb = kChunk - 16 + 16 * lane;
            if (parts == 1) {
                while (mset) {
                    const uint32_t j = (uint32_t)__builtin_ctz(mset);
                    wq16[o++] = (uint16_t)(j + (j < 16 ? pa : pb));
                    mset &= mset - 1;
                }
            } else {
                const uint32_t pj = jb < 16 ? pa : pb;  // a part's bits lie in one chunk
                while (mset) {
                    const uint32_t j = jb + (uint32_t)__builtin_ctz(mset);
                    wq16[o++] = (uint16_t)(j + pj);
                    mset &= mset - 1;
                }
            }
            wave_sync();
            // ---- stage 2 as in chunk(), for a window without boundaries:
            // positions below top have the bytes the filters read
            const uint32_t need = pfx4 ? 4u : 3u;
            const uint32_t top = min(2 * kChunk + 16, nrel + 1u - need);
            if constexpr (P4) {
                // without branches until the record: lanes past the queue
                // read its last entry (so every lookup stays inside its
                // table) and fail
                const uint32_t sh = 32u - im.pfx4_log2;
                for (uint32_t r0 = 0; r0 < qn; r0 += 64) {
                    const uint32_t e = r0 + lane;
                    const uint32_t pl = wq16[min(e, qn - 1u)];
                    const uint32_t a4 = pl & ~3u;
                    const uint32_t d0 = *(const uint32_t *)(wtext + a4);
                    const uint32_t d1 = *(const uint32_t *)(wtext + a4 + 4);
                    const uint32_t by = __builtin_amdgcn_alignbyte(d1, d0, pl);  // B[pl..pl+3]
                    const uint32_t t8 = by >> 8;
                    const uint32_t h1 = __umul24(by, im.pfx4_m1) + t8;
                    const uint32_t h2 = __umul24(t8, im.pfx4_m2) + by;
                    const uint32_t wd = *(const uint32_t *)(pfx4_base + ((h1 >> (sh + 5u)) << 2));
                    const uint32_t code = __builtin_amdgcn_perm(0u, by, 0x0c0c0001u);
                    const uint2 lv = s_lvl[code >> 5];
                    const uint32_t v = lv.y + (uint32_t)__builtin_popcount(__builtin_amdgcn_ubfe(lv.x, 0, code));
                    const uint32_t lim = min(nrel - pl, 0xffffu);
                    const uint32_t entry = (uint32_t)(g * kChunk + pl) | (lim << 16);
                    // both filter bits, e < qn and pl < top (sign bits of the
                    // differences) in one word, so that no branch splits the
                    // round before its ballot
                    const uint32_t ok = (wd >> ((h1 >> sh) & 31u)) & (wd >> (h2 >> 27)) &
                                        ((e - qn) >> 31) & ((pl - top) >> 31);
                    const bool pass2 = (ok & 1u) != 0;
                    push_cand(u, pass2, __ballot(pass2), entry, v, pl);
                }
            } else {
                for (uint32_t r0 = 0; r0 < qn; r0 += 64) {
                    const uint32_t e = r0 + lane;
                    bool pass2 = false;
                    uint32_t entry = 0, v = 0, pl = 0;
                    if (e < qn) {
                        pl = wq16[e];
                        const uint32_t a4 = pl & ~3u;
                        const uint32_t d0 = *(const uint32_t *)(wtext + a4);
                        const uint32_t d1 = *(const uint32_t *)(wtext + a4 + 4);
                        const uint32_t by = __builtin_amdgcn_alignbyte(d1, d0, pl);  // B[pl..pl+3]
                        const uint32_t lim = min(nrel - pl, 0xffffu);
                        pass2 = pl < top;
                        stage2_check(by, pass2, v);
                        entry = (uint32_t)(g * kChunk + pl) | (lim << 16);
                    }
                    push_cand(u, pass2, __ballot(pass2), entry, v, pl);
                }
            }
            wave_sync();
        }
        __builtin_amdgcn_s_setprio(0);
        // the unit's last two chunks: hand over its candidates
        if (g + 2 == nch && lane_at(u) == 0) a.cand_count[u] = cn;
        advance(cc);
        advance(cc);
    };

    // Three chunks in flight: the loads of the chunk two ahead are issued
    // before a chunk is filtered.  The loop runs over whole groups of three
    // with its one exit at the bottom (slot variables keep their registers
    // and every wait counts only the loads issued after its own); the
    // chunks past the wave's last are loaded at the text's last block and
    // skipped.
    const uint32_t u0 = blockIdx.x * waves + wave;
    uint32_t n_wave = 0;  // chunks of this wave
    if (u0 < n_u) {
        const uint32_t nu = (n_u - u0 + ustride - 1) / ustride;
        n_wave = (nu - 1) * G + unit_chunks(u0 + (nu - 1) * ustride);
    }
    Cur cc = start_at(u0), pc = cc;
    if constexpr (PAIR) {
        // two pairs of chunks in flight, the loop over whole groups of two
        // pairs with its one exit at the bottom
        Slot sa = load_slot(pc);
        advance(pc);
        Slot sb = load_slot(pc);
        advance(pc);
        Slot sc = load_slot(pc);
        advance(pc);
        Slot sd = load_slot(pc);
        advance(pc);
        for (uint32_t grp = 0; grp < (n_wave + 3) / 4; grp++) {
            pair(sa, sb, cc);
            sa = load_slot(pc);
            advance(pc);
            sb = load_slot(pc);
            advance(pc);
            pair(sc, sd, cc);
            sc = load_slot(pc);
            advance(pc);
            sd = load_slot(pc);
            advance(pc);
        }
    } else {
        Slot sa = load_slot(pc);
        advance(pc);
        Slot sb = load_slot(pc);
        advance(pc);
        for (uint32_t grp = 0; grp < (n_wave + 2) / 3; grp++) {
            const Slot sc = load_slot(pc);
            advance(pc);
            chunk(sa, cc);
            sa = load_slot(pc);
            advance(pc);
            chunk(sb, cc);
            sb = load_slot(pc);
            advance(pc);
            chunk(sc, cc);
        }
    }
}

// Walks of the split path: one wave per unit walks the unit's candidates
// (stage-2 survivors, in position order) and stages its matches in (pos, id)
// order as the fused kernel does.  Lanes walk independently: a lane whose
// walk ends takes the unit's next candidate, so the wave's time follows the
// total number of steps rather than the longest walk of each group of 64.
// One step reads the node record and the text byte together.  A unit whose
// candidates or matches overflowed is redone from the root.
constexpr uint32_t kWalkMcap = 128;

__global__ __launch_bounds__(64 * kWalkWaves, 4) void walk_units(const ScanArgs a) {
    __shared__ __align__(16) uint2 s_match[kWalkWaves][kWalkMcap];
    __shared__ __align__(16) uint2 s_sorted[kWalkWaves][kWalkMcap];
    __shared__ uint32_t s_bnd[kWalkWaves][kWin / 32 + 2];
    const ImageView &im = a.im;
    const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t u = (uint64_t)blockIdx.x * kWalkWaves + wave;
    if (u >= a.n_tiles) return;
    const uint64_t hi_valid = a.shift + a.total;
    const uint64_t unit_lo = u * a.group * kChunk;
    const uint64_t left = hi_valid > unit_lo ? hi_valid - unit_lo : 0;
    const uint32_t nch = (uint32_t)min((uint64_t)a.group, (left + kChunk - 1) / kChunk);
    uint2 *wm = s_match[wave];
    const uint32_t cn = a.cand_count[u];
    // a batch unit inside one text (the texts holding its first chunk and
    // the chunk after it are the same): its matches need no search for their
    // text; the loads overlap the walks
    UnitText ut;
    if (a.offsets) {
        const uint64_t c0 = u * a.group, c1 = c0 + nch;
        if (c1 < a.n_plan) {
            const uint32_t t0 = a.tile_first_text[c0];
            if (t0 == a.tile_first_text[c1]) {
                ut.known = true;
                ut.tid = t0;
                ut.start = a.offsets[t0] + a.shift;
            }
        }
    }
    if (cn <= a.cand_cap) {
        const uint4 *cl = a.cand + u * a.cand_cap;
        const uint32_t K = im.K;
        uint32_t mn = 0, next = 64;  // matches so far, next candidate to hand out
        bool live = lane < cn;
        uint32_t pr = 0, lim = 0, v = 0, d = 0, t0 = 0, t1 = 0, navail = 0;
        uint2 hit = make_uint2(0, 0);
        // a candidate: position, text limit, depth-K node, and the text bytes
        // B[pos+K .. pos+K+navail) that its window held
        auto take = [&](uint32_t e) {
            const uint4 c = cl[e];
            pr = c.x & 0xffffu;
            lim = c.x >> 16;
            v = c.y;
            t0 = c.z;
            t1 = c.w;
            d = K;
            const uint32_t q = (pr & (kChunk - 1)) + K;
            navail = q < kWin ? min(kWin - q, 8u) : 0u;
        };
        if (live) take(lane);
        while (__ballot(live) != 0) {
            bool done = false;
            if (live) {
                const uint64_t p = unit_lo + pr;
                const uint4 r = im.node[v];
                // the text byte at depth d: from the candidate when it holds it
                const uint32_t i = d - K;
                uint32_t cb = 0;
                if (d < lim)
                    cb = i < navail ? (((i < 4 ? t0 : t1) >> (8 * (i & 3))) & 0xffu) : (uint32_t)a.base[p + d];
                if (r.z & kTermFlagD) hit = make_uint2(r.w, r.z >> kCountShiftD);
                const uint32_t nc = r.z & 0xffffu;
                if (nc == 0 || d >= lim) {
                    done = true;
                } else if (r.z & kSkipFlagD) {
                    // no pattern ends inside a single-child run: it matches
                    // whole or the walk ends with nothing more to report
                    const uint32_t len = r.z >> kSkipShiftD;
                    if (d + len > lim) {
                        done = true;
                    } else if (p + d + len + 36 <= hi_valid) {
                        const bool leaf = (r.z & kLeafEndD) != 0;
                        if (!chain_equal_g(a.base, p + d, im.chain, leaf ? r.x & 0xffffffu : r.x, len)) {
                            done = true;
                        } else if (leaf) {
                            // the run ends at a leaf: its pattern list is in the record
                            hit = make_uint2(r.w, r.x >> 24);
                            done = true;
                        } else {
                            v = r.w;
                            d += len;
                        }
                    } else if (cb == im.label[r.y - 1]) {
                        v = r.y;
                        d++;
                    } else {
                        done = true;
                    }
                } else if (nc <= 4) {
                    const uint32_t x = r.x ^ (cb * 0x01010101u);
                    const uint32_t m = (x - 0x01010101u) & ~x & 0x80808080u;  // lowest flag = first zero byte
                    const uint32_t j = m ? (uint32_t)__builtin_ctz(m) >> 3 : 4u;
                    if (j < nc) {
                        v = r.y + j;
                        d++;
                    } else {
                        done = true;
                    }
                } else {
                    const uint8_t *lab = im.label + (r.y - 1);
                    uint32_t lo = 0, hi = nc;
                    while (lo < hi) {
                        const uint32_t mid = (lo + hi) >> 1;
                        if (lab[mid] < cb) lo = mid + 1; else hi = mid;
                    }
                    if (lo < nc && lab[lo] == cb) {
                        v = r.y + lo;
                        d++;
                    } else {
                        done = true;
                    }
                }
            }
            // finished walks: keep their matches, take the next candidates
            const bool got = done && hit.y != 0;
            const unsigned long long mk = __ballot(got);
            if (got) {
                const uint32_t slot = mn + mbcnt(mk);
                if (slot < kWalkMcap) wm[slot] = make_uint2(pr | (hit.y << 16), hit.x);
            }
            mn += (uint32_t)__popcll(mk);
            const unsigned long long md = __ballot(done);
            if (done) {
                const uint32_t e = next + mbcnt(md);
                live = e < cn;
                hit = make_uint2(0, 0);
                if (live) take(e);
            }
            next += (uint32_t)__popcll(md);
        }
        wave_sync();
        if (mn <= kWalkMcap) {
            emit_unit(a, u, unit_lo, wm, mn, s_sorted[wave], ut);
            return;
        }
    }
    unit_from_root(a, u, unit_lo, nch, s_bnd[wave]);
}

// ------------------------------------------------------------------ launchers

// modes 1 and 2: byte symbols, K = 2, the third byte folded to 8 or 16 bits
// (and not the four-symbol filter, which the split kernel prefers)
static bool byte_table_mode(const ScanArgs &a) {
    return a.q16_words == 0 && a.im.identity && a.im.K == 2 && (a.fold == 8 || a.fold == 16) &&
           a.im.fold_syms == 1;
}

void wave_lds_layout(ScanArgs &a, uint32_t waves, uint32_t lds_limit, bool split) {
    uint32_t off = 0;
    auto take = [&](uint32_t bytes) {
        const uint32_t o = off;
        off += (bytes + 15u) & ~15u;
        return o;
    };
    a.ftab_bytes = (uint32_t)((a.fold && a.im.K) ? ((1ull << (a.im.b * a.im.K)) * (a.fold / 8)) : 0);
    // mode 3: the four-symbol filter takes the table's place; the level
    // index stays in global memory (only survivors of both filters read it)
    if (a.q16_words) a.ftab_bytes = 4 * a.q16_words;
    a.ftab_bytes = (a.ftab_bytes + 15u) & ~15u;
    a.off_ftab = take(a.ftab_bytes);
    a.lvl_lds = a.q16_words ? 0u : a.im.lvl_words;
    // level index: (bit map, first node) per 32 codes
    a.off_bits = take(8 * a.lvl_lds);
    a.off_rank = a.off_bits;
    a.root_words = a.im.K == 0 ? std::max(1u, (1u << a.im.b) / 32) : 0u;
    a.off_root = take(4 * a.root_words);
    a.off_krec = take(4 * a.krec_words);
    a.off_pfx4 = take(4 * a.pfx4_words);
    a.off_sym = take(a.im.identity ? 0 : 256);
    a.off_wave = off;
    // the split filter kernel keeps no candidate or match lists in LDS
    a.mcap = split ? 0 : 64;
    a.ccap = split ? 0 : 128;
    // the split kernels of modes 1 and 2 filter chunks in pairs: a 2 KiB
    // window and a queue of half the size
    const bool pair = split && byte_table_mode(a);
    a.woff_bnd = ((pair ? 2 * kChunk : kWin) + 16 + 15) & ~15u;
    a.woff_queue = a.woff_bnd + ((4 * (kWin / 32 + 2) + 15) & ~15u);
    a.woff_cand = a.woff_queue + std::max(pair ? 2 * kQ1 : 4 * kQ1, 8 * a.mcap);
    a.woff_match = a.woff_cand + 8 * a.ccap;
    a.wave_bytes = a.woff_match + 8 * a.mcap;
    a.lds_total = off + waves * a.wave_bytes;
    (void)lds_limit;
}

// 0..2: fused kernels; 3..5: the split filter kernels of modes 0..2; 6: the
// split filter kernel of mode 3 (four-symbol alphabets); 7, 8: the split
// filter kernels of modes 1 and 2 with the prefix-4 filter.  The split
// kernels of modes 1..3 (4, 5, 6, 7, 8) come in two forms: for one text, and
// for batches (9, 10, 13, 11, 12), which read the plan's boundaries per
// chunk.
int wave_mode(const ScanArgs &a) {
    const int split = a.cand != nullptr ? 3 : 0;
    if (a.off_ftab != 0) return split;  // modes 1..3 need the table at LDS address 0
    if (split && a.q16_words) return a.chunk_info ? 13 : 6;
    const bool p4 = split && a.pfx4_words != 0;
    if (byte_table_mode(a)) {
        const int m = (a.fold == 8 ? 1 : 2) + (p4 ? 6 : split);
        if (!split || !a.chunk_info) return m;
        return m <= 5 ? m + 5 : m + 4;
    }
    return split;
}

// modes 3..5 are the split variants of modes 0..2, 6 of mode 3, 7 and 8 of
// modes 1 and 2 with the prefix-4 filter, 9..13 the batch forms of 4, 5, 7,
// 8 and 6
static const void *wave_fn_for(int mode) {
    switch (mode) {
        case 1: return (const void *)scan_waves<1, false>;
        case 2: return (const void *)scan_waves<2, false>;
        case 3: return (const void *)scan_waves<0, true>;
        case 4: return (const void *)scan_waves<1, true, false, 1>;
        case 5: return (const void *)scan_waves<2, true, false, 1>;
        case 6: return (const void *)scan_waves<3, true, false, 1>;
        case 7: return (const void *)scan_waves<1, true, true, 1>;
        case 8: return (const void *)scan_waves<2, true, true, 1>;
        case 9: return (const void *)scan_waves<1, true, false, 2>;
        case 10: return (const void *)scan_waves<2, true, false, 2>;
        case 11: return (const void *)scan_waves<1, true, true, 2>;
        case 12: return (const void *)scan_waves<2, true, true, 2>;
        case 13: return (const void *)scan_waves<3, true, false, 2>;
        default: return (const void *)scan_waves<0, false>;
    }
}

hipError_t prepare_wave_kernel(int mode, uint32_t lds_bytes) {
    // modes 1 and 2 address the filter table at LDS address 0: the kernel
    // must have no static LDS in front of the dynamic area
    hipFuncAttributes attr;
    hipError_t e = hipFuncGetAttributes(&attr, wave_fn_for(mode));
    if (e != hipSuccess) return e;
    if (attr.sharedSizeBytes != 0) return hipErrorInvalidKernelFile;
    return hipFuncSetAttribute(wave_fn_for(mode), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds_bytes);
}

hipError_t launch_scan_waves(const ScanArgs &a, uint32_t waves, uint32_t grid, hipStream_t s) {
    const int mode = wave_mode(a);
    const dim3 block(64 * waves);
    const void *fn = wave_fn_for(mode);
    ScanArgs arg = a;
    void *args[] = {(void *)&arg};
    const hipError_t e = hipLaunchKernel(fn, dim3(grid), block, args, a.lds_total, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

hipError_t launch_walk_units(const ScanArgs &a, hipStream_t s) {
    if (a.n_tiles == 0) return hipSuccess;
    const uint64_t grid = (a.n_tiles + kWalkWaves - 1) / kWalkWaves;
    if (grid > 0x7fffffffull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(walk_units, dim3((uint32_t)grid), dim3(64 * kWalkWaves), 0, s, a);
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
