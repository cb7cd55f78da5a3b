// C ABI of the scanner: trie objects, device images, workspaces, scans,
// batched scans, graph capture and autotuning.  Every step of a scan runs in
// the kernels of kernels.hip; this file only plans launches and owns memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/pfac.h"
#include "kernels.hpp"
#include "trie.hpp"

using namespace pfac;

static thread_local int g_last_hip = 0;
static int hip_fail(hipError_t e);

// PFAC_TRACE_ERRORS=1 in the environment: every failing HIP call is named
// on stderr (diagnostics only; the return codes do not change).
static bool trace_errors() {
    static const bool on = [] {
        const char *v = std::getenv("PFAC_TRACE_ERRORS");
        return v && v[0] && v[0] != '0';
    }();
    return on;
}

static int hip_fail_at(hipError_t e, const char *what, int line) {
    if (trace_errors())
        std::fprintf(stderr, "pfac: %s failed (line %d): %s\n", what, line, hipGetErrorString(e));
    return hip_fail(e);
}

static int hip_fail(hipError_t e) {
    g_last_hip = (int)e;
    // the error is reported here (and by pfac_last_hip_error); clear the
    // runtime's last-error state so that the caller's next HIP call does not
    // see it again
    (void)hipGetLastError();
    return e == hipErrorOutOfMemory ? PFAC_ENOMEM : PFAC_EDEVICE;
}

#define HIP_TRY(expr)                                                \
    do {                                                             \
        hipError_t e_ = (expr);                                      \
        if (e_ != hipSuccess) return hip_fail_at(e_, #expr, __LINE__); \
    } while (0)

struct DeviceBuf {
    void *p = nullptr;
    size_t bytes = 0;
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    // grow to at least `need` bytes; contents are not preserved.  Work still
    // queued on any stream may use the old buffer: the device drains first.
    hipError_t reserve(size_t need) {
        if (need <= bytes) return hipSuccess;
        if (p) (void)hipDeviceSynchronize();
        release();
        size_t want = std::max<size_t>(need, 256);
        hipError_t e = hipMalloc(&p, want);
        if (e != hipSuccess) {
            p = nullptr;
            return e;
        }
        bytes = want;
        return hipSuccess;
    }
};

constexpr uint64_t kNoSize = ~0ull;

struct pfac_trie {
    CrsTrie crs;
    DeviceImageHost img;
    pfac_tuning tuning{1, 16, 16, 8, 0, 16, 16, 1};
    uint32_t lds_limit = 160 * 1024;  // dynamic LDS a workgroup may use (gfx950; queried on the device)
    bool host_only = false;
    int device = -1;
    int n_cu = 0;
    DeviceBuf dev;
    ImageView view{};
    uint32_t halo = 16;
    double build_s = 0, upload_s = 0;
    std::map<uint32_t, pfac_tuning> tuned;  // by log2 size bucket
    std::mutex mu;
    // size of the merged DAG, computed on the first stats call
    mutable std::mutex dag_mu;
    mutable uint64_t dag_nodes = kNoSize, dag_edges = 0;
    // captured graphs and servers that read the current device image
    mutable std::atomic<int> pins{0};
    // servers, whose worker reads the whole tuning at every launch
    mutable std::atomic<int> tuning_pins{0};
};

struct pfac_workspace {
    DeviceBuf stage, unit_count, unit_off, blocksum, tile_first, inline_stage, misc;
    DeviceBuf cand, cand_count;  // split wave kernels: walk candidates per unit
    DeviceBuf chunk_info;        // wave kernels, batches: text boundaries per 1 KiB chunk
    hipEvent_t ev_start = nullptr, ev_stop = nullptr;  // optional kernel timing
    // launch shape of the last main scan kernel (grid, block, dynamic LDS):
    // graphs find its node by it
    uint32_t main_grid = 0, main_block = 0, main_lds = 0;
    // misc: [0] stage cursor, [1] running total, [2] per-launch count
    unsigned long long *cursor() { return (unsigned long long *)misc.p; }
    unsigned long long *running() { return (unsigned long long *)misc.p + 1; }
    uint64_t *tmp_count() { return (uint64_t *)misc.p + 2; }
};

struct pfac_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    pfac_workspace *ws = nullptr;     // its own scratch, captured with it
    const pfac_trie *t = nullptr;     // pinned: its image may not be replaced
    // event-record nodes around the main scan kernel (captured when the
    // workspace passed at creation had timing events), else NULL
    hipGraphNode_t n_start = nullptr, n_stop = nullptr;
    hipEvent_t ev_own[2] = {nullptr, nullptr};  // recorded by those nodes at capture
};

extern "C" int pfac_last_hip_error(void) { return g_last_hip; }

extern "C" const char *pfac_strerror(int code) {
    switch (code) {
        case PFAC_OK: return "ok";
        case PFAC_EINVAL: return "invalid argument";
        case PFAC_EEMPTY: return "empty pattern";
        case PFAC_ENOMEM: return "out of memory";
        case PFAC_EDEVICE: return "HIP error";
        case PFAC_ETRUNC: return "more matches than capacity";
        case PFAC_ENODEV: return "trie has no device image";
        case PFAC_EBUSY: return "busy";
        default: return "unknown error";
    }
}

// ------------------------------------------------------------- device image

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static int upload_image(pfac_trie *t) {
    const DeviceImageHost &I = t->img;
    size_t o_node = 0;
    size_t o_label = align256(o_node + I.node.size() * 4);
    size_t o_pptr = align256(o_label + I.label.size() + 16);
    size_t o_pids = align256(o_pptr + I.pout_ptr.size() * 4);
    size_t o_lvl = align256(o_pids + I.pout_ids.size() * 4);
    size_t o_sym = align256(o_lvl + std::max<size_t>(I.lvl.size(), 2) * 4);
    size_t o_ftab = align256(o_sym + 256);
    size_t o_root = align256(o_ftab + std::max<size_t>(I.ftab.size(), 16));
    size_t o_chain = align256(o_root + std::max<size_t>(I.root_bits.size(), 1) * 4);
    size_t o_krec = align256(o_chain + std::max<size_t>(I.chain.size(), 64));
    size_t o_pfx4 = align256(o_krec + std::max<size_t>(I.krec.size(), 1) * 4);
    size_t o_q16 = align256(o_pfx4 + std::max<size_t>(I.pfx4.size(), 1) * 4);
    size_t o_qfp = align256(o_q16 + std::max<size_t>(I.q16.size(), 1) * 4);
    size_t o_top = align256(o_qfp + std::max<size_t>(I.qfp.size(), 16) * 2);
    size_t o_tail = align256(o_top + std::max<size_t>(I.top.size(), 1) * 4);
    size_t o_tailb = align256(o_tail + std::max<size_t>(I.tail.size(), 4) * 4);
    size_t o_dnode = align256(o_tailb + std::max<size_t>(I.tail_bytes.size(), 64));
    size_t o_dlabel = align256(o_dnode + std::max<size_t>(I.dnode.size(), 4) * 4);
    size_t o_dchild = align256(o_dlabel + std::max<size_t>(I.dlabel.size(), 1) + 16);
    size_t o_dradd = align256(o_dchild + std::max<size_t>(I.dchild.size(), 1) * 4);
    size_t o_rlist = align256(o_dradd + std::max<size_t>(I.dradd.size(), 1) * 4);
    size_t o_ldag = align256(o_rlist + std::max<size_t>(I.rank_list.size(), 2) * 4);
    size_t total = align256(o_ldag + std::max<size_t>(I.lvl_dag.size(), 2) * 4);
    auto t0 = std::chrono::steady_clock::now();
    // the new image is built beside the old one, which stays usable if this fails
    DeviceBuf fresh;
    HIP_TRY(fresh.reserve(total));
    uint8_t *b = (uint8_t *)fresh.p;
#define CP(expr)                                   \
    do {                                           \
        hipError_t e_ = (expr);                    \
        if (e_ != hipSuccess) return e_;           \
    } while (0)
    auto copy_all = [&]() -> hipError_t {
        CP(hipMemcpy(b + o_node, I.node.data(), I.node.size() * 4, hipMemcpyHostToDevice));
        CP(hipMemcpy(b + o_label, I.label.data(), I.label.size(), hipMemcpyHostToDevice));
        CP(hipMemcpy(b + o_pptr, I.pout_ptr.data(), I.pout_ptr.size() * 4, hipMemcpyHostToDevice));
        CP(hipMemcpy(b + o_pids, I.pout_ids.data(), I.pout_ids.size() * 4, hipMemcpyHostToDevice));
        if (!I.lvl.empty())
            CP(hipMemcpy(b + o_lvl, I.lvl.data(), I.lvl.size() * 4, hipMemcpyHostToDevice));
        CP(hipMemcpy(b + o_sym, I.sym.data(), 256, hipMemcpyHostToDevice));
        if (!I.ftab.empty())
            CP(hipMemcpy(b + o_ftab, I.ftab.data(), I.ftab.size(), hipMemcpyHostToDevice));
        if (!I.krec.empty())
            CP(hipMemcpy(b + o_krec, I.krec.data(), I.krec.size() * 4, hipMemcpyHostToDevice));
        if (!I.chain.empty())
            CP(hipMemcpy(b + o_chain, I.chain.data(), I.chain.size(), hipMemcpyHostToDevice));
        if (!I.pfx4.empty())
            CP(hipMemcpy(b + o_pfx4, I.pfx4.data(), I.pfx4.size() * 4, hipMemcpyHostToDevice));
        if (!I.q16.empty())
            CP(hipMemcpy(b + o_q16, I.q16.data(), I.q16.size() * 4, hipMemcpyHostToDevice));
        if (!I.qfp.empty())
            CP(hipMemcpy(b + o_qfp, I.qfp.data(), I.qfp.size() * 2, hipMemcpyHostToDevice));
        if (!I.root_bits.empty())
            CP(hipMemcpy(b + o_root, I.root_bits.data(), I.root_bits.size() * 4, hipMemcpyHostToDevice));
        if (!I.top.empty())
            CP(hipMemcpy(b + o_top, I.top.data(), I.top.size() * 4, hipMemcpyHostToDevice));
        if (!I.tail.empty())
            CP(hipMemcpy(b + o_tail, I.tail.data(), I.tail.size() * 4, hipMemcpyHostToDevice));
        if (!I.tail_bytes.empty())
            CP(hipMemcpy(b + o_tailb, I.tail_bytes.data(), I.tail_bytes.size(), hipMemcpyHostToDevice));
        if (I.dag) {
            CP(hipMemcpy(b + o_dnode, I.dnode.data(), I.dnode.size() * 4, hipMemcpyHostToDevice));
            CP(hipMemcpy(b + o_dlabel, I.dlabel.data(), I.dlabel.size(), hipMemcpyHostToDevice));
            CP(hipMemcpy(b + o_dchild, I.dchild.data(), I.dchild.size() * 4, hipMemcpyHostToDevice));
            CP(hipMemcpy(b + o_dradd, I.dradd.data(), I.dradd.size() * 4, hipMemcpyHostToDevice));
            CP(hipMemcpy(b + o_rlist, I.rank_list.data(), I.rank_list.size() * 4, hipMemcpyHostToDevice));
            if (!I.lvl_dag.empty())
                CP(hipMemcpy(b + o_ldag, I.lvl_dag.data(), I.lvl_dag.size() * 4, hipMemcpyHostToDevice));
        }
        return hipSuccess;
    };
#undef CP
    const hipError_t ce = copy_all();
    if (ce != hipSuccess) {
        fresh.release();
        return hip_fail(ce);
    }
    // no kernel may still be reading the image it replaces
    if (t->dev.p) (void)hipDeviceSynchronize();
    std::swap(t->dev, fresh);
    fresh.release();
    ImageView &v = t->view;
    v.node = (const uint4 *)(b + o_node);
    v.label = b + o_label;
    v.pout_ptr = (const uint32_t *)(b + o_pptr);
    v.pout_ids = (const uint32_t *)(b + o_pids);
    v.lvl = (const uint32_t *)(b + o_lvl);
    v.sym = b + o_sym;
    v.ftab = b + o_ftab;
    v.root_bits = (const uint32_t *)(b + o_root);
    v.chain = b + o_chain;
    v.krec = (const uint32_t *)(b + o_krec);
    v.pfx4 = (const uint32_t *)(b + o_pfx4);
    v.pfx4_log2 = I.pfx4_log2;
    v.pfx4_mul = kPfx4Mul;
    v.pfx4_m1 = kPfx4M1;
    v.pfx4_m2 = kPfx4M2;
    v.q16 = (const uint32_t *)(b + o_q16);
    v.qfp = (const uint4 *)(b + o_qfp);
    v.q16_lw = I.q16_lw;
    v.qfp_lb = I.qfp_lb;
    v.qa = I.qa;
    v.qb = I.qb;
    v.qalph = I.qalph;
    v.q16_mul = kQ16Mul;
    v.top = (const uint32_t *)(b + o_top);
    v.top_nodes = I.top_nodes;
    v.top_rw = I.top_rw;
    v.tail = (const uint4 *)(b + o_tail);
    v.tail_bytes = b + o_tailb;
    v.dnode = (const uint4 *)(b + o_dnode);
    v.dlabel = b + o_dlabel;
    v.dchild = (const uint32_t *)(b + o_dchild);
    v.dradd = (const uint32_t *)(b + o_dradd);
    v.rank_list = (const uint2 *)(b + o_rlist);
    v.lvl_dag = (const uint2 *)(b + o_ldag);
    v.dag = I.dag;
    v.fold_syms = I.fold_syms;
    v.K = I.K;
    v.b = I.b;
    v.identity = I.identity;
    v.lvl_words = I.lvl_words;
    v.lvl_start = I.lvl_start;
    v.max_len = (uint32_t)std::min<uint64_t>(t->crs.max_len, 0xffffffffu);
    v.n_nodes = t->crs.n_nodes();
    t->upload_s =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return PFAC_OK;
}

static void set_halo(pfac_trie *t) {
    uint64_t need = t->crs.max_len ? t->crs.max_len - 1 : 0;
    uint64_t h = (need + 15) & ~15ull;
    t->halo = (uint32_t)std::max<uint64_t>(16, std::min<uint64_t>(h, kHaloCap));
}

static int build_common(const uint8_t *data, const uint64_t *offsets, uint32_t k, uint32_t flags,
                        pfac_trie **out) {
    if (!out) return PFAC_EINVAL;
    *out = nullptr;
    if (flags & ~PFAC_BUILD_HOST_ONLY) return PFAC_EINVAL;
    if (k > 0 && (!offsets || (!data && offsets[k] != offsets[0]))) return PFAC_EINVAL;
    for (uint32_t j = 0; j < k; j++) {
        if (offsets[j + 1] < offsets[j]) return PFAC_EINVAL;
        if (offsets[j + 1] == offsets[j]) return PFAC_EEMPTY;
    }
    pfac_trie *t = new (std::nothrow) pfac_trie();
    if (!t) return PFAC_ENOMEM;
    auto t0 = std::chrono::steady_clock::now();
    std::string err;
    try {
        if (!build_crs(data, offsets, k, t->crs, err)) {
            delete t;
            return PFAC_EINVAL;
        }
        pack_image(t->crs, t->tuning.index_bits, t->tuning.fold_bits, t->tuning.trunc_depth, t->tuning.dag,
                       t->img);
    } catch (const std::bad_alloc &) {
        delete t;
        return PFAC_ENOMEM;
    }
    // default launch: the split filter + walk kernels where the byte-symbol
    // two-level filter applies (few walk candidates); the fused wave kernel
    // otherwise (small alphabets and short patterns leave many candidates)
    if (t->img.identity && t->img.K == 2) t->tuning.kernel = 3;
    if (t->img.pfx4_log2) t->tuning.child_check = 2;
    if (t->img.q16_lw) t->tuning.kernel = 3;  // four-symbol alphabets: the 16-symbol filter
    t->build_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    set_halo(t);
    t->host_only = (flags & PFAC_BUILD_HOST_ONLY) != 0;
    if (!t->host_only) {
        hipError_t e = hipGetDevice(&t->device);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&t->n_cu, hipDeviceAttributeMultiprocessorCount, t->device);
        int lds = 0;
        if (e == hipSuccess &&
            hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, t->device) == hipSuccess &&
            lds > 0)
            t->lds_limit = (uint32_t)lds;
        if (e != hipSuccess) {
            delete t;
            return hip_fail(e);
        }
        int rc = upload_image(t);
        if (rc != PFAC_OK) {
            t->dev.release();
            delete t;
            return rc;
        }
    }
    *out = t;
    return PFAC_OK;
}

extern "C" int pfac_build_packed(const uint8_t *data, const uint64_t *offsets, uint32_t n_patterns,
                                 uint32_t flags, pfac_trie **out) {
    return build_common(data, offsets, n_patterns, flags, out);
}

extern "C" int pfac_build(const uint8_t *const *patterns, const uint64_t *lengths,
                          uint32_t n_patterns, uint32_t flags, pfac_trie **out) {
    if (!out) return PFAC_EINVAL;
    *out = nullptr;
    if (n_patterns > 0 && (!patterns || !lengths)) return PFAC_EINVAL;
    std::vector<uint64_t> off(n_patterns + 1, 0);
    for (uint32_t j = 0; j < n_patterns; j++) {
        if (lengths[j] == 0) return PFAC_EEMPTY;
        if (!patterns[j]) return PFAC_EINVAL;
        off[j + 1] = off[j] + lengths[j];
    }
    std::vector<uint8_t> data;
    try {
        data.resize(off[n_patterns]);
    } catch (const std::bad_alloc &) {
        return PFAC_ENOMEM;
    }
    for (uint32_t j = 0; j < n_patterns; j++)
        std::memcpy(data.data() + off[j], patterns[j], lengths[j]);
    return build_common(data.data(), off.data(), n_patterns, flags, out);
}

// LDS layout of the kernel a scan runs with the current tuning: the wave
// kernel asked for (kernel 1 or 2) where it applies and fits, dropping to
// fewer waves per workgroup, then dropping the LDS child records, until its
// tables and per-wave areas fit; the tile kernel otherwise.  *wave_out says
// which one it is.
// Kernel 3 (auto) picks by launch size.  On MI355X, one-text scans of 64 KiB
// to 64 MiB with 100, 10,000 and 20,000 patterns put the split wave kernels
// ahead of the tile kernel from 8 MiB on (their three launches and the
// persistent grid do not pay off below); under that the one-launch tile
// kernel is fastest with 4 bytes per lane below 1 MiB and 8 from there.
// The split kernels take units of up to 64 chunks (on the 2.2 GiB batch of
// 65,600 texts and 20,000 patterns, 16-chunk units cost 7% more per scan and
// 32-chunk units 2%: more units mean more walk waves and emissions).
constexpr uint64_t kAutoSplitBytes = 8ull << 20;
constexpr uint64_t kAutoWideLanes = 1ull << 20;
constexpr uint32_t kAutoUnitChunks = 64;

// Chunks per unit for a wave-kernel launch over `chunks` 1 KiB chunks on
// `waves` resident waves.  Units go to the waves one by one (wave w takes
// units w, w + waves, ...), so the wave with the most chunks bounds the
// filter kernel, while every unit costs the walk kernel a wave: take the
// largest G in 1 .. gmax whose most loaded wave is within 2% of the best G's.
// On MI355X, c4's 65,536 small texts (40,000 chunks, 4,096 waves) scan in
// 56 us with G = 10 (one unit of at most 10 chunks per wave) against 67 us
// with G = 4 (up to three units); the 2.2 GiB batch takes G = 63 (567 chunks
// on the most loaded wave against 576 with G = 64: 1% faster).
static uint32_t balanced_unit_chunks(uint64_t chunks, uint64_t waves, uint32_t gmax) {
    uint64_t m[65] = {0}, best = ~0ull;
    gmax = std::min<uint32_t>(std::max<uint32_t>(gmax, 1), 64);
    for (uint32_t G = 1; G <= gmax; G++) {
        const uint64_t U = (chunks + G - 1) / G;         // units
        const uint64_t k = (U + waves - 1) / waves;      // most units of one wave
        const uint64_t nk = U - (k - 1) * waves;         // waves with k units
        const uint64_t last = chunks - (U - 1) * G;      // chunks of the last unit
        m[G] = nk == 1 ? (k - 1) * G + last : k * G;
        best = std::min(best, m[G]);
    }
    uint32_t g = 1;
    for (uint32_t G = 1; G <= gmax; G++)
        if (m[G] <= best + best / 50) g = G;
    return g;
}

// The tuning a launch over `total` bytes runs with: kernel 3 resolved, and
// for the wave kernels the chunks per unit (at most the tuning's) that
// spread the launch's units evenly over the grid's waves (output units are
// independent; a launch of few chunks, such as a batch of small texts,
// needs small units to fill the grid).
static pfac_tuning launch_tuning(const pfac_trie *t, uint64_t total) {
    pfac_tuning tn = t->tuning;
    if (tn.kernel == 3) {
        if (total >= kAutoSplitBytes) {
            tn.kernel = 2;
            tn.chunks_per_unit = kAutoUnitChunks;
        } else {
            tn.kernel = 0;
            tn.bytes_per_lane = total < kAutoWideLanes ? 4 : 8;
        }
    }
    if (tn.kernel == 1 || tn.kernel == 2) {
        // chunks of the frame (the text and at most 15 bytes before it)
        const uint64_t chunks =
            total >= (1ull << 50) ? (1ull << 40) : std::max<uint64_t>(1, (total + 15 + kWaveChunk - 1) / kWaveChunk);
        const uint64_t waves = (uint64_t)std::max(t->n_cu, 1) * std::max<uint32_t>(tn.wg_per_cu, 1) * tn.waves_per_wg;
        tn.chunks_per_unit = balanced_unit_chunks(chunks, waves, tn.chunks_per_unit);
    }
    return tn;
}

static ScanArgs layout_for(const pfac_trie *t, const pfac_tuning &tn, uint32_t *waves_out = nullptr,
                           bool *wave_out = nullptr) {
    auto common = [&]() {
        ScanArgs a{};
        a.im = t->view;
        a.im.lvl_words = t->img.lvl_words;
        a.im.identity = t->img.identity;
        a.im.K = t->img.K;
        a.im.b = t->img.b;
        a.im.fold_syms = t->img.fold_syms;
        a.halo = t->halo;
        return a;
    };
    // tails and the merged DAG are walked by the tile kernel only, and the
    // wave kernels' walk limits are 16-bit
    const bool wave_ok = (tn.kernel == 1 || tn.kernel == 2) && !t->img.trunc_depth &&
                         !t->img.dag && t->crs.max_len <= 0xffff;
    if (wave_ok) {
        ScanArgs a = common();
        a.fold = t->img.fold_bits;
        a.group = tn.chunks_per_unit;
        // child_check 2: the prefix-4 filter where the image has one, else
        // the child records; dropped last when the layout does not fit
        const bool pfx4 = tn.child_check == 2 && t->img.pfx4_log2 != 0;
        // the split kernel filters four-symbol alphabets with the 16-symbol
        // filter when the image has one
        a.q16_words = (tn.kernel == 2 && t->img.q16_lw) ? (1u << t->img.q16_lw) : 0u;
        for (int with_rec = (tn.child_check && t->img.K) ? 1 : 0; with_rec >= 0; with_rec--) {
            a.krec_words = with_rec && !pfx4 ? (uint32_t)t->img.krec.size() : 0u;
            a.pfx4_words = with_rec && pfx4 ? (uint32_t)t->img.pfx4.size() : 0u;
            for (uint32_t waves = tn.waves_per_wg; waves >= 4; waves -= 4) {
                wave_lds_layout(a, waves, t->lds_limit, tn.kernel == 2);
                if (a.lds_total <= t->lds_limit) {
                    if (waves_out) *waves_out = waves;
                    if (wave_out) *wave_out = true;
                    return a;
                }
            }
        }
    }
    ScanArgs a = common();
    a.top_words = tn.top_nodes && t->img.K ? (uint32_t)t->img.top.size() : 0u;
    lds_layout(a, tn.bytes_per_lane);
    if (waves_out) *waves_out = std::max(4u, tn.waves_per_wg);
    if (wave_out) *wave_out = false;
    return a;
}

// the layout of large launches (statistics, checks)
static ScanArgs layout_for(const pfac_trie *t, uint32_t *waves_out = nullptr, bool *wave_out = nullptr) {
    return layout_for(t, launch_tuning(t, ~0ull), waves_out, wave_out);
}

static bool use_wave_kernel(const pfac_trie *t, const pfac_tuning &tn, uint32_t *waves_out);

extern "C" int pfac_trie_stats(const pfac_trie *t, pfac_stats *o) {
    if (!t || !o) return PFAC_EINVAL;
    std::memset(o, 0, sizeof(*o));
    const CrsTrie &c = t->crs;
    uint64_t N = c.n_nodes(), E = c.n_edges();
    o->nodes = N;
    o->edges = E;
    o->n_patterns = c.k;
    o->min_len = c.min_len;
    o->max_len = c.max_len;
    o->depth = c.level_start.size() >= 2 ? c.level_start.size() - 2 : 0;
    o->bytes_crs = 4 * (N + 1) + E + 4 * E + 4 * (N + 1) + 4ull * c.k;
    o->crs_elements = 2 * E + N + 1;
    o->bytes_dense256 = 1024 * N;
    o->bytes_bitmap36 = 36 * N;
    o->bytes_device = t->dev.bytes;
    o->alphabet_size = t->img.alphabet;
    o->symbol_bits = t->img.b;
    o->index_depth = t->img.K;
    o->lds_bytes = layout_for(t).lds_total;
    // (kernel 3: the kernel of large launches)
    const pfac_tuning large = launch_tuning(t, ~0ull);
    uint32_t waves = large.waves_per_wg;
    o->scan_kernel = use_wave_kernel(t, large, &waves) ? large.kernel : 0u;
    o->scan_waves = o->scan_kernel ? waves : kWG / 64;
    // the wave kernels' filter stages for this tuning
    o->stage1 = 0;
    o->stage2 = 0;
    if (o->scan_kernel) {
        const ScanArgs a = layout_for(t);
        if (a.q16_words) {
            o->stage1 = 3;
            o->stage2 = 3;
        } else {
            if (t->img.identity && t->img.K == 2 && t->img.fold_syms == 1)
                o->stage1 = a.fold == 8 ? 1u : a.fold == 16 ? 2u : 0u;
            o->stage2 = a.pfx4_words ? 2u : a.krec_words ? 1u : 0u;
        }
    }
    o->build_seconds = t->build_s;
    o->upload_seconds = t->upload_s;
    uint32_t bc = 0;
    while ((1u << bc) < std::max(t->img.alphabet, 2u)) bc++;
    o->bytes_bitmap_narrow = N * ((((uint64_t)1 << bc) + 7) / 8 + 4);
    o->bytes_level_index = 8ull * t->img.lvl_words;
    o->bytes_top_nodes = 4ull * t->img.top.size();
    o->trunc_depth = t->img.trunc_depth;
    o->bytes_nodes = 4ull * t->img.node.size();
    o->bytes_tails = 4ull * t->img.tail.size() + t->img.tail_bytes.size();
    {
        // the merged DAG in CRS form: row pointers, labels, children, rank
        // added per edge, terminal flags, and the k ids in string order
        std::lock_guard<std::mutex> lock(t->dag_mu);
        if (t->dag_nodes == kNoSize) dag_size(c, t->dag_nodes, t->dag_edges);
        o->dag_nodes = t->dag_nodes;
        o->dag_edges = t->dag_edges;
        o->bytes_dag_crs = 4 * (t->dag_nodes + 1) + 9 * t->dag_edges + 4 * (t->dag_nodes + 1) + 4ull * c.k;
    }
    return PFAC_OK;
}

extern "C" int pfac_trie_export(const pfac_trie *t, uint32_t *row_ptr, uint8_t *labels,
                                uint32_t *child, uint32_t *term_ptr, uint32_t *term_ids) {
    if (!t) return PFAC_EINVAL;
    const CrsTrie &c = t->crs;
    if (row_ptr) std::memcpy(row_ptr, c.row_ptr.data(), c.row_ptr.size() * 4);
    if (labels && !c.labels.empty()) std::memcpy(labels, c.labels.data(), c.labels.size());
    if (child)
        for (uint32_t e = 0; e < c.n_edges(); e++) child[e] = e + 1;
    if (term_ptr) std::memcpy(term_ptr, c.term_ptr.data(), c.term_ptr.size() * 4);
    if (term_ids && !c.term_ids.empty()) std::memcpy(term_ids, c.term_ids.data(), c.term_ids.size() * 4);
    return PFAC_OK;
}

extern "C" void pfac_trie_free(pfac_trie *t) {
    if (!t) return;
    t->dev.release();
    delete t;
}

extern "C" int pfac_trie_get_tuning(const pfac_trie *t, pfac_tuning *out) {
    if (!t || !out) return PFAC_EINVAL;
    *out = t->tuning;
    return PFAC_OK;
}

extern "C" int pfac_trie_launch_kernel(const pfac_trie *t, uint64_t total_bytes, uint32_t *kernel,
                                       pfac_tuning *tuning) {
    if (!t || !kernel) return PFAC_EINVAL;
    const pfac_tuning tn = launch_tuning(t, total_bytes);
    uint32_t waves = tn.waves_per_wg;
    *kernel = use_wave_kernel(t, tn, &waves) ? tn.kernel : 0u;
    if (tuning) *tuning = tn;
    return PFAC_OK;
}

static bool valid_tuning(const pfac_tuning *p) {
    return p->kernel <= 3 &&
           (p->bytes_per_lane == 4 || p->bytes_per_lane == 8 || p->bytes_per_lane == 16) &&
           p->index_bits >= 1 && p->index_bits <= 18 &&
           (p->fold_bits == 0 || p->fold_bits == 8 || p->fold_bits == 16) && p->wg_per_cu <= 8 &&
           (p->waves_per_wg == 4 || p->waves_per_wg == 8 || p->waves_per_wg == 12 ||
            p->waves_per_wg == 16) &&
           p->chunks_per_unit >= 1 && p->chunks_per_unit <= 64 && p->child_check <= 2 &&
           p->top_nodes <= 1 && p->trunc_depth <= 255 && p->dag <= 1 &&
           !(p->dag && (p->top_nodes || p->trunc_depth));
}

static bool same_tuning(const pfac_tuning &a, const pfac_tuning &b) {
    return std::memcmp(&a, &b, sizeof(pfac_tuning)) == 0;
}

extern "C" int pfac_trie_set_tuning(pfac_trie *t, const pfac_tuning *tn) {
    if (!t || !tn || !valid_tuning(tn)) return PFAC_EINVAL;
    // a server's worker thread reads the tuning at every launch
    if (t->tuning_pins.load() > 0 && !same_tuning(*tn, t->tuning)) return PFAC_EBUSY;
    const bool repack = tn->index_bits != t->tuning.index_bits || tn->fold_bits != t->tuning.fold_bits ||
                        tn->trunc_depth != t->tuning.trunc_depth || tn->dag != t->tuning.dag;
    // captured graphs and servers read the device image they started with
    if (repack && t->pins.load() > 0) return PFAC_EBUSY;
    // the new image is built aside; the trie changes only once it is complete
    DeviceImageHost fresh;
    if (repack) {
        try {
            pack_image(t->crs, tn->index_bits, tn->fold_bits, tn->trunc_depth, tn->dag, fresh);
        } catch (const std::bad_alloc &) {
            return PFAC_ENOMEM;
        }
        std::swap(t->img, fresh);  // `fresh` keeps the previous image
    }
    const pfac_tuning old = t->tuning;
    t->tuning = *tn;
    if (layout_for(t, launch_tuning(t, 0)).lds_total > t->lds_limit ||
        layout_for(t, launch_tuning(t, ~0ull)).lds_total > t->lds_limit) {
        // the kernel this tuning selects does not fit in LDS (e.g. bitmapped
        // top nodes or a level index too large): the previous tuning and
        // image stay
        t->tuning = old;
        if (repack) std::swap(t->img, fresh);
        return PFAC_EINVAL;
    }
    if (repack && !t->host_only) {
        const int rc = upload_image(t);
        if (rc != PFAC_OK) {  // the previous device image is still in place
            t->tuning = old;
            std::swap(t->img, fresh);
        }
        return rc;
    }
    return PFAC_OK;
}

// ---------------------------------------------------------------- workspace

extern "C" int pfac_workspace_create(pfac_workspace **out) {
    if (!out) return PFAC_EINVAL;
    pfac_workspace *w = new (std::nothrow) pfac_workspace();
    if (!w) return PFAC_ENOMEM;
    hipError_t e = w->misc.reserve(256);
    if (e == hipSuccess) e = hipMemset(w->misc.p, 0, 256);
    if (e != hipSuccess) {
        delete w;
        *out = nullptr;
        return hip_fail(e);
    }
    *out = w;
    return PFAC_OK;
}

extern "C" void pfac_workspace_free(pfac_workspace *w) {
    if (!w) return;
    w->stage.release();
    w->unit_count.release();
    w->unit_off.release();
    w->blocksum.release();
    w->tile_first.release();
    w->chunk_info.release();
    w->inline_stage.release();
    w->cand.release();
    w->cand_count.release();
    w->misc.release();
    delete w;
}

// Scratch sizes of a scan over n_tiles units (or 1 KiB chunks of the wave
// kernels, at least as many) with room for `capacity` staged matches; split:
// also the candidate lists of the split wave kernels.
struct WsSizes {
    uint64_t unit_count, unit_off, tile_first, chunk_info, blocksum, stage, inline_stage, cand,
        cand_count;
};

static WsSizes ws_sizes(uint64_t n_tiles, uint64_t capacity, bool split) {
    const uint64_t n_sums = std::max<uint64_t>(1, (n_tiles + (1u << kSumShift) - 1) >> kSumShift);
    WsSizes z{};
    z.unit_count = std::max<uint64_t>(n_tiles, 1) * 4;
    z.unit_off = std::max<uint64_t>(n_tiles, 1) * 8;
    z.tile_first = std::max<uint64_t>(n_tiles, 1) * 4;
    z.chunk_info = std::max<uint64_t>(n_tiles, 1) * 8;
    z.blocksum = n_sums * 8;
    z.stage = std::max<uint64_t>(capacity, 1) * sizeof(pfac_match);
    // wave kernels: max(kInlineCap, kInlinePerChunk * G) slots per unit of G
    // chunks, at most kInlineCap per chunk
    z.inline_stage = (n_tiles + 64) * kInlineCap * sizeof(pfac_match);
    z.cand = split ? (n_tiles + 64) * kCandPerChunk * 16 : 0;
    z.cand_count = split ? std::max<uint64_t>(n_tiles, 1) * 4 : 0;
    return z;
}

static int ws_reserve(pfac_workspace *w, uint64_t n_tiles, uint64_t capacity, bool split) {
    const WsSizes z = ws_sizes(n_tiles, capacity, split);
    HIP_TRY(w->unit_count.reserve(z.unit_count));
    HIP_TRY(w->unit_off.reserve(z.unit_off));
    HIP_TRY(w->tile_first.reserve(z.tile_first));
    HIP_TRY(w->chunk_info.reserve(z.chunk_info));
    HIP_TRY(w->blocksum.reserve(z.blocksum));
    HIP_TRY(w->stage.reserve(z.stage));
    HIP_TRY(w->inline_stage.reserve(z.inline_stage));
    if (split) {
        HIP_TRY(w->cand.reserve(z.cand));
        HIP_TRY(w->cand_count.reserve(z.cand_count));
    }
    return PFAC_OK;
}

extern "C" int pfac_workspace_set_timing(pfac_workspace *w, void *start_event, void *stop_event) {
    if (!w || (!start_event) != (!stop_event)) return PFAC_EINVAL;
    w->ev_start = (hipEvent_t)start_event;
    w->ev_stop = (hipEvent_t)stop_event;
    return PFAC_OK;
}

extern "C" int pfac_workspace_reserve(pfac_workspace *w, uint64_t max_bytes, uint32_t max_texts,
                                      uint64_t max_matches) {
    (void)max_texts;
    if (!w) return PFAC_EINVAL;
    // sizes whose byte counts would not even fit in 64 bits cannot be allocated
    if (max_bytes > (1ull << 56) || max_matches > (1ull << 56)) return PFAC_ENOMEM;
    uint64_t n_tiles = (max_bytes + 16 + kWG * 4 - 1) / (kWG * 4);  // smallest tile
    return ws_reserve(w, n_tiles, max_matches, true);
}

// ---------------------------------------------------------------------- scan

struct Launch {
    const pfac_trie *t;
    pfac_workspace *w;
    const uint8_t *text;
    uint64_t total;
    const uint64_t *offsets;    // device, NULL for one text
    uint32_t n_texts;
    uint32_t text_id0;
    pfac_match *out;
    uint64_t capacity;
    uint64_t *n_matches;
    uint32_t *counts;
    const unsigned long long *base_dev;
    hipStream_t s;
};

static uint64_t tiles_for(uint64_t total, uint64_t shift, uint32_t tile) {
    return total ? (shift + total + tile - 1) / tile : 0;
}


static uint32_t unit_bytes(const pfac_trie *t, const pfac_tuning &tn) {
    return use_wave_kernel(t, tn, nullptr) ? kWaveChunk * tn.chunks_per_unit : kWG * tn.bytes_per_lane;
}

// Opt a kernel into more than 64 KiB of dynamic LDS (once per size).
static hipError_t grant_lds(int slot, uint32_t bytes, hipError_t (*fn)(int, uint32_t), int arg) {
    static std::mutex mu;
    static uint32_t granted[32] = {};
    std::lock_guard<std::mutex> lock(mu);
    if (granted[slot] >= bytes) return hipSuccess;
    hipError_t e = fn(arg, bytes);
    if (e == hipSuccess) granted[slot] = bytes;
    return e;
}

static hipError_t prep_tile(int bpl, uint32_t bytes) { return prepare_kernels((uint32_t)bpl, bytes); }
static hipError_t prep_wave(int mode, uint32_t bytes) { return prepare_wave_kernel(mode, bytes); }

// Wave kernel when asked for, applicable and its LDS layout fits; the tile
// kernel otherwise.
static bool use_wave_kernel(const pfac_trie *t, const pfac_tuning &tn, uint32_t *waves_out) {
    bool wave = false;
    (void)layout_for(t, tn, waves_out, &wave);
    return wave;
}

static bool uses_split(const pfac_trie *t, const pfac_tuning &tn) {
    return tn.kernel == 2 && use_wave_kernel(t, tn, nullptr);
}

// How a scan of `total` bytes at `text` is cut with the trie's tuning:
// output units (tiles, or units of G chunks), batch-plan units (1 KiB chunks
// of the wave kernels, else tiles), and which kernels run.
struct ScanShape {
    bool wave_kernel, split;
    uint32_t waves, tile, plan_unit;
    uint64_t shift, n_tiles, n_plan;
    uint64_t ws_units() const { return std::max(n_tiles, n_plan); }
};

static ScanShape scan_shape(const pfac_trie *t, const pfac_tuning &tn, const void *text, uint64_t total) {
    ScanShape h{};
    h.waves = tn.waves_per_wg;
    h.wave_kernel = use_wave_kernel(t, tn, &h.waves);
    h.split = h.wave_kernel && tn.kernel == 2;
    h.tile = h.wave_kernel ? kWaveChunk * tn.chunks_per_unit : kWG * tn.bytes_per_lane;
    h.shift = (uintptr_t)text & 15;
    h.n_tiles = tiles_for(total, h.shift, h.tile);
    if (t->crs.k == 0) h.n_tiles = 0;  // nothing can match
    h.plan_unit = h.wave_kernel ? kWaveChunk : h.tile;
    h.n_plan = h.n_tiles ? tiles_for(total, h.shift, h.plan_unit) : 0;
    return h;
}

static int enqueue_scan(const Launch &L, bool reserve) {
    const pfac_trie *t = L.t;
    const pfac_tuning tn = launch_tuning(t, L.total);
    const ScanShape h = scan_shape(t, tn, L.text, L.total);
    uint32_t waves = h.waves;
    const bool wave_kernel = h.wave_kernel;
    const bool split = h.split;
    const uint32_t bpl = tn.bytes_per_lane;
    const uintptr_t addr = (uintptr_t)L.text;
    const uint64_t shift = h.shift;
    const uint64_t n_tiles = h.n_tiles;
    // the batch plan is per 1 KiB chunk for the wave kernel, per tile otherwise
    const uint32_t plan_unit = h.plan_unit;
    const uint64_t n_plan = h.n_plan;
    if (reserve) {
        int rc = ws_reserve(L.w, h.ws_units(), L.capacity, split);
        if (rc != PFAC_OK) return rc;
    }
    pfac_workspace *w = L.w;
    const uint32_t n_sums = (uint32_t)std::max<uint64_t>(1, (n_tiles + (1u << kSumShift) - 1) >> kSumShift);

    ScanArgs a = layout_for(t, tn, &waves);
    a.im = t->view;
    a.base = (const uint8_t *)(addr - shift);
    a.shift = shift;
    a.total = L.total;
    a.offsets = L.offsets;
    a.n_texts = L.n_texts;
    a.text_id0 = L.text_id0;
    a.tile_first_text = L.offsets ? (const uint32_t *)w->tile_first.p : nullptr;
    a.chunk_info = L.offsets && wave_kernel ? (const uint2 *)w->chunk_info.p : nullptr;
    a.n_plan = n_plan;
    a.plan_shift = (uint32_t)__builtin_ctz(plan_unit);
    a.n_tiles = n_tiles;
    a.stage = (pfac_match *)w->stage.p;
    a.stage_cap = std::min<uint64_t>(L.capacity, w->stage.bytes / sizeof(pfac_match));
    a.stage_cursor = w->cursor();
    a.unit_count = (uint32_t *)w->unit_count.p;
    a.unit_off = (unsigned long long *)w->unit_off.p;
    a.blocksum = (unsigned long long *)w->blocksum.p;
    a.counts = L.counts;
    a.inline_stage = (pfac_match *)w->inline_stage.p;
    a.inline_cap = wave_kernel ? std::max(kInlineCap, kInlinePerChunk * tn.chunks_per_unit) : 0;
    if (split) {
        a.cand = (uint4 *)w->cand.p;
        a.cand_count = (uint32_t *)w->cand_count.p;
        a.cand_cap = a.group * kCandPerChunk;
    }
    if (a.lds_total > t->lds_limit) return PFAC_EINVAL;
    // the wave kernels count 1 KiB chunks in 32 bits
    if (wave_kernel && n_plan >= (1ull << 31)) return PFAC_EINVAL;

    a.n_sums = n_sums;
    // the split filter kernel clears the block sums and the cursor itself
    if (!(split && n_tiles)) HIP_TRY(launch_reset(a.stage_cursor, a.blocksum, n_sums, L.s));
    if (L.counts) HIP_TRY(launch_fill_u32(L.counts, L.total, 0, L.s));
    if (n_tiles) {
        if (L.offsets)
            HIP_TRY(launch_plan(L.offsets, L.n_texts, shift, n_plan, plan_unit,
                                (uint32_t *)w->tile_first.p, (uint2 *)a.chunk_info, L.s));
        int per_cu = (int)tn.wg_per_cu;
        int occ;
        uint64_t want;
        if (wave_kernel) {
            const int mode = wave_mode(a);
            if (a.lds_total > 64 * 1024) HIP_TRY(grant_lds(4 + mode, a.lds_total, prep_wave, mode));
            occ = max_wave_wg_per_cu(a, waves);
            want = (n_tiles + waves - 1) / waves;
        } else {
            const int slot = bpl == 4 ? 0 : bpl == 8 ? 1 : 2;
            if (a.lds_total > 64 * 1024) HIP_TRY(grant_lds(slot, a.lds_total, prep_tile, (int)bpl));
            occ = max_wg_per_cu(bpl, a.lds_total, a.top_words ? 1 : a.im.dag ? 2 : 0);
            want = n_tiles;
        }
        if (per_cu == 0 || per_cu > occ) per_cu = occ;
        const uint64_t resident = (uint64_t)std::max(1, t->n_cu) * (uint64_t)per_cu;
        const uint32_t grid = (uint32_t)std::min<uint64_t>(want, resident);
        // under stream capture the timing events become event-record nodes
        // of the graph (recorded again at every replay)
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        if (w->ev_start) HIP_TRY(hipStreamIsCapturing(L.s, &cap));
        const unsigned ev_flags = cap == hipStreamCaptureStatusActive ? hipEventRecordExternal : 0u;
        if (w->ev_start) HIP_TRY(hipEventRecordWithFlags(w->ev_start, L.s, ev_flags));
        w->main_grid = grid;
        w->main_block = wave_kernel ? 64 * waves : kWG;
        w->main_lds = a.lds_total;
        if (wave_kernel)
            HIP_TRY(launch_scan_waves(a, waves, grid, L.s));
        else
            HIP_TRY(launch_scan(a, bpl, grid, L.s));
        if (w->ev_stop) HIP_TRY(hipEventRecordWithFlags(w->ev_stop, L.s, ev_flags));
        if (split) HIP_TRY(launch_walk_units(a, L.s));
    }
    FinishArgs f{};
    f.unit_count = a.unit_count;
    f.unit_off = a.unit_off;
    f.blocksum = a.blocksum;
    f.stage = a.stage;
    f.stage_cap = a.stage_cap;
    f.n_tiles = n_tiles;
    f.n_sums = n_sums;
    f.out = L.out;
    f.capacity = L.out ? L.capacity : 0;
    f.n_matches = L.n_matches;
    f.base_dev = L.base_dev;
    f.inline_stage = a.inline_stage;
    f.inline_cap = a.inline_cap;
    HIP_TRY(launch_finish(f, L.s));
    return PFAC_OK;
}

static int check_scan_args(const pfac_trie *t, pfac_workspace *w, const void *text, uint64_t n,
                           const void *out, uint64_t capacity, const void *n_matches) {
    if (!t || !w || !n_matches) return PFAC_EINVAL;
    if (t->host_only) return PFAC_ENODEV;
    if (n > 0 && !text) return PFAC_EINVAL;
    if (capacity > 0 && !out) return PFAC_EINVAL;
    return PFAC_OK;
}

extern "C" int pfac_scan(const pfac_trie *t, pfac_workspace *w, const uint8_t *text_dev,
                         uint64_t n, pfac_match *out_dev, uint64_t capacity,
                         uint64_t *n_matches_dev, uint32_t *counts_dev, void *stream) {
    int rc = check_scan_args(t, w, text_dev, n, out_dev, capacity, n_matches_dev);
    if (rc) return rc;
    Launch L{t, w, text_dev, n, nullptr, 1, 0, out_dev, capacity, n_matches_dev, counts_dev,
             nullptr, (hipStream_t)stream};
    return enqueue_scan(L, true);
}

// ------------------------------------------------- scan without allocation

// Scratch of pfac_scan_noalloc: one array in every device's memory, taken
// from the code object when the library is loaded on that device and held
// until the process ends.  Host code reaches it only through the device
// address that hipGetSymbolAddress returns on each device; the array's
// name itself is a host-side stand-in.
constexpr uint64_t kNoAllocScratch = 64ull << 20;
static __device__ __align__(256) uint8_t scratch[kNoAllocScratch];
constexpr int kMaxDevices = 256;
static std::mutex g_scratch_mu;
static uint8_t *g_scratch_dev[kMaxDevices] = {};

// The scratch's device address on the current device, looked up once per
// device with that device current.
static int noalloc_scratch(uint8_t **out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return PFAC_EINVAL;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_dev[dev] = (uint8_t *)p;
    }
    *out = g_scratch_dev[dev];
    return PFAC_OK;
}

extern "C" int pfac_scan_noalloc(const pfac_trie *t, const uint8_t *text_dev, uint64_t n,
                                 pfac_match *out_dev, uint64_t capacity, uint64_t *n_matches_dev,
                                 uint32_t *counts_dev, void *stream) {
    if (!t || !n_matches_dev) return PFAC_EINVAL;
    if (t->host_only) return PFAC_ENODEV;
    if (n > 0 && !text_dev) return PFAC_EINVAL;
    if (capacity > 0 && !out_dev) return PFAC_EINVAL;
    // the workspace pfac_scan would reserve, carved out of the scratch
    const ScanShape h = scan_shape(t, launch_tuning(t, n), text_dev, n);
    if (h.ws_units() > (1ull << 40) || capacity > (1ull << 40)) return PFAC_EINVAL;
    const WsSizes z = ws_sizes(h.ws_units(), capacity, h.split);
    uint8_t *base = nullptr;
    int rc = noalloc_scratch(&base);
    if (rc != PFAC_OK) return rc;
    pfac_workspace w{};
    uint64_t off = 0;
    auto take = [&](DeviceBuf &b, uint64_t bytes) {
        b.p = base + off;
        b.bytes = bytes;
        off += (bytes + 255) & ~255ull;
    };
    take(w.misc, 256);
    take(w.unit_count, z.unit_count);
    take(w.unit_off, z.unit_off);
    take(w.tile_first, z.tile_first);
    take(w.chunk_info, z.chunk_info);
    take(w.blocksum, z.blocksum);
    take(w.stage, z.stage);
    take(w.inline_stage, z.inline_stage);
    if (h.split) {
        take(w.cand, z.cand);
        take(w.cand_count, z.cand_count);
    }
    if (off > kNoAllocScratch) return PFAC_EINVAL;  // text or capacity beyond the scratch
    Launch L{t, &w, text_dev, n, nullptr, 1, 0, out_dev, capacity, n_matches_dev, counts_dev,
             nullptr, (hipStream_t)stream};
    // every buffer is in place: the scan allocates nothing (the DeviceBufs
    // are not owned and are dropped without release)
    return enqueue_scan(L, false);
}

extern "C" int pfac_scan_sync(const pfac_trie *t, pfac_workspace *w, const uint8_t *text_dev,
                              uint64_t n, pfac_match *out_dev, uint64_t capacity,
                              uint64_t *n_matches_host, uint32_t *counts_dev, void *stream) {
    if (!n_matches_host || !w) return PFAC_EINVAL;
    uint64_t *dcount = w->tmp_count();
    int rc = pfac_scan(t, w, text_dev, n, out_dev, capacity, dcount, counts_dev, stream);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(n_matches_host, dcount, 8, hipMemcpyDeviceToHost, (hipStream_t)stream));
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    return *n_matches_host > capacity ? PFAC_ETRUNC : PFAC_OK;
}

extern "C" int pfac_scan_batch(const pfac_trie *t, pfac_workspace *w, const uint8_t *texts_dev,
                               const uint64_t *offsets_dev, uint32_t n_texts, uint64_t total_bytes,
                               pfac_match *out_dev, uint64_t capacity, uint64_t *n_matches_dev,
                               void *stream) {
    int rc = check_scan_args(t, w, texts_dev, total_bytes, out_dev, capacity, n_matches_dev);
    if (rc) return rc;
    if (!offsets_dev || (n_texts == 0 && total_bytes != 0)) return PFAC_EINVAL;
    Launch L{t, w, texts_dev, total_bytes, offsets_dev, n_texts, 0, out_dev, capacity,
             n_matches_dev, nullptr, nullptr, (hipStream_t)stream};
    return enqueue_scan(L, true);
}

extern "C" int pfac_scan_batch_plain(const pfac_trie *t, pfac_workspace *w,
                                     const uint8_t *texts_dev, const uint64_t *offsets_host,
                                     uint32_t n_texts, pfac_match *out_dev, uint64_t capacity,
                                     uint64_t *n_matches_dev, void *stream) {
    uint64_t total = (n_texts && offsets_host) ? offsets_host[n_texts] - offsets_host[0] : 0;
    int rc = check_scan_args(t, w, texts_dev, total, out_dev, capacity, n_matches_dev);
    if (rc) return rc;
    if (!offsets_host) return PFAC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    uint64_t max_tiles = 0;
    bool split = false;
    for (uint32_t i = 0; i < n_texts; i++) {
        if (offsets_host[i + 1] < offsets_host[i]) return PFAC_EINVAL;
        const uint64_t n = offsets_host[i + 1] - offsets_host[i];
        const pfac_tuning tn = launch_tuning(t, n);
        max_tiles = std::max(max_tiles, tiles_for(n, 15, std::min(unit_bytes(t, tn), kWaveChunk)));
        split = split || uses_split(t, tn);
    }
    rc = ws_reserve(w, max_tiles, capacity, split);
    if (rc) return rc;
    HIP_TRY(launch_fill_u32((uint32_t *)w->running(), 2, 0, s));
    for (uint32_t i = 0; i < n_texts; i++) {
        const uint64_t n = offsets_host[i + 1] - offsets_host[i];
        if (n == 0) continue;
        Launch L{t, w, texts_dev + offsets_host[i], n, nullptr, 1, i, out_dev, capacity,
                 w->tmp_count(), nullptr, w->running(), s};
        rc = enqueue_scan(L, false);
        if (rc) return rc;
        HIP_TRY(launch_add_running(w->running(), w->tmp_count(), s));
    }
    HIP_TRY(launch_copy_u64(n_matches_dev, w->running(), s));
    return PFAC_OK;
}

namespace pfac {
// Servers keep the image and the tuning of their trie while they run
// (declared in server.hip).
void trie_pin(const pfac_trie *t, int delta) {
    t->pins += delta;
    t->tuning_pins += delta;
}
uint64_t workspace_device_bytes(const pfac_workspace *w) {
    if (!w) return 0;
    return w->stage.bytes + w->unit_count.bytes + w->unit_off.bytes + w->blocksum.bytes +
           w->tile_first.bytes + w->chunk_info.bytes + w->inline_stage.bytes + w->misc.bytes + w->cand.bytes +
           w->cand_count.bytes;
}
}  // namespace pfac

// ------------------------------------------------------------------- graphs

// The event-record nodes of the timing events in a captured graph.
static int find_timing_nodes(pfac_graph *g) {
    size_t n = 0;
    HIP_TRY(hipGraphGetNodes(g->graph, nullptr, &n));
    std::vector<hipGraphNode_t> nodes(n);
    if (n) HIP_TRY(hipGraphGetNodes(g->graph, nodes.data(), &n));
    for (hipGraphNode_t nd : nodes) {
        hipGraphNodeType ty;
        HIP_TRY(hipGraphNodeGetType(nd, &ty));
        if (ty != hipGraphNodeTypeEventRecord) continue;
        hipEvent_t ev = nullptr;
        HIP_TRY(hipGraphEventRecordNodeGetEvent(nd, &ev));
        if (ev == g->ws->ev_start) g->n_start = nd;
        if (ev == g->ws->ev_stop) g->n_stop = nd;
    }
    // an empty batch launches no scan kernel, so it has no timing nodes
    return PFAC_OK;
}

// Event-record nodes added around the main scan kernel of a captured graph:
// the kernel node is the one launched with the scan's grid, block and
// dynamic LDS (no other kernel of a scan uses dynamic LDS); the start node
// takes over its dependencies and the stop node its dependents.
static int add_timing_nodes(pfac_graph *g) {
    size_t n = 0;
    HIP_TRY(hipGraphGetNodes(g->graph, nullptr, &n));
    std::vector<hipGraphNode_t> nodes(n);
    if (n) HIP_TRY(hipGraphGetNodes(g->graph, nodes.data(), &n));
    hipGraphNode_t k = nullptr;
    for (hipGraphNode_t nd : nodes) {
        hipGraphNodeType ty;
        HIP_TRY(hipGraphNodeGetType(nd, &ty));
        if (ty != hipGraphNodeTypeKernel) continue;
        hipKernelNodeParams kp{};
        HIP_TRY(hipGraphKernelNodeGetParams(nd, &kp));
        if (kp.sharedMemBytes == 0 || kp.sharedMemBytes != g->ws->main_lds ||
            kp.blockDim.x != g->ws->main_block || kp.gridDim.x != g->ws->main_grid)
            continue;
        if (k) return PFAC_EINVAL;  // not unique
        k = nd;
    }
    if (!k) return PFAC_OK;  // an empty batch launches no scan kernel
    size_t ni = 0, no = 0;
    HIP_TRY(hipGraphNodeGetDependencies(k, nullptr, &ni));
    HIP_TRY(hipGraphNodeGetDependentNodes(k, nullptr, &no));
    std::vector<hipGraphNode_t> in(ni), after(no);
    if (ni) HIP_TRY(hipGraphNodeGetDependencies(k, in.data(), &ni));
    if (no) HIP_TRY(hipGraphNodeGetDependentNodes(k, after.data(), &no));
    hipGraphNode_t ns = nullptr, ne = nullptr;
    HIP_TRY(hipGraphAddEventRecordNode(&ns, g->graph, ni ? in.data() : nullptr, ni, g->ev_own[0]));
    for (size_t i = 0; i < ni; i++) HIP_TRY(hipGraphRemoveDependencies(g->graph, &in[i], &k, 1));
    HIP_TRY(hipGraphAddDependencies(g->graph, &ns, &k, 1));
    HIP_TRY(hipGraphAddEventRecordNode(&ne, g->graph, &k, 1, g->ev_own[1]));
    for (size_t i = 0; i < no; i++) {
        HIP_TRY(hipGraphRemoveDependencies(g->graph, &k, &after[i], 1));
        HIP_TRY(hipGraphAddDependencies(g->graph, &ne, &after[i], 1));
    }
    g->n_start = ns;
    g->n_stop = ne;
    return PFAC_OK;
}

extern "C" int pfac_graph_create_batch(const pfac_trie *t, pfac_workspace *w,
                                       const uint8_t *texts_dev, const uint64_t *offsets_dev,
                                       uint32_t n_texts, uint64_t total_bytes,
                                       pfac_match *out_dev, uint64_t capacity,
                                       uint64_t *n_matches_dev, void *stream, pfac_graph **out) {
    if (!out) return PFAC_EINVAL;
    *out = nullptr;
    // the graph gets scratch of its own: `w` stays free for other scans and
    // lends the graph only its timing events
    pfac_graph *g = new (std::nothrow) pfac_graph();
    if (!g) return PFAC_ENOMEM;
    int rc = pfac_workspace_create(&g->ws);
    if (rc == PFAC_OK)
        rc = check_scan_args(t, g->ws, texts_dev, total_bytes, out_dev, capacity, n_matches_dev);
    if (rc == PFAC_OK && !offsets_dev) rc = PFAC_EINVAL;
    if (rc == PFAC_OK)
    {
        const pfac_tuning tn = launch_tuning(t, total_bytes);
        if (rc == PFAC_OK)
            rc = ws_reserve(g->ws, tiles_for(total_bytes, 15, std::min(unit_bytes(t, tn), kWaveChunk)),
                            capacity, uses_split(t, tn));
    }
    if (rc != PFAC_OK) {
        pfac_graph_free(g);
        return rc;
    }
    g->t = t;
    t->pins++;
    (void)stream;  // the capture runs on a stream of the library's own
    hipStream_t s = nullptr;
    hipError_t ec = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (ec != hipSuccess) {
        pfac_graph_free(g);
        return hip_fail_at(ec, "hipStreamCreateWithFlags", __LINE__);
    }
    // With the caller's timing events set, event-record nodes around the
    // main kernel record two events of the graph's own (plain hipEventCreate
    // events), pointed at the caller's events once the graph is
    // instantiated.  The nodes are added to the captured graph (method 0)
    // or, where the runtime refuses that, captured from event records
    // (method 1); if both fail the graph is captured without them
    // (pfac_graph_set_timing then returns PFAC_EINVAL).
    const bool timed = w && w->ev_start && w->ev_stop;
    for (int method = timed ? 0 : 2; method <= 2; method++) {
        g->ws->ev_start = g->ws->ev_stop = nullptr;
        g->n_start = g->n_stop = nullptr;
        rc = PFAC_OK;
        if (method < 2) {
            for (hipEvent_t &e : g->ev_own)
                if (!e && hipEventCreate(&e) != hipSuccess) e = nullptr;
            if (!g->ev_own[0] || !g->ev_own[1]) {
                (void)hipGetLastError();
                continue;
            }
            if (method == 1) {
                g->ws->ev_start = g->ev_own[0];
                g->ws->ev_stop = g->ev_own[1];
            }
        }
        hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            Launch L{t, g->ws, texts_dev, total_bytes, offsets_dev, n_texts, 0, out_dev, capacity,
                     n_matches_dev, nullptr, nullptr, s};
            rc = enqueue_scan(L, false);
            hipGraph_t graph = nullptr;
            hipError_t e2 = hipStreamEndCapture(s, &graph);
            g->graph = graph;
            if (rc == PFAC_OK && e2 != hipSuccess) rc = hip_fail_at(e2, "hipStreamEndCapture", __LINE__);
            if (rc == PFAC_OK && method == 0) rc = add_timing_nodes(g);
            if (rc == PFAC_OK && method == 1) rc = find_timing_nodes(g);
            if (rc == PFAC_OK) {
                e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
                if (e != hipSuccess) rc = hip_fail_at(e, "hipGraphInstantiate", __LINE__);
            }
            // replays record the caller's events from the start
            if (rc == PFAC_OK && g->n_start && g->n_stop)
                rc = pfac_graph_set_timing(g, w->ev_start, w->ev_stop);
        } else {
            rc = hip_fail_at(e, "hipStreamBeginCapture", __LINE__);
        }
        g->ws->ev_start = g->ws->ev_stop = nullptr;
        if (rc == PFAC_OK || method == 2) break;
        // drop the failed attempt and try the next method
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
        if (g->graph) (void)hipGraphDestroy(g->graph);
        g->exec = nullptr;
        g->graph = nullptr;
        g->n_start = g->n_stop = nullptr;
        (void)hipGetLastError();
    }
    hipStream_t own = s;
    if (own) (void)hipStreamDestroy(own);
    if (rc != PFAC_OK) {
        pfac_graph_free(g);
        return rc;
    }
    *out = g;
    return PFAC_OK;
}

extern "C" int pfac_graph_set_timing(pfac_graph *g, void *start_event, void *stop_event) {
    if (!g || !g->exec || !start_event || !stop_event) return PFAC_EINVAL;
    if (!g->n_start || !g->n_stop) return PFAC_EINVAL;  // captured without timing events
    HIP_TRY(hipGraphExecEventRecordNodeSetEvent(g->exec, g->n_start, (hipEvent_t)start_event));
    HIP_TRY(hipGraphExecEventRecordNodeSetEvent(g->exec, g->n_stop, (hipEvent_t)stop_event));
    return PFAC_OK;
}

extern "C" int pfac_graph_launch(pfac_graph *g, void *stream) {
    if (!g || !g->exec) return PFAC_EINVAL;
    HIP_TRY(hipGraphLaunch(g->exec, (hipStream_t)stream));
    return PFAC_OK;
}

extern "C" void pfac_graph_free(pfac_graph *g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    pfac_workspace_free(g->ws);
    for (hipEvent_t e : g->ev_own)
        if (e) (void)hipEventDestroy(e);
    if (g->t) g->t->pins--;
    delete g;
}

// ----------------------------------------------------------------- autotune

static uint32_t size_bucket(uint64_t n) {
    uint32_t b = 0;
    while ((1ull << b) < n && b < 63) b++;
    return b;
}

// One scan of the text (or batch) being tuned for: writes up to `cap`
// matches to out and the count to *dcount, asynchronously on `stream`.
typedef int (*tune_scan_fn)(const void *ctx, const pfac_trie *t, pfac_workspace *w,
                            pfac_match *out, uint64_t cap, uint64_t *dcount, void *stream);

static int tune_scan_sync(const void *ctx, tune_scan_fn scan, const pfac_trie *t, pfac_workspace *w,
                          pfac_match *out, uint64_t cap, uint64_t *n_host, void *stream) {
    uint64_t *dcount = w->tmp_count();
    int rc = scan(ctx, t, w, out, cap, dcount, stream);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(n_host, dcount, 8, hipMemcpyDeviceToHost, (hipStream_t)stream));
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    return *n_host > cap ? PFAC_ETRUNC : PFAC_OK;
}

// Time every candidate tuning on one input, keep the fastest whose match
// list equals the starting tuning's, cache it under `key`.
static int autotune_common(pfac_trie *t, pfac_workspace *w, const void *ctx, tune_scan_fn scan,
                           uint32_t key, void *stream, pfac_tuning *best) {
    if (t->host_only) return PFAC_ENODEV;
    // a server reads this trie's tuning at every launch
    if (t->tuning_pins.load() > 0) return PFAC_EBUSY;
    std::lock_guard<std::mutex> lock(t->mu);
    auto it = t->tuned.find(key);
    if (it != t->tuned.end()) {
        *best = it->second;
        return pfac_trie_set_tuning(t, best);
    }
    hipStream_t s = (hipStream_t)stream;
    const pfac_tuning start = t->tuning;
    uint64_t *dcount = w->tmp_count();

    // reference list with the starting parameters
    uint64_t ref_n = 0;
    int rc = tune_scan_sync(ctx, scan, t, w, nullptr, 0, &ref_n, stream);
    if (rc != PFAC_OK && rc != PFAC_ETRUNC) return rc;
    const uint64_t cap = ref_n;
    pfac_match *dref = nullptr, *dcand = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&] {
        if (dref) (void)hipFree(dref);
        if (dcand) (void)hipFree(dcand);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    if (cap) {
        hipError_t e = hipMalloc(&dref, cap * sizeof(pfac_match));
        if (e == hipSuccess) e = hipMalloc(&dcand, cap * sizeof(pfac_match));
        if (e != hipSuccess) {
            cleanup();
            return hip_fail(e);
        }
    }
    {
        hipError_t e = hipEventCreate(&e0);
        if (e == hipSuccess) e = hipEventCreate(&e1);
        if (e != hipSuccess) {
            cleanup();
            return hip_fail(e);
        }
    }
    std::vector<pfac_match> href, hcand;
    try {
        href.resize(cap);
        hcand.resize(cap);
    } catch (const std::bad_alloc &) {
        cleanup();
        return PFAC_ENOMEM;
    }
    uint64_t got = 0;
    rc = tune_scan_sync(ctx, scan, t, w, dref, cap, &got, stream);
    if (rc == PFAC_OK && cap)
        if (hipMemcpy(href.data(), dref, cap * sizeof(pfac_match), hipMemcpyDeviceToHost) != hipSuccess)
            rc = PFAC_EDEVICE;
    if (rc != PFAC_OK) {
        cleanup();
        return rc;
    }

    std::vector<pfac_tuning> cands;
    for (uint32_t bits : {12u, 16u, 18u}) {
        for (uint32_t fold : {8u, 16u, 0u})
            for (uint32_t kernel : {1u, 2u})
                for (uint32_t waves : {8u, 16u})
                    for (uint32_t g : {4u, 16u, 32u, 64u})
                        for (uint32_t cc : {0u, 1u, 2u})
                            cands.push_back({kernel, 16, bits, fold, 0, waves, g, cc});
        for (uint32_t bpl : {8u, 16u}) cands.push_back({0, bpl, bits, 8, 0, 16, 16, 1});
    }
    // a truncated image is a footprint choice: keep it, and scan it with the
    // tile kernel, the only one whose walk verifies tails
    if (start.trunc_depth) {
        cands.erase(std::remove_if(cands.begin(), cands.end(),
                                   [](const pfac_tuning &c) { return c.kernel != 0; }),
                    cands.end());
        for (auto &c : cands) c.trunc_depth = start.trunc_depth;
    }
    float best_ms = 1e30f;
    pfac_tuning best_t = start;
    std::vector<uint64_t> seen;  // (bytes per lane, index depth, wg per CU) already timed
    for (const pfac_tuning &c : cands) {
        if (pfac_trie_set_tuning(t, &c) != PFAC_OK) continue;
        // index widths that give the same depth K and symbol width repeat a point
        const uint64_t k = ((uint64_t)c.kernel << 60) | ((uint64_t)c.bytes_per_lane << 48) |
                           ((uint64_t)t->img.K << 40) | ((uint64_t)t->img.b << 32) |
                           ((uint64_t)t->img.fold_bits << 24) | ((uint64_t)c.waves_per_wg << 16) |
                           ((uint64_t)c.chunks_per_unit << 8) | ((uint64_t)c.child_check << 4) |
                           c.wg_per_cu;
        if (std::find(seen.begin(), seen.end(), k) != seen.end()) continue;
        seen.push_back(k);
        uint64_t cn = 0;
        if (tune_scan_sync(ctx, scan, t, w, dcand, cap, &cn, stream) != PFAC_OK) continue;
        if (cn != ref_n) continue;
        if (cap && (hipMemcpy(hcand.data(), dcand, cap * sizeof(pfac_match), hipMemcpyDeviceToHost) != hipSuccess ||
                    std::memcmp(hcand.data(), href.data(), cap * sizeof(pfac_match)) != 0))
            continue;
        std::vector<float> ms;
        for (int rep = 0; rep < 5; rep++) {
            (void)hipEventRecord(e0, s);
            if (scan(ctx, t, w, dcand, cap, dcount, stream) != PFAC_OK) break;
            (void)hipEventRecord(e1, s);
            (void)hipEventSynchronize(e1);
            float m = 0;
            (void)hipEventElapsedTime(&m, e0, e1);
            ms.push_back(m);
        }
        if (ms.size() < 5) continue;
        std::sort(ms.begin(), ms.end());
        if (ms[2] < best_ms) {
            best_ms = ms[2];
            best_t = c;
        }
    }
    cleanup();
    t->tuned[key] = best_t;
    *best = best_t;
    return pfac_trie_set_tuning(t, &best_t);
}

struct TuneText {
    const uint8_t *text;
    uint64_t n;
};

static int tune_scan_text(const void *ctx, const pfac_trie *t, pfac_workspace *w, pfac_match *out,
                          uint64_t cap, uint64_t *dcount, void *stream) {
    const TuneText *x = (const TuneText *)ctx;
    return pfac_scan(t, w, x->text, x->n, out, cap, dcount, nullptr, stream);
}

struct TuneBatch {
    const uint8_t *texts;
    const uint64_t *offsets;
    uint32_t n_texts;
    uint64_t total;
};

static int tune_scan_batch(const void *ctx, const pfac_trie *t, pfac_workspace *w, pfac_match *out,
                           uint64_t cap, uint64_t *dcount, void *stream) {
    const TuneBatch *x = (const TuneBatch *)ctx;
    return pfac_scan_batch(t, w, x->texts, x->offsets, x->n_texts, x->total, out, cap, dcount, stream);
}

extern "C" int pfac_autotune(pfac_trie *t, pfac_workspace *w, const uint8_t *text_dev, uint64_t n,
                             void *stream, pfac_tuning *best) {
    if (!t || !w || (!text_dev && n) || !best) return PFAC_EINVAL;
    const TuneText x{text_dev, n};
    return autotune_common(t, w, &x, tune_scan_text, size_bucket(n), stream, best);
}

extern "C" int pfac_autotune_batch(pfac_trie *t, pfac_workspace *w, const uint8_t *texts_dev,
                                   const uint64_t *offsets_dev, uint32_t n_texts,
                                   uint64_t total_bytes, void *stream, pfac_tuning *best) {
    if (!t || !w || !offsets_dev || (!texts_dev && total_bytes) || !best ||
        (n_texts == 0 && total_bytes != 0))
        return PFAC_EINVAL;
    const TuneBatch x{texts_dev, offsets_dev, n_texts, total_bytes};
    // batches are cached apart from single texts, by total size and mean text size
    const uint32_t key = (1u << 16) | (size_bucket(n_texts ? total_bytes / n_texts : 0) << 8) |
                         size_bucket(total_bytes);
    return autotune_common(t, w, &x, tune_scan_batch, key, stream, best);
}
