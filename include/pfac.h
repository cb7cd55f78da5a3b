/*
 * pfac.h - C ABI of the MI355X (gfx950) failure-less Aho-Corasick scanner.
 *
 * The library answers the problem of Background, "Multi-Pattern Matching":
 * given patterns P_0..P_{k-1} and a text T, report every (start position i,
 * pattern j) with T[i .. i+|P_j|) == P_j.  It does so with the failure-less
 * walk of Background, "Parallel Failure-Less Aho-Corasick" (one GPU lane per
 * start byte, walking the trie from the root until the first mismatch and
 * reporting every pattern that ends on the way), over the trie of Design and
 * Implementation: built breadth first, level by level (step I), stored as a
 * row-major array (step II) and compressed as a compressed-row-storage matrix
 * (the CRS step): row_ptr per node, the edge label as column index and the
 * child as value.
 *
 * Conventions shared by every call:
 *   - Functions return PFAC_OK (0) or a negative PFAC_E* code.
 *   - pattern_id is the 0-based index of the pattern in the build call.
 *   - pos is the 0-based byte offset of the match inside its own text.
 *   - Results are sorted by (text_id, pos, pattern_id), ascending; every match
 *     is reported exactly once, duplicate patterns under each of their ids.
 *   - No match crosses the end of a text.
 *   - Pointers named *_dev are device (HBM) addresses on the current HIP
 *     device; *_host are host addresses.  `stream` is a hipStream_t (NULL =
 *     the default stream).  All scan calls are asynchronous on `stream`
 *     unless their name ends in _sync.
 *   - The caller owns every buffer it passes; the library owns the objects
 *     it returns until the matching *_free call.
 *   - A trie changes only through pfac_trie_set_tuning and pfac_autotune,
 *     which may rebuild and re-upload its device image: they must not run
 *     while a scan with that trie is in flight or being issued.  Otherwise a
 *     trie may be shared by many streams and threads.  A workspace
 *     serializes: calls that share a workspace must be issued on one stream
 *     (or otherwise ordered); calls on different workspaces may overlap.
 */
#ifndef PFAC_H
#define PFAC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PFAC_OK 0
#define PFAC_EINVAL (-1)   /* NULL pointer, bad size or bad flag */
#define PFAC_EEMPTY (-2)   /* a pattern of length 0 */
#define PFAC_ENOMEM (-3)   /* host or device allocation failed */
#define PFAC_EDEVICE (-4)  /* a HIP call failed; see pfac_last_hip_error() */
#define PFAC_ETRUNC (-5)   /* more matches than `capacity`; the count is still exact */
#define PFAC_ENODEV (-6)   /* the trie was built without a device image */
#define PFAC_EBUSY (-7)    /* serving: over budget / queue full, retry later */

/* pfac_build flags */
#define PFAC_BUILD_HOST_ONLY 1u  /* build the CRS trie on the host only; no HIP call */

/* One match: 16 bytes, naturally aligned. */
typedef struct {
    uint64_t pos;          /* start offset inside text `text_id` */
    uint32_t pattern_id;   /* index of the pattern in the build call */
    uint32_t text_id;      /* index of the text in the batch (0 for single-text scans) */
} pfac_match;

typedef struct pfac_trie pfac_trie;
typedef struct pfac_workspace pfac_workspace;
typedef struct pfac_graph pfac_graph;
typedef struct pfac_server pfac_server;

/* Sizes and footprint of a built trie (Design and Implementation; Results). */
typedef struct {
    uint64_t nodes;            /* N = distinct non-empty prefixes + 1 (the root) */
    uint64_t edges;            /* nnz = N - 1 */
    uint64_t n_patterns;       /* k */
    uint64_t min_len, max_len; /* shortest / longest pattern (0 when k = 0) */
    uint64_t depth;            /* levels below the root = max_len */
    uint64_t bytes_crs;        /* row_ptr + labels + child + term_ptr + term_ids */
    uint64_t crs_elements;     /* 2 nnz + N + 1 (row_ptr, col_ind, val) */
    uint64_t bytes_dense256;   /* uncompressed node x 256 int32 transition table = 1024 N */
    uint64_t bytes_bitmap36;   /* 256-bit bitmap + 4-byte offset per node = 36 N */
    uint64_t bytes_device;     /* device image actually resident in HBM */
    uint32_t alphabet_size;    /* distinct bytes used by the patterns */
    uint32_t symbol_bits;      /* bits per symbol in the level index */
    uint32_t index_depth;      /* K: levels resolved by the level index in LDS */
    uint32_t lds_bytes;        /* dynamic LDS per workgroup of the scan kernel */
    uint32_t scan_kernel;      /* kernels the current tuning launches: 0 = tile, 1 = fused
                                  wave kernel, 2 = split filter + walk kernels */
    uint32_t scan_waves;       /* waves per workgroup it launches with (after LDS fitting) */
    uint32_t stage1;           /* wave kernels' first filter: 0 = rolling code over K symbols (or
                                  the tile kernel), 1 / 2 = two-byte table with the third byte
                                  folded to 8 / 16 bits, 3 = 16-symbol filter */
    uint32_t stage2;           /* second filter: 0 = none, 1 = child labels of depth-K nodes,
                                  2 = prefix-4 filter, 3 = alphabet bytes + 16-bit fingerprint */
    double build_seconds;      /* host build time (not part of scan timing) */
    double upload_seconds;     /* host -> device copy time of the image */
    uint64_t bytes_bitmap_narrow; /* every node as a bitmapped node (Design and Implementation,
                                     bitmapped-node figure) with the bitmap narrowed to the
                                     2^b symbols used, b = ceil(log2 alphabet), in whole bytes,
                                     + a 4-byte first-child offset (= bytes_bitmap36 for b = 8) */
    uint64_t bytes_level_index;   /* LDS bytes of the level index at depth K (bitmap + ranks) */
    uint64_t bytes_top_nodes;     /* LDS bytes of the same K levels as bitmapped nodes (nodes of
                                     depths 0 .. K-1, bitmap over the index's 2^symbol_bits
                                     symbols padded to 32-bit words, + first child) */
    uint64_t trunc_depth;         /* depth the device image is truncated at (0 = whole trie) */
    uint64_t bytes_nodes;         /* 16-byte node records in the device image */
    uint64_t bytes_tails;         /* truncated image: tail entries + the pattern bytes after the
                                     truncation depth that the walk verifies */
    uint64_t dag_nodes;           /* the trie with equal subtries merged (Design and
                                     Implementation, steps IV and V: suffix and end-node
                                     merging): nodes ... */
    uint64_t dag_edges;           /* ... and edges */
    uint64_t bytes_dag_crs;       /* that DAG in CRS form with exact pattern ids: row pointers,
                                     labels, children, rank added per edge, terminal flags and
                                     the k ids in sorted-string order */
} pfac_stats;

/* Launch parameters chosen by hand or by pfac_autotune. */
typedef struct {
    uint32_t kernel;           /* 0 = tile kernel (workgroup tiles), 1 = fused wave kernel
                                  (filter, walks and emission in one kernel), 2 = split wave
                                  kernels (filter kernel writes walk candidates, a walk kernel
                                  runs them; for alphabets of at most four bytes it uses the
                                  16-symbol filter when every pattern has 16 bytes or more),
                                  3 = by launch size: 2 with units of up to 64 chunks
                                  for launches (a text, or a whole batch) of 8 MiB or more,
                                  else 0 with 4 bytes per lane below 1 MiB and 8 from
                                  there (the default for byte
                                  alphabets with K = 2 and for alphabets of at most four
                                  bytes).  Statistics report the kernel of large launches */
    uint32_t bytes_per_lane;   /* tile kernel: start positions per lane per tile: 4, 8 or 16 */
    uint32_t index_bits;       /* level-index width in bits (1..18); depth K = bits / symbol_bits */
    uint32_t fold_bits;        /* wave kernel prefix filter: 0 (level bitmap), 8 or 16 bits per node */
    uint32_t wg_per_cu;        /* resident workgroups per compute unit (0 = occupancy max) */
    uint32_t waves_per_wg;     /* wave kernel: 4, 8, 12 or 16 waves per workgroup (fewer when
                                  the LDS tables leave no room) */
    uint32_t chunks_per_unit;  /* wave kernel: at most this many 1 KiB chunks per output
                                  unit, 1..64; each launch takes the number up to it that
                                  spreads its units most evenly over the grid's waves (a
                                  batch of small texts takes small units and fills the GPU) */
    uint32_t child_check;      /* wave kernel second stage: 0 = none, 1 = check the byte after
                                  the level index against the depth-K node's child labels in
                                  LDS when they fit, 2 = the prefix-4 filter (two hashed bits
                                  per distinct 4-byte pattern prefix; byte alphabets with every
                                  pattern of 4 bytes or more, the default there), else as 1 */
    uint32_t top_nodes;        /* tile kernel: how the first K levels are resolved in LDS:
                                  0 = the level index (one lookup of the K-symbol code),
                                  1 = bitmapped nodes of depths 0 .. K-1 (Design and
                                  Implementation, bitmapped-node figure: K dependent lookups,
                                  child = first child + set bits below the symbol).  Setting 1
                                  fails with PFAC_EINVAL when those nodes do not fit in LDS */
    uint32_t trunc_depth;      /* 0 = the whole trie on the device; D = 1..255: the device image
                                  keeps only nodes of depths 0..D (Design and Implementation,
                                  step III, truncation) and each depth-D node with children
                                  lists the terminal nodes below it; the walk verifies the text
                                  against their pattern bytes, longest first, so results stay
                                  exact.  Scans then use the tile kernel (kernel is ignored) and
                                  the level index depth is at most D */
    uint32_t dag;              /* 1 = the device image is the merged DAG (steps IV and V) with
                                  pattern identities kept on the edges: each edge adds the
                                  number of distinct pattern strings sorting before its subtrie,
                                  so a walk sums to the rank of its deepest pattern string, whose
                                  root-path pattern list the image keeps.  Scans use the tile
                                  kernel; cannot be combined with top_nodes or trunc_depth
                                  (PFAC_EINVAL) */
} pfac_tuning;

/* ----------------------------------------------------------------- errors */

/* Last HIP error code seen by this thread (0 = hipSuccess). */
int pfac_last_hip_error(void);
/* Static description of a PFAC_E* code. */
const char *pfac_strerror(int code);

/* ------------------------------------------------------------------ build */

/*
 * Build the CRS trie of `n_patterns` patterns (Design and Implementation,
 * steps I, II, VI and the CRS step) and, unless PFAC_BUILD_HOST_ONLY, upload
 * its device image to the current HIP device.  Pattern j is
 * patterns[j][0 .. lengths[j]).  The bytes are copied; the caller may free
 * them on return.  n_patterns = 0 is valid (nothing ever matches).
 * Errors: PFAC_EINVAL (out == NULL, or n_patterns > 0 with NULL arrays),
 * PFAC_EEMPTY (some lengths[j] == 0), PFAC_ENOMEM, PFAC_EDEVICE.
 */
int pfac_build(const uint8_t *const *patterns, const uint64_t *lengths, uint32_t n_patterns,
               uint32_t flags, pfac_trie **out);

/*
 * Same as pfac_build with the patterns stored back to back:
 * pattern j = data[offsets[j] .. offsets[j+1]); offsets has n_patterns + 1
 * entries, non-decreasing.
 */
int pfac_build_packed(const uint8_t *data, const uint64_t *offsets, uint32_t n_patterns,
                      uint32_t flags, pfac_trie **out);

int pfac_trie_stats(const pfac_trie *t, pfac_stats *out);

/*
 * Copy the CRS arrays into caller-allocated host arrays (any may be NULL):
 *   row_ptr[N+1]   edges of node v are row_ptr[v] .. row_ptr[v+1]
 *   labels[N-1]    edge label (unsigned byte), ascending within a row
 *   child[N-1]     child node of each edge (breadth-first numbering makes
 *                  child[e] == e + 1)
 *   term_ptr[N+1]  pattern ids ending at node v are term_ids[term_ptr[v] ..
 *   term_ids[k]    term_ptr[v+1]), ascending
 * Nodes are numbered breadth first, children by ascending label.
 */
int pfac_trie_export(const pfac_trie *t, uint32_t *row_ptr, uint8_t *labels, uint32_t *child,
                     uint32_t *term_ptr, uint32_t *term_ids);

/* Free a trie and its device image.  NULL is ignored.  Graphs captured
 * with it must be freed first. */
void pfac_trie_free(pfac_trie *t);

/* Current / new launch parameters.  Setting them may rebuild the device
 * image on the host and re-upload it (synchronous: no scan with this trie
 * may be in flight).  The wave kernels (kernel 1, 2) run where they apply
 * (whole, unmerged images with patterns of at most 65,535 bytes) and their
 * tables fit in LDS; the tile kernel runs otherwise.  Errors: PFAC_EINVAL
 * (NULL, a field out of range, dag combined with top_nodes or trunc_depth,
 * or a tuning whose kernel does not fit in LDS, e.g. bitmapped top nodes or
 * a level index too large; the previous tuning and image stay), PFAC_EBUSY
 * (the image would be rebuilt while a captured graph reads it, or the tuning
 * would change at all while a server uses the trie), PFAC_ENOMEM,
 * PFAC_EDEVICE. */
int pfac_trie_get_tuning(const pfac_trie *t, pfac_tuning *out);
int pfac_trie_set_tuning(pfac_trie *t, const pfac_tuning *tuning);

/* The kernels a launch over `total_bytes` bytes (one text, or a whole
 * batch) runs with the current tuning, with kernel 3 resolved by that size:
 * *kernel = 0 (tile kernel), 1 (fused wave kernel) or 2 (split filter +
 * walk kernels); *tuning (may be NULL) = the tuning that launch uses.
 * Host only.  Errors: PFAC_EINVAL (NULL trie or kernel). */
int pfac_trie_launch_kernel(const pfac_trie *t, uint64_t total_bytes, uint32_t *kernel,
                            pfac_tuning *tuning);

/* -------------------------------------------------------------- workspace */

/* Device scratch for scans: match staging, per-tile counts, plan tables.
 * It grows on demand (hipMalloc) and is reused across calls. */
int pfac_workspace_create(pfac_workspace **out);
void pfac_workspace_free(pfac_workspace *w);
/* Pre-size the scratch for texts of up to `max_bytes` bytes, `max_texts`
 * texts and `max_matches` matches, so later scans allocate nothing.  Growing
 * a workspace (here or inside a scan that needs more) first waits for the
 * whole device, since queued work may still use the old buffers: reserve
 * before capturing a stream that scans with it.
 * Errors: PFAC_EINVAL (w NULL), PFAC_ENOMEM (the device cannot hold it; the
 * workspace stays usable for smaller scans), PFAC_EDEVICE. */
int pfac_workspace_reserve(pfac_workspace *w, uint64_t max_bytes, uint32_t max_texts,
                           uint64_t max_matches);

/*
 * Instrumentation: when both events are set (hipEvent_t, NULL to clear),
 * every later scan on this workspace records `start_event` on its stream
 * right before the main scan kernel (the tile kernel, the fused wave kernel,
 * or the filter kernel of the split pair) and `stop_event` right after it,
 * so the caller can time that kernel alone.  The events are only recorded,
 * never created or destroyed, by the library.
 */
int pfac_workspace_set_timing(pfac_workspace *w, void *start_event, void *stop_event);

/* ------------------------------------------------------------------- scan */

/*
 * Scan one text of n bytes at text_dev.  Writes the sorted matches to
 * out_dev[0 .. min(count, capacity)) and the exact count to *n_matches_dev
 * (device uint64).  If counts_dev is not NULL it receives the number of
 * matches starting at each position, counts_dev[0 .. n).  Asynchronous on
 * `stream`; n = 0 and an empty trie are valid.  When the count exceeds
 * capacity the output contents are unspecified: grow and scan again.
 * Errors: PFAC_EINVAL, PFAC_ENODEV, PFAC_ENOMEM, PFAC_EDEVICE.
 */
int pfac_scan(const pfac_trie *t, pfac_workspace *w, const uint8_t *text_dev, uint64_t n,
              pfac_match *out_dev, uint64_t capacity, uint64_t *n_matches_dev,
              uint32_t *counts_dev, void *stream);

/*
 * pfac_scan for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid the allocator.
 * Same arguments, results and errors as pfac_scan without the workspace:
 * its scratch (per-unit counts and offsets, walk candidates, match staging)
 * lives in one 64 MiB array that the library holds in each device's memory
 * from its load until the process ends, so no call allocates or frees
 * anything.  The scratch a scan needs grows with n and capacity: about
 * 700 bytes per KiB of text plus 16 bytes per unit of capacity (a 32 MiB
 * text with capacity 2^20 fits); a call whose needs exceed 64 MiB returns
 * PFAC_EINVAL before touching the device.  Every call on a device uses the
 * same array: calls that may overlap on one device (different streams or
 * threads) race and must be ordered by the caller; a call on one stream
 * after another is safe.  The array keeps the previous call's contents;
 * the scan clears what it needs cleared.
 */
int pfac_scan_noalloc(const pfac_trie *t, const uint8_t *text_dev, uint64_t n,
                      pfac_match *out_dev, uint64_t capacity, uint64_t *n_matches_dev,
                      uint32_t *counts_dev, void *stream);

/* pfac_scan, then wait for `stream` and return the count in *n_matches_host;
 * returns PFAC_ETRUNC when it exceeds capacity. */
int pfac_scan_sync(const pfac_trie *t, pfac_workspace *w, const uint8_t *text_dev, uint64_t n,
                   pfac_match *out_dev, uint64_t capacity, uint64_t *n_matches_host,
                   uint32_t *counts_dev, void *stream);

/*
 * Scan a batch of texts stored back to back in one device buffer: text i is
 * texts_dev[offsets[i] .. offsets[i+1]), offsets_dev has n_texts + 1
 * non-decreasing device uint64 entries with offsets[0] == 0 and
 * offsets[n_texts] == total_bytes (empty texts are allowed).  One persistent
 * launch covers every text; tiles span text boundaries and every walk stops
 * at the end of its own text.  Results carry text_id.  Asynchronous.
 */
int pfac_scan_batch(const pfac_trie *t, pfac_workspace *w, const uint8_t *texts_dev,
                    const uint64_t *offsets_dev, uint32_t n_texts, uint64_t total_bytes,
                    pfac_match *out_dev, uint64_t capacity, uint64_t *n_matches_dev,
                    void *stream);

/*
 * Baseline for the batched scan: one pfac_scan launch per text, in order,
 * each writing at the running output offset.  Needs the offsets on the host
 * (offsets_host, n_texts + 1 entries) to size every launch; writes the total
 * count to *n_matches_dev.  Same output as pfac_scan_batch.
 */
int pfac_scan_batch_plain(const pfac_trie *t, pfac_workspace *w, const uint8_t *texts_dev,
                          const uint64_t *offsets_host, uint32_t n_texts,
                          pfac_match *out_dev, uint64_t capacity, uint64_t *n_matches_dev,
                          void *stream);

/*
 * Capture pfac_scan_batch with these exact arguments into a HIP graph and
 * instantiate it.  Replays read the texts, offsets and outputs at the same
 * device addresses, so the caller may refill them between replays as long
 * as n_texts and total_bytes stay the same.  The graph allocates and owns
 * its own scratch, so `w` (which may be NULL) stays free for other scans; only
 * its timing events, if set, are taken over (see pfac_graph_set_timing).  While the graph exists the trie's device image is pinned:
 * a pfac_trie_set_tuning that would rebuild it (index_bits, fold_bits,
 * trunc_depth or dag changed, as the autotuner may do) fails with
 * PFAC_EBUSY, and the trie must outlive the graph.  Replays of one graph
 * must not overlap each other.  The capture runs on a stream the library
 * creates for it; `stream` is not used (replays take theirs in
 * pfac_graph_launch).
 */
int pfac_graph_create_batch(const pfac_trie *t, pfac_workspace *w, const uint8_t *texts_dev,
                            const uint64_t *offsets_dev, uint32_t n_texts, uint64_t total_bytes,
                            pfac_match *out_dev, uint64_t capacity, uint64_t *n_matches_dev,
                            void *stream, pfac_graph **out);
int pfac_graph_launch(pfac_graph *g, void *stream);

/*
 * Kernel timing inside replays: when `w` had timing events set
 * (pfac_workspace_set_timing) at pfac_graph_create_batch, the graph records
 * them right before and right after its main scan kernel at every replay.
 * This call makes later replays record these two events (hipEvent_t)
 * instead, so each replay can be timed with events of its own.  PFAC_EINVAL
 * for NULL arguments or a graph captured without timing events (or without
 * a scan kernel: an empty batch).
 */
int pfac_graph_set_timing(pfac_graph *g, void *start_event, void *stop_event);
void pfac_graph_free(pfac_graph *g);

/*
 * Time a grid of launch parameters on the given text (device buffer, n
 * bytes), keep the fastest in the trie and return it in *best.  Every
 * candidate's match list is checked against the current parameters' list;
 * a candidate that disagrees is discarded.  Results are cached per
 * (trie, size bucket) for the life of the trie.  Synchronous.
 */
int pfac_autotune(pfac_trie *t, pfac_workspace *w, const uint8_t *text_dev, uint64_t n,
                  void *stream, pfac_tuning *best);

/*
 * pfac_autotune for the batched launch: every candidate scans the batch
 * (texts_dev, offsets_dev, n_texts, total_bytes as in pfac_scan_batch) and
 * its list is checked against the starting tuning's.  Cached per (trie,
 * total size bucket, mean text size bucket), apart from single texts.
 * Synchronous.  PFAC_EBUSY while a server uses the trie.
 */
int pfac_autotune_batch(pfac_trie *t, pfac_workspace *w, const uint8_t *texts_dev,
                        const uint64_t *offsets_dev, uint32_t n_texts, uint64_t total_bytes,
                        void *stream, pfac_tuning *best);

/* ---------------------------------------------------------------- serving */

/*
 * Continuous-batching scan server over one resident trie.
 *   arena_dev / arena_bytes: caller-owned device memory the server carves
 *     into text slots and result buffers (it allocates no text memory itself);
 *   budget_bytes: cap on text bytes + reserved result bytes in flight
 *     (<= arena_bytes);
 *   max_batch: most requests in one batched launch;
 *   compute_stream / copy_stream: scans run on the first, host<->device
 *     copies on the second, so copies overlap scans.
 * A worker thread admits queued requests in arrival order as budget and
 * slots free up, copies them to the device, and launches one batched scan
 * over every request whose copy has landed while the previous batch runs.
 * The trie must outlive the server, and its tuning and device image are
 * fixed while the server exists: pfac_trie_set_tuning with a different
 * tuning, and pfac_autotune / pfac_autotune_batch, fail with PFAC_EBUSY.
 * Device memory: the arena, plus the scratch of two batch slots that the
 * server allocates itself (reported by pfac_server_stats).
 */
int pfac_server_create(const pfac_trie *t, void *arena_dev, uint64_t arena_bytes,
                       uint64_t budget_bytes, uint32_t max_batch, void *compute_stream,
                       void *copy_stream, pfac_server **out);

/*
 * Queue a scan of text_host[0 .. n).  The bytes are read until the request
 * completes, so the buffer must stay valid until pfac_server_wait or
 * pfac_server_cancel returns PFAC_OK for it.  Returns the request id in *request_id.  PFAC_EINVAL if a single
 * request can never fit the budget.
 */
int pfac_server_submit(pfac_server *s, const uint8_t *text_host, uint64_t n,
                       uint64_t *request_id);

/*
 * Wait for a request (timeout_ms < 0: forever).  On PFAC_OK, *n_matches holds
 * its match count and, if out_host is not NULL, up to `capacity` matches are
 * copied there (text_id = 0, positions relative to the request's text).
 * PFAC_ETRUNC when the count exceeds capacity (count still exact).
 * latency_s (optional) receives submit-to-completion seconds.  Returns
 * PFAC_EBUSY on timeout (the request stays queued and may be waited for
 * again).  Each request may be waited for once, by one thread at a time:
 * PFAC_EINVAL for an id already waited for, cancelled, unknown, or being
 * waited for by another thread.
 */
int pfac_server_wait(pfac_server *s, uint64_t request_id, int64_t timeout_ms,
                     pfac_match *out_host, uint64_t capacity, uint64_t *n_matches,
                     double *latency_s);

/*
 * Withdraw a request that is not being waited for.  A request still queued
 * for the budget is dropped at once; one admitted but not yet in a batch
 * leaves the ring once its copy has landed; one whose batch is running is
 * finished by the device and its matches are dropped (the call returns when
 * that batch ends); a completed one has its matches dropped.  After
 * PFAC_OK the text buffer is no longer read and the id is released: waiting
 * for it or cancelling it again returns PFAC_EINVAL.  PFAC_EINVAL also for
 * an unknown id and for a request another thread is waiting for.
 */
int pfac_server_cancel(pfac_server *s, uint64_t request_id);

/* Counters since creation: requests completed, batches launched, text bytes
 * scanned; and device_bytes, the device memory the server allocated itself
 * beyond the caller's arena: the scratch of its two batch slots, each sized
 * for a batch of budget_bytes of text (about 0.65 bytes per text byte:
 * per-chunk counts, inline records and walk candidates) plus match staging
 * for the slot's output capacity (16 bytes per record).  Any pointer may be
 * NULL. */
int pfac_server_stats(const pfac_server *s, uint64_t *requests, uint64_t *batches,
                      uint64_t *bytes, uint64_t *device_bytes);

/* Finish every queued request, stop the worker and free the server.  No other
 * call on the server may run during or after it. */
void pfac_server_free(pfac_server *s);

#ifdef __cplusplus
}
#endif

#endif /* PFAC_H */
