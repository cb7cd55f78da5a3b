// Continuous-batching scan server over one resident trie.
//
// Requests are admitted in arrival order into a byte ring in caller-provided
// device memory while the budget (text bytes in flight) allows.  Their
// host-to-device copies run on a copy stream; the admitted requests that are
// contiguous in the ring and not yet scanned form the next batched scan on
// the compute stream, which waits on the device for their copies.  Two batch
// slots alternate, so a batch is launched while the previous one still runs
// and new requests keep arriving and copying in the meantime.  When a batch
// completes its matches are copied back on the server's own stream, split
// per request by text id, and the ring space and budget of its requests are
// released.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/pfac.h"
#include "text_ring.hpp"

namespace pfac {
// +1 / -1: a server runs on the trie's current device image and tuning
// (defined with the trie)
void trie_pin(const pfac_trie *t, int delta);
// device bytes a workspace holds
uint64_t workspace_device_bytes(const pfac_workspace *w);
}  // namespace pfac

namespace {

using clk = std::chrono::steady_clock;

enum class St { Queued, Copying, Scanning, Done };

struct Req {
    uint64_t id = 0;
    const uint8_t *host = nullptr;
    uint64_t n = 0;
    clk::time_point t_submit, t_done;
    St st = St::Queued;
    pfac::TextRing::Span span;  // its bytes in the ring (admitted requests)
    hipEvent_t copied = nullptr;
    std::vector<pfac_match> res;
    uint64_t n_matches = 0;
    int rc = PFAC_OK;
    bool claimed = false;     // a caller waits for it or cancels it
    bool orphan = false;      // released by its caller while still in the ring:
                              // the worker frees it when it leaves the ring
};

void free_req(Req *r) {
    if (r->copied) (void)hipEventDestroy(r->copied);
    delete r;
}

struct Slot {
    uint64_t *offsets_dev = nullptr;   // max_batch + 1
    pfac_match *out_dev = nullptr;
    uint64_t out_cap = 0;
    uint64_t *count_dev = nullptr;
    uint64_t *offsets_host = nullptr;  // pinned
    pfac_match *out_host = nullptr;    // pinned
    uint64_t *count_host = nullptr;    // pinned
    pfac_workspace *ws = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<Req *> reqs;
};

}  // namespace

struct pfac_server {
    const pfac_trie *t = nullptr;
    uint8_t *ring = nullptr;
    uint64_t ring_bytes = 0;
    uint32_t max_batch = 1;
    hipStream_t cs = nullptr, xs = nullptr;
    hipStream_t ds = nullptr;  // own stream for result copies (device to host)
    int device = 0;
    Slot slot[2];

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    uint64_t next_id = 1;
    std::deque<Req *> queue;     // submitted, not admitted (arrival order)
    std::deque<Req *> in_ring;   // admitted, ring order
    std::map<uint64_t, Req *> by_id;
    pfac::TextRing place{0, 0};  // where admitted texts sit in `ring`
    uint64_t stat_req = 0, stat_batches = 0, stat_bytes = 0;
    std::thread worker;

    void admit_locked() {
        while (!queue.empty()) {
            Req *r = queue.front();
            uint64_t off = 0, pad = 0;
            if (!place.fits(r->n, off, pad)) break;
            queue.pop_front();
            r->span = place.place(r->n, off, pad, in_ring.empty());
            in_ring.push_back(r);
            r->st = St::Copying;
            if (hipMemcpyAsync(ring + off, r->host, r->n, hipMemcpyHostToDevice, xs) != hipSuccess ||
                hipEventRecord(r->copied, xs) != hipSuccess) {
                // no batch takes it; its ring bytes are released in ring order
                // once the copy stream has drained past it
                (void)hipStreamSynchronize(xs);
                (void)hipGetLastError();
                r->rc = PFAC_EDEVICE;
                r->st = St::Done;
                r->t_done = clk::now();
                release_locked();
                cv_done.notify_all();
            }
        }
    }

    void release_locked() {
        while (!in_ring.empty() && in_ring.front()->st == St::Done) {
            Req *r = in_ring.front();
            in_ring.pop_front();
            place.release(r->span, in_ring.empty());
            if (r->orphan) free_req(r);
        }
    }

    // The caller is done with r (waited for or cancelled, and Done): free it,
    // or, while it still holds ring bytes behind requests not yet done,
    // leave that to release_locked.  Called with the lock held.
    void retire_locked(Req *r) {
        if (std::find(in_ring.begin(), in_ring.end(), r) != in_ring.end())
            r->orphan = true;
        else
            free_req(r);
    }

    // Admitted requests not yet scanned, contiguous in the ring, in ring
    // order, up to max_batch.  Their copies may still be in flight: the scan
    // waits for them on the device.
    void form_batch_locked(std::vector<Req *> &b) {
        b.clear();
        for (Req *r : in_ring) {
            if (r->st == St::Scanning || r->st == St::Done) {
                if (b.empty()) continue;
                break;
            }
            if (r->st != St::Copying) break;
            if (!b.empty()) {
                const Req *p = b.back();
                if (p->span.off + p->n != r->span.off) break;  // ring wrapped
            }
            b.push_back(r);
            if (b.size() >= max_batch) break;
        }
    }

    int launch(Slot &S, std::vector<Req *> &b) {
        const uint64_t base = b.front()->span.off;
        S.offsets_host[0] = 0;
        for (size_t i = 0; i < b.size(); i++)
            S.offsets_host[i + 1] = S.offsets_host[i] + b[i]->n;
        const uint64_t total = S.offsets_host[b.size()];
        hipError_t e = hipMemcpyAsync(S.offsets_dev, S.offsets_host, 8 * (b.size() + 1),
                                      hipMemcpyHostToDevice, cs);
        if (e != hipSuccess) return PFAC_EDEVICE;
        // the scan starts once every text of the batch has landed
        for (Req *r : b)
            if (r->st == St::Copying && hipStreamWaitEvent(cs, r->copied, 0) != hipSuccess)
                return PFAC_EDEVICE;
        int rc = pfac_scan_batch(t, S.ws, ring + base, S.offsets_dev, (uint32_t)b.size(), total,
                                 S.out_dev, S.out_cap, S.count_dev, cs);
        if (rc != PFAC_OK) return rc;
        if (hipMemcpyAsync(S.count_host, S.count_dev, 8, hipMemcpyDeviceToHost, cs) != hipSuccess)
            return PFAC_EDEVICE;
        if (hipEventRecord(S.done, cs) != hipSuccess) return PFAC_EDEVICE;
        S.reqs = b;
        S.busy = true;
        for (Req *r : b) r->st = St::Scanning;
        stat_batches++;
        stat_bytes += total;
        return PFAC_OK;
    }

    // A request of a batch whose matches overflowed the slot: scan it alone.
    void rescan_alone(Req *r, pfac_workspace *ws) {
        uint64_t n = 0;
        r->rc = pfac_scan_sync(t, ws, ring + r->span.off, r->n, nullptr, 0, &n, nullptr, cs);
        if (r->rc != PFAC_OK && r->rc != PFAC_ETRUNC) return;
        r->rc = PFAC_OK;
        r->res.resize(n);
        if (n == 0) return;
        pfac_match *d = nullptr;
        if (hipMalloc(&d, n * sizeof(pfac_match)) != hipSuccess) {
            r->rc = PFAC_ENOMEM;
            return;
        }
        uint64_t n2 = 0;
        r->rc = pfac_scan_sync(t, ws, ring + r->span.off, r->n, d, n, &n2, nullptr, cs);
        if (r->rc == PFAC_OK &&
            hipMemcpy(r->res.data(), d, n * sizeof(pfac_match), hipMemcpyDeviceToHost) != hipSuccess)
            r->rc = PFAC_EDEVICE;
        (void)hipFree(d);
        r->n_matches = n;
    }

    void complete(Slot &S) {
        const uint64_t cnt = *S.count_host;
        std::vector<uint64_t> start(S.reqs.size() + 1, 0);
        if (cnt <= S.out_cap) {
            int copy_rc = PFAC_OK;
            if (cnt) {
                // the batch has ended (its event was seen): copy on our own stream,
                // behind nothing queued on the compute or copy streams
                if (hipMemcpyAsync(S.out_host, S.out_dev, cnt * sizeof(pfac_match),
                                   hipMemcpyDeviceToHost, ds) != hipSuccess ||
                    hipStreamSynchronize(ds) != hipSuccess) {
                    (void)hipGetLastError();
                    copy_rc = PFAC_EDEVICE;
                }
            }
            // records are sorted by text id: split by a linear sweep
            uint64_t k = 0;
            for (size_t i = 0; i < S.reqs.size(); i++) {
                Req *r = S.reqs[i];
                r->rc = copy_rc;
                if (copy_rc != PFAC_OK) continue;
                uint64_t a = k;
                while (k < cnt && S.out_host[k].text_id == i) k++;
                r->res.assign(S.out_host + a, S.out_host + k);
                for (auto &m : r->res) m.text_id = 0;
                r->n_matches = k - a;
            }
        } else {
            for (Req *r : S.reqs) rescan_alone(r, S.ws);
        }
        const auto now = clk::now();
        std::lock_guard<std::mutex> lock(mu);
        for (Req *r : S.reqs) {
            r->t_done = now;
            r->st = St::Done;
            stat_req++;
        }
        S.reqs.clear();
        S.busy = false;
        release_locked();
        cv_done.notify_all();
    }

    void run() {
        (void)hipSetDevice(device);
        std::vector<Req *> b;
        int turn = 0;
        for (;;) {
            bool did = false;
            for (int q = 0; q < 2; q++) {
                Slot &S = slot[(turn + q) & 1];
                if (S.busy && hipEventQuery(S.done) == hipSuccess) {
                    complete(S);
                    did = true;
                }
            }
            {
                std::unique_lock<std::mutex> lock(mu);
                admit_locked();
                Slot &S = slot[turn & 1];
                if (!S.busy) {
                    form_batch_locked(b);
                    if (!b.empty()) {
                        int rc = launch(S, b);
                        if (rc != PFAC_OK) {
                            // part of the batch may have been queued: let the
                            // compute stream and the batch's copies finish
                            // before its requests end and their ring bytes
                            // (and host texts) are given back
                            (void)hipStreamSynchronize(cs);
                            for (Req *r : b)
                                if (r->copied) (void)hipEventSynchronize(r->copied);
                            (void)hipGetLastError();
                            for (Req *r : b) {
                                r->rc = rc;
                                r->st = St::Done;
                                r->t_done = clk::now();
                            }
                            release_locked();
                            cv_done.notify_all();
                        } else {
                            turn++;
                        }
                        did = true;
                    }
                }
                if (stop && queue.empty() && in_ring.empty() && !slot[0].busy && !slot[1].busy)
                    break;
                // poll briefly while work is on the device, sleep when idle
                const bool busy = slot[0].busy || slot[1].busy || !in_ring.empty();
                if (!did) {
                    if (busy)
                        cv_work.wait_for(lock, std::chrono::microseconds(5));
                    else
                        cv_work.wait_for(lock, std::chrono::milliseconds(2));
                }
            }
        }
    }
};

extern "C" int pfac_server_create(const pfac_trie *t, void *arena_dev, uint64_t arena_bytes,
                                  uint64_t budget_bytes, uint32_t max_batch, void *compute_stream,
                                  void *copy_stream, pfac_server **out) {
    if (!out) return PFAC_EINVAL;
    *out = nullptr;
    if (!t || !arena_dev || max_batch == 0 || budget_bytes == 0 || budget_bytes > arena_bytes)
        return PFAC_EINVAL;
    pfac_stats st;
    if (pfac_trie_stats(t, &st) != PFAC_OK || st.bytes_device == 0) return PFAC_ENODEV;
    pfac_server *s = new (std::nothrow) pfac_server();
    if (!s) return PFAC_ENOMEM;
    s->t = t;
    s->max_batch = max_batch;
    s->cs = (hipStream_t)compute_stream;
    s->xs = (hipStream_t)copy_stream;
    (void)hipGetDevice(&s->device);
    if (hipStreamCreateWithFlags(&s->ds, hipStreamNonBlocking) != hipSuccess) {
        delete s;
        return PFAC_EDEVICE;
    }
    // arena: [ text ring (budget) | slot 0 | slot 1 ]
    uint8_t *a = (uint8_t *)arena_dev;
    const uint64_t rest = arena_bytes - budget_bytes;
    const uint64_t per_slot = rest / 2;
    const uint64_t off_bytes = ((8ull * (max_batch + 1)) + 255) & ~255ull;
    if (per_slot < off_bytes + 256 + 64 * sizeof(pfac_match)) {
        delete s;
        return PFAC_EINVAL;
    }
    s->ring = a;
    s->ring_bytes = budget_bytes;
    s->place = pfac::TextRing(budget_bytes, budget_bytes);
    int rc = PFAC_OK;
    for (int q = 0; q < 2 && rc == PFAC_OK; q++) {
        Slot &S = s->slot[q];
        uint8_t *p = a + budget_bytes + q * per_slot;
        p = (uint8_t *)(((uintptr_t)p + 255) & ~(uintptr_t)255);
        S.offsets_dev = (uint64_t *)p;
        S.count_dev = (uint64_t *)(p + off_bytes);
        S.out_dev = (pfac_match *)(p + off_bytes + 256);
        S.out_cap = (per_slot - off_bytes - 512) / sizeof(pfac_match);
        if (hipHostMalloc((void **)&S.offsets_host, 8 * (max_batch + 1)) != hipSuccess ||
            hipHostMalloc((void **)&S.out_host, S.out_cap * sizeof(pfac_match)) != hipSuccess ||
            hipHostMalloc((void **)&S.count_host, 8) != hipSuccess ||
            hipEventCreateWithFlags(&S.done, hipEventDisableTiming) != hipSuccess)
            rc = PFAC_ENOMEM;
        if (rc == PFAC_OK) rc = pfac_workspace_create(&S.ws);
        if (rc == PFAC_OK) rc = pfac_workspace_reserve(S.ws, budget_bytes, max_batch, S.out_cap);
    }
    if (rc != PFAC_OK) {
        for (auto &S : s->slot) {
            if (S.offsets_host) (void)hipHostFree(S.offsets_host);
            if (S.out_host) (void)hipHostFree(S.out_host);
            if (S.count_host) (void)hipHostFree(S.count_host);
            if (S.done) (void)hipEventDestroy(S.done);
            pfac_workspace_free(S.ws);
        }
        (void)hipStreamDestroy(s->ds);
        delete s;
        return rc;
    }
    pfac::trie_pin(t, +1);
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return PFAC_OK;
}

extern "C" int pfac_server_submit(pfac_server *s, const uint8_t *text_host, uint64_t n,
                                  uint64_t *request_id) {
    if (!s || !request_id || (n && !text_host)) return PFAC_EINVAL;
    if (n > s->ring_bytes) return PFAC_EINVAL;
    Req *r = new (std::nothrow) Req();
    if (!r) return PFAC_ENOMEM;
    r->host = text_host;
    r->n = n;
    r->t_submit = clk::now();
    if (n && hipEventCreateWithFlags(&r->copied, hipEventDisableTiming) != hipSuccess) {
        delete r;
        return PFAC_EDEVICE;
    }
    std::lock_guard<std::mutex> lock(s->mu);
    if (s->stop) {
        if (r->copied) (void)hipEventDestroy(r->copied);
        delete r;
        return PFAC_EINVAL;
    }
    r->id = s->next_id++;
    s->by_id[r->id] = r;
    if (n == 0) {
        r->st = St::Done;
        r->t_done = r->t_submit;
        s->stat_req++;
    } else {
        s->queue.push_back(r);
        s->cv_work.notify_one();
    }
    *request_id = r->id;
    return PFAC_OK;
}

extern "C" int pfac_server_wait(pfac_server *s, uint64_t request_id, int64_t timeout_ms,
                                pfac_match *out_host, uint64_t capacity, uint64_t *n_matches,
                                double *latency_s) {
    if (!s || !n_matches) return PFAC_EINVAL;
    std::unique_lock<std::mutex> lock(s->mu);
    auto it = s->by_id.find(request_id);
    if (it == s->by_id.end()) return PFAC_EINVAL;
    Req *r = it->second;
    if (r->claimed) return PFAC_EINVAL;  // another thread waits for it or cancels it
    // while claimed nobody else erases the entry, so `it` stays valid
    r->claimed = true;
    auto done = [&] { return r->st == St::Done; };
    if (timeout_ms < 0) {
        s->cv_done.wait(lock, done);
    } else if (!s->cv_done.wait_for(lock, std::chrono::milliseconds(timeout_ms), done)) {
        r->claimed = false;
        return PFAC_EBUSY;
    }
    s->by_id.erase(it);
    // Done: the worker no longer writes r, and does not free it before it
    // is retired below, so the results are copied unlocked
    lock.unlock();
    int rc = r->rc;
    *n_matches = r->n_matches;
    if (rc == PFAC_OK && out_host)
        std::memcpy(out_host, r->res.data(), std::min(capacity, r->n_matches) * sizeof(pfac_match));
    if (latency_s) *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
    if (rc == PFAC_OK && r->n_matches > capacity) rc = PFAC_ETRUNC;
    lock.lock();
    s->retire_locked(r);
    return rc;
}

extern "C" int pfac_server_cancel(pfac_server *s, uint64_t request_id) {
    if (!s) return PFAC_EINVAL;
    std::unique_lock<std::mutex> lock(s->mu);
    auto it = s->by_id.find(request_id);
    if (it == s->by_id.end() || it->second->claimed) return PFAC_EINVAL;
    Req *r = it->second;
    r->claimed = true;  // from here on nobody else erases or frees it
    switch (r->st) {
    case St::Queued:  // never admitted: no copy was issued
        s->queue.erase(std::find(s->queue.begin(), s->queue.end(), r));
        break;
    case St::Copying: {
        // admitted but in no batch yet: batches skip it from now on and its
        // ring bytes are released in ring order
        r->st = St::Done;
        s->release_locked();
        s->cv_work.notify_one();
        // its copy may still read the text: wait for it unlocked (r is not
        // an orphan yet, so the worker does not free it meanwhile)
        const hipEvent_t ev = r->copied;
        lock.unlock();
        (void)hipEventSynchronize(ev);
        lock.lock();
        break;
    }
    case St::Scanning:  // its batch runs to the end; the results are dropped
        s->cv_done.wait(lock, [&] { return r->st == St::Done; });
        break;
    case St::Done:
        break;
    }
    s->by_id.erase(it);
    s->retire_locked(r);
    return PFAC_OK;
}

extern "C" int pfac_server_stats(const pfac_server *s, uint64_t *requests, uint64_t *batches,
                                 uint64_t *bytes, uint64_t *device_bytes) {
    if (!s) return PFAC_EINVAL;
    pfac_server *m = const_cast<pfac_server *>(s);
    std::lock_guard<std::mutex> lock(m->mu);
    if (requests) *requests = s->stat_req;
    if (batches) *batches = s->stat_batches;
    if (bytes) *bytes = s->stat_bytes;
    if (device_bytes) {
        uint64_t d = 0;
        for (const Slot &S : s->slot) d += pfac::workspace_device_bytes(S.ws);
        *device_bytes = d;
    }
    return PFAC_OK;
}

extern "C" void pfac_server_free(pfac_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lock(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    for (auto &S : s->slot) {
        if (S.offsets_host) (void)hipHostFree(S.offsets_host);
        if (S.out_host) (void)hipHostFree(S.out_host);
        if (S.count_host) (void)hipHostFree(S.count_host);
        if (S.done) (void)hipEventDestroy(S.done);
        pfac_workspace_free(S.ws);
    }
    // the worker has drained the ring (freeing its orphans): what is left
    // are requests nobody waited for or cancelled
    for (auto &kv : s->by_id) free_req(kv.second);
    if (s->ds) (void)hipStreamDestroy(s->ds);
    pfac::trie_pin(s->t, -1);
    delete s;
}
