// Randomized check of the serving ring's placement (TextRing), on the CPU:
// requests arrive in order with random sizes, are placed first-come
// first-served while they fit, finish in any order (completion or
// cancellation) and leave the ring in placement order, as the server does.
// Every byte of the ring is tracked: a placement may only take free bytes
// (its text and any end bytes it holds), the bytes held never exceed the
// budget, the ring's count equals the bytes held, and an empty ring always
// takes the next request (no request waits forever).
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <random>
#include <vector>

#include "../../paper_1702_03657_amd/csrc/text_ring.hpp"

using pfac::TextRing;

struct Live {
    TextRing::Span span;
    uint64_t pad_lo = 0;  // end bytes held: [pad_lo, size) when span.len > span.n
    bool done = false;
    int id = 0;
};

static int fail(const char *what, int seed, long step) {
    std::printf("FAIL %s (seed %d, step %ld)\n", what, seed, step);
    return 1;
}

static int run(int seed, uint64_t size, uint64_t budget, long steps, uint64_t max_n) {
    std::mt19937_64 rng(seed);
    TextRing ring(size, budget);
    std::vector<int> owner(size, -1);
    std::deque<uint64_t> queue;  // sizes waiting, arrival order
    std::deque<Live> live;       // placement order
    uint64_t tail_seen = 0;      // end of the newest placed text
    int next_id = 0;
    long placed = 0, wrapped = 0;
    for (long step = 0; step < steps; step++) {
        const unsigned op = (unsigned)(rng() % 8);
        if (op < 3) {  // a request arrives (sizes skewed small)
            const uint64_t n = 1 + (rng() % 3 == 0 ? rng() % max_n : rng() % (max_n / 8 + 1));
            queue.push_back(n);
        } else if (op < 6 && !live.empty()) {  // one finishes, any of them
            live[rng() % live.size()].done = true;
        } else if (op == 6 && !queue.empty()) {  // one still queued is cancelled
            queue.erase(queue.begin() + (long)(rng() % queue.size()));
        }
        // leave in placement order
        while (!live.empty() && live.front().done) {
            const Live l = live.front();
            live.pop_front();
            for (uint64_t b = l.span.off; b < l.span.off + l.span.n; b++) {
                if (owner[b] != l.id) return fail("released bytes not owned", seed, step);
                owner[b] = -1;
            }
            if (l.span.len > l.span.n)
                for (uint64_t b = l.pad_lo; b < size; b++) {
                    if (owner[b] != l.id) return fail("released end bytes not owned", seed, step);
                    owner[b] = -1;
                }
            ring.release(l.span, live.empty());
        }
        // admit first-come first-served
        while (!queue.empty()) {
            uint64_t off = 0, pad = 0;
            if (!ring.fits(queue.front(), off, pad)) {
                if (live.empty()) return fail("empty ring refused a request", seed, step);
                break;
            }
            const uint64_t n = queue.front();
            queue.pop_front();
            Live l;
            l.id = next_id++;
            l.span = ring.place(n, off, pad, live.empty());
            if (l.span.off != off || l.span.n != n || l.span.len != n + pad)
                return fail("span differs from the place chosen", seed, step);
            if (off + n > size) return fail("text past the end of the ring", seed, step);
            for (uint64_t b = off; b < off + n; b++) {
                if (owner[b] != -1) return fail("placed over held bytes", seed, step);
                owner[b] = l.id;
            }
            if (pad) {
                if (off != 0) return fail("end bytes held by a text not at 0", seed, step);
                l.pad_lo = size - pad;
                if (l.pad_lo != tail_seen) return fail("end bytes do not start at the tail", seed, step);
                for (uint64_t b = l.pad_lo; b < size; b++) {
                    if (owner[b] != -1) return fail("end bytes already held", seed, step);
                    owner[b] = l.id;
                }
                wrapped++;
            }
            tail_seen = off + n;
            live.push_back(l);
            placed++;
        }
        if (live.empty()) tail_seen = 0;
        uint64_t held = 0;
        for (const Live &l : live) held += l.span.len;
        if (held != ring.used()) return fail("count differs from the bytes held", seed, step);
        if (held > budget) return fail("over budget", seed, step);
    }
    std::printf("seed %d size %llu budget %llu: %ld placed, %ld wrapped\n", seed,
                (unsigned long long)size, (unsigned long long)budget, placed, wrapped);
    if (placed < steps / 20 || wrapped == 0) return fail("too little exercised", seed, steps);
    return 0;
}

int main() {
    int bad = 0;
    for (int seed = 1; seed <= 6; seed++) {
        bad |= run(seed, 1000, 1000, 40000, 1000);  // requests up to the whole ring
        bad |= run(seed + 100, 4096, 4096, 40000, 300);
        bad |= run(seed + 200, 777, 777, 40000, 50);  // many small requests
        bad |= run(seed + 300, 1000, 700, 40000, 700);  // a budget below the ring size
    }
    if (bad) return 1;
    std::printf("ok\n");
    return 0;
}
