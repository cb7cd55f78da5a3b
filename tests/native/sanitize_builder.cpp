// Host trie builder under AddressSanitizer / UndefinedBehaviorSanitizer:
// seeded pattern sets of several alphabets and length mixes (length-1
// patterns, duplicates, long runs) built into CRS tries and packed into every
// device-image variant (level index widths, prefix-filter folds, bitmapped
// top nodes, truncation depths, the merged DAG).  Exits non-zero on a failed
// invariant; the sanitizers abort on a memory or UB error.
#include <cstdint>
#include <cstdio>
#include <random>
#include <string>
#include <vector>

#include "../../paper_1702_03657_amd/csrc/trie.hpp"

using namespace pfac;

static int fail(const char *what, int seed) {
    std::fprintf(stderr, "invariant failed: %s (seed %d)\n", what, seed);
    return 1;
}

int main() {
    const char *alphabets[] = {"\x01\x02", "ACGT", "abcdefghijklmnop", nullptr};
    for (int seed = 0; seed < 24; seed++) {
        std::mt19937 rng(1000 + seed);
        const char *al = alphabets[seed % 4];
        const int asz = al ? (int)std::string(al).size() : 256;
        const uint32_t k = 1 + rng() % 300;
        const uint32_t lo = (uint32_t)(seed % 3 == 0 ? 1 : 1 + rng() % 8), hi = lo + rng() % 40;
        std::vector<uint8_t> data;
        std::vector<uint64_t> off(1, 0);
        for (uint32_t j = 0; j < k; j++) {
            uint32_t len = lo + rng() % (hi - lo + 1);
            if (j > 0 && rng() % 10 == 0) {  // a duplicate or a prefix of an earlier pattern
                const uint32_t i = rng() % j;
                const uint64_t a = off[i], b = off[i + 1];
                const uint64_t n = 1 + rng() % (b - a);
                data.insert(data.end(), data.begin() + a, data.begin() + a + n);
            } else {
                for (uint32_t q = 0; q < len; q++)
                    data.push_back(al ? (uint8_t)al[rng() % asz] : (uint8_t)(rng() & 0xff));
            }
            off.push_back(data.size());
        }
        CrsTrie T;
        std::string err;
        if (!build_crs(data.data(), off.data(), k, T, err)) return fail("build", seed);
        if (T.row_ptr.back() != T.n_edges() || T.term_ptr.back() != k) return fail("csr sizes", seed);
        uint64_t dn = 0, de = 0;
        dag_size(T, dn, de);
        if (dn > T.n_nodes() || de > T.n_edges() || dn == 0) return fail("dag size", seed);
        for (uint32_t bits : {1u, 8u, 12u, 16u, 18u})
            for (uint32_t fold : {0u, 8u, 16u})
                for (uint32_t trunc : {0u, 1u, 3u, 8u})
                    for (uint32_t dag : {0u, 1u}) {
                        if (dag && trunc) continue;
                        DeviceImageHost I;
                        pack_image(T, bits, fold, trunc, dag, I);
                        if (I.node.size() % 4 || I.tail.size() % 4) return fail("record sizes", seed);
                        if (I.top.size() != (size_t)I.top_nodes * I.top_rw) return fail("top size", seed);
                        if (dag && I.dnode.size() / 4 != dn) return fail("dag nodes", seed);
                        if (I.K > T.min_len || (trunc && I.trunc_depth && I.K > trunc))
                            return fail("index depth", seed);
                    }
    }
    std::puts("builder sanitizer run: ok");
    return 0;
}
