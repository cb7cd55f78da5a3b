/* The oracle under AddressSanitizer / UndefinedBehaviorSanitizer: its three
 * matchers on seeded random batches (several alphabets, short and long
 * patterns, threads and chunking), the match counts of the three compared,
 * and a small exhaustive run.  Exits non-zero on a disagreement. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void *orc_match(int algo, const uint8_t *text, const uint64_t *toff, uint32_t n_texts,
                const uint8_t *pdata, const uint64_t *poff, uint32_t k,
                uint64_t lo, uint64_t hi, int threads, uint64_t chunk, double *timing);
uint64_t orc_count(const void *h);
void orc_free(void *h);
int64_t orc_exhaustive(int sigma, int max_plen, int max_npat, int max_tlen, int threads,
                       uint64_t *n_cases);

static uint64_t rnd(uint64_t *s) {
    *s ^= *s << 13; *s ^= *s >> 7; *s ^= *s << 17;
    return *s;
}

int main(void) {
    uint64_t s = 88172645463325252ull;
    for (int trial = 0; trial < 30; trial++) {
        const int sigma = (int[]){2, 4, 16, 256}[trial % 4];
        const uint32_t k = 1 + (uint32_t)(rnd(&s) % 200);
        uint64_t *poff = malloc((k + 1) * sizeof(uint64_t));
        uint8_t *pdata = malloc((size_t)k * 64);
        poff[0] = 0;
        for (uint32_t j = 0; j < k; j++) {
            uint64_t len = 1 + rnd(&s) % (trial % 3 == 0 ? 4 : 40);
            for (uint64_t q = 0; q < len; q++) pdata[poff[j] + q] = (uint8_t)(rnd(&s) % sigma);
            poff[j + 1] = poff[j] + len;
        }
        const uint32_t n_texts = 1 + (uint32_t)(rnd(&s) % 5);
        uint64_t *toff = malloc((n_texts + 1) * sizeof(uint64_t));
        toff[0] = 0;
        for (uint32_t i = 0; i < n_texts; i++) toff[i + 1] = toff[i] + rnd(&s) % 20000;
        uint8_t *text = malloc(toff[n_texts] + 1);
        for (uint64_t i = 0; i < toff[n_texts]; i++) text[i] = (uint8_t)(rnd(&s) % sigma);
        uint64_t n[3];
        for (int algo = 1; algo <= 3; algo++) {
            double tm[2];
            void *h = orc_match(algo, text, toff, n_texts, pdata, poff, k, 0, UINT64_MAX,
                                1 + trial % 4, 1 + rnd(&s) % 5000, tm);
            if (!h) { fprintf(stderr, "match failed (trial %d algo %d)\n", trial, algo); return 1; }
            n[algo - 1] = orc_count(h);
            orc_free(h);
        }
        if (n[0] != n[1] || n[0] != n[2]) {
            fprintf(stderr, "counts differ (trial %d): %llu %llu %llu\n", trial,
                    (unsigned long long)n[0], (unsigned long long)n[1], (unsigned long long)n[2]);
            return 1;
        }
        free(poff); free(pdata); free(toff); free(text);
    }
    uint64_t cases = 0;
    if (orc_exhaustive(2, 2, 2, 6, 2, &cases) != 0 || cases == 0) {
        fprintf(stderr, "exhaustive run disagreed\n");
        return 1;
    }
    puts("oracle sanitizer run: ok");
    return 0;
}
