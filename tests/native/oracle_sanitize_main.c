/*
 * Driver for a sanitizer build of the CPU oracle (test infrastructure): runs
 * oracle_trellis, oracle_branch_metrics, oracle_pb_geometry and oracle_decode
 * over edge-case streams (n = 1, D >= n, L >= T, L = 0, unterminated ends,
 * hard input, several threads, block sub-ranges, all optional outputs) with
 * symbols from a fixed linear congruential generator, so that AddressSanitizer
 * and UndefinedBehaviorSanitizer see every code path.  Exit status 0 when all
 * calls return as expected; the sanitizers abort on any memory or UB error.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_trellis(int K, int R, const uint32_t *gen, int32_t *next, int32_t *label);
int oracle_branch_metrics(int R, int input_kind, const uint8_t *syms, int64_t n_stages, int64_t *bm);
int64_t oracle_num_blocks(int64_t n, int64_t D);
void oracle_pb_geometry(int64_t n, int64_t T, int64_t D, int64_t L, int64_t b, int64_t *out);
int oracle_decode(int K, int R, const uint32_t *gen, int D, int L, int terminated, int input_kind,
                  const uint8_t *syms, int64_t n, int64_t pb_first, int64_t pb_count, uint8_t *bits,
                  int64_t *final_pm, uint8_t *dec_out, int nthreads);

static uint32_t lcg = 12345u;
static uint8_t next_byte(void)
{
    lcg = lcg * 1664525u + 1013904223u;
    return (uint8_t)(lcg >> 24);
}

struct code { int K, R; uint32_t gen[4]; };

int main(void)
{
    const struct code codes[] = {
        {3, 2, {07, 05}}, {7, 2, {0171, 0133}}, {7, 3, {0133, 0171, 0165}}, {9, 3, {0557, 0663, 0711}},
        {5, 4, {025, 027, 033, 037}}, {6, 2, {046, 073}},
    };
    const int64_t ns[] = {1, 2, 7, 64, 333, 1000};
    const int Ds[] = {1, 3, 8, 64, 100, 4096};
    const int Ls[] = {0, 1, 5, 42, 2000};
    int failures = 0, calls = 0;
    for (size_t ci = 0; ci < sizeof(codes) / sizeof(codes[0]); ++ci) {
        const struct code *c = &codes[ci];
        const int N = 1 << (c->K - 1);
        int32_t *next = malloc(sizeof(int32_t) * 2 * N), *label = malloc(sizeof(int32_t) * 2 * N);
        if (oracle_trellis(c->K, c->R, c->gen, next, label) != 0) ++failures;
        for (size_t ni = 0; ni < sizeof(ns) / sizeof(ns[0]); ++ni)
        for (size_t di = 0; di < sizeof(Ds) / sizeof(Ds[0]); ++di)
        for (size_t li = 0; li < sizeof(Ls) / sizeof(Ls[0]); ++li)
        for (int term = 0; term < 2; ++term) {
            const int64_t n = ns[ni];
            const int D = Ds[di], L = Ls[li];
            /* keep each case small: blocks x forward stages x states */
            {
                const int64_t t = n + (term ? c->K - 1 : 0);
                const int64_t span = (int64_t)D + 2 * L < t ? (int64_t)D + 2 * L : t;
                if (oracle_num_blocks(n, D) * span * N > 4000000) continue;
            }
            const int kind = (int)((ni + di + li + (size_t)term) & 1);
            const int64_t T = n + (term ? c->K - 1 : 0);
            const int64_t nsym = T * c->R;
            uint8_t *syms = malloc((size_t)nsym);
            for (int64_t i = 0; i < nsym; ++i) syms[i] = kind ? (next_byte() & 1) : next_byte();
            int64_t *bm = malloc(sizeof(int64_t) * (size_t)T << c->R);
            if (oracle_branch_metrics(c->R, kind, syms, T, bm) != 0) ++failures;
            const int64_t nb = oracle_num_blocks(n, D);
            int64_t geo[4];
            for (int64_t b = 0; b < nb; b += (nb > 3 ? nb - 1 : 1)) oracle_pb_geometry(n, T, D, L, b, geo);
            /* whole stream with every output, then a middle sub-range on threads */
            uint8_t *bits = malloc((size_t)n);
            int64_t *pm = malloc(sizeof(int64_t) * (size_t)nb * N);
            uint8_t *dec = malloc((size_t)nb * (size_t)(D + L) * (size_t)N);
            if (oracle_decode(c->K, c->R, c->gen, D, L, term, kind, syms, n, 0, nb, bits, pm, dec, 1) != 0)
                ++failures;
            const int64_t first = nb / 2, cnt = nb - first;
            if (oracle_decode(c->K, c->R, c->gen, D, L, term, kind, syms, n, first, cnt, bits, NULL, NULL, 3) != 0)
                ++failures;
            /* invalid ranges must be refused */
            if (oracle_decode(c->K, c->R, c->gen, D, L, term, kind, syms, n, 0, nb + 1, bits, NULL, NULL, 1) != -1)
                ++failures;
            calls += 3;
            free(dec);
            free(pm);
            free(bits);
            free(bm);
            free(syms);
        }
        free(next);
        free(label);
    }
    printf("oracle sanitizer run: %d calls, %d failures\n", calls, failures);
    return failures ? 1 : 0;
}
