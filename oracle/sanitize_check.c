/*
 * sanitize_check.c -- TEST INFRASTRUCTURE ONLY: a driver that runs the oracle's entry
 * points over small inputs so that the oracle can be built and run under
 * AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_oracle_sanitize.py).
 *
 * It covers the tree build (leaf limits 1, 8, 64, coincident particles, a particle on
 * the box edge), every MAC mode, both truncation functions, orders 0..8, the targeted
 * run, the interaction-list and cell exports, and the brute-force sum; it checks that a
 * tiny opening angle reproduces the brute-force sum (every pair inside r_cut is then
 * summed directly).  Exit status 0 means every run finished and every check held.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    double box, rs, rcut, theta, G;
    int p, ncrit, mac_mode, split;
} orc_params;

void *orc_fmm(const orc_params *P, long n, const double *pos, const double *mass, long ntarget,
              const long *targets, double *acc, int nthreads);
void orc_free(void *h);
void orc_stats(const void *h, long *out16);
int orc_ncell(const void *h);
long orc_nlist(const void *h, int kind);
void orc_copy_list(const void *h, int kind, uint64_t *out);
void orc_copy_cells(const void *h, int64_t *out, long *orig);
int orc_bruteforce(const orc_params *P, double rc, long n, const double *pos, const double *mass, long ntarget,
                   const long *targets, double *out, int nthreads);

static uint64_t g_state = 88172645463325252ull;

static double uniform01(void) /* xorshift64*, 53-bit mantissa */
{
    g_state ^= g_state >> 12;
    g_state ^= g_state << 25;
    g_state ^= g_state >> 27;
    return (double)((g_state * 2685821657736338717ull) >> 11) * (1.0 / 9007199254740992.0);
}

/* n particles: half uniform, half in three small blobs; a few duplicates and a particle
 * exactly on the upper box edge (wrapped to 0) */
static void make_input(long n, double *pos, double *m)
{
    const double c[3][3] = {{0.2, 0.3, 0.7}, {0.8, 0.8, 0.1}, {0.5, 0.05, 0.5}};
    for (long i = 0; i < n; ++i) {
        for (int a = 0; a < 3; ++a) {
            double v = uniform01();
            if (i % 2) v = c[i % 3][a] + 0.02 * (uniform01() - 0.5);
            pos[3 * i + a] = v;
        }
        m[i] = 1.0 / n;
    }
    for (int a = 0; a < 3; ++a) {
        pos[3 * 5 + a] = pos[3 * 4 + a];
        pos[3 * 7 + a] = pos[3 * 4 + a];
    }
    pos[0] = 1.0;
}

static int run_one(const orc_params *P, long n, const double *pos, const double *m, int targeted)
{
    double *acc = (double *)calloc((size_t)n * 3, sizeof(double));
    long tg[64], nt = 0;
    if (targeted)
        for (long i = 0; i < n && nt < 64; i += 37) tg[nt++] = i;
    void *h = orc_fmm(P, n, pos, m, targeted ? nt : n, targeted ? tg : NULL, acc, 2);
    if (!h) {
        fprintf(stderr, "orc_fmm rejected p=%d ncrit=%d mode=%d split=%d\n", P->p, P->ncrit, P->mac_mode, P->split);
        free(acc);
        return 1;
    }
    long st[16];
    orc_stats(h, st);
    int nc = orc_ncell(h);
    int64_t *cells = (int64_t *)malloc((size_t)(nc > 0 ? nc : 1) * 5 * sizeof(int64_t));
    long *orig = (long *)malloc((size_t)n * sizeof(long));
    orc_copy_cells(h, cells, orig);
    for (int k = 0; k < 2; ++k) {
        long nl = orc_nlist(h, k);
        uint64_t *l = (uint64_t *)malloc((size_t)(nl > 0 ? nl : 1) * 3 * sizeof(uint64_t));
        orc_copy_list(h, k, l);
        free(l);
    }
    int bad = 0;
    for (long i = 0; i < 3 * n; ++i)
        if (!isfinite(acc[i])) bad = 1;
    orc_free(h);
    free(cells);
    free(orig);
    free(acc);
    return bad;
}

int main(void)
{
    const long n = 3000;
    double *pos = (double *)malloc(n * 3 * sizeof(double)), *m = (double *)malloc(n * sizeof(double));
    make_input(n, pos, m);
    int fails = 0, runs = 0;
    const int ncrits[3] = {1, 8, 64};
    for (int split = 0; split <= 1; ++split)
        for (int mode = 0; mode < 8; ++mode)
            for (int q = 0; q < 3; ++q) {
                orc_params P = {1.0, 0.02, 0.09, 0.5, 1.0, (mode + q) % 9, ncrits[q], mode, split};
                fails += run_one(&P, n, pos, m, q == 1);
                ++runs;
            }
    for (int p = 0; p <= 8; ++p) {
        orc_params P = {1.0, 0.02, 0.09, 0.45, 1.0, p, 16, 0, 0};
        fails += run_one(&P, n, pos, m, p & 1);
        ++runs;
    }
    /* tiny opening angle: no pair is accepted, the FMM is the brute-force sum */
    orc_params P = {1.0, 0.02, 0.09, 1e-3, 1.0, 4, 8, 0, 0};
    double *a = (double *)calloc(n * 3, sizeof(double)), *b = (double *)calloc(n * 3, sizeof(double));
    void *h = orc_fmm(&P, n, pos, m, n, NULL, a, 2);
    if (!h || orc_bruteforce(&P, P.rcut, n, pos, m, n, NULL, b, 2) != 0) {
        fails++;
    } else {
        double worst = 0.0, scale = 0.0;
        for (long i = 0; i < 3 * n; ++i) {
            double d = fabs(a[i] - b[i]);
            worst = d > worst ? d : worst;
            scale = fabs(b[i]) > scale ? fabs(b[i]) : scale;
        }
        if (!(worst <= 1e-12 * scale)) {
            fprintf(stderr, "theta -> 0 differs from brute force: %g of %g\n", worst, scale);
            fails++;
        }
    }
    if (h) orc_free(h);
    free(a);
    free(b);
    free(pos);
    free(m);
    printf("%d runs, %d failures\n", runs + 1, fails);
    return fails ? 1 : 0;
}
