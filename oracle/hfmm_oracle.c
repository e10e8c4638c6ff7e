/*
 * hfmm_oracle.c -- FP64 CPU oracle of the truncated Cartesian FMM used for the
 * short-range gravity of the hybrid PM-FMM method (Q. Wang, "A Hybrid Fast
 * Multipole Method for Cosmological N-body Simulations", arXiv:2006.14952).
 *
 * TEST INFRASTRUCTURE ONLY. This library exists to check the GPU library. Only
 * the test-suite, the smoke check and the CPU-baseline leg of the benchmark load
 * it. It shares no code, header, table or helper with the GPU path.
 *
 * Everything is double precision and written to be read against the paper:
 *   prefactors f_(p) = (r^-1 d/dr)^p [erfc(r/2r_s)/r]    Sec. 2.2 (closed form, recurrence)
 *   derivative tensor D_n = grad^n psi                    Sec. 2.1 (M2L equation), Sec. 2.2
 *   P2M, M2M, M2L, L2L, L2P                               Sec. 2.1, Eqs. (1), (2), (3), (5), (6)
 *   octree with a leaf-size limit                         Sec. 2.1 (particle packs)
 *   dual traversal with the three-item MAC                Sec. 2.3
 *   P2P with the truncated force law g(r)                 Sec. 2.2
 *   brute-force hard-cut minimum-image sum                (plain definition of the result)
 *
 * Readings of the paper that this file takes (each is listed in the design notes):
 *   - erfc argument is r/(2 r_s) everywhere (Sec. 2.2 potential and force law).
 *   - The recurrence printed in Sec. 2.2 has an index shift and a missing sign;
 *     the form used here is
 *         -r^2 f_(p) = (2p-1) f_(p-1) + (-1)^(p-1) exp(-r^2/4r_s^2) / (2^(p-1) sqrt(pi) r_s^(2p-1)),
 *     which reproduces the explicit f_(2), f_(3), f_(4) and the general closed form.
 *   - D_n of the truncated kernel is not traceless; the full Cartesian tensor is
 *     built from the prefactors (Hermite-type product formula for a radial function).
 *   - Expansion centres are geometric cube centres (Sec. 2.1 allows geometric or mass centre).
 *   - MAC item 3 "transition region": default STRICT reading (open while the pair's
 *     maximum distance exceeds r_cut and its minimum distance does not); mac_mode 1
 *     takes the literal S_c > r_cut > S_m test.
 *   - theta = L / S_c, accepted at equality.
 * Departure from the paper (not a reading): Sec. 2.3 defines L = L_B, the side of the
 * source cell; by default L here is the larger side of the two cells, because with L_B
 * alone a large leaf sink meets tiny adjacent sources whose local expansions do not
 * converge in p.  mac_mode bit 1 restores the paper's L_B (with bit 0 as well, the MAC
 * exactly as printed).
 *   - mac_mode bit 2: the conventional MAC the cost comparison of Sec. 3 measures against:
 *     item 2 alone decides (no neglect beyond r_cut, no forced opening across it).
 *   - Periodicity: 27 root images; r_cut < box/2 makes the image of any pair unique.
 *   - A pair contributes iff 0 < r^2 < r_cut^2 (hard cut, no softening).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PMAX 12
#define ORC_MAXLEVEL 21
#define ORC_NCOEF_MAX ((ORC_PMAX + 1) * (ORC_PMAX + 2) * (ORC_PMAX + 3) / 6)

/* ------------------------------------------------------------------------- */
/* Multi-indices n = (nx, ny, nz), ordered by total degree, then nx descending,
 * then ny descending.  idx(n) = d(d+1)(d+2)/6 + t(t+1)/2 + nz with d = |n|, t = ny + nz. */

int orc_ncoef(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }

static int mi_index(int nx, int ny, int nz)
{
    int d = nx + ny + nz, t = ny + nz;
    return d * (d + 1) * (d + 2) / 6 + t * (t + 1) / 2 + nz;
}

static int g_mi[ORC_NCOEF_MAX][3];
static double g_fact[2 * ORC_PMAX + 2];
static int g_tables_ready = 0;

static void init_tables(void)
{
    if (g_tables_ready) return;
    for (int d = 0; d <= ORC_PMAX; ++d)
        for (int nx = d; nx >= 0; --nx)
            for (int ny = d - nx; ny >= 0; --ny) {
                int nz = d - nx - ny, k = mi_index(nx, ny, nz);
                g_mi[k][0] = nx; g_mi[k][1] = ny; g_mi[k][2] = nz;
            }
    g_fact[0] = 1.0;
    for (int i = 1; i < 2 * ORC_PMAX + 2; ++i) g_fact[i] = g_fact[i - 1] * i;
    g_tables_ready = 1;
}

void orc_multi_indices(int p, int *out /* ncoef(p) x 3 */)
{
    init_tables();
    for (int k = 0; k < orc_ncoef(p); ++k)
        for (int a = 0; a < 3; ++a) out[3 * k + a] = g_mi[k][a];
}

static double mfact(int k) { return g_fact[g_mi[k][0]] * g_fact[g_mi[k][1]] * g_fact[g_mi[k][2]]; }

static double ipow(double x, int e)
{
    double r = 1.0;
    for (int i = 0; i < e; ++i) r *= x;
    return r;
}

/* x^n for all |n| <= p */
static void monomials(int p, const double x[3], double *out)
{
    for (int k = 0; k < orc_ncoef(p); ++k)
        out[k] = ipow(x[0], g_mi[k][0]) * ipow(x[1], g_mi[k][1]) * ipow(x[2], g_mi[k][2]);
}

/* ------------------------------------------------------------------------- */
/* Prefactors (Sec. 2.2).  f_(0) = erfc(r/2r_s)/r is the truncated potential;
 * f_(1) r is the truncated force law g(r). */

static double dfact_odd(int k) /* k!! for odd k >= -1 */
{
    double r = 1.0;
    for (int i = k; i > 1; i -= 2) r *= i;
    return r;
}

/* General closed form of Sec. 2.2, with x = r / r_s:
 *   (-1)^p r_s^(2p+1) f_(p)(x) = (2p-1)!!/x^(2p+1) erfc(x/2)
 *                              + sum_{q=1..p} 2^(q-p) (2p-1)!!/(2p-2q+1)!! exp(-x^2/4)/(sqrt(pi) x^(2q)) */
void orc_prefactors_closed(int p, double r, double rs, double *f)
{
    double x = r / rs, e = exp(-0.25 * x * x), ec = erfc(0.5 * x);
    for (int k = 0; k <= p; ++k) {
        double s = dfact_odd(2 * k - 1) / ipow(x, 2 * k + 1) * ec;
        for (int q = 1; q <= k; ++q)
            s += ldexp(1.0, q - k) * dfact_odd(2 * k - 1) / dfact_odd(2 * k - 2 * q + 1) * e
                 / (sqrt(M_PI) * ipow(x, 2 * q));
        f[k] = ((k & 1) ? -1.0 : 1.0) * s / ipow(rs, 2 * k + 1);
    }
}

/* Successive prefactors by the recurrence of Sec. 2.2 (corrected reading, see header). */
void orc_prefactors_recur(int p, double r, double rs, double *f)
{
    double e = exp(-r * r / (4.0 * rs * rs));
    f[0] = erfc(r / (2.0 * rs)) / r;
    for (int k = 1; k <= p; ++k) {
        double src = ((k - 1) & 1 ? -1.0 : 1.0) * e / (ldexp(1.0, k - 1) * sqrt(M_PI) * ipow(rs, 2 * k - 1));
        f[k] = -((2 * k - 1) * f[k - 1] + src) / (r * r);
    }
}

/* Polynomial split (the alternative truncation function of Sec. 5): with x = r / r_cut,
 *   phi_s(r) = g(x) / r,  g(x) = 1 - 15/8 x + 5/4 x^3 - 3/8 x^5  (x < 1),  0 beyond.
 * Reading: the paper names no polynomial; this one is the lowest-degree g whose
 * complement (1 - g)/r holds only even powers of r (a smooth long range) and that
 * vanishes with its first two derivatives at r_cut.  Then
 *   phi_s = 1/r + sum_m c_m r^(2m) / r_cut^(2m+1),  c = (-15/8, 5/4, -3/8),
 * and the same operator gives the prefactors in closed form:
 *   f_(p) = (-1)^p (2p-1)!!/r^(2p+1) + sum_{m >= p} c_m 2^p m!/(m-p)! r^(2m-2p) / r_cut^(2m+1)
 * (valid for r < r_cut, where every expansion of the method is used). */
static const double kPolyC[3] = {-15.0 / 8.0, 5.0 / 4.0, -3.0 / 8.0};

void orc_prefactors_poly(int p, double r, double rc, double *f)
{
    for (int k = 0; k <= p; ++k) {
        double s = ((k & 1) ? -1.0 : 1.0) * dfact_odd(2 * k - 1) / ipow(r, 2 * k + 1);
        for (int m = k; m < 3; ++m) {
            double fall = 1.0; /* m! / (m-k)! */
            for (int i = 0; i < k; ++i) fall *= (double)(m - i);
            s += kPolyC[m] * ldexp(fall, k) * ipow(r, 2 * m - 2 * k) / ipow(rc, 2 * m + 1);
        }
        f[k] = s;
    }
}

/* Force factor of the polynomial split: f_(1) = -1/r^3 + 5/(2 r_c^3) - 3 r^2/(2 r_c^5). */
double orc_f1_poly(double r, double rc)
{
    return -1.0 / (r * r * r) + 2.5 / (rc * rc * rc) - 1.5 * r * r / (rc * rc * rc * rc * rc);
}

/* Newtonian prefactor, Sec. 2.1 Eq. (4): (-1)^n (2n-1)!!/r^(2n+1). */
void orc_prefactors_newton(int p, double r, double *f)
{
    for (int k = 0; k <= p; ++k) f[k] = ((k & 1) ? -1.0 : 1.0) * dfact_odd(2 * k - 1) / ipow(r, 2 * k + 1);
}

/* ------------------------------------------------------------------------- */
/* Derivative tensor D_n(R) = d^n/dR^n psi(|R|) for |n| <= p.  For a radial function
 * psi(r) = F(r^2/2) one has F^(k) = f_(k), and the n-th derivative is
 *   D_n = sum_{k <= n/2} f_(|n|-|k|) prod_i n_i! / (2^k_i k_i! (n_i-2k_i)!) R_i^(n_i-2k_i).
 * rs <= 0 selects the Newtonian kernel 1/r (Eq. (4)). */
void orc_dtensor_split(int p, const double R[3], double rs, double rc, int split, double *D)
{
    init_tables();
    double r = sqrt(R[0] * R[0] + R[1] * R[1] + R[2] * R[2]);
    double f[ORC_PMAX + 1];
    if (split == 1) orc_prefactors_poly(p, r, rc, f);
    else if (rs > 0) orc_prefactors_recur(p, r, rs, f);
    else orc_prefactors_newton(p, r, f);
    for (int k = 0; k < orc_ncoef(p); ++k) {
        const int *n = g_mi[k];
        double s = 0.0;
        for (int kx = 0; 2 * kx <= n[0]; ++kx)
            for (int ky = 0; 2 * ky <= n[1]; ++ky)
                for (int kz = 0; 2 * kz <= n[2]; ++kz) {
                    int kk[3] = {kx, ky, kz};
                    double c = 1.0;
                    for (int i = 0; i < 3; ++i)
                        c *= g_fact[n[i]] / (ldexp(1.0, kk[i]) * g_fact[kk[i]] * g_fact[n[i] - 2 * kk[i]])
                             * ipow(R[i], n[i] - 2 * kk[i]);
                    s += f[n[0] + n[1] + n[2] - kx - ky - kz] * c;
                }
        D[k] = s;
    }
}

/* ------------------------------------------------------------------------- */
/* Expansion operators of Sec. 2.1. All of them ADD into their output. */

/* Eq. (1): M_m(z) += sum_a mu_a (-1)^|m| / m! (x_a - z)^m */
void orc_p2m(int p, long n, const double *x, const double *mu, const double z[3], double *M)
{
    init_tables();
    double mono[ORC_NCOEF_MAX];
    for (long a = 0; a < n; ++a) {
        double d[3] = {x[3 * a] - z[0], x[3 * a + 1] - z[1], x[3 * a + 2] - z[2]};
        monomials(p, d, mono);
        for (int k = 0; k < orc_ncoef(p); ++k) {
            int deg = g_mi[k][0] + g_mi[k][1] + g_mi[k][2];
            M[k] += mu[a] * ((deg & 1) ? -1.0 : 1.0) / mfact(k) * mono[k];
        }
    }
}

/* Eq. (2): M_m(z + x) += sum_{n <= m} x^n / n! M_{m-n}(z)   (x = new centre - old centre) */
void orc_m2m(int p, const double *Mold, const double x[3], double *Mnew)
{
    init_tables();
    for (int k = 0; k < orc_ncoef(p); ++k) {
        const int *m = g_mi[k];
        double s = 0.0;
        for (int nx = 0; nx <= m[0]; ++nx)
            for (int ny = 0; ny <= m[1]; ++ny)
                for (int nz = 0; nz <= m[2]; ++nz) {
                    int kn = mi_index(nx, ny, nz);
                    s += ipow(x[0], nx) * ipow(x[1], ny) * ipow(x[2], nz) / mfact(kn)
                         * Mold[mi_index(m[0] - nx, m[1] - ny, m[2] - nz)];
                }
        Mnew[k] += s;
    }
}

void orc_dtensor(int p, const double R[3], double rs, double *D) { orc_dtensor_split(p, R, rs, 0.0, 0, D); }

/* Eq. (3): L_n(z_sink) += sum_{|m| <= p-|n|} M_m(z_src) D_{n+m}(z_sink - z_src) */
void orc_m2l_split(int p, const double *M, const double R[3], double rs, double rc, int split, double *L)
{
    init_tables();
    double D[ORC_NCOEF_MAX];
    orc_dtensor_split(p, R, rs, rc, split, D);
    for (int k = 0; k < orc_ncoef(p); ++k) {
        const int *n = g_mi[k];
        int dn = n[0] + n[1] + n[2];
        double s = 0.0;
        for (int j = 0; j < orc_ncoef(p - dn); ++j) {
            const int *m = g_mi[j];
            s += M[j] * D[mi_index(n[0] + m[0], n[1] + m[1], n[2] + m[2])];
        }
        L[k] += s;
    }
}

void orc_m2l(int p, const double *M, const double R[3], double rs, double *L)
{
    orc_m2l_split(p, M, R, rs, 0.0, 0, L);
}

/* Eq. (5): L_n(z + x) += sum_{|m| <= p-|n|} x^m / m! L_{m+n}(z)   (x = new centre - old centre) */
void orc_l2l(int p, const double *Lold, const double x[3], double *Lnew)
{
    init_tables();
    double mono[ORC_NCOEF_MAX];
    monomials(p, x, mono);
    for (int k = 0; k < orc_ncoef(p); ++k) {
        const int *n = g_mi[k];
        int dn = n[0] + n[1] + n[2];
        double s = 0.0;
        for (int j = 0; j < orc_ncoef(p - dn); ++j) {
            const int *m = g_mi[j];
            s += mono[j] / mfact(j) * Lold[mi_index(n[0] + m[0], n[1] + m[1], n[2] + m[2])];
        }
        Lnew[k] += s;
    }
}

/* Eq. (6) and its gradient, at y = x_b - z: pot = sum_{|n|<=p} L_n y^n/n!,
 * grad_k = sum_{|n|<=p-1} L_{n+e_k} y^n/n!. */
void orc_l2p(int p, const double *L, const double y[3], double *pot, double *grad)
{
    init_tables();
    double mono[ORC_NCOEF_MAX];
    monomials(p, y, mono);
    double s = 0.0;
    for (int k = 0; k < orc_ncoef(p); ++k) s += L[k] * mono[k] / mfact(k);
    if (pot) *pot = s;
    if (grad) {
        grad[0] = grad[1] = grad[2] = 0.0;
        if (p >= 1)
            for (int k = 0; k < orc_ncoef(p - 1); ++k) {
                const int *n = g_mi[k];
                double w = mono[k] / mfact(k);
                grad[0] += L[mi_index(n[0] + 1, n[1], n[2])] * w;
                grad[1] += L[mi_index(n[0], n[1] + 1, n[2])] * w;
                grad[2] += L[mi_index(n[0], n[1], n[2] + 1)] * w;
            }
    }
}

/* Truncated force factor f_(1)(r) (Sec. 2.2 force law divided by r):
 * g(r) = f_(1)(r) r,  f_(1) = -[erfc(r/2r_s) + r/(r_s sqrt(pi)) exp(-r^2/4r_s^2)] / r^3 */
double orc_f1(double r, double rs)
{
    double u = r / (2.0 * rs);
    return -(erfc(u) + r / (rs * sqrt(M_PI)) * exp(-u * u)) / (r * r * r);
}

/* ------------------------------------------------------------------------- */
/* Parameters and solver state */

typedef struct {
    double box, rs, rcut, theta, G;
    int p, ncrit, mac_mode; /* bit 0: literal item 3 (S_c); bit 1: source-only size in item 2;
                               bit 2: conventional MAC (item 2 alone) */
    int split;              /* 0: Gaussian (erfc) split of Sec. 2.2; 1: polynomial split */
} orc_params;

/* pair force factor f_(1)(r) of the split in use */
static double f1_of(const orc_params *P, double r)
{
    if (P->split == 1) return r < P->rcut ? orc_f1_poly(r, P->rcut) : 0.0; /* compact support */
    return orc_f1(r, P->rs);
}

typedef struct {
    int level, ix, iy, iz;   /* cube [i h, (i+1) h) per axis, h = box / 2^level */
    long beg, end;           /* range in the cell-ordered particle array */
    int child, nchild;       /* children are contiguous: child .. child+nchild-1 */
    int parent;
    int active;              /* contains at least one requested target */
} ocell;

typedef struct { int a, b, s; } opair; /* sink cell, source cell, image index 0..26 */

typedef struct {
    opair *v; long n, cap;
} oplist;

static void plist_push(oplist *l, int a, int b, int s)
{
    if (l->n == l->cap) {
        l->cap = l->cap ? 2 * l->cap : 1024;
        l->v = (opair *)realloc(l->v, (size_t)l->cap * sizeof(opair));
    }
    l->v[l->n].a = a; l->v[l->n].b = b; l->v[l->n].s = s; l->n++;
}

typedef struct {
    orc_params P;
    long n;
    double *x;         /* wrapped positions, cell order, n x 3 */
    double *m;         /* masses, cell order */
    long *orig;        /* cell order -> input index */
    int *coord;        /* integer coordinates at the finest level, cell order, n x 3 */
    ocell *cell; int ncell, cellcap;
    double *M, *L;     /* ncell x ncoef */
    oplist m2l, p2p;
    long stats[16];
    double seconds;
    double phase[5];   /* seconds: tree, traversal, upward, M2L, downward + P2P */
} orc_state;

/* stats slots */
enum { ST_NCELL, ST_NLEAF, ST_MAXLEVEL, ST_NM2L, ST_NP2P, ST_P2P_PAIRS, ST_P2P_INCUT,
       ST_NPRUNE, ST_NVISIT, ST_NSPLIT_SINK, ST_NSPLIT_SRC, ST_NFORCEOPEN };

static int new_cell(orc_state *S)
{
    if (S->ncell == S->cellcap) {
        S->cellcap = S->cellcap ? 2 * S->cellcap : 1024;
        S->cell = (ocell *)realloc(S->cell, (size_t)S->cellcap * sizeof(ocell));
    }
    memset(&S->cell[S->ncell], 0, sizeof(ocell));
    return S->ncell++;
}

static double cell_h(const orc_state *S, int c) { return ldexp(S->P.box, -S->cell[c].level); }

static void cell_centre(const orc_state *S, int c, double z[3])
{
    double h = cell_h(S, c);
    z[0] = (S->cell[c].ix + 0.5) * h;
    z[1] = (S->cell[c].iy + 0.5) * h;
    z[2] = (S->cell[c].iz + 0.5) * h;
}

static int is_leaf(const orc_state *S, int c) { return S->cell[c].nchild == 0; }

/* Octree with a leaf-size limit (Sec. 2.1 "particle packs"; the octree replaces the
 * paper's ORB tree).  A cell is split into its eight octants while it holds more than
 * ncrit particles and is above the finest level; empty octants are dropped; children
 * are ordered by octant o = 4 bx + 2 by + bz.  Cells are created breadth-first, level by
 * level: the cells of one level own disjoint particle ranges, so their counting sorts
 * run in parallel; their children are then appended in cell order. */
static int octant_of(const int *coord, int shift)
{
    return (((coord[0] >> shift) & 1) << 2) | (((coord[1] >> shift) & 1) << 1) | ((coord[2] >> shift) & 1);
}

static void build_tree(orc_state *S)
{
    long n = S->n;
    const double scale = ldexp(1.0, ORC_MAXLEVEL);
    const int imax = (1 << ORC_MAXLEVEL) - 1;
    #pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            int c = (int)floor(S->x[3 * i + a] / S->P.box * scale);
            if (c < 0) c = 0;
            if (c > imax) c = imax;
            S->coord[3 * i + a] = c;
        }
    int root = new_cell(S);
    S->cell[root].beg = 0; S->cell[root].end = n; S->cell[root].parent = -1;
    long *tmp = (long *)malloc((size_t)(n > 0 ? n : 1) * sizeof(long));
    double *tx = (double *)malloc((size_t)(n > 0 ? n : 1) * 4 * sizeof(double));
    int *tc = (int *)malloc((size_t)(n > 0 ? n : 1) * 3 * sizeof(int));
    int lbeg = 0;
    while (lbeg < S->ncell) {                   /* one level: cells lbeg .. lend-1 */
        const int lend = S->ncell;
        long (*bucket)[9] = (long (*)[9])calloc((size_t)(lend - lbeg), sizeof(long[9]));
        #pragma omp parallel for schedule(dynamic, 1)
        for (int c = lbeg; c < lend; ++c) {
            ocell cc = S->cell[c];
            long cnt = cc.end - cc.beg;
            long *bk = bucket[c - lbeg];
            if (cnt <= S->P.ncrit || cc.level >= ORC_MAXLEVEL) continue;
            int shift = ORC_MAXLEVEL - 1 - cc.level;
            for (long i = cc.beg; i < cc.end; ++i) bk[octant_of(&S->coord[3 * i], shift) + 1]++;
            for (int o = 0; o < 8; ++o) bk[o + 1] += bk[o];
            long pos[8];
            for (int o = 0; o < 8; ++o) pos[o] = cc.beg + bk[o];
            for (long i = cc.beg; i < cc.end; ++i) {  /* stable counting sort by octant */
                long d = pos[octant_of(&S->coord[3 * i], shift)]++;
                tmp[d] = S->orig[i];
                for (int a = 0; a < 3; ++a) { tx[4 * d + a] = S->x[3 * i + a]; tc[3 * d + a] = S->coord[3 * i + a]; }
                tx[4 * d + 3] = S->m[i];
            }
            for (long i = cc.beg; i < cc.end; ++i) {
                S->orig[i] = tmp[i];
                for (int a = 0; a < 3; ++a) { S->x[3 * i + a] = tx[4 * i + a]; S->coord[3 * i + a] = tc[3 * i + a]; }
                S->m[i] = tx[4 * i + 3];
            }
        }
        for (int c = lbeg; c < lend; ++c) {     /* children in cell order, octant order */
            const long *bk = bucket[c - lbeg];
            if (bk[8] == 0) continue;           /* not split */
            ocell cc = S->cell[c];
            int first = -1, nch = 0;
            for (int o = 0; o < 8; ++o) {
                if (bk[o + 1] == bk[o]) continue;
                int k = new_cell(S);
                ocell *ch = &S->cell[k];
                ch->level = cc.level + 1;
                ch->ix = 2 * cc.ix + ((o >> 2) & 1);
                ch->iy = 2 * cc.iy + ((o >> 1) & 1);
                ch->iz = 2 * cc.iz + (o & 1);
                ch->beg = cc.beg + bk[o];
                ch->end = cc.beg + bk[o + 1];
                ch->parent = c;
                if (first < 0) first = k;
                nch++;
            }
            S->cell[c].child = first;
            S->cell[c].nchild = nch;
        }
        free(bucket);
        lbeg = lend;
    }
    free(tmp); free(tx); free(tc);
}

/* ------------------------------------------------------------------------- */
/* Dual tree traversal with the modified MAC of Sec. 2.3.
 *
 * For a sink A and a source B shifted by image s (B occupies its cube + s*box):
 *   R   = c_A - (c_B + s box)                  centre separation, S_c = |R|
 *   S_m = |max(|R_i| - (h_A+h_B)/2, 0)|        minimum distance of the two cubes
 *   S_M = |  |R_i| + (h_A+h_B)/2  |            maximum distance of the two cubes
 * item 1: S_m > r_cut                    -> neglect the pair
 * item 3: strict  S_M > r_cut            -> must open (transition region straddles r_cut)
 *         literal S_c > r_cut            -> must open
 * item 2: L <= theta S_c                 -> M2L, with L = max(h_A, h_B) by default and
 *         L = h_B (source side only) with mac_mode bit 1
 * otherwise open the larger cell (sink on ties); two leaves -> P2P.
 * mac_mode bit 2 (conventional MAC): items 1 and 3 are skipped, item 2 alone decides.
 *
 * Why L = max(h_A, h_B) by default: the traversal keeps the two sides within a factor
 * two of each other except when the sink is a leaf, where it keeps opening the source.
 * A large leaf sink can then meet a tiny adjacent source with h_B <= theta S_c while
 * the source lies closer to some sink particles than to the sink centre, and the local
 * expansion diverges there (errors of order one that do not fall with p).  Taking the
 * larger side restores h_A, h_B <= theta S_c and convergence in p.
 *
 * Distances are evaluated exactly: every centre is an odd multiple of h/2, so in units
 * of u = box / 2^(l+1), l the finer of the two levels, all of R, the cube half-widths
 * and hence S_c^2, S_m^2, S_M^2 are integers.  Comparisons use the thresholds
 * (r_cut/u)^2 and theta^2 computed once per level in double precision. */

typedef struct {
    double cut2[ORC_MAXLEVEL + 1]; /* (r_cut / u_l)^2, u_l = box/2^(l+1) */
    double theta2;
} orc_mac;

static void mac_setup(const orc_params *P, orc_mac *mac)
{
    for (int l = 0; l <= ORC_MAXLEVEL; ++l) {
        double u = ldexp(P->box, -(l + 1));
        mac->cut2[l] = (P->rcut * P->rcut) / (u * u);
    }
    mac->theta2 = P->theta * P->theta;
}

static void image_of(int s, int sh[3]) { sh[0] = s / 9 - 1; sh[1] = (s / 3) % 3 - 1; sh[2] = s % 3 - 1; }

/* returns 0 prune, 1 M2L, 2 open */
static int mac_decide(const orc_state *S, const orc_mac *mac, int A, int B, int s, long *nforce)
{
    const ocell *a = &S->cell[A], *b = &S->cell[B];
    int l = a->level > b->level ? a->level : b->level;
    int64_t wa = (int64_t)1 << (l - a->level), wb = (int64_t)1 << (l - b->level);
    int sh[3]; image_of(s, sh);
    int ia[3] = {a->ix, a->iy, a->iz}, ib[3] = {b->ix, b->iy, b->iz};
    int64_t sc2 = 0, sm2 = 0, sM2 = 0;
    int64_t half = wa + wb; /* (h_A + h_B)/2 in units of u */
    for (int i = 0; i < 3; ++i) {
        int64_t R = (2 * (int64_t)ia[i] + 1) * wa - (2 * (int64_t)ib[i] + 1) * wb
                    - (int64_t)sh[i] * ((int64_t)1 << (l + 1));
        int64_t aR = R < 0 ? -R : R;
        int64_t g = aR - half; if (g < 0) g = 0;
        int64_t G = aR + half;
        sc2 += R * R; sm2 += g * g; sM2 += G * G;
    }
    double cut2 = mac->cut2[l];
    if (!(S->P.mac_mode & 4)) {                                     /* truncated MAC */
        if ((double)sm2 > cut2) return 0;                           /* item 1 */
        int straddle = (S->P.mac_mode & 1) ? ((double)sc2 > cut2) : ((double)sM2 > cut2);
        if (straddle) { if (nforce) (*nforce)++; return 2; }        /* item 3 */
    }
    /* item 2: size L = larger side of the pair (default) or the source side alone
     * (mac_mode bit 1, the literal Sec. 2.3 wording) */
    int64_t w = (S->P.mac_mode & 2) ? wb : (wa > wb ? wa : wb);
    double hl2 = (double)(4 * w * w);                               /* (L / u)^2 */
    if (hl2 <= mac->theta2 * (double)sc2) return 1;
    return 2;
}

static void traverse(orc_state *S, const orc_mac *mac, int A, int B, int s)
{
    if (!S->cell[A].active) return;
    S->stats[ST_NVISIT]++;
    int d = mac_decide(S, mac, A, B, s, &S->stats[ST_NFORCEOPEN]);
    if (d == 0) { S->stats[ST_NPRUNE]++; return; }
    if (d == 1) { plist_push(&S->m2l, A, B, s); return; }
    int la = is_leaf(S, A), lb = is_leaf(S, B);
    if (la && lb) { plist_push(&S->p2p, A, B, s); return; }
    if (!la && (S->cell[A].level <= S->cell[B].level || lb)) {
        S->stats[ST_NSPLIT_SINK]++;
        for (int c = 0; c < S->cell[A].nchild; ++c) traverse(S, mac, S->cell[A].child + c, B, s);
    } else {
        S->stats[ST_NSPLIT_SRC]++;
        for (int c = 0; c < S->cell[B].nchild; ++c) traverse(S, mac, A, S->cell[B].child + c, s);
    }
}

static int cmp_pair(const void *x, const void *y)
{
    const opair *a = (const opair *)x, *b = (const opair *)y;
    if (a->a != b->a) return a->a < b->a ? -1 : 1;
    if (a->b != b->b) return a->b < b->b ? -1 : 1;
    return (a->s > b->s) - (a->s < b->s);
}

/* ------------------------------------------------------------------------- */
/* P2P (Sec. 2.1 last paragraph, force law of Sec. 2.2): for sink leaf A and source
 * leaf B shifted by image s, a_i += m_j f_(1)(r) d with d = x_i - x_j - s box, for
 * 0 < r^2 < r_cut^2. */
static void p2p_leaf_pair(const orc_state *S, int A, int B, int s, double *acc, long *npairs, long *nin)
{
    int sh[3]; image_of(s, sh);
    double L = S->P.box, rc2 = S->P.rcut * S->P.rcut;
    const ocell *a = &S->cell[A], *b = &S->cell[B];
    for (long i = a->beg; i < a->end; ++i) {
        double ax = 0, ay = 0, az = 0;
        for (long j = b->beg; j < b->end; ++j) {
            double dx = (S->x[3 * i] - S->x[3 * j]) - sh[0] * L;
            double dy = (S->x[3 * i + 1] - S->x[3 * j + 1]) - sh[1] * L;
            double dz = (S->x[3 * i + 2] - S->x[3 * j + 2]) - sh[2] * L;
            double r2 = dx * dx + dy * dy + dz * dz;
            (*npairs)++;
            if (!(r2 > 0.0 && r2 < rc2)) continue;
            (*nin)++;
            double w = S->m[j] * f1_of(&S->P, sqrt(r2));
            ax += w * dx; ay += w * dy; az += w * dz;
        }
        acc[3 * i] += ax; acc[3 * i + 1] += ay; acc[3 * i + 2] += az;
    }
}

static double now_seconds(void)
{
    struct timespec t;
    clock_gettime(CLOCK_MONOTONIC, &t);
    return t.tv_sec + 1e-9 * t.tv_nsec;
}

/* Run the whole truncated FMM.  targets == NULL means every particle; otherwise only
 * the requested particles get forces, only sink cells containing one of them are
 * traversed, and multipoles are formed only for the cells those sinks read (the M2L
 * sources and their subtrees): the per-sink work is exactly that of the full run.  The
 * traversal, which reads cell geometry only, runs before the upward pass so that these
 * cells are known.  acc (n x 3, input order) is overwritten for targets and left
 * untouched elsewhere.  Returns a state handle holding the tree, lists, statistics and
 * per-phase times (free with orc_free). */
void *orc_fmm(const orc_params *P, long n, const double *pos, const double *mass, long ntarget,
              const long *targets, double *acc, int nthreads)
{
    init_tables();
    if (P->p < 0 || P->p > ORC_PMAX || P->ncrit < 1 || !(P->theta > 0) || !(P->rcut < 0.5 * P->box) ||
        P->split < 0 || P->split > 1)
        return NULL;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    double t0 = now_seconds();
    orc_state *S = (orc_state *)calloc(1, sizeof(orc_state));
    S->P = *P; S->n = n;
    size_t nn = (size_t)(n > 0 ? n : 1);
    S->x = (double *)malloc(nn * 3 * sizeof(double));
    S->m = (double *)malloc(nn * sizeof(double));
    S->orig = (long *)malloc(nn * sizeof(long));
    S->coord = (int *)malloc(nn * 3 * sizeof(int));
    #pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) {
        for (int a = 0; a < 3; ++a) {          /* wrap into [0, box) */
            double v = pos[3 * i + a] - P->box * floor(pos[3 * i + a] / P->box);
            if (v >= P->box) v = 0.0;
            S->x[3 * i + a] = v;
        }
        S->m[i] = mass[i];
        S->orig[i] = i;
    }
    build_tree(S);
    const int np = orc_ncoef(P->p);

    /* mark active cells */
    if (!targets) {
        for (int c = 0; c < S->ncell; ++c) S->cell[c].active = 1;
    } else {
        long *where = (long *)malloc(nn * sizeof(long));
        for (long i = 0; i < n; ++i) where[S->orig[i]] = i;
        char *want = (char *)calloc(nn, 1);
        for (long t = 0; t < ntarget; ++t) want[where[targets[t]]] = 1;
        for (int c = S->ncell - 1; c >= 0; --c) {
            if (is_leaf(S, c)) {
                for (long i = S->cell[c].beg; i < S->cell[c].end; ++i)
                    if (want[i]) { S->cell[c].active = 1; break; }
            }
            if (S->cell[c].active && S->cell[c].parent >= 0) S->cell[S->cell[c].parent].active = 1;
        }
        free(where); free(want);
    }

    S->phase[0] = now_seconds() - t0;        /* tree */

    /* dual traversal from the 27 root images (it reads cell geometry only, so the lists
     * can be made before the multipoles) */
    double t1 = now_seconds();
    orc_mac mac; mac_setup(P, &mac);
    if (n > 0)
        for (int s = 0; s < 27; ++s) traverse(S, &mac, 0, 0, s);
    if (S->m2l.n) qsort(S->m2l.v, (size_t)S->m2l.n, sizeof(opair), cmp_pair);  /* an empty list has no array */
    if (S->p2p.n) qsort(S->p2p.v, (size_t)S->p2p.n, sizeof(opair), cmp_pair);
    S->phase[1] = now_seconds() - t1;

    /* upward pass: P2M at leaves, M2M to parents (Sec. 2.1), for the cells whose
     * multipoles are read: the M2L sources and everything below them (all cells in a
     * full run).  Parents have smaller ids than children (breadth-first creation). */
    t1 = now_seconds();
    S->M = (double *)calloc((size_t)S->ncell * np, sizeof(double));
    S->L = (double *)calloc((size_t)S->ncell * np, sizeof(double));
    char *need = (char *)calloc((size_t)(S->ncell > 0 ? S->ncell : 1), 1);
    if (!targets) {
        memset(need, 1, (size_t)S->ncell);
    } else {
        for (long e = 0; e < S->m2l.n; ++e) need[S->m2l.v[e].b] = 1;
        for (int c = 1; c < S->ncell; ++c)
            if (need[S->cell[c].parent]) need[c] = 1;
    }
    #pragma omp parallel for schedule(dynamic, 16)
    for (int c = 0; c < S->ncell; ++c) {
        if (!need[c] || !is_leaf(S, c)) continue;
        double z[3]; cell_centre(S, c, z);
        orc_p2m(P->p, S->cell[c].end - S->cell[c].beg, S->x + 3 * S->cell[c].beg, S->m + S->cell[c].beg, z,
                S->M + (size_t)c * np);
    }
    for (int lend = S->ncell; lend > 0;) {     /* levels bottom-up; a level is a contiguous id range */
        int lbeg = lend - 1;
        while (lbeg > 0 && S->cell[lbeg - 1].level == S->cell[lend - 1].level) --lbeg;
        #pragma omp parallel for schedule(dynamic, 16)
        for (int c = lbeg; c < lend; ++c) {
            if (!need[c] || is_leaf(S, c)) continue;
            double zp[3]; cell_centre(S, c, zp);
            for (int k = 0; k < S->cell[c].nchild; ++k) {
                int ch = S->cell[c].child + k;
                double zc[3]; cell_centre(S, ch, zc);
                double x[3] = {zp[0] - zc[0], zp[1] - zc[1], zp[2] - zc[2]};
                orc_m2m(P->p, S->M + (size_t)ch * np, x, S->M + (size_t)c * np);
            }
        }
        lend = lbeg;
    }
    free(need);
    S->phase[2] = now_seconds() - t1;
    t1 = now_seconds();

    /* M2L grouped by sink (lists sorted by sink) */
    {
        long nl = S->m2l.n;
        long *start = (long *)malloc((size_t)(S->ncell + 1) * sizeof(long));
        for (int c = 0; c <= S->ncell; ++c) start[c] = 0;
        for (long e = 0; e < nl; ++e) start[S->m2l.v[e].a + 1]++;
        for (int c = 0; c < S->ncell; ++c) start[c + 1] += start[c];
        #pragma omp parallel for schedule(dynamic, 16)
        for (int c = 0; c < S->ncell; ++c) {
            double za[3]; cell_centre(S, c, za);
            for (long e = start[c]; e < start[c + 1]; ++e) {
                int B = S->m2l.v[e].b, sh[3]; image_of(S->m2l.v[e].s, sh);
                double zb[3]; cell_centre(S, B, zb);
                double R[3] = {za[0] - (zb[0] + sh[0] * P->box), za[1] - (zb[1] + sh[1] * P->box),
                               za[2] - (zb[2] + sh[2] * P->box)};
                orc_m2l_split(P->p, S->M + (size_t)B * np, R, P->rs, P->rcut, P->split, S->L + (size_t)c * np);
            }
        }
        free(start);
    }

    S->phase[3] = now_seconds() - t1;
    t1 = now_seconds();

    /* downward pass: L2L parent -> child (parents first) */
    for (int c = 1; c < S->ncell; ++c) {
        if (!S->cell[c].active) continue;
        int pa = S->cell[c].parent;
        double zp[3], zc[3]; cell_centre(S, pa, zp); cell_centre(S, c, zc);
        double x[3] = {zc[0] - zp[0], zc[1] - zp[1], zc[2] - zp[2]};
        orc_l2l(P->p, S->L + (size_t)pa * np, x, S->L + (size_t)c * np);
    }

    /* L2P and P2P per sink leaf */
    double *accs = (double *)calloc(nn * 3, sizeof(double));
    {
        long np2p = S->p2p.n;
        long *start = (long *)malloc((size_t)(S->ncell + 1) * sizeof(long));
        for (int c = 0; c <= S->ncell; ++c) start[c] = 0;
        for (long e = 0; e < np2p; ++e) start[S->p2p.v[e].a + 1]++;
        for (int c = 0; c < S->ncell; ++c) start[c + 1] += start[c];
        long pairs = 0, incut = 0;
        #pragma omp parallel for schedule(dynamic, 4) reduction(+ : pairs, incut)
        for (int c = 0; c < S->ncell; ++c) {
            if (!is_leaf(S, c) || !S->cell[c].active) continue;
            double z[3]; cell_centre(S, c, z);
            for (long i = S->cell[c].beg; i < S->cell[c].end; ++i) {
                double y[3] = {S->x[3 * i] - z[0], S->x[3 * i + 1] - z[1], S->x[3 * i + 2] - z[2]}, g[3];
                orc_l2p(P->p, S->L + (size_t)c * np, y, NULL, g);
                accs[3 * i] += g[0]; accs[3 * i + 1] += g[1]; accs[3 * i + 2] += g[2];
            }
            long pl = 0, il = 0;
            for (long e = start[c]; e < start[c + 1]; ++e)
                p2p_leaf_pair(S, c, S->p2p.v[e].b, S->p2p.v[e].s, accs, &pl, &il);
            pairs += pl; incut += il;
        }
        S->stats[ST_P2P_PAIRS] = pairs; S->stats[ST_P2P_INCUT] = incut;
        free(start);
    }
    if (!targets) {
        for (long i = 0; i < n; ++i)
            for (int a = 0; a < 3; ++a) acc[3 * S->orig[i] + a] = P->G * accs[3 * i + a];
    } else {
        long *where = (long *)malloc(nn * sizeof(long));
        for (long i = 0; i < n; ++i) where[S->orig[i]] = i;
        for (long t = 0; t < ntarget; ++t) {
            long i = where[targets[t]];
            for (int a = 0; a < 3; ++a) acc[3 * targets[t] + a] = P->G * accs[3 * i + a];
        }
        free(where);
    }
    free(accs);
    S->phase[4] = now_seconds() - t1;
    S->seconds = now_seconds() - t0;

    int nleaf = 0, maxl = 0;
    for (int c = 0; c < S->ncell; ++c) {
        if (is_leaf(S, c)) nleaf++;
        if (S->cell[c].level > maxl) maxl = S->cell[c].level;
    }
    S->stats[ST_NCELL] = S->ncell; S->stats[ST_NLEAF] = nleaf; S->stats[ST_MAXLEVEL] = maxl;
    S->stats[ST_NM2L] = S->m2l.n; S->stats[ST_NP2P] = S->p2p.n;
    return S;
}

void orc_free(void *h)
{
    orc_state *S = (orc_state *)h;
    if (!S) return;
    free(S->x); free(S->m); free(S->orig); free(S->coord); free(S->cell);
    free(S->M); free(S->L); free(S->m2l.v); free(S->p2p.v); free(S);
}

void orc_stats(const void *h, long *out16) { memcpy(out16, ((const orc_state *)h)->stats, 16 * sizeof(long)); }
double orc_seconds(const void *h) { return ((const orc_state *)h)->seconds; }
void orc_phase_seconds(const void *h, double *out5) { memcpy(out5, ((const orc_state *)h)->phase, 5 * sizeof(double)); }
int orc_ncell(const void *h) { return ((const orc_state *)h)->ncell; }
long orc_nlist(const void *h, int kind) { const orc_state *S = (const orc_state *)h; return kind ? S->p2p.n : S->m2l.n; }

/* Cell key: (1 << 3 level) | morton(ix, iy, iz) with x the most significant bit of
 * every octal digit.  Unique over all levels. */
static uint64_t cell_key(const ocell *c)
{
    uint64_t k = 1;
    for (int b = c->level - 1; b >= 0; --b)
        k = (k << 3) | ((uint64_t)((c->ix >> b) & 1) << 2) | ((uint64_t)((c->iy >> b) & 1) << 1)
            | (uint64_t)((c->iz >> b) & 1);
    return k;
}

/* Interaction list as (sink key, source key, image) triples; kind 0 = M2L, 1 = P2P. */
void orc_copy_list(const void *h, int kind, uint64_t *out /* nlist x 3 */)
{
    const orc_state *S = (const orc_state *)h;
    const oplist *l = kind ? &S->p2p : &S->m2l;
    for (long e = 0; e < l->n; ++e) {
        out[3 * e] = cell_key(&S->cell[l->v[e].a]);
        out[3 * e + 1] = cell_key(&S->cell[l->v[e].b]);
        out[3 * e + 2] = (uint64_t)l->v[e].s;
    }
}

/* Cells as (key, level, beg, end, nchild) rows, and the cell-order permutation. */
void orc_copy_cells(const void *h, int64_t *out /* ncell x 5 */, long *orig /* n */)
{
    const orc_state *S = (const orc_state *)h;
    for (int c = 0; c < S->ncell; ++c) {
        out[5 * c] = (int64_t)cell_key(&S->cell[c]);
        out[5 * c + 1] = S->cell[c].level;
        out[5 * c + 2] = S->cell[c].beg;
        out[5 * c + 3] = S->cell[c].end;
        out[5 * c + 4] = S->cell[c].nchild;
    }
    if (orig) memcpy(orig, S->orig, (size_t)S->n * sizeof(long));
}

/* ------------------------------------------------------------------------- */
/* Brute-force minimum-image sum: the plain definition that the truncated FMM
 * approximates,  a_i = G sum_{j, 0 < |d_ij|^2 < rc^2} m_j f_(1)(|d_ij|) d_ij,
 * d_ij = x_i - x_j - box * round((x_i - x_j)/box).  A cell list with cells no
 * smaller than rc keeps it O(N * neighbours); rc < box/2. */
int orc_bruteforce(const orc_params *P, double rc, long n, const double *pos, const double *mass, long ntarget,
                   const long *targets, double *acc_out /* ntarget x 3 */, int nthreads)
{
    if (!(rc < 0.5 * P->box) || !(rc > 0) || P->split < 0 || P->split > 1) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    double L = P->box;
    int nc = (int)floor(L / rc);
    if (nc < 1) nc = 1;
    if (nc > 256) nc = 256;
    long ncells = (long)nc * nc * nc;
    double *x = (double *)malloc((size_t)(n > 0 ? n : 1) * 3 * sizeof(double));
    int *cid = (int *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int));
    long *head = (long *)malloc((size_t)(ncells + 1) * sizeof(long));
    long *sorted = (long *)malloc((size_t)(n > 0 ? n : 1) * sizeof(long));
    for (long c = 0; c <= ncells; ++c) head[c] = 0;
    for (long i = 0; i < n; ++i) {
        int ci[3];
        for (int a = 0; a < 3; ++a) {
            double v = pos[3 * i + a] - L * floor(pos[3 * i + a] / L);
            if (v >= L) v = 0.0;
            x[3 * i + a] = v;
            ci[a] = (int)floor(v / L * nc);
            if (ci[a] >= nc) ci[a] = nc - 1;
        }
        cid[i] = (ci[0] * nc + ci[1]) * nc + ci[2];
        head[cid[i] + 1]++;
    }
    for (long c = 0; c < ncells; ++c) head[c + 1] += head[c];
    {
        long *fill = (long *)malloc((size_t)ncells * sizeof(long));
        for (long c = 0; c < ncells; ++c) fill[c] = head[c];
        for (long i = 0; i < n; ++i) sorted[fill[cid[i]]++] = i;
        free(fill);
    }
    double rc2 = rc * rc;
    #pragma omp parallel for schedule(dynamic, 64)
    for (long t = 0; t < ntarget; ++t) {
        long i = targets ? targets[t] : t;
        int ci = cid[i] / (nc * nc), cj = (cid[i] / nc) % nc, ck = cid[i] % nc;
        int span = nc >= 3 ? 1 : 0;
        double ax = 0, ay = 0, az = 0;
        for (int di = -span; di <= span; ++di)
            for (int dj = -span; dj <= span; ++dj)
                for (int dk = -span; dk <= span; ++dk) {
                    long c;
                    if (span) {
                        int a = (ci + di + nc) % nc, b = (cj + dj + nc) % nc, e = (ck + dk + nc) % nc;
                        c = ((long)a * nc + b) * nc + e;
                    }
                    long lo = span ? head[c] : 0, hi = span ? head[c + 1] : n;
                    for (long q = lo; q < hi; ++q) {
                        long j = span ? sorted[q] : q;
                        double d[3];
                        for (int a = 0; a < 3; ++a) {
                            double v = x[3 * i + a] - x[3 * j + a];
                            d[a] = v - L * round(v / L);
                        }
                        double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                        if (!(r2 > 0.0 && r2 < rc2)) continue;
                        double w = mass[j] * f1_of(P, sqrt(r2));
                        ax += w * d[0]; ay += w * d[1]; az += w * d[2];
                    }
                }
        acc_out[3 * t] = P->G * ax; acc_out[3 * t + 1] = P->G * ay; acc_out[3 * t + 2] = P->G * az;
    }
    free(x); free(cid); free(head); free(sorted);
    return 0;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
