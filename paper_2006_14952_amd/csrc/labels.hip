// Training data for the learned acceptance / order selector: features of candidate pairs
// and the smallest expansion order whose error the method itself measures to be within
// a target.
//
// For a candidate pair (sink A, source B, image) the label kernel computes, for every
// particle i of A, the exact truncated force from B's particles (the P2P of the pair) and
// the expansion result M2L + L2P at each order p = 2..8 (FP64, multipoles of order 8
// truncated: terms with |n| + |m| <= p).  The error of order p is
//     e_p = max_i |a_i^(p) - a_i^direct| / |a_i^ref|,
// a_i^ref being the particle's total short-range force (from a full evaluation).  The
// label is the class of the smallest p with e_p <= eps (class p - 1), or 0 (open).
#include "expand_impl.h"
#include "mlp.h"

namespace hfmm {

struct LabelArgs {
    const Cell *cells;
    int ncell;
    const int *head, *cnt;  // candidate lists (kind 3)
    const uint32_t *items;
    const int *next;
    const double *xs, *ys, *zs, *ms;
    const double *M;  // FP64 scaled multipoles, stride ncoef(8)
    const double *aref;  // total short-range acceleration, SoA 3 x n in Morton order
    int n;
    double box, rs, rcut, eps;
    float *feats;
    int *labels;
    float *errs;  // 7 per candidate, may be null
    int *counter;
    int cap;
    double maxpairs;  // candidates with n_A n_B above this are skipped (cost bound)
    int stride;       // label candidates with (A + entry) % stride == 0 only
    uint64_t *pairs;  // (sink key, source key, image) per labelled candidate, may be null
};

__device__ inline uint64_t dev_cell_key(const Cell &c)
{
    uint64_t k = 1;
    int ix = cell_ix(c);
    for (int b = cell_level(c) - 1; b >= 0; --b)
        k = (k << 3) | ((uint64_t)((ix >> b) & 1) << 2) | ((uint64_t)((c.iy >> b) & 1) << 1) |
            (uint64_t)((c.iz >> b) & 1);
    return k;
}

__global__ __launch_bounds__(64) void k_labels(LabelArgs a)
{
    constexpr int P = 8, NC = ncoef(8), NC7 = ncoef(7);
    constexpr Tab<8> tb{};
    constexpr PairTab<8> pt{};
    const int lane = threadIdx.x;
    for (int A = blockIdx.x; A < a.ncell; A += gridDim.x) {
        const int nl = a.cnt[A];
        if (nl == 0) continue;
        const Cell ca = a.cells[A];
        const int la = cell_level(ca);
        const double hA = ldexp(a.box, -la);
        const double cx = (cell_ix(ca) + 0.5) * hA, cy = (ca.iy + 0.5) * hA, cz = (ca.iz + 0.5) * hA;
        const double mA0 = a.M[(size_t)A * NC];
        int chunk = a.head[A];
        for (int e0 = 0; e0 < nl; e0 += 64) {
            if (e0 > 0) chunk = a.next[chunk];
            const int e = e0 + lane;
            if (e >= nl) continue;
            if ((A + e) % a.stride != 0) continue;
            const uint32_t it = a.items[(size_t)chunk * kChunk + lane];
            const int B = (int)(it >> 5), s = (int)(it & 31);
            const Cell cb = a.cells[B];
            const int lb = cell_level(cb);
            if ((double)(ca.end - ca.beg) * (double)(cb.end - cb.beg) > a.maxpairs) continue;
            const int4 ga = reinterpret_cast<const int4 *>(a.cells)[2 * A];
            const int4 gbv = reinterpret_cast<const int4 *>(a.cells)[2 * B];
            PairGeo g = pair_geo(ga, gbv, s);
            float f[kFeat];
            pair_features(g, la, lb, a.box, a.rs, a.rcut, mA0, cell_features<double>(a.M + (size_t)B * NC), f);
            // expansion in units of h_A: Rh = R / h_A, split scale r_s / h_A, rho = h_B / h_A
            double inv2wa = 0.5 / g.wa;
            double Rx = g.R[0] * inv2wa, Ry = g.R[1] * inv2wa, Rz = g.R[2] * inv2wa;
            double fk[P + 1], D[NC], L[NC];
            prefactors<P, double>(Rx * Rx + Ry * Ry + Rz * Rz, a.rs / hA, 0, fk);
            dtensor<P, double>(Rx, Ry, Rz, fk, D);
            const double rho = ldexp(1.0, la - lb);
            const double *Mb = a.M + (size_t)B * NC;
            for (int k = 0; k < NC; ++k) L[k] = 0.0;
            // source image shift of B's particles
            const double shx = (double)(s / 9 - 1) * a.box, shy = (double)((s / 3) % 3 - 1) * a.box,
                         shz = (double)(s % 3 - 1) * a.box;
            double emax[7] = {0, 0, 0, 0, 0, 0, 0};
            // running contraction by total degree d = |n| + |m|; after degree d, L = L^(d)
            double Ld[7][NC];  // L^(p) for p = 2..8 (kept to evaluate each particle once)
            for (int d = 0; d <= P; ++d) {
                for (int q = 0; q < PairTab<8>::NT; ++q) {
                    int kn = pt.n[q], km = pt.m[q];
                    if (tb.d[kn] + tb.d[km] != d) continue;
                    double rp = 1.0;
                    for (int r = 0; r < tb.d[km]; ++r) rp *= rho;
                    L[kn] += rp * Mb[km] * D[pt.nm[q]];
                }
                if (d >= 2)
                    for (int k = 0; k < NC; ++k) Ld[d - 2][k] = L[k];
            }
            for (int i = ca.beg; i < ca.end; ++i) {
                double ax = 0, ay = 0, az = 0;
                for (int j = cb.beg; j < cb.end; ++j) {
                    double dx = a.xs[i] - (a.xs[j] + shx), dy = a.ys[i] - (a.ys[j] + shy),
                           dz = a.zs[i] - (a.zs[j] + shz);
                    double r2 = dx * dx + dy * dy + dz * dz;
                    if (!(r2 > 0.0 && r2 < a.rcut * a.rcut)) continue;
                    double r = sqrt(r2), u = r / (2.0 * a.rs);
                    double w = -a.ms[j] * (erfc(u) + r / (a.rs * 1.7724538509055160273) * exp(-u * u)) / (r2 * r);
                    ax += w * dx; ay += w * dy; az += w * dz;
                }
                double yx = (a.xs[i] - cx) / hA, yy = (a.ys[i] - cy) / hA, yz = (a.zs[i] - cz) / hA;
                double mono[NC7];
                mono[0] = 1.0;
                for (int k = 1; k < NC7; ++k) {
                    double yv = tb.ax[k] == 0 ? yx : (tb.ax[k] == 1 ? yy : yz);
                    mono[k] = mono[tb.par[k]] * yv;
                }
                for (int k = 1; k < NC7; ++k) mono[k] *= tb.invf[k];
                double ref = sqrt(a.aref[i] * a.aref[i] + a.aref[(size_t)a.n + i] * a.aref[(size_t)a.n + i] +
                                  a.aref[2 * (size_t)a.n + i] * a.aref[2 * (size_t)a.n + i]);
                ref = ref > 0 ? ref : 1e-300;
                for (int p = 2; p <= P; ++p) {
                    double gx = 0, gy = 0, gz = 0;
                    for (int k = 0; k < ncoef(p - 1); ++k) {
                        int x = tb.x[k], y = tb.y[k], z = tb.z[k];
                        gx += Ld[p - 2][midx(x + 1, y, z)] * mono[k];
                        gy += Ld[p - 2][midx(x, y + 1, z)] * mono[k];
                        gz += Ld[p - 2][midx(x, y, z + 1)] * mono[k];
                    }
                    double sc = 1.0 / (hA * hA);
                    double ex = gx * sc - ax, ey = gy * sc - ay, ez = gz * sc - az;
                    double err = sqrt(ex * ex + ey * ey + ez * ez) / ref;
                    emax[p - 2] = fmax(emax[p - 2], err);
                }
            }
            int cls = 0;
            for (int p = 2; p <= P; ++p)
                if (emax[p - 2] <= a.eps) {
                    cls = p - 1;
                    break;
                }
            int o = atomicAdd(a.counter, 1);
            if (o >= a.cap) continue;
            for (int k = 0; k < kFeat; ++k) a.feats[(size_t)o * kFeat + k] = f[k];
            a.labels[o] = cls;
            if (a.errs)
                for (int p = 0; p < 7; ++p) a.errs[(size_t)o * 7 + p] = (float)emax[p];
            if (a.pairs) {
                a.pairs[3 * (size_t)o] = dev_cell_key(ca);
                a.pairs[3 * (size_t)o + 1] = dev_cell_key(cb);
                a.pairs[3 * (size_t)o + 2] = (uint64_t)s;
            }
        }
    }
}

// caller-order (n, 3) -> Morton-order SoA
__global__ void k_to_sorted_soa(const double *__restrict__ acc, const int *__restrict__ perm, int n,
                                double *__restrict__ out)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    size_t o = 3 * (size_t)perm[i];
    out[i] = acc[o];
    out[(size_t)n + i] = acc[o + 1];
    out[2 * (size_t)n + i] = acc[o + 2];
}

int sort_soa(fmm_tree *t, const double *acc, double *out, hipStream_t st)
{
    int n = (int)t->n;
    if (n == 0) return 0;
    k_to_sorted_soa<<<(n + 255) / 256, 256, 0, st>>>(acc, ptr<int>(t->perm), n, out);
    return hip_check(hipGetLastError(), "sort soa");
}

int run_labels(fmm_tree *t, const fmm_params *P, const double *aref_sorted, double eps, int stride, float *feats,
               int *labels, float *errs, uint64_t *pairs, int cap, int *dcounter, hipStream_t st)
{
    LabelArgs a;
    a.cells = ptr<Cell>(t->cells);
    a.ncell = t->ncell;
    a.head = ptr<int>(t->lhead) + 3 * (size_t)t->ncell;
    a.cnt = ptr<int>(t->lcnt) + 3 * (size_t)t->ncell;
    a.items = ptr<uint32_t>(t->litems[3]);
    a.next = ptr<int>(t->lnext[3]);
    a.xs = ptr<double>(t->xs);
    a.ys = ptr<double>(t->ys);
    a.zs = ptr<double>(t->zs);
    a.ms = ptr<double>(t->ms);
    a.M = ptr<double>(t->Mc);
    a.aref = aref_sorted;
    a.n = (int)t->n;
    a.box = t->box;
    a.rs = P->r_s;
    a.rcut = P->r_cut;
    a.eps = eps;
    a.feats = feats;
    a.labels = labels;
    a.errs = errs;
    a.counter = dcounter;
    a.cap = cap;
    a.maxpairs = 262144.0;
    a.stride = stride > 0 ? stride : 1;
    a.pairs = pairs;
    int g = t->ncell < 16384 ? t->ncell : 16384;
    k_labels<<<g, 64, 0, st>>>(a);
    return hip_check(hipGetLastError(), "labels");
}

}  // namespace hfmm
