// P2P: direct truncated interaction between a sink leaf and the leaves of its P2P list
// (Sec. 2.1 last paragraph; force law of Sec. 2.2):  a_i += m_j f_(1)(r) d, d = x_i - x_j - s box,
// counted iff 0 < r^2 < r_cut^2.
//
// One 64-lane wave per sink leaf.  Sources of up to 64 list entries are laid out as one
// stream of slots (a wave prefix sum over the entry sizes); slots are staged 64 at a
// time in LDS.  A sink leaf of n_A <= 64 particles occupies n2 = pow2ceil(n_A) lanes;
// the wave holds 64 / n2 copies of the sink, each copy walking a different subset of
// the staged sources, and the copies are summed with cross-lane shuffles at the end.
//
// FP64 form: absolute FP64 positions, erfc/exp from the device math library.
// FP32 form: FP32 coordinates relative to each particle's leaf centre, the exact
// centre offset c_B + s box - c_A added when staging, and
//   f_(1)(r) = -1/r^3 + S(t)/(8 r_s^3),  t = 2 r^2/r_cut^2 - 1,
// with S(t) = (4/sqrt(pi)) int_0^1 q^2 exp(-v q^2) dq (v = r^2/4r_s^2) replaced by a
// degree-10 polynomial fitted on the host; sums per staged chunk are added to a
// Kahan-compensated per-particle accumulator.
#include <math.h>

#include <vector>

#include "state.h"

namespace hfmm {

__device__ __forceinline__ int wave_incl_scan(int v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    return v;
}

// largest e in [0, ne) with pref[e] <= slot (pref non-decreasing, pref[0] = 0)
__device__ __forceinline__ int find_entry(const int *pref, int ne, int slot)
{
    int lo = 0, hi = ne - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (pref[mid] <= slot) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int pow2ceil(int v)
{
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

struct P2PArgs {
    const Cell *cells;
    const int *leaves;
    int nleaf;
    const int *head;  // P2P list kind: head/cnt offset by ncell already
    const int *cnt;
    const uint32_t *items;
    const int *next;
    const double *xs, *ys, *zs, *ms;
    const float4 *rel;
    double box;
    double *nearf;  // 3 x n SoA
    int n;
};

// ---------------------------------------------------------------------------
// FP64

__global__ __launch_bounds__(64) void k_p2p_f64(P2PArgs a, P2PConst k)
{
    __shared__ double4 src[64];
    __shared__ int ebeg[64], epref[64];
    __shared__ double esh[64][3];
    const int lane = threadIdx.x;
    const int A = a.leaves[blockIdx.x];
    const Cell ca = a.cells[A];
    const int nA = ca.end - ca.beg;
    const int nlist = a.cnt[A];
    int chunk = a.head[A];
    const double rc2 = k.rc2d, inv2rs = 0.5 / k.rs, c1 = 1.0 / (k.rs * 1.7724538509055160273);

    for (int ib = 0; ib < nA; ib += 64) {
        const int ns = min(64, nA - ib);
        const int n2 = pow2ceil(ns), G = 64 / n2;
        const int si = lane & (n2 - 1), g = lane / n2;
        const bool valid = si < ns;
        const int i = ca.beg + ib + (valid ? si : 0);
        const double xi = a.xs[i], yi = a.ys[i], zi = a.zs[i];
        double ax = 0, ay = 0, az = 0;
        for (int eb = 0; eb < nlist; eb += 64) {
            const int ne = min(64, nlist - eb);
            int cntj = 0;
            if (lane < ne) {
                uint32_t it = a.items[(size_t)chunk * kChunk + lane];
                int s = (int)(it & 31);
                Cell cb = a.cells[it >> 5];
                cntj = cb.end - cb.beg;
                ebeg[lane] = cb.beg;
                esh[lane][0] = (double)(s / 9 - 1) * a.box;
                esh[lane][1] = (double)((s / 3) % 3 - 1) * a.box;
                esh[lane][2] = (double)(s % 3 - 1) * a.box;
            }
            const int incl = wave_incl_scan(cntj);
            if (lane < ne) epref[lane] = incl - cntj;
            const int total = __shfl(incl, 63, 64);
            __syncthreads();
            for (int cb0 = 0; cb0 < total; cb0 += 64) {
                const int slot = cb0 + lane;
                double4 v = make_double4(1e30, 1e30, 1e30, 0.0);
                if (slot < total) {
                    int e = find_entry(epref, ne, slot);
                    int j = ebeg[e] + slot - epref[e];
                    v = make_double4(a.xs[j] + esh[e][0], a.ys[j] + esh[e][1], a.zs[j] + esh[e][2], a.ms[j]);
                }
                src[lane] = v;
                __syncthreads();
                for (int q = g; q < 64; q += G) {
                    const double4 s = src[q];
                    double dx = xi - s.x, dy = yi - s.y, dz = zi - s.z;
                    double r2 = dx * dx + dy * dy + dz * dz;
                    bool in = r2 > 0.0 && r2 < rc2;
                    double rr2 = in ? r2 : 1.0;
                    double r = sqrt(rr2);
                    double u = r * inv2rs;
                    double h = erfc(u) + r * c1 * exp(-u * u);
                    double w = in ? -s.w * h / (rr2 * r) : 0.0;
                    ax += w * dx;
                    ay += w * dy;
                    az += w * dz;
                }
                __syncthreads();
            }
            if (eb + 64 < nlist) chunk = a.next[chunk];
        }
        for (int o = n2; o < 64; o <<= 1) {
            ax += __shfl_xor(ax, o, 64);
            ay += __shfl_xor(ay, o, 64);
            az += __shfl_xor(az, o, 64);
        }
        if (g == 0 && valid) {
            a.nearf[i] = ax;
            a.nearf[(size_t)a.n + i] = ay;
            a.nearf[2 * (size_t)a.n + i] = az;
        }
    }
}

// ---------------------------------------------------------------------------
// FP32

__device__ __forceinline__ void kahan_add(float &s, float &c, float v)
{
    float y = v - c;
    float t = s + y;
    c = (t - s) - y;
    s = t;
}

__global__ __launch_bounds__(64) void k_p2p_f32(P2PArgs a, P2PConst k)
{
    __shared__ float4 src[64];
    __shared__ int ebeg[64], epref[64];
    __shared__ float eoff[64][3];
    const int lane = threadIdx.x;
    const int A = a.leaves[blockIdx.x];
    const Cell ca = a.cells[A];
    const int la = cell_level(ca);
    const double hA = ldexp(a.box, -la);
    const double cax = (ca.ix + 0.5) * hA, cay = (ca.iy + 0.5) * hA, caz = (ca.iz + 0.5) * hA;
    const int nA = ca.end - ca.beg;
    const int nlist = a.cnt[A];
    int chunk = a.head[A];

    for (int ib = 0; ib < nA; ib += 64) {
        const int ns = min(64, nA - ib);
        const int n2 = pow2ceil(ns), G = 64 / n2;
        const int si = lane & (n2 - 1), g = lane / n2;
        const bool valid = si < ns;
        const int i = ca.beg + ib + (valid ? si : 0);
        const float4 me = a.rel[i];
        float sx = 0, sy = 0, sz = 0, cx = 0, cy = 0, cz = 0;
        for (int eb = 0; eb < nlist; eb += 64) {
            const int ne = min(64, nlist - eb);
            int cntj = 0;
            if (lane < ne) {
                uint32_t it = a.items[(size_t)chunk * kChunk + lane];
                int s = (int)(it & 31);
                Cell cb = a.cells[it >> 5];
                double hB = ldexp(a.box, -cell_level(cb));
                cntj = cb.end - cb.beg;
                ebeg[lane] = cb.beg;
                // exact in FP64: dyadic centres and integer image shifts
                eoff[lane][0] = (float)((cb.ix + 0.5) * hB + (double)(s / 9 - 1) * a.box - cax);
                eoff[lane][1] = (float)((cb.iy + 0.5) * hB + (double)((s / 3) % 3 - 1) * a.box - cay);
                eoff[lane][2] = (float)((cb.iz + 0.5) * hB + (double)(s % 3 - 1) * a.box - caz);
            }
            const int incl = wave_incl_scan(cntj);
            if (lane < ne) epref[lane] = incl - cntj;
            const int total = __shfl(incl, 63, 64);
            __syncthreads();
            for (int cb0 = 0; cb0 < total; cb0 += 64) {
                const int slot = cb0 + lane;
                float4 v = make_float4(1e18f, 1e18f, 1e18f, 0.0f);
                if (slot < total) {
                    int e = find_entry(epref, ne, slot);
                    float4 r = a.rel[ebeg[e] + slot - epref[e]];
                    v = make_float4(r.x + eoff[e][0], r.y + eoff[e][1], r.z + eoff[e][2], r.w);
                }
                src[lane] = v;
                __syncthreads();
                float px = 0, py = 0, pz = 0;
                for (int q = g; q < 64; q += G) {
                    const float4 s = src[q];
                    float dx = me.x - s.x, dy = me.y - s.y, dz = me.z - s.z;
                    float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                    float rinv = __frsqrt_rn(r2);
                    float t = fmaf(r2, k.two_over_rc2, -1.0f);
                    float S = k.c[kP2PPoly - 1];
#pragma unroll
                    for (int c = kP2PPoly - 2; c >= 0; --c) S = fmaf(S, t, k.c[c]);
                    float rinv2 = rinv * rinv;
                    float f1 = fmaf(S, k.inv8rs3, -rinv2 * rinv);
                    float w = (r2 < k.rc2 && r2 > 0.0f) ? s.w * f1 : 0.0f;
                    px = fmaf(w, dx, px);
                    py = fmaf(w, dy, py);
                    pz = fmaf(w, dz, pz);
                }
                kahan_add(sx, cx, px);
                kahan_add(sy, cy, py);
                kahan_add(sz, cz, pz);
                __syncthreads();
            }
            if (eb + 64 < nlist) chunk = a.next[chunk];
        }
        double ax = (double)sx - (double)cx, ay = (double)sy - (double)cy, az = (double)sz - (double)cz;
        for (int o = n2; o < 64; o <<= 1) {
            ax += __shfl_xor(ax, o, 64);
            ay += __shfl_xor(ay, o, 64);
            az += __shfl_xor(az, o, 64);
        }
        if (g == 0 && valid) {
            a.nearf[i] = ax;
            a.nearf[(size_t)a.n + i] = ay;
            a.nearf[2 * (size_t)a.n + i] = az;
        }
    }
}

// ---------------------------------------------------------------------------
// host: fit of S(t) on [-1, 1] at Chebyshev points (interpolation, solved in FP64)

static double S_of_v(double v)
{
    // S(v) = (erf(u) - 2u/sqrt(pi) e^{-u^2}) / u^3, u = sqrt(v); series near 0
    if (v < 0.09) {
        double s = 0, term = 1;  // sum (-1)^k v^k / (k! (2k+3))
        for (int k = 0; k < 30; ++k) {
            s += term / (2 * k + 3);
            term *= -v / (k + 1);
        }
        return 4.0 / sqrt(M_PI) * s;
    }
    double u = sqrt(v);
    return (erf(u) - 2.0 * u / sqrt(M_PI) * exp(-v)) / (u * u * u);
}

void p2p_setup(const fmm_params *P, P2PConst &k)
{
    const int m = kP2PPoly;
    double vcut = (P->r_cut * P->r_cut) / (4.0 * P->r_s * P->r_s);
    double Amat[kP2PPoly][kP2PPoly + 1];
    for (int i = 0; i < m; ++i) {
        double t = cos(M_PI * (i + 0.5) / m);
        double v = (t + 1.0) * 0.5 * vcut;
        double pw = 1.0;
        for (int j = 0; j < m; ++j) { Amat[i][j] = pw; pw *= t; }
        Amat[i][m] = S_of_v(v);
    }
    for (int c = 0; c < m; ++c) {  // Gaussian elimination with partial pivoting
        int piv = c;
        for (int r = c + 1; r < m; ++r)
            if (fabs(Amat[r][c]) > fabs(Amat[piv][c])) piv = r;
        for (int j = 0; j <= m; ++j) { double tmp = Amat[c][j]; Amat[c][j] = Amat[piv][j]; Amat[piv][j] = tmp; }
        for (int r = 0; r < m; ++r) {
            if (r == c) continue;
            double f = Amat[r][c] / Amat[c][c];
            for (int j = c; j <= m; ++j) Amat[r][j] -= f * Amat[c][j];
        }
    }
    for (int j = 0; j < m; ++j) k.c[j] = (float)(Amat[j][m] / Amat[j][j]);
    k.inv8rs3 = (float)(1.0 / (8.0 * P->r_s * P->r_s * P->r_s));
    k.two_over_rc2 = (float)(2.0 / (P->r_cut * P->r_cut));
    k.rc2 = (float)(P->r_cut * P->r_cut);
    k.rs = P->r_s;
    k.rc2d = P->r_cut * P->r_cut;
}

int p2p(fmm_tree *t, const fmm_params *P, hipStream_t st)
{
    if (t->nleaf == 0) return 0;
    P2PConst k;
    p2p_setup(P, k);
    P2PArgs a;
    a.cells = ptr<Cell>(t->cells);
    a.leaves = ptr<int>(t->leaves);
    a.nleaf = t->nleaf;
    a.head = ptr<int>(t->lhead) + t->ncell;
    a.cnt = ptr<int>(t->lcnt) + t->ncell;
    a.items = ptr<uint32_t>(t->litems[1]);
    a.next = ptr<int>(t->lnext[1]);
    a.xs = ptr<double>(t->xs);
    a.ys = ptr<double>(t->ys);
    a.zs = ptr<double>(t->zs);
    a.ms = ptr<double>(t->ms);
    a.rel = ptr<float4>(t->rel32);
    a.box = t->box;
    a.nearf = ptr<double>(t->nearf);
    a.n = (int)t->n;
    if (P->precision) k_p2p_f32<<<t->nleaf, 64, 0, st>>>(a, k);
    else k_p2p_f64<<<t->nleaf, 64, 0, st>>>(a, k);
    return hip_check(hipGetLastError(), "p2p");
}

}  // namespace hfmm
