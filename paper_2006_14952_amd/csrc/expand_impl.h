// Expansion operators of Sec. 2.1 (Eqs. (1), (2), (3), (5), (6)) with the truncated
// kernel of Sec. 2.2, templated on the order P and the arithmetic type T.
//
// Coefficients are stored scaled by the cell side h so that FP32 keeps its range at
// every level:  Mh_m = M_m / h^|m|,  Lh_n = L_n h^(|n|+1).  In these units
//   P2M  Mh_m  = sum_a mu_a (-1)^|m|/m! ((x_a - z)/h)^m
//   M2M  Mh_m(parent) = 2^-|m| sum_{n<=m} xh^n/n! Mh_{m-n}(child),  xh = (z_p - z_c)/h_c = +-1/2
//   M2L  Lh_n(A) += sum_{|m|<=P-|n|} rho^|m| Mh_m(B) Dh_{n+m}(Rh),  rho = h_B/h_A, Rh = R/h_A,
//        Dh_j = h_A^(|j|+1) D_j(R) = derivatives in h_A units with split scale r_s/h_A
//   L2L  Lh_n(child) += 2^-(|n|+1) sum_{|m|<=P-|n|} xh^m/m! Lh_{n+m}(parent),  xh = +-1/4
//   L2P  grad Psi = h^-2 sum_{|n|<=P-1} Lh_{n+e_k} yh^n/n!,  yh = (x - z)/h
// The derivative tensor is built with the radial recurrence
//   D^(m)_n = R_a D^(m+1)_{n-e_a} + (n_a - 1) D^(m+1)_{n-2e_a},   D^(m)_0 = f_(m)(r),
// (f_(m) = (r^-1 d/dr)^m of the truncated potential), from the prefactor recurrence of
// Sec. 2.2 in its corrected form  -r^2 f_(k) = (2k-1) f_(k-1) + (-1)^(k-1) e^(-r^2/4r_s^2)/(2^(k-1) sqrt(pi) r_s^(2k-1)).
#pragma once
#include "state.h"

namespace hfmm {

// ---------------------------------------------------------------------------
// compile-time tables

template <int P> struct Tab {
    static constexpr int NC = ncoef(P);
    int x[NC], y[NC], z[NC], d[NC];
    int ax[NC], par[NC], par2[NC], na[NC];  // first non-zero axis a, index of n-e_a, of n-2e_a (-1), n_a
    double invf[NC];                        // 1 / n!
    double sgn_invf[NC];                    // (-1)^|n| / n!
    constexpr Tab() : x(), y(), z(), d(), ax(), par(), par2(), na(), invf(), sgn_invf()
    {
        for (int dd = 0; dd <= P; ++dd)
            for (int a = dd; a >= 0; --a)
                for (int b = dd - a; b >= 0; --b) {
                    int c = dd - a - b, k = midx(a, b, c);
                    x[k] = a; y[k] = b; z[k] = c; d[k] = dd;
                    double f = 1.0;
                    for (int i = 2; i <= a; ++i) f *= i;
                    for (int i = 2; i <= b; ++i) f *= i;
                    for (int i = 2; i <= c; ++i) f *= i;
                    invf[k] = 1.0 / f;
                    sgn_invf[k] = (dd & 1) ? -1.0 / f : 1.0 / f;
                    if (dd == 0) { ax[k] = 0; par[k] = -1; par2[k] = -1; na[k] = 0; continue; }
                    int e[3] = {a, b, c};
                    int q = e[0] ? 0 : (e[1] ? 1 : 2);
                    ax[k] = q; na[k] = e[q];
                    e[q] -= 1;
                    par[k] = midx(e[0], e[1], e[2]);
                    if (e[q] >= 1) { e[q] -= 1; par2[k] = midx(e[0], e[1], e[2]); }
                    else par2[k] = -1;
                }
    }
};

constexpr int binom(int n, int k)
{
    int r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

// (n, m) pairs with |n| + |m| <= P, m outer: used by M2L (L_n += M_m D_{n+m}) and L2L.
template <int P> struct PairTab {
    static constexpr int NT = binom(P + 6, 6);
    short n[NT], m[NT], nm[NT];
    int mstart[ncoef(P) + 1];  // pairs with source index m occupy mstart[m] .. mstart[m+1]-1
    constexpr PairTab() : n(), m(), nm(), mstart()
    {
        Tab<P> T{};
        int t = 0;
        for (int km = 0; km < ncoef(P); ++km)
            for (int kn = 0; kn < ncoef(P - T.d[km]); ++kn) {
                n[t] = (short)kn; m[t] = (short)km;
                nm[t] = (short)midx(T.x[kn] + T.x[km], T.y[kn] + T.y[km], T.z[kn] + T.z[km]);
                if (kn == 0) mstart[km] = t;
                ++t;
            }
        mstart[ncoef(P)] = t;
    }
};

// M2L contraction for source indices KB .. KB+MB-1: the block of the source multipole is
// loaded (scaled by rho^|m|) and consumed before the next block is loaded, so that only
// L, D and one block are live.
template <int P, class T, int KB, int MB>
__device__ __forceinline__ void m2l_contract(const T *__restrict__ Mb, const T *rp, const T *D, T *acc)
{
    constexpr Tab<P> tb{};
    constexpr PairTab<P> pt{};
    constexpr int NC = ncoef(P);
    constexpr int KE = KB + MB < NC ? KB + MB : NC;
    T Ms[MB];
#pragma unroll
    for (int k = KB; k < KE; ++k) Ms[k - KB] = Mb[k] * rp[tb.d[k]];
    asm volatile("" ::: "memory");
#pragma unroll
    for (int q = pt.mstart[KB]; q < pt.mstart[KE]; ++q) acc[pt.n[q]] += Ms[pt.m[q] - KB] * D[pt.nm[q]];
    if constexpr (KE < NC) m2l_contract<P, T, KE, MB>(Mb, rp, D, acc);
}

// (m, n) pairs with n <= m componentwise, |m| <= P: used by M2M.
template <int P> struct SubTab {
    static constexpr int NT = binom(P + 6, 6);
    short m[NT], n[NT], mn[NT];
    constexpr SubTab() : m(), n(), mn()
    {
        Tab<P> T{};
        int t = 0;
        for (int km = 0; km < ncoef(P); ++km)
            for (int a = 0; a <= T.x[km]; ++a)
                for (int b = 0; b <= T.y[km]; ++b)
                    for (int c = 0; c <= T.z[km]; ++c) {
                        m[t] = (short)km; n[t] = (short)midx(a, b, c);
                        mn[t] = (short)midx(T.x[km] - a, T.y[km] - b, T.z[km] - c);
                        ++t;
                    }
    }
};

// monomials y^n / n! for |n| <= P (scaled by w)
template <int P, class T> __device__ __forceinline__ void monomials(T yx, T yy, T yz, T w, T *mono)
{
    constexpr Tab<P> tb{};
    const T yv[3] = {yx, yy, yz};
    mono[0] = w;
#pragma unroll
    for (int k = 1; k < Tab<P>::NC; ++k) mono[k] = mono[tb.par[k]] * yv[tb.ax[k]];
#pragma unroll
    for (int k = 1; k < Tab<P>::NC; ++k) mono[k] *= (T)tb.invf[k];
}

__device__ __forceinline__ float d_erfc(float x) { return erfcf(x); }
__device__ __forceinline__ double d_erfc(double x) { return erfc(x); }
__device__ __forceinline__ float d_exp(float x) { return __expf(x); }
__device__ __forceinline__ double d_exp(double x) { return exp(x); }
__device__ __forceinline__ float d_sqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double d_sqrt(double x) { return sqrt(x); }

// Truncated prefactors f_(0..P) at squared distance r2, a = the split's scale (any units,
// the same as r2's).  Polynomial split, phi_s = 1/r + sum_m c_m r^(2m)/a^(2m+1) with
// c = (-15/8, 5/4, -3/8): f_(k) = (-1)^k (2k-1)!!/r^(2k+1) + the k-fold (r^-1 d/dr) of the
// polynomial, which ends at k = 2.
template <int P, class T> __device__ __forceinline__ void prefactors(T r2, T rs, int kind, T *f)
{
    if (kind == 1) {
        const T r = d_sqrt(r2), inv_r2 = (T)1 / r2, ia = (T)1 / rs, ia2 = ia * ia;
        T nk = (T)1 / r;
        f[0] = nk + ia * ((T)(-15.0 / 8.0) + r2 * ia2 * ((T)1.25 - (T)0.375 * r2 * ia2));
#pragma unroll
        for (int k = 1; k <= P; ++k) {
            nk = -(T)(2 * k - 1) * nk * inv_r2;
            T pk = 0;
            if (k == 1) pk = ia2 * ia * ((T)2.5 - (T)1.5 * r2 * ia2);
            if (k == 2) pk = (T)(-3) * ia2 * ia2 * ia;
            f[k] = nk + pk;
        }
        return;
    }
    T r = d_sqrt(r2);
    T inv_r2 = (T)1 / r2;
    T e = d_exp(-r2 / ((T)4 * rs * rs));
    f[0] = d_erfc(r / ((T)2 * rs)) / r;
    T src = e / ((T)1.7724538509055160273 * rs);  // k = 1 source term
    T step = (T)(-0.5) / (rs * rs);
#pragma unroll
    for (int k = 1; k <= P; ++k) {
        f[k] = -((T)(2 * k - 1) * f[k - 1] + src) * inv_r2;
        src *= step;
    }
}

// Dh_j for |j| <= P from the radial recurrence, in place: at level m the entries are
// rewritten in decreasing index (hence non-increasing degree) order, so every read of
// degree |n|-1 or |n|-2 still sees level m+1.
template <int P, class T> __device__ __forceinline__ void dtensor(T Rx, T Ry, T Rz, const T *f, T *D)
{
    constexpr Tab<P> tb{};
    const T Rv[3] = {Rx, Ry, Rz};
    D[0] = f[P];
#pragma unroll
    for (int m = P - 1; m >= 0; --m) {
#pragma unroll
        for (int k = ncoef(P - m) - 1; k >= 1; --k) {
            T v = Rv[tb.ax[k]] * D[tb.par[k]];
            if (tb.par2[k] >= 0) v += (T)(tb.na[k] - 1) * D[tb.par2[k]];
            D[k] = v;
        }
        D[0] = f[m];
    }
}

// ---------------------------------------------------------------------------
// kernels

// Separation R = z_A - (z_B + image shift) in units of h_A, from the cells' integer
// coordinates (exact): R / h_A = R_int / (2 w_A), R_int in units of box / 2^(l+1).
template <class T> __device__ __forceinline__ void pair_sep(const Cell &ca, const Cell &cb, int s, T &Rx, T &Ry, T &Rz)
{
    const int la = cell_level(ca), lb = cell_level(cb);
    const int l = la > lb ? la : lb;
    const int64_t wa = (int64_t)1 << (l - la), wb = (int64_t)1 << (l - lb);
    const int sh[3] = {s / 9 - 1, (s / 3) % 3 - 1, s % 3 - 1};
    const T inv2wa = (T)(0.5 / (double)wa);
    Rx = (T)((2 * (int64_t)cell_ix(ca) + 1) * wa - (2 * (int64_t)cell_ix(cb) + 1) * wb - (int64_t)sh[0] * ((int64_t)2 << l)) * inv2wa;
    Ry = (T)((2 * (int64_t)ca.iy + 1) * wa - (2 * (int64_t)cb.iy + 1) * wb - (int64_t)sh[1] * ((int64_t)2 << l)) * inv2wa;
    Rz = (T)((2 * (int64_t)ca.iz + 1) * wa - (2 * (int64_t)cb.iz + 1) * wb - (int64_t)sh[2] * ((int64_t)2 << l)) * inv2wa;
}

__device__ __forceinline__ double cell_h(const Cell &c, double box) { return ldexp(box, -cell_level(c)); }

// One thread per leaf.  The FP32 form reads each particle's leaf-relative FP32 record
// (x - c, m), one 16-byte load, instead of four FP64 arrays: the same values (the FP64
// difference rounded to FP32, then scaled by the power of two 1/h for a box of power-of-two
// size), a quarter of the loads and half the bytes.
template <int P, class T>
__global__ __launch_bounds__(64) void k_p2m(const Cell *__restrict__ cells, const int *__restrict__ leaves, int nleaf,
                                            const double *__restrict__ xs, const double *__restrict__ ys,
                                            const double *__restrict__ zs, const double *__restrict__ ms,
                                            const float4 *__restrict__ rel, double box, T *__restrict__ M)
{
    constexpr int NC = Tab<P>::NC;
    constexpr Tab<P> tb{};
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nleaf) return;
    int c = leaves[t];
    Cell cc = cells[c];
    double h = cell_h(cc, box), ih = 1.0 / h;
    double cx = (cell_ix(cc) + 0.5) * h, cy = (cc.iy + 0.5) * h, cz = (cc.iz + 0.5) * h;
    T acc[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) acc[k] = 0;
    for (int i = cc.beg; i < cc.end; ++i) {
        T mono[NC];
        if constexpr (sizeof(T) == 4) {
            const float4 r = rel[i];
            const T s = (T)ih;
            monomials<P, T>(r.x * s, r.y * s, r.z * s, r.w, mono);
        } else {
            monomials<P, T>((T)((xs[i] - cx) * ih), (T)((ys[i] - cy) * ih), (T)((zs[i] - cz) * ih), (T)ms[i], mono);
        }
#pragma unroll
        for (int k = 0; k < NC; ++k) acc[k] += mono[k];
    }
    T *out = M + (size_t)c * NC;
#pragma unroll
    for (int k = 0; k < NC; ++k) out[k] = (tb.d[k] & 1) ? -acc[k] : acc[k];
}

template <int P, class T>
__global__ __launch_bounds__(64) void k_m2m(const Cell *__restrict__ cells, const int *__restrict__ inner, int lbeg,
                                            int ln, T *__restrict__ M)
{
    constexpr int NC = Tab<P>::NC;
    constexpr Tab<P> tb{};
    constexpr SubTab<P> st{};
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ln) return;
    int c = inner[lbeg + t];
    Cell cc = cells[c];
    int nch = cell_nchild(cc);
    if (nch == 0) return;
    T acc[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) acc[k] = 0;
    for (int q = 0; q < nch; ++q) {
        int ch = cc.child + q;
        Cell cq = cells[ch];
        T mono[NC], Mc[NC];
        monomials<P, T>((T)(0.5 - (cell_ix(cq) & 1)), (T)(0.5 - (cq.iy & 1)), (T)(0.5 - (cq.iz & 1)), (T)1, mono);
        const T *src = M + (size_t)ch * NC;
#pragma unroll
        for (int k = 0; k < NC; ++k) Mc[k] = src[k];
#pragma unroll
        for (int e = 0; e < SubTab<P>::NT; ++e) acc[st.m[e]] += mono[st.n[e]] * Mc[st.mn[e]];
    }
    T *out = M + (size_t)c * NC;
#pragma unroll
    for (int k = 0; k < NC; ++k) out[k] = acc[k] * (T)(1.0 / (double)(1 << tb.d[k]));
}

template <int P, class T>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(P >= 7 ? 1 : 2))) void k_m2l(
    const Cell *__restrict__ cells, int ncell, const int *__restrict__ head, const int *__restrict__ cnt,
    const uint32_t *__restrict__ items, const int *__restrict__ next, const T *__restrict__ M, T *__restrict__ L,
    double box, Split sp, int stride, int accumulate, const unsigned char *__restrict__ ord)
{
    // M and L hold ncoef(order of storage) coefficients per cell (stride); this kernel
    // reads and writes the first ncoef(P) of them (multi-indices are ordered by degree).
    // ord != nullptr: a list of mixed orders, of which the entries of order P are taken.
    constexpr int NC = Tab<P>::NC;
    constexpr Tab<P> tb{};
    constexpr PairTab<P> pt{};
    int A = blockIdx.x * blockDim.x + threadIdx.x;
    if (A >= ncell) return;
    int nl = cnt[A];
    T acc[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) acc[k] = 0;
    if (nl > 0) {
        Cell ca = cells[A];
        int la = cell_level(ca);
        T rsh = (T)(sp.scale / cell_h(ca, box));
        int chunk = head[A], taken = 0;
        for (int e = 0; e < nl; ++e) {
            if (e > 0 && (e & (kChunk - 1)) == 0) chunk = next[chunk];
            const size_t at = (size_t)chunk * kChunk + (e & (kChunk - 1));
            if (ord && ord[at] != P) continue;
            ++taken;
            uint32_t it = items[at];
            int B = (int)(it >> 5), s = (int)(it & 31);
            Cell cb = cells[B];
            int lb = cell_level(cb);
            T Rx, Ry, Rz;
            pair_sep<T>(ca, cb, s, Rx, Ry, Rz);
            T f[P + 1], D[NC];
            prefactors<P, T>(Rx * Rx + Ry * Ry + Rz * Rz, rsh, sp.kind, f);
            dtensor<P, T>(Rx, Ry, Rz, f, D);
            T rho = (T)ldexp(1.0, la - lb);
            T rp[P + 1];
            rp[0] = 1;
#pragma unroll
            for (int k = 1; k <= P; ++k) rp[k] = rp[k - 1] * rho;
            const T *Mb = M + (size_t)B * stride;
            m2l_contract<P, T, 0, 16>(Mb, rp, D, acc);
        }
        if (taken == 0) nl = 0;
    }
    if (accumulate && nl == 0) return;
    T *out = L + (size_t)A * stride;
    if (accumulate) {
#pragma unroll
        for (int k = 0; k < NC; ++k) out[k] += acc[k];
    } else {
#pragma unroll
        for (int k = 0; k < NC; ++k) out[k] = acc[k];
    }
}

template <int P, class T>
__global__ __launch_bounds__(64) void k_l2l(const Cell *__restrict__ cells, int lbeg, int ln, T *__restrict__ L)
{
    constexpr int NC = Tab<P>::NC;
    constexpr Tab<P> tb{};
    constexpr PairTab<P> pt{};
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ln) return;
    int c = lbeg + t;
    Cell cc = cells[c];
    T mono[NC], Lp[NC], acc[NC];
    monomials<P, T>((T)(0.25 * ((cell_ix(cc) & 1) ? 1 : -1)), (T)(0.25 * ((cc.iy & 1) ? 1 : -1)),
                    (T)(0.25 * ((cc.iz & 1) ? 1 : -1)), (T)1, mono);
    const T *src = L + (size_t)cc.parent * NC;
#pragma unroll
    for (int k = 0; k < NC; ++k) { Lp[k] = src[k]; acc[k] = 0; }
#pragma unroll
    for (int q = 0; q < PairTab<P>::NT; ++q) acc[pt.n[q]] += mono[pt.m[q]] * Lp[pt.nm[q]];
    T *out = L + (size_t)c * NC;
#pragma unroll
    for (int k = 0; k < NC; ++k) out[k] += acc[k] * (T)(1.0 / (double)(2 << tb.d[k]));
}

// L2P (gradient of Eq. (6)), plus the near field, times G, written in caller order.
template <int P, class T>
__global__ __launch_bounds__(256) void k_l2p(const Cell *__restrict__ cells, const int *__restrict__ leaf_of, int n,
                                             const double *__restrict__ xs, const double *__restrict__ ys,
                                             const double *__restrict__ zs, const T *__restrict__ L,
                                             const double *__restrict__ nearf, const int *__restrict__ perm, double box,
                                             double G, double *__restrict__ acc, int accumulate)
{
    constexpr int NC = Tab<P>::NC;
    constexpr int NC1 = P > 0 ? ncoef(P - 1) : 1;
    constexpr Tab<P> tb{};
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = leaf_of[i];
    Cell cc = cells[c];
    double h = cell_h(cc, box), ih = 1.0 / h;
    double g[3] = {0, 0, 0};
    if (P > 0) {
        T mono[NC1];
        monomials<(P > 0 ? P - 1 : 0), T>((T)((xs[i] - (cell_ix(cc) + 0.5) * h) * ih), (T)((ys[i] - (cc.iy + 0.5) * h) * ih),
                                          (T)((zs[i] - (cc.iz + 0.5) * h) * ih), (T)1, mono);
        const T *Lc = L + (size_t)c * NC;
        T gx = 0, gy = 0, gz = 0;
#pragma unroll
        for (int k = 0; k < NC1; ++k) {
            int a = tb.x[k], b = tb.y[k], z = tb.z[k];
            gx += Lc[midx(a + 1, b, z)] * mono[k];
            gy += Lc[midx(a, b + 1, z)] * mono[k];
            gz += Lc[midx(a, b, z + 1)] * mono[k];
        }
        double s = ih * ih;
        g[0] = (double)gx * s;
        g[1] = (double)gy * s;
        g[2] = (double)gz * s;
    }
    size_t o = 3 * (size_t)perm[i];
    const double r0 = G * (g[0] + nearf[i]), r1 = G * (g[1] + nearf[(size_t)n + i]),
                 r2 = G * (g[2] + nearf[2 * (size_t)n + i]);
    if (accumulate) {
        acc[o] += r0;
        acc[o + 1] += r1;
        acc[o + 2] += r2;
    } else {
        acc[o] = r0;
        acc[o + 1] = r1;
        acc[o + 2] = r2;
    }
}

// ---------------------------------------------------------------------------
// High orders (P >= 7).  Order 8 has 165 coefficients: a thread cannot hold a cell's
// expansion, a derivative tensor and a source block in registers at once.  M2M and L2L
// therefore run a wave per cell, and M2L (FP32) a lane per interaction pair.

// A Cartesian translation factorises into three one-dimensional shifts: with monomial
// weights w_a(i) = h_a^i / i!,
//   M2M  M'_m = sum_{i <= m_x} w_x(i) sum_{j <= m_y} w_y(j) sum_{k <= m_z} w_z(k) M_{m - (i,j,k)}
//   L2L  L'_n = sum_i w_x(i) sum_j w_y(j) sum_k w_z(k) L_{n + (i,j,k)}   (|n + (i,j,k)| <= P)
// so the operators are applied as three in-place passes along x, y and z (about half the
// multiply-adds of the direct double sum, and no second coefficient array).  A pass
// along `ax` visits the multi-indices in an order where every source is still unmodified:
// descending component ax for M2M (sources have a smaller component), ascending for L2L.
template <int P, int AX, bool UP> struct AxisOrder {
    int k[ncoef(P)];
    constexpr AxisOrder() : k()
    {
        Tab<P> T{};
        int q = 0;
        for (int v = 0; v <= P; ++v) {
            int comp = UP ? P - v : v;
            for (int kk = 0; kk < ncoef(P); ++kk) {
                int c = AX == 0 ? T.x[kk] : (AX == 1 ? T.y[kk] : T.z[kk]);
                if (c == comp) k[q++] = kk;
            }
        }
    }
};

template <int P, class T, int AX, bool UP> __device__ __forceinline__ void shift_axis(T *C, const T *w)
{
    constexpr Tab<P> tb{};
    constexpr AxisOrder<P, AX, UP> ao{};
#pragma unroll
    for (int q = 0; q < ncoef(P); ++q) {
        const int k = ao.k[q];
        const int a = tb.x[k], b = tb.y[k], c = tb.z[k];
        const int comp = AX == 0 ? a : (AX == 1 ? b : c);
        T sum = C[k];
        if (UP) {
#pragma unroll
            for (int i = 1; i <= comp; ++i)
                sum += w[i] * C[midx(AX == 0 ? a - i : a, AX == 1 ? b - i : b, AX == 2 ? c - i : c)];
        } else {
#pragma unroll
            for (int i = 1; i <= P - tb.d[k]; ++i)
                sum += w[i] * C[midx(AX == 0 ? a + i : a, AX == 1 ? b + i : b, AX == 2 ? c + i : c)];
        }
        C[k] = sum;
    }
}

// w[i] = (s h)^i / i!, i = 0..P, s = +1 or -1
template <int P, class T> __device__ __forceinline__ void shift_weights(T h, bool neg, T *w)
{
    T v = 1;
    w[0] = 1;
#pragma unroll
    for (int i = 1; i <= P; ++i) {
        v *= h / (T)i;
        w[i] = (neg && (i & 1)) ? -v : v;
    }
}

// M2M for the parents of one level, a thread per parent: each child's multipole is
// shifted in registers (x-hat = +-1/2 in child units) and added to the parent.
template <int P, class T>
__global__ __launch_bounds__(64) void k_m2m_axis(const Cell *__restrict__ cells, const int *__restrict__ inner, int lbeg,
                                                 int ln, T *__restrict__ M)
{
    constexpr int NC = ncoef(P);
    constexpr Tab<P> tb{};
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ln) return;
    const int c = inner[lbeg + t];
    const Cell cc = cells[c];
    const int nch = cell_nchild(cc);
    if (nch == 0) return;
    T *out = M + (size_t)c * NC;
    // FP32: the sum over the children is kept in this thread's LDS row (odd stride NC, no
    // bank conflicts) and written once, instead of a read-modify-write of the parent's
    // coefficients in global memory per child
    constexpr bool kLds = sizeof(T) == 4;
    __shared__ T accs[kLds ? 64 * NC : 1];
    T *acc = kLds ? accs + threadIdx.x * NC : out;
    for (int q = 0; q < nch; ++q) {
        const int ch = cc.child + q;
        const Cell cq = cells[ch];
        T C[NC], wx[P + 1], wy[P + 1], wz[P + 1];
        const T *src = M + (size_t)ch * NC;
#pragma unroll
        for (int k = 0; k < NC; ++k) C[k] = src[k];
        shift_weights<P, T>((T)0.5, cell_ix(cq) & 1, wx);
        shift_weights<P, T>((T)0.5, cq.iy & 1, wy);
        shift_weights<P, T>((T)0.5, cq.iz & 1, wz);
        shift_axis<P, T, 0, true>(C, wx);
        shift_axis<P, T, 1, true>(C, wy);
        shift_axis<P, T, 2, true>(C, wz);
        if (q == 0) {
#pragma unroll
            for (int k = 0; k < NC; ++k) acc[k] = C[k] * (T)(1.0 / (double)(1 << tb.d[k]));
        } else {
#pragma unroll
            for (int k = 0; k < NC; ++k) acc[k] += C[k] * (T)(1.0 / (double)(1 << tb.d[k]));
        }
    }
    if constexpr (kLds) {
#pragma unroll
        for (int k = 0; k < NC; ++k) out[k] = acc[k];
    }
}

// L2L for the cells of one level, a thread per child: the parent's local expansion is
// shifted to the child centre (x-hat = +-1/4 in parent units) and added.
template <int P, class T>
__global__ __launch_bounds__(64) void k_l2l_axis(const Cell *__restrict__ cells, int lbeg, int ln, T *__restrict__ L)
{
    constexpr int NC = ncoef(P);
    constexpr Tab<P> tb{};
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ln) return;
    const int c = lbeg + t;
    const Cell cc = cells[c];
    T C[NC], wx[P + 1], wy[P + 1], wz[P + 1];
    const T *src = L + (size_t)cc.parent * NC;
#pragma unroll
    for (int k = 0; k < NC; ++k) C[k] = src[k];
    shift_weights<P, T>((T)0.25, !(cell_ix(cc) & 1), wx);
    shift_weights<P, T>((T)0.25, !(cc.iy & 1), wy);
    shift_weights<P, T>((T)0.25, !(cc.iz & 1), wz);
    shift_axis<P, T, 0, false>(C, wx);
    shift_axis<P, T, 1, false>(C, wy);
    shift_axis<P, T, 2, false>(C, wz);
    T *dst = L + (size_t)c * NC;
#pragma unroll
    for (int k = 0; k < NC; ++k) dst[k] += C[k] * (T)(1.0 / (double)(2 << tb.d[k]));
}

// M2L of the high orders, a lane per pair of the flattened pair array (each sink's pairs
// contiguous).  A lane builds its pair's derivative tensor in registers.  Outputs of
// degree >= P - 2 need source coefficients of degree <= 2 only: they are summed one at a
// time from the first ten coefficients and staged in LDS, a chunk of rows at a time, for
// the wave reduction.  The other outputs take the whole source multipole, streamed in
// blocks of MB coefficients (the next block is loaded while the current one is used):
// the kLo lowest outputs (degree <= 2) in registers, the rest (degree 3 .. P - 3) in LDS,
// one row per lane.  A reduction sums each output over the runs of lanes that share a
// sink and adds the sums into L with one atomic per run.
constexpr int kLo = 10;  // outputs of degree <= 2

// Orders whose M2L takes the lane-per-pair kernel: FP32 from order 3 up, FP64 from 3 to 6
// (an order-7/8 FP64 derivative tensor does not fit in registers).
template <int P, class T> constexpr bool pair_m2l() { return P >= 3 && (sizeof(T) == 4 || P <= 6); }

// First output of degree >= P - 2 past the register outputs, and the LDS row counts.
template <int P> constexpr int m2l_hi_begin() { return P >= 3 && ncoef(P - 3) > kLo ? ncoef(P - 3) : kLo; }
template <int P> constexpr int m2l_mid_rows() { return m2l_hi_begin<P>() - kLo; }
template <int P> constexpr int m2l_hi_chunk()
{
    return m2l_mid_rows<P>() > 32 ? m2l_mid_rows<P>() : (ncoef(P) - m2l_hi_begin<P>() < 32 ? ncoef(P) - m2l_hi_begin<P>() : 32);
}

// Terms of one source block KB .. KB+MB-1 for the outputs below NE, in output-major order:
// (output n, source k, derivative index n + k), with flags marking the first and last
// term of each output.
template <int P> constexpr int block_terms(int kb, int ke, int ne)
{
    Tab<P> T{};
    int c = 0;
    for (int n = 0; n < ne; ++n)
        for (int k = kb; k < ke; ++k)
            if (T.d[k] + T.d[n] <= P) ++c;
    return c;
}

template <int P, int KB, int MB, int NE> struct BlockTab {
    static constexpr int KE = KB + MB < ncoef(P) ? KB + MB : ncoef(P);
    static constexpr int NQ = block_terms<P>(KB, KE, NE);
    short n[NQ], k[NQ], nm[NQ];
    bool first[NQ], last[NQ];
    constexpr BlockTab() : n(), k(), nm(), first(), last()
    {
        Tab<P> T{};
        int q = 0;
        for (int kn = 0; kn < NE; ++kn) {
            int q0 = q;
            for (int km = KB; km < KE; ++km)
                if (T.d[km] + T.d[kn] <= P) {
                    n[q] = (short)kn;
                    k[q] = (short)(km - KB);
                    nm[q] = (short)midx(T.x[kn] + T.x[km], T.y[kn] + T.y[km], T.z[kn] + T.z[km]);
                    first[q] = q == q0;
                    last[q] = false;
                    ++q;
                }
            if (q > q0) last[q - 1] = true;
        }
    }
};

// Terms of the outputs N0 .. N1-1 (all of degree >= P - 2): (output n - N0, source k < 10,
// derivative index n + k), output-major, flags as in BlockTab.
template <int P> constexpr int hi_terms(int n0, int n1)
{
    Tab<P> T{};
    int c = 0;
    for (int n = n0; n < n1; ++n)
        for (int k = 0; k < kLo; ++k)
            if (T.d[k] + T.d[n] <= P) ++c;
    return c;
}

template <int P, int N0, int N1> struct HiTab {
    static constexpr int NQ = hi_terms<P>(N0, N1);
    short n[NQ], k[NQ], nm[NQ];
    bool last[NQ];
    constexpr HiTab() : n(), k(), nm(), last()
    {
        Tab<P> T{};
        int q = 0;
        for (int kn = N0; kn < N1; ++kn) {
            int q0 = q;
            for (int km = 0; km < kLo; ++km)
                if (T.d[km] + T.d[kn] <= P) {
                    n[q] = (short)(kn - N0);
                    k[q] = (short)km;
                    nm[q] = (short)midx(T.x[kn] + T.x[km], T.y[kn] + T.y[km], T.z[kn] + T.z[km]);
                    last[q] = false;
                    ++q;
                }
            if (q > q0) last[q - 1] = true;
        }
    }
};

template <int P, class T, int KB, int MB, int NE>
__device__ __forceinline__ void m2l_pair_block(const T *__restrict__ Mb, const T *rp, const T *D, T *lo, T *row,
                                               const T *Mcur)
{
    constexpr Tab<P> tb{};
    constexpr BlockTab<P, KB, MB, NE> bt{};
    constexpr int NC = ncoef(P);
    constexpr int KE = BlockTab<P, KB, MB, NE>::KE;
    constexpr int KE2 = KE + MB < NC ? KE + MB : NC;
    T Mnext[MB];
    if constexpr (KE < NC) {
#pragma unroll
        for (int k = KE; k < KE2; ++k) Mnext[k - KE] = Mb[k];
    }
    T Ms[MB];
#pragma unroll
    for (int k = KB; k < KE; ++k) Ms[k - KB] = Mcur[k - KB] * rp[tb.d[k]];
    T a = 0;
#pragma unroll
    for (int q = 0; q < BlockTab<P, KB, MB, NE>::NQ; ++q) {
        const int n = bt.n[q];
        if (bt.first[q]) a = n < kLo ? lo[n] : row[n - kLo];
        a += Ms[bt.k[q]] * D[bt.nm[q]];
        if (bt.last[q]) {
            if (n < kLo) lo[n] = a;
            else row[n - kLo] = a;
        }
    }
    if constexpr (KE < NC) m2l_pair_block<P, T, KE, MB, NE>(Mb, rp, D, lo, row, Mnext);
}

// Sum the staged rows 0 .. NROWS-1 (lane j's values at buf[j * STR + r]) over the runs of
// lanes with the same sink sid[j] and add each sum to output `out0 + r` of that sink.
// With fewer than 64 rows, a power of two of threads share a row, each summing a
// contiguous range of lanes (a run cut by a range boundary is added in two parts).  When
// the whole wave holds one sink (`one`, wave-uniform; the pairs of a sink are contiguous),
// the sums take no run tests and their loads are independent.
template <class T, int STR, int NROWS>
__device__ __forceinline__ void m2l_reduce_rows(const T *buf, const int *sid, bool one, int out0, T *L, int stride)
{
    constexpr int NP = NROWS > 32 ? 1 : NROWS > 16 ? 2 : NROWS > 8 ? 4 : NROWS > 4 ? 8 : NROWS > 2 ? 16 : NROWS > 1 ? 32 : 64;
    constexpr int SPAN = 64 / NP;
    for (int t = threadIdx.x; t < NROWS * NP; t += 64) {
        const int r = t % NROWS, j0 = (t / NROWS) * SPAN;
        if (one) {
            T s0 = 0, s1 = 0;
#pragma unroll
            for (int k = 0; k < SPAN; k += 2) {
                s0 += buf[(j0 + k) * STR + r];
                if (k + 1 < SPAN) s1 += buf[(j0 + k + 1) * STR + r];
            }
            atomicAdd(&L[(size_t)sid[j0] * stride + out0 + r], s0 + s1);
            continue;
        }
        T sum = 0;
        int cur = sid[j0];
        for (int j = j0; j < j0 + SPAN; ++j) {
            const int a = sid[j];
            if (a != cur) {
                if (cur >= 0) atomicAdd(&L[(size_t)cur * stride + out0 + r], sum);
                sum = 0;
                cur = a;
            }
            sum += buf[j * STR + r];
        }
        if (cur >= 0) atomicAdd(&L[(size_t)cur * stride + out0 + r], sum);
    }
}

// The outputs N0 .. NC-1 in chunks of HC: each output of a chunk summed in a register,
// staged, reduced.
template <int P, class T, int N0, int HC, int STR>
__device__ __forceinline__ void m2l_hi_outputs(const T *Ms, const T *D, T *buf, const int *sid, bool one, T *L,
                                               int stride)
{
    constexpr int NC = ncoef(P);
    constexpr int N1 = N0 + HC < NC ? N0 + HC : NC;
    constexpr HiTab<P, N0, N1> ht{};
    T *row = buf + threadIdx.x * STR;
    T a = 0;
#pragma unroll
    for (int q = 0; q < HiTab<P, N0, N1>::NQ; ++q) {
        a += Ms[ht.k[q]] * D[ht.nm[q]];
        if (ht.last[q]) {
            row[ht.n[q]] = a;
            a = 0;
        }
    }
    __syncthreads();
    m2l_reduce_rows<T, STR, N1 - N0>(buf, sid, one, N0, L, stride);
    __syncthreads();
    if constexpr (N1 < NC) m2l_hi_outputs<P, T, N1, HC, STR>(Ms, D, buf, sid, one, L, stride);
}

// Shared memory of one 64-pair block of the pair kernel.
template <int P, class T> struct M2LPairShared {
    static constexpr int NMID = m2l_mid_rows<P>(), HC = m2l_hi_chunk<P>();
    static constexpr int STR = (NMID > HC ? NMID : HC) | 1;  // odd row stride: no bank conflicts
    T buf[64 * STR];
    int sid[64];
};

// Pairs blk*64 .. blk*64+63 of the flattened array (one 64-lane wave).
template <int P, class T>
__device__ __forceinline__ void m2l_pairs_block(const Cell *__restrict__ cells, const int2 *__restrict__ pairs,
                                                int64_t npair, const T *__restrict__ M, T *__restrict__ L, double box,
                                                Split sp, int stride, int64_t blk, M2LPairShared<P, T> &sh)
{
    constexpr int NC = ncoef(P), NHB = m2l_hi_begin<P>(), NMID = m2l_mid_rows<P>(), HC = m2l_hi_chunk<P>();
    constexpr int STR = M2LPairShared<P, T>::STR;
    constexpr int MB = 16;
    T *buf = sh.buf;
    int *sid = sh.sid;
    const int lane = threadIdx.x;
    const int64_t idx = blk * 64 + lane;
    T D[NC], rp[P + 1], M0[MB];
#pragma unroll
    for (int k = 0; k < NC; ++k) D[k] = 0;
#pragma unroll
    for (int k = 0; k < MB; ++k) M0[k] = 0;
#pragma unroll
    for (int k = 0; k <= P; ++k) rp[k] = 0;
    int A = -1;
    const T *Mb = M;
    if (idx < npair) {
        const int2 pr = pairs[idx];
        A = pr.x;
        const uint32_t it = (uint32_t)pr.y;
        const int B = (int)(it >> 5), s = (int)(it & 31);
        const Cell ca = cells[A], cb = cells[B];
        Mb = M + (size_t)B * stride;
#pragma unroll
        for (int k = 0; k < MB; ++k) M0[k] = Mb[k];
        T Rx, Ry, Rz;
        pair_sep<T>(ca, cb, s, Rx, Ry, Rz);
        T f[P + 1];
        prefactors<P, T>(Rx * Rx + Ry * Ry + Rz * Rz, (T)(sp.scale / cell_h(ca, box)), sp.kind, f);
        dtensor<P, T>(Rx, Ry, Rz, f, D);
        const T rho = (T)ldexp(1.0, cell_level(ca) - cell_level(cb));
        rp[0] = 1;
#pragma unroll
        for (int k = 1; k <= P; ++k) rp[k] = rp[k - 1] * rho;
    }
    sid[lane] = A;
    // every lane holds the same sink: the pairs of a sink are contiguous, so equal ends suffice
    const int A0 = __builtin_amdgcn_readlane(A, 0);
    const bool one = A0 >= 0 && A0 == __builtin_amdgcn_readlane(A, 63);
    // outputs of degree >= P - 2 from the source coefficients of degree <= 2
    {
        constexpr Tab<P> tb{};
        T Ms[kLo];
#pragma unroll
        for (int k = 0; k < kLo; ++k) Ms[k] = M0[k] * rp[tb.d[k]];
        __syncthreads();
        m2l_hi_outputs<P, T, NHB, HC, STR>(Ms, D, buf, sid, one, L, stride);
    }
    // the other outputs from the whole source multipole
    T *row = buf + lane * STR;
#pragma unroll
    for (int k = 0; k < NMID; ++k) row[k] = 0;
    T lo[kLo];
#pragma unroll
    for (int k = 0; k < kLo; ++k) lo[k] = 0;
    if (idx < npair) m2l_pair_block<P, T, 0, MB, NHB>(Mb, rp, D, lo, row, M0);
    __syncthreads();
    if constexpr (NMID > 0) {
        m2l_reduce_rows<T, STR, NMID>(buf, sid, one, kLo, L, stride);
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < kLo; ++k) row[k] = lo[k];
    __syncthreads();
    m2l_reduce_rows<T, STR, kLo>(buf, sid, one, 0, L, stride);
}

template <int P, class T>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 1 : P >= 7 ? 2 : 3))) void k_m2l_pairs(
    const Cell *__restrict__ cells, const int2 *__restrict__ pairs, int64_t npair, const T *__restrict__ M,
    T *__restrict__ L, double box, Split sp, int stride)
{
    __shared__ M2LPairShared<P, T> sh;
    m2l_pairs_block<P, T>(cells, pairs, npair, M, L, box, sp, stride, xcd_order(blockIdx.x, gridDim.x), sh);
}

int flatten_pairs(fmm_tree *t, int kind, int64_t npair, hipStream_t st);

// ---------------------------------------------------------------------------
// dispatch over P and precision

template <template <int, class> class F, class T, class... Args> int dispatch_p(int p, Args &&...args)
{
    switch (p) {
    case 0: return F<0, T>::run(args...);
    case 1: return F<1, T>::run(args...);
    case 2: return F<2, T>::run(args...);
    case 3: return F<3, T>::run(args...);
    case 4: return F<4, T>::run(args...);
    case 5: return F<5, T>::run(args...);
    case 6: return F<6, T>::run(args...);
    case 7: return F<7, T>::run(args...);
    case 8: return F<8, T>::run(args...);
    }
    return set_error(FMM_ERR_ARG, "expansion order %d not compiled", p);
}

static inline int nblk(int64_t n, int b) { return (int)((n + b - 1) / b); }

template <int P, class T> struct Upward {
    static int run(fmm_tree *t, hipStream_t st)
    {
        constexpr int NC = ncoef(P);
        if (int rc = grow(t->Mc, (size_t)t->ncell * NC * sizeof(T)) | grow(t->Lc, (size_t)t->ncell * NC * sizeof(T)))
            return rc;
        k_p2m<P, T><<<nblk(t->nleaf, 64), 64, 0, st>>>(ptr<Cell>(t->cells), ptr<int>(t->leaves), t->nleaf,
                                                       ptr<double>(t->xs), ptr<double>(t->ys), ptr<double>(t->zs),
                                                       ptr<double>(t->ms), ptr<float4>(t->rel32), t->box, ptr<T>(t->Mc));
        // M2M over the cells with children only, level by level (inner[] holds them in cell
        // order; those of level l follow the lvl_beg[l] - leaf_lvl[l] before it): at 134M
        // seven cells in eight are leaves, whose threads would idle
        for (int l = t->nlevel - 2; l >= 0; --l) {
            const int lb = t->lvl_beg[l] - t->leaf_lvl[l], ln = t->lvl_beg[l + 1] - t->leaf_lvl[l + 1] - lb;
            if (ln <= 0) continue;
            if constexpr (P >= 7)
                k_m2m_axis<P, T><<<nblk(ln, 64), 64, 0, st>>>(ptr<Cell>(t->cells), ptr<int>(t->inner), lb, ln,
                                                               ptr<T>(t->Mc));
            else
                k_m2m<P, T><<<nblk(ln, 64), 64, 0, st>>>(ptr<Cell>(t->cells), ptr<int>(t->inner), lb, ln,
                                                          ptr<T>(t->Mc));
        }
        return hip_check(hipGetLastError(), "upward pass");
    }
};

template <int P, class T> struct M2L {
    // Coefficient storage of order `pstore`.  learned == 0: the plain M2L list (kind 0);
    // learned != 0: the entries of order P of the learned selector's list, whose pairs
    // flatten_learned has already laid out by order (the pair kernel adds to L).
    // mfma != 0 (FP32, orders 4..8, plain list): pairs of cells on one level on the matrix
    // cores (m2l_mfma.hip), the others by the lane-per-pair kernel below.
    // det != 0: the thread-per-sink kernel below for every order (a fixed summation order).
    static int run(fmm_tree *t, Split sp, int learned, int pstore, int accumulate, int mfma, int det, hipStream_t st)
    {
        const int kind = learned ? kKindOrd : 0;
        if constexpr (pair_m2l<P, T>()) if (!det) {
            const int64_t np = learned ? t->stats.n_m2l_by_order[P - 2] : t->n_m2l;
            if (!accumulate)
                if (int rc = zero_async(t->Lc.p, (size_t)t->ncell * ncoef(pstore) * sizeof(T), st)) return rc;
            if (np == 0) return hip_check(hipGetLastError(), "m2l");
            if constexpr (sizeof(T) == 4 && P >= 4) {
                if (mfma && !learned && !accumulate && pstore == P) {
                    int64_t nother = 0;
                    if (int rc = m2l_mfma_split_and_run(t, P, sp, &nother, st)) return rc;
                    if (nother > 0)
                        k_m2l_pairs<P, T><<<(unsigned)((nother + 63) / 64), 64, 0, st>>>(
                            ptr<Cell>(t->cells), ptr<int2>(t->m2l_pairs), nother, ptr<T>(t->Mc), ptr<T>(t->Lc),
                            t->box, sp, ncoef(pstore));
                    return hip_check(hipGetLastError(), "m2l pairs");
                }
            }
            if (!learned)
                if (int rc = flatten_pairs(t, kind, np, st)) return rc;
            const int2 *pairs = ptr<int2>(t->m2l_pairs) + (learned ? t->lseg[P - 2] : 0);
            k_m2l_pairs<P, T><<<(unsigned)((np + 63) / 64), 64, 0, st>>>(ptr<Cell>(t->cells), pairs, np, ptr<T>(t->Mc),
                                                                       ptr<T>(t->Lc), t->box, sp, ncoef(pstore));
            return hip_check(hipGetLastError(), "m2l pairs");
        }
        size_t off = (size_t)kind * t->ncell;
        k_m2l<P, T><<<nblk(t->ncell, 64), 64, 0, st>>>(
            ptr<Cell>(t->cells), t->ncell, ptr<int>(t->lhead) + off, ptr<int>(t->lcnt) + off,
            ptr<uint32_t>(t->litems[kind]), ptr<int>(t->lnext[kind]), ptr<T>(t->Mc), ptr<T>(t->Lc), t->box, sp,
            ncoef(pstore), accumulate, learned ? ptr<unsigned char>(t->lord) : nullptr);
        return hip_check(hipGetLastError(), "m2l");
    }
};

template <int P, class T> struct L2L {
    static int run(fmm_tree *t, hipStream_t st)
    {
        for (int l = 1; l < t->nlevel; ++l) {
            int lb = t->lvl_beg[l], ln = t->lvl_beg[l + 1] - lb;
            if constexpr (P >= 7)
                k_l2l_axis<P, T><<<nblk(ln, 64), 64, 0, st>>>(ptr<Cell>(t->cells), lb, ln, ptr<T>(t->Lc));
            else
                k_l2l<P, T><<<nblk(ln, 64), 64, 0, st>>>(ptr<Cell>(t->cells), lb, ln, ptr<T>(t->Lc));
        }
        return hip_check(hipGetLastError(), "l2l");
    }
};

template <int P, class T> struct L2P {
    static int run(fmm_tree *t, double G, double *acc, int accumulate, hipStream_t st)
    {
        k_l2p<P, T><<<nblk(t->n, 256), 256, 0, st>>>(ptr<Cell>(t->cells), ptr<int>(t->leaf_of), (int)t->n,
                                                     ptr<double>(t->xs), ptr<double>(t->ys), ptr<double>(t->zs),
                                                     ptr<T>(t->Lc), ptr<double>(t->nearf), ptr<int>(t->perm), t->box,
                                                     G, acc, accumulate);
        return hip_check(hipGetLastError(), "l2p");
    }
};

template <class T> int upward_t(fmm_tree *t, int p, hipStream_t st) { return dispatch_p<Upward, T>(p, t, st); }
template <class T>
int m2l_t(fmm_tree *t, int p, Split sp, int learned, int pstore, int accumulate, int mfma, int det, hipStream_t st)
{
    return dispatch_p<M2L, T>(p, t, sp, learned, pstore, accumulate, mfma, det, st);
}
template <class T> int l2l_t(fmm_tree *t, int p, hipStream_t st) { return dispatch_p<L2L, T>(p, t, st); }
template <class T> int l2p_t(fmm_tree *t, int p, double G, double *acc, int accumulate, hipStream_t st)
{
    return dispatch_p<L2P, T>(p, t, G, acc, accumulate, st);
}

}  // namespace hfmm
