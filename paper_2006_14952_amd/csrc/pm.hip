// Long-range force by the particle-mesh method (Sec. 2.2): the Poisson Green function
// filtered by exp(-k^2 r_s^2), so that PM + the erfc-truncated short range sums to
// Newtonian gravity (the split of the force law g(r) of Sec. 2.2).
//
//   deposit -> rho(x);  FFT;  phi_k = -4 pi G rho_k exp(-k^2 r_s^2) / (k^2 W(k)^2);
//   a_k = -i k phi_k (three components);  inverse FFTs;  interpolation.
// The mass assignment is cloud-in-cell by default, or the higher-order triangular-shaped
// cloud (TSC) or piecewise cubic (PCS) B-spline schemes (fmm_params.pm_assign 3, 4);
// W(k) = prod_i sinc^p(k_i Delta / 2) is the window of the order-p scheme, divided out
// once for the deposit and once for the interpolation.  With the polynomial split the filter is the
// transform of its smoothing density 15/(8 pi r_c^3)(1 - r^2/r_c^2) (r < r_c):
// 15 (3 sin u - 3 u cos u - u^2 sin u) / u^5, u = k r_cut.  The k = 0 mode is dropped (mean density is
// cancelled by the expanding background).  FFTs are hipFFT (double precision).
#include <hipfft/hipfft.h>
#include <math.h>

#include <map>
#include <mutex>

#include "state.h"

namespace hfmm {

struct PMPlan {
    int mesh = 0;
    hipfftHandle r2c = 0, c2r = 0;
    DevBuf rho, rhok, work, amesh;
};

static std::mutex g_pm_mu;
static std::map<int, PMPlan *> g_pm;  // one plan set per mesh size per process

static int pm_plan(int mesh, PMPlan **out)
{
    std::lock_guard<std::mutex> lk(g_pm_mu);
    auto it = g_pm.find(mesh);
    if (it != g_pm.end()) {
        *out = it->second;
        return 0;
    }
    PMPlan *p = new PMPlan();
    p->mesh = mesh;
    if (hipfftPlan3d(&p->r2c, mesh, mesh, mesh, HIPFFT_D2Z) != HIPFFT_SUCCESS ||
        hipfftPlan3d(&p->c2r, mesh, mesh, mesh, HIPFFT_Z2D) != HIPFFT_SUCCESS) {
        delete p;
        return set_error(FMM_ERR_HIP, "hipfftPlan3d(%d) failed", mesh);
    }
    size_t nr = (size_t)mesh * mesh * mesh, nc = (size_t)mesh * mesh * (mesh / 2 + 1);
    int rc = grow(p->rho, nr * 8) | grow(p->rhok, nc * 16) | grow(p->work, nc * 16) | grow(p->amesh, 3 * nr * 8);
    if (rc) {
        delete p;
        return rc;
    }
    g_pm[mesh] = p;
    *out = p;
    return 0;
}

// Mass-assignment weights of the B-spline schemes on the cell-centred mesh (node i at
// (i + 0.5) Delta): ORDER 2 cloud-in-cell, 3 triangular-shaped cloud, 4 piecewise cubic.
// The particle touches nodes i0 .. i0 + ORDER - 1 (mod M) with weights w[0 .. ORDER-1].
template <int ORDER> __device__ __forceinline__ void assign_weights(double x, double inv_d, int M, int &i0, double *w)
{
    const double g = x * inv_d - 0.5;
    double first;
    if constexpr (ORDER == 2) {
        const double f = floor(g), t = g - f;
        w[0] = 1.0 - t;
        w[1] = t;
        first = f;
    } else if constexpr (ORDER == 3) {
        const double c = floor(g + 0.5), dx = g - c;  // nearest node, dx in [-1/2, 1/2)
        w[0] = 0.5 * (0.5 - dx) * (0.5 - dx);
        w[1] = 0.75 - dx * dx;
        w[2] = 0.5 * (0.5 + dx) * (0.5 + dx);
        first = c - 1.0;
    } else {
        const double f = floor(g), t = g - f, t2 = t * t, t3 = t2 * t, u = 1.0 - t;
        w[0] = u * u * u / 6.0;
        w[1] = (4.0 - 6.0 * t2 + 3.0 * t3) / 6.0;
        w[2] = (1.0 + 3.0 * t + 3.0 * t2 - 3.0 * t3) / 6.0;
        w[3] = t3 / 6.0;
        first = f - 1.0;
    }
    const int i = (int)first;
    i0 = ((i % M) + M) % M;
}

// Particle sources of the PM step: the caller's (n,3) positions and masses, or the
// octree's Morton-ordered SoA copies (wrapped), whose output rows are perm[p].  In Morton
// order neighbouring threads deposit into neighbouring mesh cells.
struct CallerOrder {
    const double *pos, *mass;
    __device__ double x(int p, int a) const { return pos[3 * (size_t)p + a]; }
    __device__ double m(int p) const { return mass[p]; }
    __device__ size_t row(int p) const { return 3 * (size_t)p; }
};
struct MortonOrder {
    const double *xs, *ys, *zs, *ms;
    const int *perm;
    __device__ double x(int p, int a) const { return a == 0 ? xs[p] : (a == 1 ? ys[p] : zs[p]); }
    __device__ double m(int p) const { return ms[p]; }
    __device__ size_t row(int p) const { return 3 * (size_t)perm[p]; }
};

template <class S, int ORDER>
__global__ void k_deposit(S src, int n, double box, int M, double inv_vol, double *__restrict__ rho)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    double inv_d = M / box;
    int i[3];
    double w[3][ORDER];
    for (int a = 0; a < 3; ++a) {
        double x = src.x(p, a);
        x -= box * floor(x / box);
        assign_weights<ORDER>(x, inv_d, M, i[a], w[a]);
    }
    double m = src.m(p) * inv_vol;
    for (int dx = 0; dx < ORDER; ++dx)
        for (int dy = 0; dy < ORDER; ++dy)
            for (int dz = 0; dz < ORDER; ++dz) {
                size_t idx = ((size_t)((i[0] + dx) % M) * M + (i[1] + dy) % M) * M + (i[2] + dz) % M;
                atomicAdd(&rho[idx], m * w[0][dx] * w[1][dy] * w[2][dz]);
            }
}

// Deterministic deposit (fmm_params.deterministic): every contribution m w / d^3 is rounded
// to an integer multiple of 2^-e and summed in 64-bit integers, whose sums do not depend on
// the order of the atomics.  e is the largest exponent with n max|m| / d^3 2^e < 2^62, so no
// partial sum overflows; a contribution's rounding is at most 2^-(e+1), below 1e-15 of the
// total |mass| / d^3 for any n up to 2^30.
template <class S> __global__ __launch_bounds__(256) void k_mass_absmax(S src, int n, unsigned long long *mx)
{
    __shared__ unsigned long long w[256];
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    // |m| >= 0: the order of the bit patterns is the order of the values
    w[threadIdx.x] = p < n ? (unsigned long long)__double_as_longlong(fabs(src.m(p))) : 0ull;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) w[threadIdx.x] = max(w[threadIdx.x], w[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0 && w[0]) atomicMax(mx, w[0]);
}

__device__ __forceinline__ int fixed_exponent(const unsigned long long *mx, int n, double inv_vol)
{
    const double bound = (double)n * __longlong_as_double((long long)*mx) * inv_vol;
    return bound > 0.0 ? 61 - ilogb(bound) : 0;
}

template <class S, int ORDER>
__global__ void k_deposit_fixed(S src, int n, double box, int M, double inv_vol, const unsigned long long *__restrict__ mx,
                                unsigned long long *__restrict__ rho)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int e = fixed_exponent(mx, n, inv_vol);
    double inv_d = M / box;
    int i[3];
    double w[3][ORDER];
    for (int a = 0; a < 3; ++a) {
        double x = src.x(p, a);
        x -= box * floor(x / box);
        assign_weights<ORDER>(x, inv_d, M, i[a], w[a]);
    }
    double m = src.m(p) * inv_vol;
    for (int dx = 0; dx < ORDER; ++dx)
        for (int dy = 0; dy < ORDER; ++dy)
            for (int dz = 0; dz < ORDER; ++dz) {
                size_t idx = ((size_t)((i[0] + dx) % M) * M + (i[1] + dy) % M) * M + (i[2] + dz) % M;
                const long long q = llrint(ldexp(m * w[0][dx] * w[1][dy] * w[2][dz], e));
                atomicAdd(&rho[idx], (unsigned long long)q);
            }
}

// The integer mesh back to FP64, in place.
__global__ void k_fixed_to_double(unsigned long long *__restrict__ rho, size_t nr, const unsigned long long *__restrict__ mx,
                                  int n, double inv_vol)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr) return;
    const int e = fixed_exponent(mx, n, inv_vol);
    const double v = ldexp((double)(long long)rho[i], -e);
    reinterpret_cast<double *>(rho)[i] = v;
}

__device__ __forceinline__ double sinc(double x) { return fabs(x) < 1e-8 ? 1.0 : sin(x) / x; }

// long-range filter at |k|^2 = k2: Gaussian split exp(-k^2 r_s^2); polynomial split the
// transform above (its series below u = 0.1, where the closed form cancels)
__device__ __forceinline__ double lr_window(double k2, double rs, int split, double rcut)
{
    if (split != 1) return exp(-k2 * rs * rs);
    const double u = sqrt(k2) * rcut, u2 = u * u;
    if (u < 0.1) return 1.0 - u2 / 14.0 + u2 * u2 / 504.0 - u2 * u2 * u2 / 33264.0;
    const double s = sin(u), c = cos(u);
    return 15.0 * (3.0 * s - 3.0 * u * c - u2 * s) / (u2 * u2 * u);
}

// a_k component `axis` from rho_k; includes the 1/M^3 of the inverse transform
__global__ void k_green_grad(const hipfftDoubleComplex *__restrict__ rhok, hipfftDoubleComplex *__restrict__ out,
                             int M, double box, double rs, int split, double rcut, double G, int axis, int order)
{
    int Mh = M / 2 + 1;
    size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t nc = (size_t)M * M * Mh;
    if (t >= nc) return;
    int kz = (int)(t % Mh), ky = (int)((t / Mh) % M), kx = (int)(t / ((size_t)Mh * M));
    int nx = kx <= M / 2 ? kx : kx - M, ny = ky <= M / 2 ? ky : ky - M, nz = kz;
    double twopi_L = 2.0 * M_PI / box, d = box / M;
    double k0 = nx * twopi_L, k1 = ny * twopi_L, k2 = nz * twopi_L;
    double k2s = k0 * k0 + k1 * k1 + k2 * k2;
    hipfftDoubleComplex r = rhok[t], o;
    if (k2s == 0.0 || (M % 2 == 0 && (nx == M / 2 || ny == M / 2 || nz == M / 2))) {
        o.x = 0; o.y = 0;  // k = 0 and the unpaired Nyquist planes carry no gradient
        out[t] = o;
        return;
    }
    const double s1 = sinc(0.5 * k0 * d) * sinc(0.5 * k1 * d) * sinc(0.5 * k2 * d);
    double W = s1;  // the assignment window: sinc^order per axis
    for (int o = 1; o < order; ++o) W *= s1;
    double phi = -4.0 * M_PI * G * lr_window(k2s, rs, split, rcut) / (k2s * W * W);
    double ka = axis == 0 ? k0 : (axis == 1 ? k1 : k2);
    double s = phi * ka / ((double)M * M * M);  // a_k = -i k phi_k
    o.x = s * r.y;
    o.y = -s * r.x;
    out[t] = o;
}

template <class S, int ORDER>
__global__ void k_interp(S src, int n, double box, int M, const double *__restrict__ am, double *__restrict__ acc)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    double inv_d = M / box;
    int i[3];
    double w[3][ORDER];
    for (int a = 0; a < 3; ++a) {
        double x = src.x(p, a);
        x -= box * floor(x / box);
        assign_weights<ORDER>(x, inv_d, M, i[a], w[a]);
    }
    size_t nr = (size_t)M * M * M;
    double g[3] = {0, 0, 0};
    for (int dx = 0; dx < ORDER; ++dx)
        for (int dy = 0; dy < ORDER; ++dy)
            for (int dz = 0; dz < ORDER; ++dz) {
                const double wt = w[0][dx] * w[1][dy] * w[2][dz];
                size_t idx = ((size_t)((i[0] + dx) % M) * M + (i[1] + dy) % M) * M + (i[2] + dz) % M;
                for (int a = 0; a < 3; ++a) g[a] += wt * am[a * nr + idx];
            }
    const size_t o = src.row(p);
    for (int a = 0; a < 3; ++a) acc[o + a] = g[a];
}

__global__ void k_add3(double *__restrict__ acc, const double *__restrict__ other, size_t n3)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n3) acc[i] += other[i];
}

__global__ void k_check_finite(const double *__restrict__ pos, size_t n3, int *bad)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n3 && !isfinite(pos[i])) *bad = 1;
}

template <class S>
static int pm_run(const fmm_params *P, int mesh, int n, S src, const double *pos_check, double *acc, hipStream_t st)
{
    PMPlan *pl;
    if (int rc = pm_plan(mesh, &pl)) return rc;
    std::lock_guard<std::mutex> lk(g_pm_mu);  // plans and mesh buffers are shared per mesh size
    size_t nr = (size_t)mesh * mesh * mesh, nc = (size_t)mesh * mesh * (mesh / 2 + 1);
    if (pos_check) {
        int *bad = ptr<int>(pl->amesh);  // scratch flag in the (not yet used) output mesh
        if (int rc = hip_check(hipMemsetAsync(bad, 0, sizeof(int), st), "pm check")) return rc;
        k_check_finite<<<(unsigned)((3 * (size_t)n + 255) / 256), 256, 0, st>>>(pos_check, 3 * (size_t)n, bad);
        int hbad = 0;
        if (hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return set_error(FMM_ERR_HIP, "pm sync");
        if (hbad) return set_error(FMM_ERR_NAN, "non-finite particle position");
    }
    if (int rc = hip_check(hipMemsetAsync(pl->rho.p, 0, nr * 8, st), "pm mesh")) return rc;
    double d = P->box / mesh;
    const int order = P->pm_assign == 0 ? 2 : P->pm_assign;
    const unsigned nb = (unsigned)((n + 255) / 256);
    const double inv_vol = 1.0 / (d * d * d);
    if (P->deterministic) {
        unsigned long long *mx = ptr<unsigned long long>(pl->amesh);  // the output mesh is not yet in use
        unsigned long long *irho = ptr<unsigned long long>(pl->rho);
        if (int rc = hip_check(hipMemsetAsync(mx, 0, 8, st), "pm mass bound")) return rc;
        k_mass_absmax<S><<<nb, 256, 0, st>>>(src, n, mx);
        if (order == 3) k_deposit_fixed<S, 3><<<nb, 256, 0, st>>>(src, n, P->box, mesh, inv_vol, mx, irho);
        else if (order == 4) k_deposit_fixed<S, 4><<<nb, 256, 0, st>>>(src, n, P->box, mesh, inv_vol, mx, irho);
        else k_deposit_fixed<S, 2><<<nb, 256, 0, st>>>(src, n, P->box, mesh, inv_vol, mx, irho);
        k_fixed_to_double<<<(unsigned)((nr + 255) / 256), 256, 0, st>>>(irho, nr, mx, n, inv_vol);
    } else if (order == 3) {
        k_deposit<S, 3><<<nb, 256, 0, st>>>(src, n, P->box, mesh, inv_vol, ptr<double>(pl->rho));
    } else if (order == 4) {
        k_deposit<S, 4><<<nb, 256, 0, st>>>(src, n, P->box, mesh, inv_vol, ptr<double>(pl->rho));
    } else {
        k_deposit<S, 2><<<nb, 256, 0, st>>>(src, n, P->box, mesh, inv_vol, ptr<double>(pl->rho));
    }
    if (hipfftSetStream(pl->r2c, st) != HIPFFT_SUCCESS || hipfftSetStream(pl->c2r, st) != HIPFFT_SUCCESS)
        return set_error(FMM_ERR_HIP, "hipfftSetStream");
    if (hipfftExecD2Z(pl->r2c, ptr<double>(pl->rho), ptr<hipfftDoubleComplex>(pl->rhok)) != HIPFFT_SUCCESS)
        return set_error(FMM_ERR_HIP, "hipfftExecD2Z");
    for (int axis = 0; axis < 3; ++axis) {
        k_green_grad<<<(unsigned)((nc + 255) / 256), 256, 0, st>>>(ptr<hipfftDoubleComplex>(pl->rhok),
                                                                  ptr<hipfftDoubleComplex>(pl->work), mesh, P->box,
                                                                  P->r_s, P->split, P->r_cut, P->G, axis, order);
        if (hipfftExecZ2D(pl->c2r, ptr<hipfftDoubleComplex>(pl->work), ptr<double>(pl->amesh) + axis * nr) !=
            HIPFFT_SUCCESS)
            return set_error(FMM_ERR_HIP, "hipfftExecZ2D");
    }
    if (order == 3) k_interp<S, 3><<<nb, 256, 0, st>>>(src, n, P->box, mesh, ptr<double>(pl->amesh), acc);
    else if (order == 4) k_interp<S, 4><<<nb, 256, 0, st>>>(src, n, P->box, mesh, ptr<double>(pl->amesh), acc);
    else k_interp<S, 2><<<nb, 256, 0, st>>>(src, n, P->box, mesh, ptr<double>(pl->amesh), acc);
    int rc = hip_check(hipGetLastError(), "pm");
    if (rc == 0) rc = hip_check(hipStreamSynchronize(st), "pm");  // mesh buffers are reused by the next call
    return rc;
}

int pm_forces(const fmm_params *P, int mesh, int64_t n64, const double *pos, const double *mass, double *acc,
              hipStream_t st)
{
    if (mesh < 8 || mesh > 1024) return set_error(FMM_ERR_ARG, "mesh must be in [8, 1024]");
    if (n64 < 0 || n64 > ((int64_t)1 << 30)) return set_error(FMM_ERR_ARG, "n out of range");
    const int n = (int)n64;
    if (n == 0) return 0;
    return pm_run(P, mesh, n, CallerOrder{pos, mass}, pos, acc, st);
}

// PM on the particles of a built tree (Morton order, already wrapped and checked).
int pm_forces_tree(const fmm_params *P, int mesh, fmm_tree *t, double *acc, hipStream_t st)
{
    if (mesh < 8 || mesh > 1024) return set_error(FMM_ERR_ARG, "mesh must be in [8, 1024]");
    if (t->n == 0) return 0;
    return pm_run(P, mesh, (int)t->n,
                  MortonOrder{ptr<double>(t->xs), ptr<double>(t->ys), ptr<double>(t->zs), ptr<double>(t->ms),
                              ptr<int>(t->perm)},
                  nullptr, acc, st);
}

int add_into(double *acc, const double *other, int64_t n3, hipStream_t st)
{
    if (n3 <= 0) return 0;
    k_add3<<<(unsigned)((n3 + 255) / 256), 256, 0, st>>>(acc, other, (size_t)n3);
    return hip_check(hipGetLastError(), "add");
}

}  // namespace hfmm
