// P2P: direct truncated interaction between a sink leaf and the leaves of its P2P list
// (Sec. 2.1 last paragraph; force law of Sec. 2.2):  a_i += m_j f_(1)(r) d, d = x_i - x_j - s box,
// counted iff 0 < r^2 < r_cut^2.
//
// One 64-lane wave per sink leaf.  The sources of up to 64 list entries form one stream
// of slots (a wave prefix sum over the entry sizes), staged 256 slots at a time in LDS.
// A sink of n_A <= C particles (the sink tile, C = 16, 32 or 64, default 32) is held
// floor(64 / n_A) times in the wave; copy g walks slots g, g + G, ... of the staged stream,
// and the copies are summed through LDS at the end.  Larger leaves are processed in
// Morton-ordered chunks of C sink particles, each culled against the box of its own
// particles: chunks of 32 against chunks of 64 culled by the leaf's box, 2M box 8.49 ->
// 7.83 ms at n_crit 48, 16.7M box 56.7 -> 51.6 ms and 134M box 480 -> 430 ms at n_crit 96
// (chunks of 16: 1% slower).
//
// FP64 form: absolute FP64 positions, erfc/exp from the device math library.
// FP32 form: FP32 coordinates relative to each particle's leaf centre, the exact
// centre offset c_B + s box - c_A added when staging, and
//   f_(1)(r) = -1/r^3 + S(t)/(8 r_s^3),  t = 2 r^2/r_cut^2 - 1,
// with S(t) = (4/sqrt(pi)) int_0^1 q^2 exp(-v q^2) dq (v = r^2/4r_s^2) replaced by a
// polynomial of degree 9, 10 or 14 fitted on the host, the lowest that meets the FP32
// tolerance at this r_cut / r_s <= 6 (its coefficients carry the factor 1/(8 r_s^3));
// the sum of each staged block is added to a Kahan-compensated per-particle accumulator.
// A listed source leaf whose particles' bounding box lies farther than r_cut from the sink
// leaf's box, and any single source particle farther than r_cut from that box, hold no
// pair inside the cutoff and are not staged (the lists themselves are unchanged).
#include <math.h>

#include <algorithm>
#include <mutex>
#include <type_traits>
#include <vector>

#include "expand_impl.h"

namespace hfmm {

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
    unsigned long long *pairs;  // listed particle pairs (sum of n_A n_B over P2P leaf pairs)
    unsigned long long *evaluated;  // particle pairs actually evaluated (FP32 form: after the box test)
    const float4 *bbox;             // per cell: lo, hi of the particles relative to the cell centre
    int first;                      // k_p2p: block b takes sink leaf leaves[first + b]
    const int *err;                 // k_p2p: if non-NULL and non-zero, the lists are void: do nothing
};

// Bounding box of each leaf's particles in the FP32 cell-relative frame.
__global__ void k_leaf_bbox(const Cell *__restrict__ cells, const int *__restrict__ leaves, int nleaf,
                            const float4 *__restrict__ rel, float4 *__restrict__ bbox)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nleaf) return;
    int c = leaves[t];
    Cell cc = cells[c];
    float lx = 0, ly = 0, lz = 0, hx = 0, hy = 0, hz = 0;
    if (cc.end > cc.beg) {
        float4 r = rel[cc.beg];
        lx = hx = r.x; ly = hy = r.y; lz = hz = r.z;
        for (int i = cc.beg + 1; i < cc.end; ++i) {
            r = rel[i];
            lx = fminf(lx, r.x); hx = fmaxf(hx, r.x);
            ly = fminf(ly, r.y); hy = fmaxf(hy, r.y);
            lz = fminf(lz, r.z); hz = fmaxf(hz, r.z);
        }
    }
    bbox[2 * (size_t)c] = make_float4(lx, ly, lz, 0.0f);
    bbox[2 * (size_t)c + 1] = make_float4(hx, hy, hz, 0.0f);
}

__device__ __forceinline__ void kahan_add(float &s, float &c, float v)
{
    float y = v - c;
    float t = s + y;
    c = (t - s) - y;
    s = t;
}

constexpr int kStage = 256;
// Sink particles per pass over a leaf's list unless fmm_params.p2p_chunk names 16 or 64: a
// leaf of more is processed in Morton-ordered chunks of this many, each tested against the
// box of its own particles.
constexpr int kSinkChunk = 32;

__device__ __forceinline__ float wave_minf(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ float wave_maxf(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

// POLY (FP32 form, polynomial split): f_(1) = -1/r^3 + 5/(2 r_c^3) - 3 r^2/(2 r_c^5) evaluated
// as -(1-x)^2 (1 + 2x + 3x^2 + 3x^3/2) / r^3, x = r / r_c: the three terms cancel near r_cut
// in FP32, the factored form does not.
// Shared memory of one sink leaf's P2P (one 64-lane wave).
template <bool F64> struct P2PShared {
    using R = typename std::conditional<F64, double, float>::type;
    using V4 = typename std::conditional<F64, double4, float4>::type;
    V4 src[kStage];
    int ebeg[64], epref[64];
    int smark[kStage];
    R eoff[64][3];
};

// P2P of sink leaf `leaves[li]`.
// CHUNK: the sink tile (16, 32 or 64 particles), a compile-time constant: a tile read at
// run time (from P2PConst, or as an extra kernel argument) changed the register allocation
// of the pair loop and cost 0.8-1.1% of the 134M box's P2P time.
template <bool F64, bool POLY, int NPC, int CHUNK>
__device__ __forceinline__ void p2p_leaf(const P2PArgs &a, const P2PConst &k, int li, P2PShared<F64> &sh)
{
    using R = typename std::conditional<F64, double, float>::type;
    using V4 = typename std::conditional<F64, double4, float4>::type;
    V4 *src = sh.src;
    int *ebeg = sh.ebeg, *epref = sh.epref, *smark = sh.smark;
    R(*eoff)[3] = sh.eoff;
    const int lane = threadIdx.x;
    const uint64_t lt = (1ull << lane) - 1ull;
    const int A = a.leaves[li];
    const Cell ca = a.cells[A];
    const double hA = ldexp(a.box, -cell_level(ca));
    const double cax = (cell_ix(ca) + 0.5) * hA, cay = (ca.iy + 0.5) * hA, caz = (ca.iz + 0.5) * hA;
    const int nA = ca.end - ca.beg;
    const int nlist = a.cnt[A];
    unsigned long long npairs = 0, nevald = 0;
    float4 alo = make_float4(0, 0, 0, 0), ahi = alo;
    if constexpr (!F64) {
        alo = a.bbox[2 * (size_t)A];
        ahi = a.bbox[2 * (size_t)A + 1];
    }

    for (int ib = 0; ib < nA; ib += CHUNK) {
        const int ns = min(CHUNK, nA - ib);
        const int G = 64 / ns, g = lane / ns, si = lane - g * ns;
        if constexpr (!F64) {
            if (nA > CHUNK) {  // one chunk of the leaf: the box of its own particles
                const float4 me = a.rel[ca.beg + ib + (lane < ns ? lane : 0)];
                alo = make_float4(wave_minf(me.x), wave_minf(me.y), wave_minf(me.z), 0.0f);
                ahi = make_float4(wave_maxf(me.x), wave_maxf(me.y), wave_maxf(me.z), 0.0f);
            }
        }
        const bool valid = g < G;
        const int i = ca.beg + ib + (valid ? si : 0);
        R xi, yi, zi;
        if constexpr (F64) {
            xi = a.xs[i]; yi = a.ys[i]; zi = a.zs[i];
        } else {
            float4 me = a.rel[i];
            xi = me.x; yi = me.y; zi = me.z;
        }
        double ax = 0, ay = 0, az = 0;              // FP64 form
        float sx = 0, sy = 0, sz = 0, cx = 0, cy = 0, cz = 0;  // FP32 form (Kahan)
        int chunk = a.head[A];
        for (int eb = 0; eb < nlist; eb += 64) {
            const int ne = min(64, nlist - eb);
            int cntj = 0, listed = 0;
            if (lane < ne) {
                uint32_t it = a.items[(size_t)chunk * kChunk + lane];
                int s = (int)(it & 31);
                Cell cb = a.cells[it >> 5];
                cntj = listed = cb.end - cb.beg;
                ebeg[lane] = cb.beg;
                double shx = (double)(s / 9 - 1) * a.box, shy = (double)((s / 3) % 3 - 1) * a.box,
                       shz = (double)(s % 3 - 1) * a.box;
                if constexpr (F64) {
                    eoff[lane][0] = shx; eoff[lane][1] = shy; eoff[lane][2] = shz;
                } else {  // exact in FP64: dyadic centres and integer image shifts
                    double hB = ldexp(a.box, -cell_level(cb));
                    const float ox = (float)((cell_ix(cb) + 0.5) * hB + shx - cax);
                    const float oy = (float)((cb.iy + 0.5) * hB + shy - cay);
                    const float oz = (float)((cb.iz + 0.5) * hB + shz - caz);
                    eoff[lane][0] = ox; eoff[lane][1] = oy; eoff[lane][2] = oz;
                    // gap between the two boxes; the margin covers FP32 rounding many times over
                    const float4 blo = a.bbox[2 * (size_t)(it >> 5)], bhi = a.bbox[2 * (size_t)(it >> 5) + 1];
                    const float gx = fmaxf(0.0f, fmaxf(alo.x - (bhi.x + ox), (blo.x + ox) - ahi.x));
                    const float gy = fmaxf(0.0f, fmaxf(alo.y - (bhi.y + oy), (blo.y + oy) - ahi.y));
                    const float gz = fmaxf(0.0f, fmaxf(alo.z - (bhi.z + oz), (blo.z + oz) - ahi.z));
                    if (gx * gx + gy * gy + gz * gz > k.rc2 * 1.0001f) cntj = 0;
                }
            }
            const int incl = wave_incl_sum(cntj);
            if (lane < ne) epref[lane] = incl - cntj;
            const int total = __builtin_amdgcn_readlane(incl, 63);
            const int ltot = F64 ? total : __builtin_amdgcn_readlane(wave_incl_sum(listed), 63);
            npairs += (unsigned long long)ns * (unsigned)ltot;
            __syncthreads();
            // FP32: the source records of a stage are loaded into registers one stage
            // ahead, so their latency is covered by the pair work of the current stage
            constexpr int kPer = kStage / 64;
            float4 rv[kPer];
            int ev[kPer];
            // slot -> list entry for the kStage slots from sbase: each entry marks the slot it
            // starts at (the largest entry wins, so entries left empty by the box test are
            // skipped), and a max-scan over the slots carries the marks forward.  Lane l
            // owns slots kPer l .. kPer l + kPer - 1.
            // ecarry: the entry holding the last slot fetched so far (it holds slot sbase
            // unless an entry starts there, which the marks then supply)
            int ecarry = 0;
            auto fetch = [&](int sbase) __attribute__((always_inline)) {
                const int nraw = min(kStage, total - sbase);
                const int efirst = ecarry;
#pragma unroll
                for (int u = 0; u < kPer; ++u) smark[kPer * lane + u] = 0;
                __syncthreads();
                if (lane < ne) {
                    const int st = epref[lane] - sbase;
                    if (st >= 0 && st < kStage) atomicMax(&smark[st], lane + 1);
                }
                __syncthreads();
                int mrun[kPer], m = 0;
#pragma unroll
                for (int u = 0; u < kPer; ++u) {
                    m = max(m, smark[kPer * lane + u]);
                    mrun[u] = m;
                }
                const int incl = wave_incl_max(m);
                const int prev = wave_shift_up1(incl);
                const int base = max(prev, efirst + 1);
#pragma unroll
                for (int u = 0; u < kPer; ++u) {
                    const int q = kPer * lane + u;
                    ev[u] = -1;
                    if (q < nraw) {
                        const int e = max(base, mrun[u]) - 1;
                        ev[u] = e;
                        rv[u] = a.rel[ebeg[e] + sbase + q - epref[e]];
                    }
                }
                ecarry = __builtin_amdgcn_readlane(ev[kPer - 1], 63);
            };
            if (!F64 && total > 0) fetch(0);
            for (int sb = 0; sb < total; sb += kStage) {
                const int nraw = min(kStage, total - sb);
                int nst = nraw;
                if constexpr (F64) {
                    for (int q = lane; q < nraw; q += 64) {
                        int slot = sb + q;
                        int e = find_entry(epref, ne, slot);
                        int j = ebeg[e] + slot - epref[e];
                        src[q] = make_double4(a.xs[j] + eoff[e][0], a.ys[j] + eoff[e][1], a.zs[j] + eoff[e][2], a.ms[j]);
                    }
                } else {
                    // a source particle farther than r_cut from the sink leaf's box meets no
                    // sink particle inside the cutoff: it is not staged (ballot compaction)
                    nst = 0;
#pragma unroll
                    for (int u = 0; u < kPer; ++u) {
                        bool keep = false;
                        float4 sv = make_float4(0, 0, 0, 0);
                        if (ev[u] >= 0) {
                            const int e = ev[u];
                            sv = make_float4(rv[u].x + eoff[e][0], rv[u].y + eoff[e][1], rv[u].z + eoff[e][2], rv[u].w);
                            const float gx = fmaxf(0.0f, fmaxf(alo.x - sv.x, sv.x - ahi.x));
                            const float gy = fmaxf(0.0f, fmaxf(alo.y - sv.y, sv.y - ahi.y));
                            const float gz = fmaxf(0.0f, fmaxf(alo.z - sv.z, sv.z - ahi.z));
                            keep = gx * gx + gy * gy + gz * gz <= k.rc2 * 1.0001f;
                        }
                        const uint64_t km = __ballot(keep);
                        if (keep) src[nst + __popcll(km & lt)] = sv;
                        nst += __popcll(km);
                    }
                    if (sb + kStage < total) fetch(sb + kStage);
                }
                nevald += (unsigned long long)ns * (unsigned)nst;
                __syncthreads();
                if (valid) {
                    if constexpr (F64) {
                        const double rc2 = k.rc2d, inv2rs = 0.5 / k.rs, c1 = 1.0 / (k.rs * 1.7724538509055160273);
                        const double irc2 = 1.0 / rc2, irc3 = irc2 / sqrt(rc2);
                        for (int q = g; q < nst; q += G) {
                            const double4 s = src[q];
                            double dx = xi - s.x, dy = yi - s.y, dz = zi - s.z;
                            double r2 = dx * dx + dy * dy + dz * dz;
                            bool in = r2 > 0.0 && r2 < rc2;
                            double rr2 = in ? r2 : 1.0;
                            double r = sqrt(rr2);
                            double w;
                            if (k.split == 1) {  // -1/r^3 + 5/(2 r_c^3) - 3 r^2/(2 r_c^5)
                                w = in ? s.w * (-1.0 / (rr2 * r) + irc3 * (2.5 - 1.5 * rr2 * irc2)) : 0.0;
                            } else {
                                double u = r * inv2rs;
                                double h = erfc(u) + r * c1 * exp(-u * u);
                                w = in ? -s.w * h / (rr2 * r) : 0.0;
                            }
                            ax += w * dx;
                            ay += w * dy;
                            az += w * dz;
                        }
                    } else {
                        float px = 0, py = 0, pz = 0;
                        // the leading coefficient as a vector operand: each Horner step then
                        // reads a single scalar
                        float clead = k.c[NPC - 1];
                        asm volatile("" : "+v"(clead));
                        auto pair = [&](const float4 s) __attribute__((always_inline)) {
                            const float dx = xi - s.x, dy = yi - s.y, dz = zi - s.z;
                            // a particle meets itself (and exact duplicates) at d = 0: the 1e-20
                            // added to r^2 keeps w finite, so w d = 0 without a separate r > 0
                            // test; for any other pair it is far below r^2's rounding
                            const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, 1e-20f)));
                            const float rinv = __frsqrt_rn(r2);
                            float f1;
                            if constexpr (POLY) {
                                const float x = r2 * rinv * k.c[0], omx = 1.0f - x;
                                const float q = fmaf(fmaf(fmaf(1.5f, x, 3.0f), x, 2.0f), x, 1.0f);
                                f1 = -(omx * omx) * q * (rinv * rinv * rinv);
                            } else {
                                const float t = fmaf(r2, k.two_over_rc2, -1.0f);
                                float S = clead;  // S(t) / (8 r_s^3)
#pragma unroll
                                for (int c = NPC - 2; c >= 0; --c) S = fmaf(S, t, k.c[c]);
                                f1 = fmaf(-rinv * rinv, rinv, S);
                            }
                            const float w = r2 < k.rc2 ? s.w * f1 : 0.0f;
                            px = fmaf(w, dx, px);
                            py = fmaf(w, dy, py);
                            pz = fmaf(w, dz, pz);
                        };
                        // four sources per step, read two at a time
                        const float4 *sp = reinterpret_cast<const float4 *>(src) + g;
                        const float4 *const send = reinterpret_cast<const float4 *>(src) + nst;
                        for (; sp + 3 * G < send; sp += 4 * G) {
                            const float4 s0 = sp[0], s1 = sp[G];
                            pair(s0);
                            pair(s1);
                            const float4 s2 = sp[2 * G], s3 = sp[3 * G];
                            pair(s2);
                            pair(s3);
                        }
                        for (; sp < send; sp += G) pair(sp[0]);
                        kahan_add(sx, cx, px);
                        kahan_add(sy, cy, py);
                        kahan_add(sz, cz, pz);
                    }
                }
                __syncthreads();
            }
            if (eb + 64 < nlist) chunk = a.next[chunk];
        }
        if constexpr (!F64) {
            ax = (double)sx - (double)cx;
            ay = (double)sy - (double)cy;
            az = (double)sz - (double)cz;
        }
        double(*red)[3] = reinterpret_cast<double(*)[3]>(&src[0]);  // staging area is free here
        red[lane][0] = ax;
        red[lane][1] = ay;
        red[lane][2] = az;
        __syncthreads();
        if (lane < ns) {
            double tx = 0, ty = 0, tz = 0;
            for (int q = 0; q < G; ++q) {
                tx += red[q * ns + lane][0];
                ty += red[q * ns + lane][1];
                tz += red[q * ns + lane][2];
            }
            int o = ca.beg + ib + lane;
            a.nearf[o] = tx;
            a.nearf[(size_t)a.n + o] = ty;
            a.nearf[2 * (size_t)a.n + o] = tz;
        }
        __syncthreads();
    }
    if (lane == 0) {
        atomicAdd(a.pairs, npairs);
        atomicAdd(a.evaluated, nevald);
    }
}

template <bool F64, bool POLY, int NPC, int CHUNK>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(F64 ? 2 : 5))) void k_p2p(P2PArgs a, P2PConst k)
{
    __shared__ P2PShared<F64> sh;
    if (a.err && *a.err) return;  // the traversal overflowed: it reruns, and so does P2P
    p2p_leaf<F64, POLY, NPC, CHUNK>(a, k, a.first + xcd_order(blockIdx.x, gridDim.x), sh);
}

// ---------------------------------------------------------------------------
// Persistent fused P2P + M2L (FP32, plain MAC): the grid holds as many 64-lane blocks as
// fit on the device at once; each block pulls items from one device counter until the
// queue is empty: first the sink leaves (P2P), then the 64-pair blocks of the flattened
// M2L array.  One launch covers both stages of every box of a forest, so no stage waits
// for the tail of another and no launch boundary falls between them.
template <bool POLY, int NPC, int P>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(P >= 7 ? 2 : (P >= 5 ? 3 : 4)))) void k_p2p_m2l_persist(
    P2PArgs a, P2PConst k, const int2 *__restrict__ pairs, int64_t npair, const float *__restrict__ M,
    float *__restrict__ L, Split sp, int stride, int *__restrict__ queue)
{
    __shared__ union {
        P2PShared<false> p;
        M2LPairShared<P, float> m;
    } sh;
    const int nleaf = a.nleaf;
    const int total = nleaf + (int)((npair + 63) / 64);
    for (;;) {
        int item = 0;
        if (threadIdx.x == 0) item = atomicAdd(queue, 1);
        item = __builtin_amdgcn_readfirstlane(__shfl(item, 0, 64));
        if (item >= total) break;
        if (item < nleaf) p2p_leaf<false, POLY, NPC, kSinkChunk>(a, k, item, sh.p);
        else m2l_pairs_block<P, float>(a.cells, pairs, npair, M, L, a.box, sp, stride, item - nleaf, sh.m);
        __syncthreads();  // the block's shared memory is reused by the next item
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

// Interpolation of S at the m Chebyshev points of t in [-1, 1] (solved in FP64), the
// coefficients of t^0 .. t^(m-1) returned in FP64.
static void fit_S(double vcut, int m, double *coef)
{
    double Amat[kP2PPolyMax][kP2PPolyMax + 1];
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
    for (int j = 0; j < m; ++j) coef[j] = Amat[j][m] / Amat[j][j];
}

// Largest error of the fit, with its coefficients rounded to FP32, in r^3 f_(1) = S u^3 - 1
// (u = r / 2 r_s): the pair force's error relative to the Newtonian one, on 4001 points.
static double fit_error(double vcut, int m, const double *coef)
{
    double worst = 0.0;
    for (int i = 0; i <= 4000; ++i) {
        const double t = -1.0 + i / 2000.0, v = (t + 1.0) * 0.5 * vcut;
        double S = (double)(float)coef[m - 1];
        for (int j = m - 2; j >= 0; --j) S = S * t + (double)(float)coef[j];
        const double e = fabs(S - S_of_v(v)) * v * sqrt(v);
        worst = e > worst ? e : worst;
    }
    return worst;
}

// Force-law constants.  FP32 form, Gaussian split: the lowest polynomial length of 10, 11, 15 whose
// checked error is at most kP2PFitTol; returns FMM_ERR_ARG for r_cut > kP2PMaxCut r_s (FP32
// cancellation near the cutoff) or if no fit meets the tolerance.  The last fit is cached
// (same vcut, same result).
int p2p_setup(const fmm_params *P, P2PConst &k)
{
    static std::mutex mu;
    static double cached_vcut = -1.0;
    static int cached_m = 0;
    static double cached[kP2PPolyMax];
    const double vcut = (P->r_cut * P->r_cut) / (4.0 * P->r_s * P->r_s);
    double coef[kP2PPolyMax] = {0};
    int m = 0;
    if (P->precision == 1 && P->split == 0) {  // the FP64 form evaluates erfc/exp: no fit, no limit
        if (P->r_cut > kP2PMaxCut * P->r_s)
            return set_error(FMM_ERR_ARG, "precision 1 supports r_cut <= %.0f r_s (r_cut / r_s = %.3g): beyond it the "
                                          "FP32 pair force loses accuracy near the cutoff; use precision 0",
                             kP2PMaxCut, P->r_cut / P->r_s);
        std::lock_guard<std::mutex> lk(mu);
        if (vcut != cached_vcut) {
            cached_m = 0;
            for (int mm : {10, 11, 15}) {
                fit_S(vcut, mm, cached);
                if (fit_error(vcut, mm, cached) <= kP2PFitTol) {
                    cached_m = mm;
                    break;
                }
            }
            cached_vcut = vcut;
        }
        m = cached_m;
        for (int j = 0; j < m; ++j) coef[j] = cached[j];
        if (m == 0)
            return set_error(FMM_ERR_ARG, "precision 1: no polynomial of degree <= 14 meets the FP32 force-law "
                                          "tolerance at r_cut / r_s = %.3g; use precision 0", P->r_cut / P->r_s);
    }
    // the kernel evaluates S(t) / (8 r_s^3): the factor is folded into the coefficients
    const double inv8rs3 = 1.0 / (8.0 * P->r_s * P->r_s * P->r_s);
    for (int j = 0; j < kP2PPolyMax; ++j) k.c[j] = j < m ? (float)(coef[j] * inv8rs3) : 0.0f;
    k.ncoef = m > 0 ? m : 11;
    k.split = P->split;
    if (P->split == 1) k.c[0] = (float)(1.0 / P->r_cut);  // polynomial split: the FP32 kernel needs 1 / r_cut only
    k.two_over_rc2 = (float)(2.0 / (P->r_cut * P->r_cut));
    k.rc2 = (float)(P->r_cut * P->r_cut);
    k.rs = P->r_s;
    k.rc2d = P->r_cut * P->r_cut;
    return 0;
}



// The FP32 form's leaf bounding boxes (they depend on the tree only).
int p2p_bbox(fmm_tree *t, const fmm_params *P, hipStream_t st)
{
    if (t->nleaf == 0 || !P->precision) return 0;
    if (int rc = grow(t->bbox, (size_t)t->ncell * 32)) return rc;
    k_leaf_bbox<<<(t->nleaf + 63) / 64, 64, 0, st>>>(ptr<Cell>(t->cells), ptr<int>(t->leaves), t->nleaf,
                                                    ptr<float4>(t->rel32), ptr<float4>(t->bbox));
    return hip_check(hipGetLastError(), "leaf boxes");
}

static void p2p_args(fmm_tree *t, P2PArgs &a)
{
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
    a.pairs = ptr<unsigned long long>(t->counters) + 1;
    a.evaluated = ptr<unsigned long long>(t->counters) + 24;
    a.bbox = ptr<float4>(t->bbox);
    a.first = 0;
    a.err = nullptr;
}

// Whether the fused persistent kernel serves these parameters: the FP32 plain form with
// the pair M2L kernel (orders 3..8) and a force law of degree 9 or 10, or the polynomial split.
bool fused_applies(const fmm_params *P)
{
    if (P->precision != 1 || P->learned || P->p < 3 || P->m2l_mfma == 2) return false;
    if (P->split == 1) return true;
    P2PConst k;
    return p2p_setup(P, k) == 0 && (k.ncoef == 10 || k.ncoef == 11);
}

template <bool POLY, int NPC, int P> static int launch_persist(fmm_tree *t, const P2PArgs &a, const P2PConst &k, Split sp,
                                                      int64_t np, int *queue, hipStream_t st)
{
    static int per_cu = 0, ncu = 0;
    if (per_cu == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_p2p_m2l_persist<POLY, NPC, P>, 64, 0) != hipSuccess ||
            per_cu <= 0)
            return set_error(FMM_ERR_HIP, "occupancy of the fused kernel");
    }
    const int64_t items = (int64_t)t->nleaf + (np + 63) / 64;
    const int64_t g = std::min<int64_t>(items, (int64_t)per_cu * ncu);
    if (g <= 0) return 0;
    k_p2p_m2l_persist<POLY, NPC, P><<<(unsigned)g, 64, 0, st>>>(a, k, ptr<int2>(t->m2l_pairs), np, ptr<float>(t->Mc),
                                                          ptr<float>(t->Lc), sp, ncoef(P), queue);
    return hip_check(hipGetLastError(), "fused p2p + m2l");
}

// P2P and M2L of a built tree (or forest) in one persistent launch on `st`.  The
// preparation (L zeroed, the M2L list flattened, the queue counter zeroed) is its own call
// so that stage timing can bracket the launch alone.
int p2p_m2l_fused_prepare(fmm_tree *t, const fmm_params *P, hipStream_t st)
{
    if (t->nleaf == 0) return 0;
    if (t->bbox.bytes < (size_t)t->ncell * 32) return set_error(FMM_ERR_STATE, "p2p: leaf boxes not computed");
    const int64_t np = t->n_m2l;
    if (int rc = zero_async(t->Lc.p, (size_t)t->ncell * ncoef(P->p) * sizeof(float), st)) return rc;
    if (np > 0)
        if (int rc = flatten_pairs(t, 0, np, st)) return rc;
    if (int rc = grow(t->m2l_ctr, 256)) return rc;
    return zero_async(ptr<int>(t->m2l_ctr) + 32, 4, st);
}

int p2p_m2l_fused_launch(fmm_tree *t, const fmm_params *P, hipStream_t st)
{
    if (t->nleaf == 0) return 0;
    P2PConst k;
    if (int rc = p2p_setup(P, k)) return rc;
    const int64_t np = t->n_m2l;
    int *queue = ptr<int>(t->m2l_ctr) + 32;
    P2PArgs a;
    p2p_args(t, a);
    const Split sp{P->split ? P->r_cut : P->r_s, P->split};
    if (P->split == 1) {
        switch (P->p) {
        case 3: return launch_persist<true, 11, 3>(t, a, k, sp, np, queue, st);
        case 4: return launch_persist<true, 11, 4>(t, a, k, sp, np, queue, st);
        case 5: return launch_persist<true, 11, 5>(t, a, k, sp, np, queue, st);
        case 6: return launch_persist<true, 11, 6>(t, a, k, sp, np, queue, st);
        case 7: return launch_persist<true, 11, 7>(t, a, k, sp, np, queue, st);
        case 8: return launch_persist<true, 11, 8>(t, a, k, sp, np, queue, st);
        }
    } else if (k.ncoef == 10) {
        switch (P->p) {
        case 3: return launch_persist<false, 10, 3>(t, a, k, sp, np, queue, st);
        case 4: return launch_persist<false, 10, 4>(t, a, k, sp, np, queue, st);
        case 5: return launch_persist<false, 10, 5>(t, a, k, sp, np, queue, st);
        case 6: return launch_persist<false, 10, 6>(t, a, k, sp, np, queue, st);
        case 7: return launch_persist<false, 10, 7>(t, a, k, sp, np, queue, st);
        case 8: return launch_persist<false, 10, 8>(t, a, k, sp, np, queue, st);
        }
    } else if (k.ncoef == 11) {
        switch (P->p) {
        case 3: return launch_persist<false, 11, 3>(t, a, k, sp, np, queue, st);
        case 4: return launch_persist<false, 11, 4>(t, a, k, sp, np, queue, st);
        case 5: return launch_persist<false, 11, 5>(t, a, k, sp, np, queue, st);
        case 6: return launch_persist<false, 11, 6>(t, a, k, sp, np, queue, st);
        case 7: return launch_persist<false, 11, 7>(t, a, k, sp, np, queue, st);
        case 8: return launch_persist<false, 11, 8>(t, a, k, sp, np, queue, st);
        }
    }
    return set_error(FMM_ERR_ARG, "fused kernel compiled for orders 3..8 and force laws of degree 9 or 10");
}

template <int CHUNK>
static void launch_p2p(const fmm_params *P, const P2PConst &k, const P2PArgs &a, int count, hipStream_t st)
{
    if (P->precision && P->split == 1) k_p2p<false, true, 11, CHUNK><<<count, 64, 0, st>>>(a, k);
    else if (P->precision && k.ncoef == 10) k_p2p<false, false, 10, CHUNK><<<count, 64, 0, st>>>(a, k);
    else if (P->precision && k.ncoef == 11) k_p2p<false, false, 11, CHUNK><<<count, 64, 0, st>>>(a, k);
    else if (P->precision) k_p2p<false, false, 15, CHUNK><<<count, 64, 0, st>>>(a, k);
    else k_p2p<true, false, 11, CHUNK><<<count, 64, 0, st>>>(a, k);
}

int p2p_range(fmm_tree *t, const fmm_params *P, int first, int count, const int *err, hipStream_t st)
{
    if (count <= 0) return 0;
    if (first < 0 || count > t->nleaf - first) return set_error(FMM_ERR_STATE, "p2p: leaf range out of bounds");
    P2PConst k;
    if (int rc = p2p_setup(P, k)) return rc;
    P2PArgs a;
    p2p_args(t, a);
    a.first = first;
    a.err = err;
    if (P->precision) {
        if (t->bbox.bytes < (size_t)t->ncell * 32) return set_error(FMM_ERR_STATE, "p2p: leaf boxes not computed");
    } else {
        a.bbox = nullptr;
    }
    if (P->precision && k.split != 1 && k.ncoef != 10 && k.ncoef != 11 && k.ncoef != 15)
        return set_error(FMM_ERR_STATE, "p2p: no kernel for a force law of %d coefficients", k.ncoef);
    if (P->p2p_chunk == 16) launch_p2p<16>(P, k, a, count, st);
    else if (P->p2p_chunk == 64) launch_p2p<64>(P, k, a, count, st);
    else launch_p2p<kSinkChunk>(P, k, a, count, st);
    return hip_check(hipGetLastError(), "p2p");
}

int p2p(fmm_tree *t, const fmm_params *P, hipStream_t st) { return p2p_range(t, P, 0, t->nleaf, nullptr, st); }

}  // namespace hfmm
