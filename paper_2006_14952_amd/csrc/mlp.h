// Learned acceptance / order selector: pair features and the MLP (16 -> 64 -> 64 -> 8,
// ReLU), shared by the training-data generator, the training kernels and the traversal.
//
// Classes: 0 = open the pair, c = 1..7 = accept with an M2L of order c + 1 (2..8).
// Parameter vector (FP32 master copy), row-major [in][out]:
//   W1 16x64 @0, b1 64 @1024, W2 64x64 @1088, b2 64 @5184, W3 64x8 @5248, b3 8 @5760.
#pragma once
#include "common.h"

namespace hfmm {

constexpr int kFeat = 16, kHid = 64, kCls = 8;
constexpr int kOffW1 = 0, kOffB1 = 1024, kOffW2 = 1088, kOffB2 = 5184, kOffW3 = 5248, kOffB3 = 5760;
constexpr int kNParam = 5768;

// Device copy of a loaded model: weights as BF16 MFMA B-operand fragments (see
// mlp_fragments), FP32 biases, feature normalisation and decoding constants.
struct MacModel {
    short w1f[4][64][4];        // [col tile][lane][4]
    short w2f[4][4][64][4];     // [k chunk][col tile][lane][4]
    short w3f[4][64][4];        // [k chunk][lane][4]   (8 classes padded to 16 columns)
    float b1[64], b2[64], b3[16];
    float mu[kFeat], isd[kFeat];
    double theta_max;           // pairs with L/S_c above this are always opened
    int safety;                 // orders added to the predicted one (0..)
    int pad;
};

// Pair geometry in units u = box / 2^(l+1) (l the finer level), exact in FP64.
struct PairGeo {
    double R[3], sc2, sm2, sM2, wa, wb;
    int l;
};

__device__ __forceinline__ PairGeo pair_geo(int4 a, int4 b, int s)
{
    PairGeo g;
    int la = xln_level(a.x), lb = xln_level(b.x);
    g.l = la > lb ? la : lb;
    g.wa = (double)(1 << (g.l - la));
    g.wb = (double)(1 << (g.l - lb));
    double half = g.wa + g.wb, img = (double)(2 << g.l);
    double sh[3] = {(double)(s / 9 - 1), (double)((s / 3) % 3 - 1), (double)(s % 3 - 1)};
    int ia[3] = {xln_ix(a.x), a.y, a.z}, ib[3] = {xln_ix(b.x), b.y, b.z};
    g.sc2 = g.sm2 = g.sM2 = 0.0;
    for (int i = 0; i < 3; ++i) {
        g.R[i] = (2.0 * ia[i] + 1.0) * g.wa - (2.0 * ib[i] + 1.0) * g.wb - sh[i] * img;
        double A = fabs(g.R[i]);
        double gm = fmax(A - half, 0.0), GM = A + half;
        g.sc2 += g.R[i] * g.R[i];
        g.sm2 += gm * gm;
        g.sM2 += GM * GM;
    }
    return g;
}

// Features of a candidate pair (see the learned-selector notes in the design notes):
// size/separation ratios, separations in units of r_s, level difference, direction,
// scale of the sink, and the low-order shape of the source multipole (scaled Mh_m,
// first 20 coefficients) relative to its mass.
template <class T>
__device__ __forceinline__ void pair_features(const PairGeo &g, int la, int lb, double box, double rs, double rcut,
                                              double mA0, const T *MB, float *f)
{
    double u = ldexp(box, -(g.l + 1));
    double Sc = sqrt(g.sc2) * u, Sm = sqrt(g.sm2) * u, SM = sqrt(g.sM2) * u;
    double hA = 2.0 * g.wa * u, hB = 2.0 * g.wb * u;
    double L = fmax(hA, hB);
    double Rm = fmax(fabs(g.R[0]), fmax(fabs(g.R[1]), fabs(g.R[2]))) * u;
    f[0] = (float)(L / Sc);
    f[1] = (float)(hA / Sc);
    f[2] = (float)(hB / Sc);
    f[3] = (float)(Sc / rs);
    f[4] = (float)(Sm / rs);
    f[5] = (float)(SM / rs);
    f[6] = (float)(rcut / rs);
    f[7] = (float)(la - lb);
    f[8] = (float)(Rm / Sc);
    f[9] = (float)log2(hA / rs);
    double m0 = (double)MB[0];
    double am0 = fabs(m0) > 0 ? fabs(m0) : 1e-300;
    double n1 = 0, n2 = 0, n3 = 0;
    for (int k = 1; k < 4; ++k) n1 += (double)MB[k] * MB[k];
    for (int k = 4; k < 10; ++k) n2 += (double)MB[k] * MB[k];
    for (int k = 10; k < 20; ++k) n3 += (double)MB[k] * MB[k];
    f[10] = (float)(sqrt(n1) / am0);
    f[11] = (float)(sqrt(n2) / am0);
    f[12] = (float)(sqrt(n3) / am0);
    f[13] = (float)log((am0 > 1e-300 ? am0 : 1e-300) / (mA0 > 1e-300 ? mA0 : 1e-300));
    f[14] = 0.0f;
    f[15] = 0.0f;
}

__device__ __forceinline__ short f2bf(float x)  // round to nearest even
{
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

typedef short short4v __attribute__((ext_vector_type(4)));
typedef float float4v __attribute__((ext_vector_type(4)));

// Logits of the 64 pairs of a wave (one per lane; lanes with valid == false still take
// part).  `act` is 64 x 64 BF16 of LDS, `out` receives 8 logits per lane.
// v_mfma_f32_16x16x16_bf16 operand layout (per lane l): A[i = l%16][k = 4(l/16)+r],
// B[k = 4(l/16)+r][j = l%16], D[i = 4(l/16)+r][j = l%16], r = 0..3.
__device__ __forceinline__ void mlp_logits_wave(const MacModel *__restrict__ M, const float *fin, short *act,
                                                float *out)
{
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    // features (normalised) -> act row `lane`, columns 0..15
    for (int k = 0; k < kFeat; ++k) act[lane * 64 + k] = f2bf((fin[k] - M->mu[k]) * M->isd[k]);
    __syncthreads();
    // layer 1: 16 -> 64, in place per row tile (row tile t reads only its own rows)
    for (int t = 0; t < 4; ++t) {
        short4v a;
        for (int r = 0; r < 4; ++r) a[r] = act[(16 * t + li) * 64 + 4 * lk + r];
        float4v c[4];
        for (int u = 0; u < 4; ++u) {
            short4v b;
            for (int r = 0; r < 4; ++r) b[r] = M->w1f[u][lane][r];
            c[u] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, float4v{0, 0, 0, 0}, 0, 0, 0);
        }
        __syncthreads();
        for (int u = 0; u < 4; ++u)
            for (int r = 0; r < 4; ++r)
                act[(16 * t + 4 * lk + r) * 64 + 16 * u + li] = f2bf(fmaxf(c[u][r] + M->b1[16 * u + li], 0.0f));
        __syncthreads();
    }
    // layer 2: 64 -> 64
    for (int t = 0; t < 4; ++t) {
        float4v c[4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
        for (int kc = 0; kc < 4; ++kc) {
            short4v a;
            for (int r = 0; r < 4; ++r) a[r] = act[(16 * t + li) * 64 + 16 * kc + 4 * lk + r];
            for (int u = 0; u < 4; ++u) {
                short4v b;
                for (int r = 0; r < 4; ++r) b[r] = M->w2f[kc][u][lane][r];
                c[u] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c[u], 0, 0, 0);
            }
        }
        __syncthreads();
        for (int u = 0; u < 4; ++u)
            for (int r = 0; r < 4; ++r)
                act[(16 * t + 4 * lk + r) * 64 + 16 * u + li] = f2bf(fmaxf(c[u][r] + M->b2[16 * u + li], 0.0f));
        __syncthreads();
    }
    // layer 3: 64 -> 8 (padded to 16); logits written as FP32 over the consumed row tile
    float *fout = reinterpret_cast<float *>(act);
    for (int t = 0; t < 4; ++t) {
        float4v c = {0, 0, 0, 0};
        for (int kc = 0; kc < 4; ++kc) {
            short4v a, b;
            for (int r = 0; r < 4; ++r) a[r] = act[(16 * t + li) * 64 + 16 * kc + 4 * lk + r];
            for (int r = 0; r < 4; ++r) b[r] = M->w3f[kc][lane][r];
            c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
        }
        __syncthreads();
        // row tile t occupies bytes [t*2048, (t+1)*2048) of act: 16 rows x 16 floats = 1 KB fits
        for (int r = 0; r < 4; ++r) fout[t * 512 + (4 * lk + r) * 16 + li] = c[r] + M->b3[li];
        __syncthreads();
    }
    const int t = lane >> 4, row = lane & 15;
    for (int k = 0; k < kCls; ++k) out[k] = fout[t * 512 + row * 16 + k];
    __syncthreads();
}

// Class -> M2L order (0 = open); the safety margin raises the order, capped at 8.
__device__ __forceinline__ int decode_order(const float *logit, int safety)
{
    int c = 0;
    for (int k = 1; k < kCls; ++k)
        if (logit[k] > logit[c]) c = k;
    if (c == 0) return 0;
    int p = c + 1 + safety;
    return p > 8 ? 8 : p;
}

}  // namespace hfmm
