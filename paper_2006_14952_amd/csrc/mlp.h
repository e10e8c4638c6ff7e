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

typedef short short4v __attribute__((ext_vector_type(4)));
typedef short short8v __attribute__((ext_vector_type(8)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef float float4v __attribute__((ext_vector_type(4)));

// The network as the inference reads it: BF16 MFMA A-operand fragments of the weights
// (see build_model), FP32 biases and feature normalisation.  Layer 1 (16 inputs) runs on
// the 16x16x16 BF16 MFMA, layers 2 and 3 (64 inputs) on the 16x16x32 one, two K steps
// each instead of four.
struct MlpWeights {
    short4v w1[4][64];      // [col tile][lane]
    short8v w2[2][4][64];   // [k chunk of 32][col tile][lane]
    short8v w3[2][64];      // [k chunk of 32][lane]
    float b1[64], b2[64], b3[16];
    float mu[kFeat], isd[kFeat];
};

// Device copy of a loaded model.
struct MacModel {
    MlpWeights w;
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

// Per-cell part of the features: the mass term of the (scaled) multipole and the norms of
// its degree-1, -2 and -3 parts (first 20 coefficients) relative to |mass|.
template <class T> __device__ __forceinline__ float4 cell_features(const T *MB)
{
    const float m0 = (float)MB[0];
    const float am0 = fabsf(m0) > 0.0f ? fabsf(m0) : 1e-30f;
    float n1 = 0, n2 = 0, n3 = 0;
    for (int k = 1; k < 4; ++k) n1 += (float)MB[k] * (float)MB[k];
    for (int k = 4; k < 10; ++k) n2 += (float)MB[k] * (float)MB[k];
    for (int k = 10; k < 20; ++k) n3 += (float)MB[k] * (float)MB[k];
    const float ia = 1.0f / am0;
    return make_float4(m0, sqrtf(n1) * ia, sqrtf(n2) * ia, sqrtf(n3) * ia);
}

// Features of a candidate pair (sink A, source B): size/separation ratios, separations in
// units of r_s, level difference, direction, scale of the sink, the low-order shape of the
// source multipole (cell_features of B) and the log of the mass ratio B : A.  mA0 is the
// mass term of A's multipole.
__device__ __forceinline__ void pair_features(const PairGeo &g, int la, int lb, double box, double rs, double rcut,
                                              double mA0, float4 cB, float *f)
{
    // geometry is exact in units u; the ratios are formed in FP32
    const float u = (float)ldexp(box, -(g.l + 1));
    const float Sc = sqrtf((float)g.sc2) * u, Sm = sqrtf((float)g.sm2) * u, SM = sqrtf((float)g.sM2) * u;
    const float hA = 2.0f * (float)g.wa * u, hB = 2.0f * (float)g.wb * u;
    const float L = fmaxf(hA, hB);
    const float Rm = fmaxf(fabsf((float)g.R[0]), fmaxf(fabsf((float)g.R[1]), fabsf((float)g.R[2]))) * u;
    const float irs = (float)(1.0 / rs), iSc = 1.0f / Sc;
    f[0] = L * iSc;
    f[1] = hA * iSc;
    f[2] = hB * iSc;
    f[3] = Sc * irs;
    f[4] = Sm * irs;
    f[5] = SM * irs;
    f[6] = (float)(rcut / rs);
    f[7] = (float)(la - lb);
    f[8] = Rm * iSc;
    f[9] = log2f(hA * irs);
    const float am0 = fabsf(cB.x) > 0.0f ? fabsf(cB.x) : 1e-30f;
    f[10] = cB.y;
    f[11] = cB.z;
    f[12] = cB.w;
    f[13] = logf(am0 / fmaxf((float)mA0, 1e-30f));
    f[14] = 0.0f;
    f[15] = 0.0f;
}

__device__ __forceinline__ short f2bf(float x)  // round to nearest even
{
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

typedef __bf16 bf2v __attribute__((ext_vector_type(2)));

// two FP32 values rounded to BF16 (nearest even, v_cvt_pk_bf16_f32), packed
__device__ __forceinline__ uint32_t pack_bf16(float a, float b)
{
    bf2v v = {(__bf16)a, (__bf16)b};
    return __builtin_bit_cast(uint32_t, v);
}

// ReLU(c + bias) of one output fragment, rounded to BF16 and packed as a B operand.
__device__ __forceinline__ short4v relu_pack(const float4v c, const float4 bias)
{
    const uint2 v = make_uint2(pack_bf16(fmaxf(c[0] + bias.x, 0.0f), fmaxf(c[1] + bias.y, 0.0f)),
                               pack_bf16(fmaxf(c[2] + bias.z, 0.0f), fmaxf(c[3] + bias.w, 0.0f)));
    return __builtin_bit_cast(short4v, v);
}

// Logits of the 64 pairs of a wave (one per lane; lanes without a pair take part with
// zero features).  `act` is 64 x 64 BF16 of LDS, `out` receives 8 logits per lane.
// MFMA operand layout (per lane l, lane group g = l/16): v_mfma_f32_16x16x16_bf16 takes
// A[i = l%16][k = 4g+r] and B[k = 4g+r][j = l%16], r = 0..3; v_mfma_f32_16x16x32_bf16 takes
// 8 values per lane, K slots (g, r), r = 0..7, paired between A and B the same way; both
// give D[i = 4g+r][j = l%16], r = 0..3.  Each layer computes the transposed product
// D = W^T act^T: the weight fragment is the A operand and the activations the B operand,
// so a lane ends with 4 consecutive outputs of one pair.  Row tile t holds pairs 16t .. 16t+15.
__device__ __forceinline__ bf8v cat_bf8(const short4v lo, const short4v hi)
{
    return __builtin_bit_cast(bf8v, __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7));
}

__device__ __forceinline__ void mlp_logits_wave(const MlpWeights &W, const float *fin, short *act, float *out)
{
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    {
        uint32_t pk[kFeat / 2];
#pragma unroll
        for (int k = 0; k < kFeat; k += 2)
            pk[k / 2] = pack_bf16((fin[k] - W.mu[k]) * W.isd[k], (fin[k + 1] - W.mu[k + 1]) * W.isd[k + 1]);
        uint4 *row = reinterpret_cast<uint4 *>(act + lane * 64);
        row[0] = make_uint4(pk[0], pk[1], pk[2], pk[3]);
        row[1] = make_uint4(pk[4], pk[5], pk[6], pk[7]);
    }
    __syncthreads();
    // The output fragment of a layer (4 consecutive outputs of one pair per lane) is laid
    // out as the next layer's B operand: two fragments side by side are the 8 K slots of a
    // 16x16x32 step (build_model orders the next layer's weights to match), so the hidden
    // activations stay in registers; only the input (one pair per lane) and the logits
    // (back to one pair per lane) pass through LDS.
    short4v h1[4][4];  // [pair tile t][output chunk u]
    {
        short4v a1[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) a1[t] = *reinterpret_cast<const short4v *>(act + (16 * t + li) * 64 + 4 * lk);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const short4v w = W.w1[u][lane];
            const float4 bias = *reinterpret_cast<const float4 *>(W.b1 + 16 * u + 4 * lk);
#pragma unroll
            for (int t = 0; t < 4; ++t)
                h1[t][u] = relu_pack(__builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w, a1[t], float4v{0, 0, 0, 0}, 0, 0, 0),
                                     bias);
        }
    }
    short4v h2[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        float4v c[4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
#pragma unroll
        for (int kc = 0; kc < 2; ++kc) {
            const bf8v w = __builtin_bit_cast(bf8v, W.w2[kc][u][lane]);
#pragma unroll
            for (int t = 0; t < 4; ++t)
                c[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, cat_bf8(h1[t][2 * kc], h1[t][2 * kc + 1]), c[t], 0, 0,
                                                               0);
        }
        const float4 bias = *reinterpret_cast<const float4 *>(W.b2 + 16 * u + 4 * lk);
#pragma unroll
        for (int t = 0; t < 4; ++t) h2[t][u] = relu_pack(c[t], bias);
    }
    // layer 3: 64 -> 8 (padded to 16 outputs)
    float4v c[4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
#pragma unroll
    for (int kc = 0; kc < 2; ++kc) {
        const bf8v w = __builtin_bit_cast(bf8v, W.w3[kc][lane]);
#pragma unroll
        for (int t = 0; t < 4; ++t)
            c[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, cat_bf8(h2[t][2 * kc], h2[t][2 * kc + 1]), c[t], 0, 0, 0);
    }
    __syncthreads();  // every lane has read its input rows before the logits overwrite them
    float *fout = reinterpret_cast<float *>(act);
    if (lk < 2) {  // classes 4 lk .. 4 lk + 3 of pair 16 t + li
        const float4 bias = *reinterpret_cast<const float4 *>(W.b3 + 4 * lk);
#pragma unroll
        for (int t = 0; t < 4; ++t)
            *reinterpret_cast<float4 *>(fout + (16 * t + li) * 8 + 4 * lk) =
                make_float4(c[t][0] + bias.x, c[t][1] + bias.y, c[t][2] + bias.z, c[t][3] + bias.w);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kCls; ++k) out[k] = fout[lane * 8 + k];
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
