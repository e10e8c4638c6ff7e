// Learned acceptance / order selector: training kernels (FP32 forward, softmax
// cross-entropy, backward, Adam), BF16 MFMA inference, model upload and loading, and
// the training-data entry point (candidate export + labels).
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "mlp.h"
#include "state.h"

namespace hfmm {

int run_labels(fmm_tree *t, const fmm_params *P, const double *aref_sorted, double eps, float *feats, int *labels,
               float *errs, int cap, int *dcounter, hipStream_t st);
int upward(fmm_tree *t, const fmm_params *P, hipStream_t st);

// ---------------------------------------------------------------------------
// model state (one model per process, on the device current at upload)

static std::mutex g_model_mu;
static MacModel g_hmodel;
static MacModel *g_dmodel = nullptr;
static bool g_have_model = false;
static uint64_t g_model_serial = 0;  // changes with every model set or cleared

uint64_t model_serial()
{
    std::lock_guard<std::mutex> lk(g_model_mu);
    return g_model_serial;
}

const MacModel *current_model(MacModel *host_copy)
{
    std::lock_guard<std::mutex> lk(g_model_mu);
    if (!g_have_model) return nullptr;
    if (host_copy) *host_copy = g_hmodel;
    return g_dmodel;
}

static short host_bf16(float x)
{
    uint32_t u;
    memcpy(&u, &x, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

// MFMA B-operand fragments: lane l holds W[k = 16 kc + 4 (l / 16) + r][j = 16 u + l % 16].
static void build_model(const float *w, const float *mu, const float *isd, double theta_max, int safety, MacModel &M)
{
    memset(&M, 0, sizeof(M));
    for (int u = 0; u < 4; ++u)
        for (int l = 0; l < 64; ++l)
            for (int r = 0; r < 4; ++r) {
                int k = 4 * (l / 16) + r, j = 16 * u + l % 16;
                M.w.w1[u][l][r] = host_bf16(w[kOffW1 + k * kHid + j]);
            }
    // 16x16x32 steps: K slot r of lane l in step kc multiplies the hidden unit that the
    // previous layer's output fragments leave there, 16 (2 kc + r / 4) + 4 (l / 16) + r % 4
    for (int kc = 0; kc < 2; ++kc)
        for (int u = 0; u < 4; ++u)
            for (int l = 0; l < 64; ++l)
                for (int r = 0; r < 8; ++r) {
                    int k = 16 * (2 * kc + r / 4) + 4 * (l / 16) + r % 4, j = 16 * u + l % 16;
                    M.w.w2[kc][u][l][r] = host_bf16(w[kOffW2 + k * kHid + j]);
                }
    for (int kc = 0; kc < 2; ++kc)
        for (int l = 0; l < 64; ++l)
            for (int r = 0; r < 8; ++r) {
                int k = 16 * (2 * kc + r / 4) + 4 * (l / 16) + r % 4, j = l % 16;
                M.w.w3[kc][l][r] = j < kCls ? host_bf16(w[kOffW3 + k * kCls + j]) : 0;
            }
    for (int j = 0; j < kHid; ++j) {
        M.w.b1[j] = w[kOffB1 + j];
        M.w.b2[j] = w[kOffB2 + j];
    }
    for (int j = 0; j < 16; ++j) M.w.b3[j] = j < kCls ? w[kOffB3 + j] : 0.0f;
    for (int k = 0; k < kFeat; ++k) {
        M.w.mu[k] = mu[k];
        M.w.isd[k] = isd[k];
    }
    M.theta_max = theta_max;
    M.safety = safety;
}

// ---------------------------------------------------------------------------
// training kernels (FP32)

__device__ __forceinline__ void fwd_one(const float *__restrict__ w, const float *xn, float *h1, float *h2, float *z)
{
    for (int j = 0; j < kHid; ++j) {
        float s = w[kOffB1 + j];
        for (int k = 0; k < kFeat; ++k) s += xn[k] * w[kOffW1 + k * kHid + j];
        h1[j] = fmaxf(s, 0.0f);
    }
    for (int j = 0; j < kHid; ++j) {
        float s = w[kOffB2 + j];
        for (int k = 0; k < kHid; ++k) s += h1[k] * w[kOffW2 + k * kHid + j];
        h2[j] = fmaxf(s, 0.0f);
    }
    for (int j = 0; j < kCls; ++j) {
        float s = w[kOffB3 + j];
        for (int k = 0; k < kHid; ++k) s += h2[k] * w[kOffW3 + k * kCls + j];
        z[j] = s;
    }
}

__global__ void k_mlp_fwd(const float *__restrict__ w, const float *__restrict__ mu, const float *__restrict__ isd,
                          const float *__restrict__ X, int B, float *__restrict__ Xn, float *__restrict__ H1,
                          float *__restrict__ H2, float *__restrict__ Z)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= B) return;
    float xn[kFeat], h1[kHid], h2[kHid], z[kCls];
    for (int k = 0; k < kFeat; ++k) xn[k] = (X[(size_t)s * kFeat + k] - mu[k]) * isd[k];
    fwd_one(w, xn, h1, h2, z);
    if (Xn)
        for (int k = 0; k < kFeat; ++k) Xn[(size_t)s * kFeat + k] = xn[k];
    if (H1)
        for (int k = 0; k < kHid; ++k) H1[(size_t)s * kHid + k] = h1[k];
    if (H2)
        for (int k = 0; k < kHid; ++k) H2[(size_t)s * kHid + k] = h2[k];
    for (int k = 0; k < kCls; ++k) Z[(size_t)s * kCls + k] = z[k];
}

// softmax cross-entropy with class weights, mean over the batch (weights sum).
// wsum_dev != nullptr: the weight sum is read from device memory (k_class_wsum), a label
// outside [0, kCls) has weight 0 and a zero weight sum gives zero loss and gradient.
__global__ void k_mlp_loss(const float *__restrict__ Z, const int *__restrict__ y, const float *__restrict__ cw, int B,
                           float wsum, const float *__restrict__ wsum_dev, float *__restrict__ dZ,
                           float *__restrict__ loss)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= B) return;
    float z[kCls], m = -3.0e38f;
    for (int k = 0; k < kCls; ++k) {
        z[k] = Z[(size_t)s * kCls + k];
        m = fmaxf(m, z[k]);
    }
    float se = 0.0f;
    for (int k = 0; k < kCls; ++k) se += expf(z[k] - m);
    int c = y[s];
    float wc;
    if (wsum_dev) {
        const float ws = *wsum_dev;
        const bool ok = c >= 0 && c < kCls && ws > 0.0f;
        wc = ok ? cw[c] / ws : 0.0f;
        c = ok ? c : 0;
    } else {
        wc = cw[c] / wsum;
    }
    atomicAdd(loss, wc * (logf(se) + m - z[c]));
    for (int k = 0; k < kCls; ++k) dZ[(size_t)s * kCls + k] = wc * (expf(z[k] - m) / se - (k == c ? 1.0f : 0.0f));
}

// Sum of the class weights of the batch's labels (labels outside [0, kCls) count 0),
// added into *wsum (which the caller cleared).
__global__ void k_class_wsum(const int *__restrict__ y, const float *__restrict__ cw, int B, float *__restrict__ wsum)
{
    float v = 0.0f;
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < B; s += gridDim.x * blockDim.x) {
        const int c = y[s];
        v += (c >= 0 && c < kCls) ? cw[c] : 0.0f;
    }
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(wsum, v);
}

// Sets n floats to zero (a kernel, not a memset: also valid inside a recorded graph).
__global__ void k_fill_zero(float *__restrict__ p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

__global__ void k_mlp_bwd_hidden(const float *__restrict__ w, const float *__restrict__ H1, const float *__restrict__ H2,
                                 const float *__restrict__ dZ, int B, float *__restrict__ dH1, float *__restrict__ dH2)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= B) return;
    float d2[kHid];
    for (int k = 0; k < kHid; ++k) {
        float v = 0.0f;
        for (int j = 0; j < kCls; ++j) v += dZ[(size_t)s * kCls + j] * w[kOffW3 + k * kCls + j];
        d2[k] = H2[(size_t)s * kHid + k] > 0.0f ? v : 0.0f;
        dH2[(size_t)s * kHid + k] = d2[k];
    }
    for (int k = 0; k < kHid; ++k) {
        float v = 0.0f;
        for (int j = 0; j < kHid; ++j) v += d2[j] * w[kOffW2 + k * kHid + j];
        dH1[(size_t)s * kHid + k] = H1[(size_t)s * kHid + k] > 0.0f ? v : 0.0f;
    }
}

// one thread per parameter: sum over the batch of input x output-gradient
__global__ void k_mlp_wgrad(const float *__restrict__ Xn, const float *__restrict__ H1, const float *__restrict__ H2,
                            const float *__restrict__ dH1, const float *__restrict__ dH2, const float *__restrict__ dZ,
                            int B, float *__restrict__ g)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kNParam) return;
    const float *in = nullptr, *dout = nullptr;
    int nin = 0, nout = 0, i = 0, j = 0;
    bool bias = false;
    if (p < kOffB1) { in = Xn; nin = kFeat; dout = dH1; nout = kHid; i = p / kHid; j = p % kHid; }
    else if (p < kOffW2) { dout = dH1; nout = kHid; j = p - kOffB1; bias = true; }
    else if (p < kOffB2) { in = H1; nin = kHid; dout = dH2; nout = kHid; i = (p - kOffW2) / kHid; j = (p - kOffW2) % kHid; }
    else if (p < kOffW3) { dout = dH2; nout = kHid; j = p - kOffB2; bias = true; }
    else if (p < kOffB3) { in = H2; nin = kHid; dout = dZ; nout = kCls; i = (p - kOffW3) / kCls; j = (p - kOffW3) % kCls; }
    else { dout = dZ; nout = kCls; j = p - kOffB3; bias = true; }
    float acc = 0.0f;
    for (int s = 0; s < B; ++s) acc += (bias ? 1.0f : in[(size_t)s * nin + i]) * dout[(size_t)s * nout + j];
    g[p] = acc;
}

__global__ void k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v,
                       int n, float lr, float b1, float b2, float eps, float wd, float c1, float c2)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    float gp = g[p] + wd * w[p];
    float mp = b1 * m[p] + (1.0f - b1) * gp;
    float vp = b2 * v[p] + (1.0f - b2) * gp * gp;
    m[p] = mp;
    v[p] = vp;
    w[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + eps);
}

// inference with the loaded model: 64 samples per wave, BF16 MFMA (as in the traversal)
__global__ __launch_bounds__(64) void k_mlp_infer(const MacModel *__restrict__ M, const float *__restrict__ X, int B,
                                                  float *__restrict__ Z)
{
    __shared__ short act[64 * 64];
    int s = blockIdx.x * 64 + threadIdx.x;
    float f[kFeat], lg[kCls];
    for (int k = 0; k < kFeat; ++k) f[k] = s < B ? X[(size_t)s * kFeat + k] : 0.0f;
    mlp_logits_wave(M->w, f, act, lg);
    if (s < B)
        for (int k = 0; k < kCls; ++k) Z[(size_t)s * kCls + k] = lg[k];
}

struct TrainScratch {
    DevBuf xn, h1, h2, z, dz, dh1, dh2;
};
static std::mutex g_train_mu;
static TrainScratch g_ts;

// Scratch of fmm_mlp_grad_noalloc: a fixed device array (one copy per GPU, held until the
// process ends) for the per-sample activations and gradients of at most kNoAllocMaxB
// samples, plus the class-weight sum.  Host code never passes the array's name to a
// kernel or copy: it uses the device address hipGetSymbolAddress returns for the device
// that is current, taken once per device.
constexpr int kNoAllocMaxB = 8192;
constexpr int kPerSample = kFeat + 4 * kHid + 2 * kCls;  // xn, h1, h2, dh1, dh2, z, dz
constexpr size_t kNoAllocFloats = (size_t)kNoAllocMaxB * kPerSample + 64;
static __device__ __align__(256) float scratch[kNoAllocFloats];
constexpr int kMaxDevices = 64;
static float *g_scratch_dev[kMaxDevices];
static std::mutex g_scratch_mu;

static int scratch_address(float **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return set_error(FMM_ERR_HIP, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return set_error(FMM_ERR_ARG, "device %d beyond the %d supported", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
            return set_error(FMM_ERR_HIP, "hipGetSymbolAddress of the training scratch");
        g_scratch_dev[dev] = static_cast<float *>(p);
    }
    *out = g_scratch_dev[dev];
    return 0;
}

}  // namespace hfmm

using namespace hfmm;

extern "C" {

int fmm_set_mac_model(const float *params, const float *mu, const float *isd, double theta_max, int safety)
{
    if (!params || !mu || !isd) {
        std::lock_guard<std::mutex> lk(g_model_mu);
        g_have_model = false;
        ++g_model_serial;
        return 0;
    }
    if (!(theta_max > 0) || !(theta_max < 0.75)) return set_error(FMM_ERR_ARG, "theta_max must be in (0, 0.75)");
    if (safety < 0 || safety > 6) return set_error(FMM_ERR_ARG, "safety must be in [0, 6]");
    MacModel M;
    build_model(params, mu, isd, theta_max, safety, M);
    std::lock_guard<std::mutex> lk(g_model_mu);
    if (!g_dmodel && hipMalloc(&g_dmodel, sizeof(MacModel)) != hipSuccess) {
        g_dmodel = nullptr;
        return set_error(FMM_ERR_NOMEM, "model allocation");
    }
    if (hipMemcpy(g_dmodel, &M, sizeof(M), hipMemcpyHostToDevice) != hipSuccess)
        return set_error(FMM_ERR_HIP, "model upload");
    g_hmodel = M;
    g_have_model = true;
    ++g_model_serial;
    return 0;
}

// File layout (little endian): "HFMMMAC1", int32 version (1), nfeat (16), hidden (64),
// nclass (8); double theta_max, eps_label; int32 safety, reserved; float mu[16], isd[16],
// params[5768] (FP32 master), adam_m[5768], adam_v[5768]; int64 step; int32 len; JSON.
int fmm_load_mac_model(const char *path)
{
    if (!path) return fmm_set_mac_model(nullptr, nullptr, nullptr, 0.0, 0);
    FILE *f = fopen(path, "rb");
    if (!f) return set_error(FMM_ERR_ARG, "cannot open model file %s", path);
    char magic[8];
    int hdr[4];
    double th[2];
    int sf[2];
    std::vector<float> mu(kFeat), isd(kFeat), w(kNParam);
    bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, "HFMMMAC1", 8) == 0 && fread(hdr, 4, 4, f) == 4 &&
              hdr[0] == 1 && hdr[1] == kFeat && hdr[2] == kHid && hdr[3] == kCls && fread(th, 8, 2, f) == 2 &&
              fread(sf, 4, 2, f) == 2 && fread(mu.data(), 4, kFeat, f) == (size_t)kFeat &&
              fread(isd.data(), 4, kFeat, f) == (size_t)kFeat && fread(w.data(), 4, kNParam, f) == (size_t)kNParam;
    fclose(f);
    if (!ok) return set_error(FMM_ERR_ARG, "%s is not a selector model file of this version", path);
    return fmm_set_mac_model(w.data(), mu.data(), isd.data(), th[0], sf[0]);
}

int fmm_mlp_forward(const float *params, const float *mu, const float *isd, const float *X, int B, float *logits,
                    void *stream)
{
    if (B < 0 || (B > 0 && (!params || !mu || !isd || !X || !logits))) return set_error(FMM_ERR_ARG, "bad arguments");
    if (B == 0) return 0;
    k_mlp_fwd<<<(B + 127) / 128, 128, 0, (hipStream_t)stream>>>(params, mu, isd, X, B, nullptr, nullptr, nullptr,
                                                                 logits);
    return hip_check(hipGetLastError(), "mlp forward");
}

int fmm_mlp_infer(const float *X, int B, float *logits, void *stream)
{
    if (B < 0 || (B > 0 && (!X || !logits))) return set_error(FMM_ERR_ARG, "bad arguments");
    const MacModel *M = current_model(nullptr);
    if (!M) return set_error(FMM_ERR_STATE, "no selector model loaded");
    if (B == 0) return 0;
    k_mlp_infer<<<(B + 63) / 64, 64, 0, (hipStream_t)stream>>>(M, X, B, logits);
    return hip_check(hipGetLastError(), "mlp infer");
}

int fmm_mlp_grad(const float *params, const float *mu, const float *isd, const float *X, const int *y,
                 const float *class_w, int B, float *grad, float *loss, void *stream)
{
    if (B <= 0 || !params || !mu || !isd || !X || !y || !class_w || !grad || !loss)
        return set_error(FMM_ERR_ARG, "bad arguments");
    hipStream_t st = (hipStream_t)stream;
    std::lock_guard<std::mutex> lk(g_train_mu);
    size_t b = (size_t)B;
    int rc = grow(g_ts.xn, b * kFeat * 4) | grow(g_ts.h1, b * kHid * 4) | grow(g_ts.h2, b * kHid * 4) |
             grow(g_ts.z, b * kCls * 4) | grow(g_ts.dz, b * kCls * 4) | grow(g_ts.dh1, b * kHid * 4) |
             grow(g_ts.dh2, b * kHid * 4);
    if (rc) return rc;
    std::vector<float> cw(kCls);
    if (hipMemcpy(cw.data(), class_w, kCls * 4, hipMemcpyDeviceToHost) != hipSuccess)
        return set_error(FMM_ERR_HIP, "class weights");
    std::vector<int> hy(B);
    if (hipMemcpy(hy.data(), y, b * 4, hipMemcpyDeviceToHost) != hipSuccess) return set_error(FMM_ERR_HIP, "labels");
    float wsum = 0.0f;
    for (int s = 0; s < B; ++s) wsum += cw[hy[s]];
    if (!(wsum > 0)) return set_error(FMM_ERR_ARG, "class weights sum to zero");
    if (int rc = hip_check(hipMemsetAsync(loss, 0, 4, st), "mlp loss")) return rc;
    unsigned nb = (unsigned)((B + 127) / 128);
    k_mlp_fwd<<<nb, 128, 0, st>>>(params, mu, isd, X, B, ptr<float>(g_ts.xn), ptr<float>(g_ts.h1), ptr<float>(g_ts.h2),
                                  ptr<float>(g_ts.z));
    k_mlp_loss<<<nb, 128, 0, st>>>(ptr<float>(g_ts.z), y, class_w, B, wsum, nullptr, ptr<float>(g_ts.dz), loss);
    k_mlp_bwd_hidden<<<nb, 128, 0, st>>>(params, ptr<float>(g_ts.h1), ptr<float>(g_ts.h2), ptr<float>(g_ts.dz), B,
                                         ptr<float>(g_ts.dh1), ptr<float>(g_ts.dh2));
    k_mlp_wgrad<<<(kNParam + 127) / 128, 128, 0, st>>>(ptr<float>(g_ts.xn), ptr<float>(g_ts.h1), ptr<float>(g_ts.h2),
                                                       ptr<float>(g_ts.dh1), ptr<float>(g_ts.dh2), ptr<float>(g_ts.dz),
                                                       B, grad);
    rc = hip_check(hipGetLastError(), "mlp grad");
    if (!rc) rc = hip_check(hipStreamSynchronize(st), "mlp grad");  // scratch is shared between calls
    return rc;
}

int fmm_mlp_grad_noalloc(const float *params, const float *mu, const float *isd, const float *X, const int *y,
                         const float *class_w, int B, float *grad, float *loss, void *stream)
{
    if (B <= 0 || !params || !mu || !isd || !X || !y || !class_w || !grad || !loss)
        return set_error(FMM_ERR_ARG, "bad arguments");
    if (B > kNoAllocMaxB)
        return set_error(FMM_ERR_ARG, "batch of %d exceeds the %d samples of the fixed scratch", B, kNoAllocMaxB);
    float *sc = nullptr;
    if (int rc = scratch_address(&sc)) return rc;
    hipStream_t st = (hipStream_t)stream;
    const size_t b = (size_t)B;
    float *xn = sc, *h1 = xn + b * kFeat, *h2 = h1 + b * kHid, *dh1 = h2 + b * kHid, *dh2 = dh1 + b * kHid,
          *z = dh2 + b * kHid, *dz = z + b * kCls;
    float *wsum = sc + (size_t)kNoAllocMaxB * kPerSample;  // past the largest batch's arrays
    const unsigned nb = (unsigned)((B + 127) / 128);
    k_fill_zero<<<1, 64, 0, st>>>(wsum, 1);
    k_fill_zero<<<1, 64, 0, st>>>(loss, 1);
    k_class_wsum<<<nb < 64 ? nb : 64, 128, 0, st>>>(y, class_w, B, wsum);
    k_mlp_fwd<<<nb, 128, 0, st>>>(params, mu, isd, X, B, xn, h1, h2, z);
    k_mlp_loss<<<nb, 128, 0, st>>>(z, y, class_w, B, 0.0f, wsum, dz, loss);
    k_mlp_bwd_hidden<<<nb, 128, 0, st>>>(params, h1, h2, dz, B, dh1, dh2);
    k_mlp_wgrad<<<(kNParam + 127) / 128, 128, 0, st>>>(xn, h1, h2, dh1, dh2, dz, B, grad);
    return hip_check(hipGetLastError(), "mlp grad (fixed scratch)");
}

int fmm_mlp_adam(float *params, const float *grad, float *m, float *v, int64_t step, float lr, float beta1, float beta2,
                 float eps, float weight_decay, void *stream)
{
    if (!params || !grad || !m || !v || step < 1) return set_error(FMM_ERR_ARG, "bad arguments");
    float c1 = 1.0f - powf(beta1, (float)step), c2 = 1.0f - powf(beta2, (float)step);
    k_adam<<<(kNParam + 255) / 256, 256, 0, (hipStream_t)stream>>>(params, grad, m, v, kNParam, lr, beta1, beta2, eps,
                                                                   weight_decay, c1, c2);
    return hip_check(hipGetLastError(), "adam");
}

}  // extern "C"
