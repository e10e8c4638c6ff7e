// Error reporting, device buffer growth and a device-wide exclusive scan.
#include <stdarg.h>
#include <stdio.h>

#include <atomic>

#include "common.h"

namespace hfmm {

static thread_local char g_msg[512] = "";

int set_error(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_msg, sizeof(g_msg), fmt, ap);
    va_end(ap);
    return code;
}

const char *last_error() { return g_msg; }
void clear_error() { g_msg[0] = 0; }

int hip_check(hipError_t e, const char *what)
{
    if (e == hipSuccess) return 0;
    return set_error(FMM_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

static std::atomic<uint64_t> g_moves{0};
uint64_t buffer_moves() { return g_moves.load(std::memory_order_relaxed); }

// Bytes the library's device buffers hold (process-wide) and the caller's bound on them.
static std::atomic<uint64_t> g_used{0}, g_limit{0};
void set_memory_limit(uint64_t bytes) { g_limit.store(bytes, std::memory_order_relaxed); }
uint64_t memory_in_use() { return g_used.load(std::memory_order_relaxed); }

int grow(DevBuf &b, size_t bytes)
{
    if (bytes <= b.bytes) return 0;
    size_t want = bytes + bytes / 4 + 256;
    const uint64_t lim = g_limit.load(std::memory_order_relaxed);
    if (lim && memory_in_use() - b.bytes + want > lim)
        return set_error(FMM_ERR_NOMEM, "device buffers would hold %llu bytes, over the limit of %llu",
                         (unsigned long long)(memory_in_use() - b.bytes + want), (unsigned long long)lim);
    g_moves.fetch_add(1, std::memory_order_relaxed);  // a recorded graph may hold the old address
    void *p = nullptr;
    if (hipMalloc(&p, want) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(FMM_ERR_NOMEM, "hipMalloc of %zu bytes failed", want);
    }
    release(b);
    g_used.fetch_add(want, std::memory_order_relaxed);
    b.p = p;
    b.bytes = want;
    return 0;
}

void release(DevBuf &b)
{
    if (b.p) {
        (void)hipFree(b.p);
        g_used.fetch_sub(b.bytes, std::memory_order_relaxed);
    }
    b.p = nullptr;
    b.bytes = 0;
}

// Grow keeping the first `used` bytes.  The caller's stream must be idle.
int grow_keep(DevBuf &b, size_t bytes, size_t used)
{
    if (bytes <= b.bytes) return 0;
    DevBuf nb;
    if (int rc = grow(nb, bytes)) return rc;
    if (b.p && used) {
        if (hipMemcpy(nb.p, b.p, used, hipMemcpyDeviceToDevice) != hipSuccess) {
            release(nb);
            return set_error(FMM_ERR_HIP, "device copy while growing a buffer");
        }
    }
    release(b);
    b = nb;
    return 0;
}

// ---------------------------------------------------------------------------
// Zero fill by one-wave workgroups: these find room on a GPU filled by another stream's
// kernel, where the runtime's fill kernel (larger workgroups) waits for whole free CUs.

__global__ __launch_bounds__(64) void k_zero(uint4 *__restrict__ p, size_t n16, uint32_t *__restrict__ tail, int ntail)
{
    const size_t stride = (size_t)gridDim.x * 64;
    for (size_t i = (size_t)blockIdx.x * 64 + threadIdx.x; i < n16; i += stride) p[i] = make_uint4(0, 0, 0, 0);
    if (blockIdx.x == 0 && (int)threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

int zero_async(void *p, size_t bytes, hipStream_t st)
{
    if (bytes == 0) return 0;
    if ((reinterpret_cast<uintptr_t>(p) & 15) || (bytes & 3))
        return set_error(FMM_ERR_ARG, "zero fill: unaligned buffer or size");
    const size_t n16 = bytes / 16;
    const int ntail = (int)((bytes - n16 * 16) / 4);
    const size_t nb = (n16 + 63) / 64;
    const unsigned grid = (unsigned)(nb == 0 ? 1 : nb < 8192 ? nb : 8192);
    k_zero<<<grid, 64, 0, st>>>(static_cast<uint4 *>(p), n16, reinterpret_cast<uint32_t *>(static_cast<char *>(p) + n16 * 16),
                               ntail);
    return hip_check(hipGetLastError(), "zero fill");
}

// ---------------------------------------------------------------------------
// Exclusive scan of int32: block-local scans of 2048 elements, a recursive scan of
// the block totals, then a uniform add.  Totals fit in int32 by construction of the
// callers (list sizes are checked against 2^31 before use).

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ __forceinline__ void scan_tile_body(const int *__restrict__ in, int *__restrict__ out, int n,
                                               int *__restrict__ tile_sum)
{
    __shared__ int lds[kScanThreads];
    const int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int i = base + k;
        v[k] = i < n ? in[i] : 0;
        s += v[k];
    }
    lds[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {  // Hillis-Steele inclusive scan of thread sums
        int t = threadIdx.x >= off ? lds[threadIdx.x - off] : 0;
        __syncthreads();
        lds[threadIdx.x] += t;
        __syncthreads();
    }
    int run = lds[threadIdx.x] - s;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int i = base + k;
        if (i < n) out[i] = run;
        run += v[k];
    }
    if (threadIdx.x == kScanThreads - 1) tile_sum[blockIdx.x] = lds[threadIdx.x];
}

__global__ __launch_bounds__(kScanThreads) void k_scan_tile(const int *__restrict__ in, int *__restrict__ out, int n,
                                                            int *__restrict__ tile_sum)
{
    scan_tile_body(in, out, n, tile_sum);
}

// The same with n = *hi - *lo read on the device (grids sized for an upper bound of n);
// tiles past n report an empty sum.
__global__ __launch_bounds__(kScanThreads) void k_scan_tile_dn(const int *__restrict__ in, int *__restrict__ out,
                                                               const int *__restrict__ lo, const int *__restrict__ hi,
                                                               int *__restrict__ tile_sum)
{
    const int n = *hi - *lo;
    if ((int64_t)blockIdx.x * kScanTile >= n) {
        if (threadIdx.x == 0) tile_sum[blockIdx.x] = 0;
        return;
    }
    scan_tile_body(in, out, n, tile_sum);
}

__global__ void k_scan_add_dn(int *__restrict__ out, const int *__restrict__ lo, const int *__restrict__ hi,
                              const int *__restrict__ tile_off)
{
    const int n = *hi - *lo;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += tile_off[i / kScanTile];
}

__global__ void k_scan_total_dn(const int *__restrict__ in, const int *__restrict__ out, const int *__restrict__ lo,
                                const int *__restrict__ hi, int *__restrict__ total)
{
    const int n = *hi - *lo;
    *total = n > 0 ? out[n - 1] + in[n - 1] : 0;
}

__global__ void k_scan_add(int *__restrict__ out, int n, const int *__restrict__ tile_off)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += tile_off[i / kScanTile];
}

__global__ void k_scan_total(const int *__restrict__ in, const int *__restrict__ out, int n, int *__restrict__ total)
{
    *total = n > 0 ? out[n - 1] + in[n - 1] : 0;
}

static int scan_rec(const int *in, int *out, int n, hipStream_t st, int *tmp)
{
    int nt = (n + kScanTile - 1) / kScanTile;
    int *sums = tmp, *offs = tmp + nt;
    k_scan_tile<<<nt, kScanThreads, 0, st>>>(in, out, n, sums);
    if (nt > 1) {
        int rc = scan_rec(sums, offs, nt, st, tmp + 2 * nt);
        if (rc) return rc;
        k_scan_add<<<(n + 255) / 256, 256, 0, st>>>(out, n, offs);
    }
    return 0;
}

static size_t scan_tmp_ints(int n)
{
    size_t need = 4;
    for (int m = n; m > 1; m = (m + kScanTile - 1) / kScanTile) need += 2 * ((m + kScanTile - 1) / kScanTile);
    return need;
}

int scan_exclusive_dn(const int *in, int *out, const int *lo, const int *hi, int n_max, int *total, hipStream_t st,
                      DevBuf &tmp)
{
    if (n_max <= 0) return 0;
    if (int rc = grow(tmp, scan_tmp_ints(n_max) * sizeof(int))) return rc;
    const int nt = (n_max + kScanTile - 1) / kScanTile;
    int *sums = static_cast<int *>(tmp.p), *offs = sums + nt;
    k_scan_tile_dn<<<nt, kScanThreads, 0, st>>>(in, out, lo, hi, sums);
    if (nt > 1) {
        if (int rc = scan_rec(sums, offs, nt, st, sums + 2 * nt)) return rc;
        k_scan_add_dn<<<(n_max + 255) / 256, 256, 0, st>>>(out, lo, hi, offs);
    }
    if (total) k_scan_total_dn<<<1, 1, 0, st>>>(in, out, lo, hi, total);
    return hip_check(hipGetLastError(), "scan");
}

int scan_exclusive(const int *in, int *out, int n, int *total, hipStream_t st, DevBuf &tmp)
{
    if (n <= 0) {
        return total ? hip_check(hipMemsetAsync(total, 0, sizeof(int), st), "scan total") : 0;
    }
    size_t need = 0;
    for (int m = n; m > 1; m = (m + kScanTile - 1) / kScanTile) need += 2 * ((m + kScanTile - 1) / kScanTile);
    need += 4;
    if (int rc = grow(tmp, need * sizeof(int))) return rc;
    if (int rc = scan_rec(in, out, n, st, static_cast<int *>(tmp.p))) return rc;
    if (total) k_scan_total<<<1, 1, 0, st>>>(in, out, n, total);
    return hip_check(hipGetLastError(), "scan");
}

}  // namespace hfmm
