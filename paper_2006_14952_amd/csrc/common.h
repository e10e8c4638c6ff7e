// Internal declarations shared by the HIP translation units of the solver.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hfmm.h"

namespace hfmm {

constexpr int kMaxLevel = FMM_MAXLEVEL;
constexpr int kPMax = FMM_PMAX;

// One octree cell: the cube [i h, (i+1) h)^3 with h = box / 2^level, holding the
// Morton-sorted particles beg..end-1.  Children are contiguous (child .. child+nchild-1)
// and ordered by octant 4 bx + 2 by + bz.  32 bytes; the first 16 hold everything the
// traversal needs (x index, level, number of children, y and z indices, first child).
struct __align__(16) Cell {
    int xln;      // ix | level << 21 | nchild << 26
    int iy, iz;
    int child;    // first child, -1 for a leaf
    int beg, end;
    int parent;   // -1 for the root
    int pad;
};

__host__ __device__ inline int pack_xln(int ix, int level, int nchild) { return ix | level << 21 | nchild << 26; }
__host__ __device__ inline int xln_ix(int v) { return v & 0x1fffff; }
__host__ __device__ inline int xln_level(int v) { return (v >> 21) & 31; }
__host__ __device__ inline int xln_nchild(int v) { return (v >> 26) & 15; }
__host__ __device__ inline int cell_ix(const Cell &c) { return xln_ix(c.xln); }
__host__ __device__ inline int cell_level(const Cell &c) { return xln_level(c.xln); }
__host__ __device__ inline int cell_nchild(const Cell &c) { return xln_nchild(c.xln); }

// Multi-indices n = (nx, ny, nz) with |n| <= p, ordered by degree, then nx descending,
// then ny descending: idx = d(d+1)(d+2)/6 + t(t+1)/2 + nz, d = |n|, t = ny + nz.
__host__ __device__ constexpr int ncoef(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }
__host__ __device__ constexpr int midx(int x, int y, int z)
{
    return (x + y + z) * (x + y + z + 1) * (x + y + z + 2) / 6 + (y + z) * (y + z + 1) / 2 + z;
}

// Traversal thresholds: every distance of a cell pair is an integer multiple of
// u_l = box / 2^(l+1), l the finer level of the pair.
struct MacConst {
    double cut2[kMaxLevel + 1];  // (r_cut / u_l)^2
    double theta2;
    int mode;
    int pad;
};

// Interaction lists are chains of kChunk-entry chunks (entry = source cell << 5 | image).
constexpr int kChunk = 64;
// A list entry keeps 27 bits for the cell index: a tree holds fewer cells than this.
constexpr int kMaxCells = 1 << 27;

// Per-call constants of the P2P force law in FP32: f_(1)(r) = -1/r^3 + S(t)/(8 r_s^3),
// t = 2 r^2 / r_cut^2 - 1, S a polynomial fitted on the host: of degree 9, 10 or 14, the
// lowest whose error in r^3 f_(1) stays below kP2PFitTol over [0, r_cut] (checked on the
// host at every fit, with the coefficients rounded to FP32; degree 9 serves r_cut up to
// about 4.6 r_s, 10 up to about 5.1 r_s, 14 up to 6 r_s: degree 12 also meets the
// tolerance there, but at 6 r_s its larger error, 5e-7 against 2e-7, put the force's p99
// against the FP64 oracle at 2.1e-5 and its maximum at 1.4e-3).  The two terms
// cancel as r^3 f_(1) = -(erfc(u) + 2u/sqrt(pi) e^(-u^2)), u = r/2r_s, falls towards r_cut:
// their FP32 rounding (about 1e-7 of 1/r^3) is 2e-5 of a pair's own force at a cutoff of
// 4.5 r_s, 2e-4 at 6 r_s and 5e-2 at 7 r_s, where particles whose force comes from pairs
// near the cutoff reach relative errors of 1e-2.  The FP32 form accepts r_cut <=
// kP2PMaxCut r_s.
constexpr int kP2PPolyMax = 15;
constexpr double kP2PFitTol = 1.0e-6;
constexpr double kP2PMaxCut = 6.0;
// The short range's truncation function: kind 0 the Gaussian split (scale = r_s), kind 1
// the polynomial split g(r/r_cut)/r (scale = r_cut).
struct Split {
    double scale;
    int kind;
};

struct P2PConst {
    float c[kP2PPolyMax];  // S(t) / (8 r_s^3), coefficients of t^0 .. t^(ncoef-1)
    int ncoef;             // 10, 11 or 15
    int split;             // 0: Gaussian split; 1: polynomial split (c[0] = 1 / r_cut, see p2p_setup)
    float two_over_rc2;
    float rc2;
    double rs, rc2d;
};

// ---------------------------------------------------------------------------
// Device buffers of one tree/evaluation.  Grown, never shrunk.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

int grow(DevBuf &b, size_t bytes);                    // 0 or FMM_ERR_NOMEM; content is lost
void release(DevBuf &b);                              // frees b (if held) and empties it
uint64_t buffer_moves();  // reallocations by grow() so far (process-wide): recorded graphs check it
void set_memory_limit(uint64_t bytes);  // bound on the bytes all DevBufs hold (0: none); grow() refuses beyond it
uint64_t memory_in_use();               // bytes all DevBufs hold now
int grow_keep(DevBuf &b, size_t bytes, size_t used);  // keeps the first `used` bytes
template <class T> inline T *ptr(DevBuf &b) { return static_cast<T *>(b.p); }

// error reporting (thread-local message)
int set_error(int code, const char *fmt, ...);
int hip_check(hipError_t e, const char *what);

// scans (int32), result is exclusive; total (device int) optional
int scan_exclusive(const int *in, int *out, int n, int *total, hipStream_t st, DevBuf &tmp);
int zero_async(void *p, size_t bytes, hipStream_t st);
// scan_exclusive of in[0 .. n), n = *hi - *lo read on the device, n <= n_max
int scan_exclusive_dn(const int *in, int *out, const int *lo, const int *hi, int n_max, int *total, hipStream_t st,
                      DevBuf &tmp);  // p 16-byte aligned, bytes a multiple of 4

// ---------------------------------------------------------------------------
// Inclusive scans over one 64-lane wave by DPP: shifts by 1, 2, 4 and 8 lanes within each
// row of 16, then lane 15 of rows 0 and 2 into rows 1 and 3, then lane 31 into rows 2
// and 3.  Lanes without a source lane take 0, the identity of both operations (the max
// is over non-negative values).  No LDS round trips.
__device__ __forceinline__ int wave_incl_sum(int vi)
{
    unsigned v = (unsigned)vi;
    v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return (int)v;
}

__device__ __forceinline__ int wave_incl_max(int vi)
{
    unsigned v = (unsigned)vi;  // unsigned: 0 is the identity, so each step fuses into one DPP max
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false));  // row_shr:1
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false));  // row_shr:2
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false));  // row_shr:4
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false));  // row_shr:8
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));  // row_bcast:15
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));  // row_bcast:31
    return (int)v;
}

// Workgroup order across the XCDs.  The workgroups of a launch are dealt to the 8 XCDs in
// turn (workgroup b to XCD b % 8), and each XCD has its own L2.  xcd_order(b, n) gives
// workgroup b of a grid of n a work position such that every XCD takes runs of kXcdRun
// consecutive positions (one run in every 8): consecutive work items (cells or leaves in
// Morton order, whose sources overlap) then share an L2, while every XCD still samples the
// whole range, so a dense region does not fall on one XCD.  Positions past the last whole
// round of 8 runs keep their own index.  A bijection of [0, n).  Measured against the plain
// order (same box, step ms; runs of 4 / 16 / 64 / 256 / 1024 tried): 2M box 9.05-9.16 ->
// 8.93-9.12, 64-box forest 12.13-12.36 -> 11.80-12.20, 16.7M box 75.2-77.7 -> 74.5-75.1,
// 134M box 690-695 -> 687 with runs of 64; runs of 1024 were slower than none.
constexpr int kXcds = 8;
constexpr int kXcdRun = 64;
__device__ __forceinline__ int xcd_order(int b, int n)
{
    const int full = n / (kXcds * kXcdRun) * (kXcds * kXcdRun);
    if (kXcdRun <= 1 || b >= full) return b;
    const int x = b % kXcds, i = b / kXcds;
    return ((i / kXcdRun) * kXcds + x) * kXcdRun + i % kXcdRun;
}

// The value of the previous lane (0 in lane 0): DPP wave_shr:1.
__device__ __forceinline__ int wave_shift_up1(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, false); }

}  // namespace hfmm
