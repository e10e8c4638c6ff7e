// Octree construction (the particle packs of Sec. 2.1, built as a Morton octree):
// wrap + 63-bit Morton keys, LSD radix sort (8-bit digits, stable), SoA gather, then
// cells level by level from the sorted keys.
#include <math.h>

#include "state.h"

namespace hfmm {

// ---------------------------------------------------------------------------
// keys

__device__ inline uint64_t spread3(uint32_t v)  // 21 bits -> every third bit
{
    uint64_t x = v & 0x1fffff;
    x = (x | x << 32) & 0x1f00000000ffffULL;
    x = (x | x << 16) & 0x1f0000ff0000ffULL;
    x = (x | x << 8) & 0x100f00f00f00f00fULL;
    x = (x | x << 4) & 0x10c30c30c30c30c3ULL;
    x = (x | x << 2) & 0x1249249249249249ULL;
    return x;
}

// Periodic wrap into [0, box) and the integer coordinate floor(x / box * 2^21).  The
// expression order (no contraction) fixes the rounding so that every implementation
// of the method assigns a particle to the same cube.
__device__ inline double wrap_coord(double x, double box)
{
#pragma clang fp contract(off)
    double v = x - box * floor(x / box);
    return v >= box ? 0.0 : v;
}

__device__ inline uint32_t grid_coord(double v, double box)
{
#pragma clang fp contract(off)
    double g = floor(v / box * 2097152.0);
    int c = (int)g;
    c = c < 0 ? 0 : c;
    c = c > 2097151 ? 2097151 : c;
    return (uint32_t)c;
}

__global__ void k_keys(const double *__restrict__ pos, int n, double box, uint64_t *__restrict__ keys,
                       uint32_t *__restrict__ idx, int *__restrict__ bad)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double x = pos[3 * (size_t)i], y = pos[3 * (size_t)i + 1], z = pos[3 * (size_t)i + 2];
    if (!isfinite(x) || !isfinite(y) || !isfinite(z)) {
        *bad = 1;
        x = y = z = 0.0;
    }
    uint32_t gx = grid_coord(wrap_coord(x, box), box), gy = grid_coord(wrap_coord(y, box), box),
             gz = grid_coord(wrap_coord(z, box), box);
    keys[i] = spread3(gx) << 2 | spread3(gy) << 1 | spread3(gz);
    idx[i] = (uint32_t)i;
}

// ---------------------------------------------------------------------------
// LSD radix sort, 8-bit digits.  A tile of 4096 keys per 256-thread block; each wave
// handles 1024 consecutive keys in 16 rounds of 64, ranking equal digits inside a
// round with ballots, so the scatter is stable.

constexpr int kRsThreads = 256;
constexpr int kRsRounds = 16;
constexpr int kRsTile = kRsThreads * kRsRounds;

// Box of original particle index v: the largest b with off[b] <= v (empty boxes skipped).
__device__ inline int box_of(const int *off, int nbox, uint32_t v)
{
    int lo = 0, hi = nbox - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= (int)v) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Radix digit of an element: 8 bits of the Morton key, or (for the passes that group the
// boxes of a batch) 8 bits of the box of its original index.
__device__ inline int rs_digit(uint64_t key, uint32_t val, int shift, const int *boxoff, int nbox)
{
    if (boxoff) return (box_of(boxoff, nbox, val) >> shift) & 0xff;
    return (int)((key >> shift) & 0xff);
}

__global__ __launch_bounds__(kRsThreads) void k_rs_hist(const uint64_t *__restrict__ keys,
                                                        const uint32_t *__restrict__ vals, int n, int shift,
                                                        const int *__restrict__ boxoff, int nbox, int nblocks,
                                                        int *__restrict__ hist)
{
    __shared__ int h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int base = blockIdx.x * kRsTile;
    for (int k = 0; k < kRsRounds; ++k) {
        int i = base + k * kRsThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[rs_digit(keys[i], vals[i], shift, boxoff, nbox)], 1);
    }
    __syncthreads();
    hist[threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Scatter of one tile: the keys are ranked by digit in registers (ballots, as before),
// placed in LDS in the tile's digit order, and written from there by consecutive threads, so
// each digit's run of the tile goes out as consecutive addresses (whole cache lines) rather
// than as one scattered 8-byte store per key.
__global__ __launch_bounds__(kRsThreads) void k_rs_scatter(const uint64_t *__restrict__ kin,
                                                           const uint32_t *__restrict__ vin, uint64_t *__restrict__ kout,
                                                           uint32_t *__restrict__ vout, int n, int shift,
                                                           const int *__restrict__ boxoff, int nbox, int nblocks,
                                                           const int *__restrict__ offs)
{
    __shared__ int cnt[4][256];
    __shared__ int boff[256];
    __shared__ int dstart[256];  // first slot of each digit in the tile ordered by digit
    __shared__ int wsum[4];
    __shared__ uint64_t skey[kRsTile];
    __shared__ uint32_t sval[kRsTile];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int k = threadIdx.x; k < 4 * 256; k += kRsThreads) (&cnt[0][0])[k] = 0;
    boff[threadIdx.x] = offs[threadIdx.x * nblocks + blockIdx.x];
    __syncthreads();
    const uint64_t lt = (1ull << lane) - 1ull;
    const int base = blockIdx.x * kRsTile + w * (kRsTile / 4);
    uint64_t key[kRsRounds];
    uint32_t val[kRsRounds];
    int pos[kRsRounds];
#pragma unroll
    for (int r = 0; r < kRsRounds; ++r) {
        int i = base + r * 64 + lane;
        bool ok = i < n;
        key[r] = ok ? kin[i] : 0;
        val[r] = ok ? vin[i] : 0;
        int d = rs_digit(key[r], val[r], shift, boxoff, nbox);
        uint64_t peers = __ballot(ok);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            uint64_t m = __ballot((d >> b) & 1);
            peers &= ((d >> b) & 1) ? m : ~m;
        }
        int old = cnt[w][d];
        int rank = __popcll(peers & lt);
        if (ok && rank == 0) cnt[w][d] = old + __popcll(peers);
        pos[r] = ok ? old + rank : -1;
    }
    __syncthreads();
    {  // per-digit prefix over the four waves, then over the digits (a block-wide scan)
        const int d = threadIdx.x;
        int run = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int c = cnt[q][d];
            cnt[q][d] = run;
            run += c;
        }
        const int incl = wave_incl_sum(run);
        if (lane == 63) wsum[w] = incl;
        __syncthreads();
        int add = 0;
        for (int q = 0; q < w; ++q) add += wsum[q];
        dstart[d] = add + incl - run;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRsRounds; ++r) {
        if (pos[r] < 0) continue;
        const int d = rs_digit(key[r], val[r], shift, boxoff, nbox);
        const int l = dstart[d] + cnt[w][d] + pos[r];
        skey[l] = key[r];
        sval[l] = val[r];
    }
    __syncthreads();
    const int ntile = min(kRsTile, n - blockIdx.x * kRsTile);
    for (int j = threadIdx.x; j < ntile; j += kRsThreads) {
        const uint64_t k = skey[j];
        const uint32_t v = sval[j];
        const int d = rs_digit(k, v, shift, boxoff, nbox);
        const int o = boff[d] + j - dstart[d];
        kout[o] = k;
        vout[o] = v;
    }
}

// Passes over the Morton key's digits first_digit .. 7, then (batches) 1 or 2 passes over
// the box index, so the order is by box, then by key; stable throughout.  Sorts the
// buffer pair t->sorted holds (t->sorted = 0 after k_keys) and sets t->sorted to the result.
static int radix_sort(fmm_tree *t, int n, int nbox, int first_digit, hipStream_t st)
{
    int nb = (n + kRsTile - 1) / kRsTile;
    if (int rc = grow(t->nch, (size_t)256 * nb * 2 * sizeof(int))) return rc;
    int *hist = ptr<int>(t->nch), *offs = hist + 256 * nb;
    const int *boxoff = ptr<int>(t->boxoff);
    int npass = 8 + (nbox > 1) + (nbox > 256);
    int cur = t->sorted;
    for (int pass = first_digit; pass < npass; ++pass) {
        bool bpass = pass >= 8;
        int shift = bpass ? 8 * (pass - 8) : 8 * pass;
        const int *bo = bpass ? boxoff : nullptr;
        k_rs_hist<<<nb, kRsThreads, 0, st>>>(ptr<uint64_t>(t->keys[cur]), ptr<uint32_t>(t->idx[cur]), n, shift, bo,
                                             nbox, nb, hist);
        if (int rc = scan_exclusive(hist, offs, 256 * nb, nullptr, st, t->scan_tmp)) return rc;
        k_rs_scatter<<<nb, kRsThreads, 0, st>>>(ptr<uint64_t>(t->keys[cur]), ptr<uint32_t>(t->idx[cur]),
                                                ptr<uint64_t>(t->keys[cur ^ 1]), ptr<uint32_t>(t->idx[cur ^ 1]), n,
                                                shift, bo, nbox, nb, offs);
        cur ^= 1;
    }
    t->sorted = cur;
    return hip_check(hipGetLastError(), "radix sort");
}

// ---------------------------------------------------------------------------
// gather into Morton order

__global__ void k_gather(const double *__restrict__ pos, const double *__restrict__ mass,
                         const uint32_t *__restrict__ idx, int n, double box, double *__restrict__ xs,
                         double *__restrict__ ys, double *__restrict__ zs, double *__restrict__ ms,
                         int *__restrict__ perm)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t j = idx[i];
    double x = pos[3 * (size_t)j], y = pos[3 * (size_t)j + 1], z = pos[3 * (size_t)j + 2];
    xs[i] = isfinite(x) ? wrap_coord(x, box) : 0.0;
    ys[i] = isfinite(y) ? wrap_coord(y, box) : 0.0;
    zs[i] = isfinite(z) ? wrap_coord(z, box) : 0.0;
    ms[i] = mass[j];
    perm[i] = (int)j;
}

// ---------------------------------------------------------------------------
// cells, level by level

// one root (level 0, the whole box) per box of the batch
__global__ void k_roots(Cell *cells, int nbox, const int *__restrict__ boxoff)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbox) return;
    Cell c;
    c.xln = pack_xln(0, 0, 0);
    c.iy = c.iz = 0;
    c.pad = 0;
    c.beg = boxoff[b];
    c.end = boxoff[b + 1];
    c.child = -1;
    c.parent = -1;
    cells[b] = c;
}

// Octant boundaries of a cell at level l: b[o] = first particle of octant o, b[8] = end.
// The seven lower bounds each search the whole particle range in lockstep (the interval
// length sequence depends on the range only), so their loads are in flight together:
// log2(n) dependent steps instead of seven times that.  Invariant per search: keys before
// base are below the target and the answer lies in [base, base + n].
__device__ inline void octant_bounds(const uint64_t *keys, const Cell &c, int l, int b[9])
{
    const int shift = 3 * (kMaxLevel - 1 - l);
    const uint64_t prefix = keys[c.beg] >> (shift + 3) << (shift + 3);
    int base[7];
    uint64_t tgt[7];
#pragma unroll
    for (int o = 0; o < 7; ++o) {
        base[o] = c.beg;
        tgt[o] = prefix | ((uint64_t)(o + 1) << shift);
    }
    int n = c.end - c.beg;  // >= 1: only cells with more than n_crit particles are split
    while (n > 1) {
        const int half = n >> 1;
#pragma unroll
        for (int o = 0; o < 7; ++o) base[o] = keys[base[o] + half] < tgt[o] ? base[o] + half : base[o];
        n -= half;
    }
    b[0] = c.beg;
#pragma unroll
    for (int o = 0; o < 7; ++o) b[o + 1] = base[o] + (keys[base[o]] < tgt[o] ? 1 : 0);
    b[8] = c.end;
}

// Level by level without host round trips: the cells of level l are lv[l] .. lv[l+1]-1
// in device memory, the cell array has room for `cap` cells, and *ovf is set (and every
// later level left empty) when a level would not fit; the host then rebuilds with room.
__global__ void k_level_init(int *__restrict__ lv, int nbox, int *__restrict__ ovf)
{
    if (threadIdx.x == 0) {
        lv[0] = 0;
        lv[1] = nbox;
        *ovf = 0;
    }
}

__global__ void k_count_children_dev(const Cell *__restrict__ cells, const int *__restrict__ lv, int l, int ncrit,
                                     const uint64_t *__restrict__ keys, int *__restrict__ nch,
                                     const int *__restrict__ ovf)
{
    if (*ovf) return;
    const int lbeg = lv[l], ln = lv[l + 1] - lbeg;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < ln; t += gridDim.x * blockDim.x) {
        Cell c = cells[lbeg + t];
        int k = 0;
        if (c.end - c.beg > ncrit && l < kMaxLevel) {
            int b[9];
            octant_bounds(keys, c, l, b);
            for (int o = 0; o < 8; ++o) k += b[o + 1] > b[o];
        }
        nch[t] = k;
    }
}

__global__ void k_make_children_dev(Cell *__restrict__ cells, const int *__restrict__ lv, int l, int ncrit,
                                    const uint64_t *__restrict__ keys, const int *__restrict__ off, int cap,
                                    int *__restrict__ ovf)
{
    if (*ovf) return;
    const int lbeg = lv[l], ln = lv[l + 1] - lbeg, nbeg = lv[l + 1];
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < ln; t += gridDim.x * blockDim.x) {
        const int ci = lbeg + t;
        Cell c = cells[ci];
        if (!(c.end - c.beg > ncrit && l < kMaxLevel)) continue;
        int b[9];
        octant_bounds(keys, c, l, b);
        int nk = 0;
        for (int o = 0; o < 8; ++o) nk += b[o + 1] > b[o];
        const int first = nbeg + off[t];
        if (first + nk > cap) {  // no room: the level is dropped and the tree rebuilt
            atomicOr(ovf, 1);
            continue;
        }
        int k = 0;
        for (int o = 0; o < 8; ++o) {
            if (b[o + 1] == b[o]) continue;
            Cell ch;
            ch.xln = pack_xln(2 * cell_ix(c) + ((o >> 2) & 1), l + 1, 0);
            ch.iy = 2 * c.iy + ((o >> 1) & 1);
            ch.iz = 2 * c.iz + (o & 1);
            ch.pad = 0;
            ch.beg = b[o];
            ch.end = b[o + 1];
            ch.child = -1;
            ch.parent = ci;
            cells[first + k] = ch;
            ++k;
        }
        c.child = first;
        c.xln = pack_xln(cell_ix(c), l, k);
        cells[ci] = c;
    }
}

// lv[l+2] = end of the next level; an overflowing level leaves the next one empty
__global__ void k_level_end(int *__restrict__ lv, int l, const int *__restrict__ total, int cap, int *__restrict__ ovf)
{
    if (threadIdx.x != 0) return;
    int e = lv[l + 1] + (*ovf ? 0 : *total);
    if (e > cap) {
        *ovf = 1;
        e = lv[l + 1];
    }
    if (*ovf) e = lv[l + 1];
    lv[l + 2] = e;
}

__global__ void k_leaf_flag(const Cell *__restrict__ cells, int ncell, int *__restrict__ flag)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < ncell) flag[c] = cell_nchild(cells[c]) == 0;
}

// Leaves before the first cell of each level (the exclusive leaf-flag scan at the level
// boundaries; the scan total past the last): the leaves of level l are
// leaves[out[l] .. out[l+1]-1], since cells, and so leaves, are stored level by level.
struct LevelBounds {
    int b[kMaxLevel + 2];
    int n;  // levels; b[0 .. n]
};

__global__ void k_leaf_levels(const int *__restrict__ off, int ncell, const int *__restrict__ total, LevelBounds lb,
                              int *__restrict__ out)
{
    const int l = threadIdx.x;
    if (l <= lb.n) out[l] = lb.b[l] < ncell ? off[lb.b[l]] : *total;
}

// Leaves and the cells with children, each in cell order (so level by level): a cell with
// children is number c - off[c] among them.
__global__ void k_leaf_compact(const Cell *__restrict__ cells, int ncell, const int *__restrict__ flag,
                               const int *__restrict__ off, int *__restrict__ leaves, int *__restrict__ inner,
                               int *__restrict__ leaf_of)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    if (!flag[c]) {
        inner[c - off[c]] = c;
        return;
    }
    leaves[off[c]] = c;
    Cell cc = cells[c];
    for (int i = cc.beg; i < cc.end; ++i) leaf_of[i] = c;
}

// FP32 particle records relative to the centre of their leaf (the FP32 form keeps FP64
// only for absolute positions and the exact cell-centre offsets).
__global__ void k_rel32(const Cell *__restrict__ cells, const int *__restrict__ leaf_of, const double *__restrict__ xs,
                        const double *__restrict__ ys, const double *__restrict__ zs, const double *__restrict__ ms,
                        int n, double box, float4 *__restrict__ rel)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Cell c = cells[leaf_of[i]];
    double h = ldexp(box, -cell_level(c));
    rel[i] = make_float4((float)(xs[i] - (cell_ix(c) + 0.5) * h), (float)(ys[i] - (c.iy + 0.5) * h),
                         (float)(zs[i] - (c.iz + 0.5) * h), (float)ms[i]);
}

static inline int blocks(int64_t n, int b) { return (int)((n + b - 1) / b); }

int tree_build(fmm_tree *t, const fmm_params *P, int64_t n64, const double *pos, const double *mass, int nbox,
               const int64_t *hoff, hipStream_t st)
{
    if (n64 < 0 || n64 > (int64_t)1 << 30) return set_error(FMM_ERR_ARG, "n = %lld out of range", (long long)n64);
    if (nbox < 1 || nbox > 65536) return set_error(FMM_ERR_ARG, "nbox = %d out of range", nbox);
    int n = (int)n64;
    t->n = n;
    t->box = P->box;
    t->ncrit = P->n_crit;
    const size_t nn = (size_t)(n > 0 ? n : 1);
    int rc = 0;
    for (int b = 0; b < 2 && !rc; ++b) rc = grow(t->keys[b], nn * 8) | grow(t->idx[b], nn * 4);
    if (!rc) rc = grow(t->xs, nn * 8) | grow(t->ys, nn * 8) | grow(t->zs, nn * 8) | grow(t->ms, nn * 8);
    if (!rc) rc = grow(t->perm, nn * 4) | grow(t->leaf_of, nn * 4) | grow(t->rel32, nn * 16) | grow(t->nearf, nn * 24);
    if (!rc) rc = grow(t->flag, 64 * sizeof(int));
    if (!rc) rc = grow(t->boxoff, (size_t)(nbox + 1) * 4);
    if (rc) return rc;
    t->nbox = nbox;
    t->hboxoff.resize(nbox + 1);
    for (int b = 0; b <= nbox; ++b) t->hboxoff[b] = hoff ? (int)hoff[b] : (b ? n : 0);
    if ((rc = hip_check(hipMemcpyAsync(t->boxoff.p, t->hboxoff.data(), (size_t)(nbox + 1) * 4, hipMemcpyHostToDevice, st),
                        "box offsets")))
        return rc;
    if (!t->host) {
        if (hipHostMalloc((void **)&t->host, kHostInts * sizeof(int), hipHostMallocDefault) != hipSuccess)
            return set_error(FMM_ERR_NOMEM, "pinned host buffer");
    }
    int *bad = ptr<int>(t->flag);
    if ((rc = hip_check(hipMemsetAsync(bad, 0, sizeof(int), st), "tree flags"))) return rc;
    // The sort starts at the key's third digit: bits 16 .. 62 order the particles exactly to
    // level 15 (a level-l octant is decided by key bits 3 (21 - l) .. 3 (21 - l) + 2).  Only
    // a tree that splits a level-15 cell needs the two lowest digits; the level loop then
    // stops at level 16, and the arrays are sorted again over every digit (a full LSD sort
    // of the partly sorted arrays) before the cells are built anew.
    constexpr int kPartialDigit = 2, kPartialLevels = 16;
    auto sort_gather = [&](int first_digit) -> int {
        if (int r = radix_sort(t, n, nbox, first_digit, st)) return r;
        k_gather<<<blocks(n, 256), 256, 0, st>>>(pos, mass, ptr<uint32_t>(t->idx[t->sorted]), n, P->box,
                                                 ptr<double>(t->xs), ptr<double>(t->ys), ptr<double>(t->zs),
                                                 ptr<double>(t->ms), ptr<int>(t->perm));
        return hip_check(hipGetLastError(), "tree sort");
    };
    bool partial = n > 0;
    if (n > 0) {
        t->sorted = 0;
        k_keys<<<blocks(n, 256), 256, 0, st>>>(pos, n, P->box, ptr<uint64_t>(t->keys[0]), ptr<uint32_t>(t->idx[0]), bad);
        if ((rc = sort_gather(kPartialDigit))) return rc;
    }
    if ((rc = hip_check(hipGetLastError(), "tree keys"))) return rc;

    // Cells level by level.  The level sizes stay on the device (lv); the host reads each
    // one back a level late through an event, only to stop the loop, so the GPU never
    // waits for it.  Room for `cap` cells: the previous tree's count or 8 n / n_crit,
    // four times more after an overflow.
    if (!t->bev_ready) {
        for (auto &e : t->bev)
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
                return set_error(FMM_ERR_HIP, "hipEventCreateWithFlags");
        t->bev_ready = true;
    }
    int *lv = bad + 8, *ovf = bad + 2;  // flag area: [0] non-finite, [1] scan total, [2] overflow, [8..] lv
    int *hl = t->host + kHostLevels;    // pinned mirror of lv
    const int nc_ = P->n_crit > 0 ? P->n_crit : 1;
    int launched = 0;
    for (;;) {  // once, or twice after a partial sort that does not reach deep enough
    const uint64_t *keys = ptr<uint64_t>(t->keys[t->sorted]);
    int64_t cap64 = (nc_ >= 2 ? 8 * (int64_t)n / nc_ : 4 * (int64_t)n) + 64 * (int64_t)nbox + 1024;
    if (t->ncell > 0) cap64 = cap64 > (int64_t)t->ncell * 5 / 4 + 1024 ? cap64 : (int64_t)t->ncell * 5 / 4 + 1024;
    const int lmax = partial ? kPartialLevels : kMaxLevel;
    for (int attempt = 0;; ++attempt) {
        if (cap64 > 0x7fffffff || attempt > 3) return set_error(FMM_ERR_NOMEM, "octree does not fit");
        const int cap = (int)cap64;
        if ((rc = grow(t->cells, sizeof(Cell) * (size_t)cap) | grow(t->nch, (size_t)cap * 2 * sizeof(int) + 64)))
            return rc;
        int *nch = ptr<int>(t->nch), *off = nch + cap;
        k_roots<<<blocks(nbox, 64), 64, 0, st>>>(ptr<Cell>(t->cells), nbox, ptr<int>(t->boxoff));
        k_level_init<<<1, 64, 0, st>>>(lv, nbox, ovf);
        hl[0] = 0;
        hl[1] = nbox;
        int64_t bound = nbox;  // the cells of level l are at most 8^l nbox (and cap)
        launched = 0;
        for (int l = 0; l < lmax && n > 0; ++l) {
            const int b = (int)bound, g = blocks(b, 256) < 4096 ? blocks(b, 256) : 4096;
            k_count_children_dev<<<g, 256, 0, st>>>(ptr<Cell>(t->cells), lv, l, P->n_crit, keys, nch, ovf);
            if ((rc = scan_exclusive_dn(nch, off, lv + l, lv + l + 1, b, bad + 1, st, t->scan_tmp))) return rc;
            k_make_children_dev<<<g, 256, 0, st>>>(ptr<Cell>(t->cells), lv, l, P->n_crit, keys, off, cap, ovf);
            k_level_end<<<1, 64, 0, st>>>(lv, l, bad + 1, cap, ovf);
            if ((rc = hip_check(hipMemcpyAsync(hl + l + 2, lv + l + 2, sizeof(int), hipMemcpyDeviceToHost, st),
                                "level size")) ||
                (rc = hip_check(hipEventRecord(t->bev[l], st), "event")))
                return rc;
            launched = l + 1;
            bound = bound * 8 < cap ? bound * 8 : cap;
            if (l >= 1) {  // the previous level's result: is level l (launched already) empty?
                if ((rc = hip_check(hipEventSynchronize(t->bev[l - 1]), "tree level"))) return rc;
                if (hl[l + 1] == hl[l]) break;
            }
        }
        if ((rc = hip_check(hipMemcpyAsync(t->host, bad, 3 * sizeof(int), hipMemcpyDeviceToHost, st), "tree flags")) ||
            (rc = hip_check(hipStreamSynchronize(st), "tree")))
            return rc;
        if (t->host[0]) return set_error(FMM_ERR_NAN, "non-finite particle position");
        if (!t->host[2]) break;
        cap64 *= 4;  // a level did not fit: rebuild with more room
    }
    if (partial && launched == kPartialLevels && hl[kPartialLevels + 1] > hl[kPartialLevels]) {
        partial = false;  // a level-15 cell splits: sort over every digit and build again
        if ((rc = sort_gather(0))) return rc;
        continue;
    }
    break;
    }
    t->lvl_beg.assign(1, 0);
    for (int l = 0; l <= launched && hl[l + 1] > hl[l]; ++l) t->lvl_beg.push_back(hl[l + 1]);
    t->nlevel = (int)t->lvl_beg.size() - 1;
    t->ncell = t->lvl_beg.back();
    if (t->ncell >= kMaxCells) {  // interaction-list entries hold the cell index in 27 bits
        const int nc = t->ncell;
        t->n = 0;  // the tree is unusable: later calls see an empty tree, never aliased entries
        t->ncell = t->nleaf = t->nlevel = 0;
        t->lvl_beg.assign(1, 0);
        t->leaf_lvl.assign(1, 0);
        t->stats.n = t->stats.n_cells = t->stats.n_leaves = t->stats.max_level = 0;
        return set_error(FMM_ERR_ARG, "octree of %d cells exceeds the %d cells an interaction-list entry can "
                                      "address (raise n_crit)", nc, kMaxCells - 1);
    }
    if (n == 0) {
        t->nleaf = 0;
        t->leaf_lvl.assign(t->nlevel + 1, 0);
        return hip_check(hipStreamSynchronize(st), "tree");
    }
    // leaves
    if ((rc = grow(t->nch, (size_t)t->ncell * 2 * sizeof(int) + 64))) return rc;
    int *flag = ptr<int>(t->nch), *off = flag + t->ncell;
    k_leaf_flag<<<blocks(t->ncell, 256), 256, 0, st>>>(ptr<Cell>(t->cells), t->ncell, flag);
    if ((rc = scan_exclusive(flag, off, t->ncell, bad + 1, st, t->scan_tmp))) return rc;
    if (t->nlevel > kMaxLevel + 1) return set_error(FMM_ERR_STATE, "octree deeper than %d levels", kMaxLevel + 1);
    LevelBounds lb;
    lb.n = t->nlevel;
    for (int l = 0; l <= t->nlevel; ++l) lb.b[l] = t->lvl_beg[l];
    int *hlev = bad + 32;  // flag area [32 ..]: leaves before each level
    k_leaf_levels<<<1, 64, 0, st>>>(off, t->ncell, bad + 1, lb, hlev);
    if ((rc = hip_check(hipMemcpyAsync(t->host, bad + 1, sizeof(int), hipMemcpyDeviceToHost, st), "leaf count")) ||
        (rc = hip_check(hipMemcpyAsync(t->host + 32, hlev, (size_t)(t->nlevel + 1) * sizeof(int),
                                       hipMemcpyDeviceToHost, st), "leaves per level")))
        return rc;
    if ((rc = hip_check(hipStreamSynchronize(st), "leaf count"))) return rc;
    t->nleaf = t->host[0];
    t->leaf_lvl.assign(t->host + 32, t->host + 32 + t->nlevel + 1);
    if ((rc = grow(t->leaves, (size_t)t->nleaf * 4 + 4) | grow(t->inner, (size_t)(t->ncell - t->nleaf) * 4 + 4))) return rc;
    k_leaf_compact<<<blocks(t->ncell, 256), 256, 0, st>>>(ptr<Cell>(t->cells), t->ncell, flag, off, ptr<int>(t->leaves),
                                                          ptr<int>(t->inner), ptr<int>(t->leaf_of));
    k_rel32<<<blocks(n, 256), 256, 0, st>>>(ptr<Cell>(t->cells), ptr<int>(t->leaf_of), ptr<double>(t->xs),
                                            ptr<double>(t->ys), ptr<double>(t->zs), ptr<double>(t->ms), n, P->box,
                                            ptr<float4>(t->rel32));
    return hip_check(hipGetLastError(), "tree leaves");
}

}  // namespace hfmm
