// M2L (Sec. 2.1, Eq. (3)) as dense contractions on the matrix cores (FP32 MFMA).
//
// For a pair of cells on one level the transfer is  Lh_n(A) += sum_m Dh_{n+m}(R) Mh_m(B),
// with R = c_A - c_B - s box in units of the cell side: an integer vector.  Every pair with
// the same level and the same R shares the matrix T_{nm} = Dh_{n+m}(R) (block triangular,
// |n| + |m| <= p), so the pairs of one R form a product  L[:, sinks] += T M[:, sources].
//
// Work layout:
//  * the M2L list is split: pairs of two cells on one level (at level <= 15, where R fits
//    the sort key) go to this kernel, laid out by sink (CSR); every other pair goes to the
//    lane-per-pair VALU kernel;
//  * a workgroup (4 waves) takes a window of 64 consecutive sinks and keeps their local
//    expansions in LDS; the window's pairs are sorted by (level, R) in LDS (bitonic), and
//    each run of equal keys is cut into tiles of up to 16 pairs (the 16 columns of a
//    v_mfma_f32_16x16x4f32 product);
//  * per tile: the derivative tensor Dh(R) is built once (one lane per tile, 16 tiles at a
//    time, into LDS), the 16 source multipoles are the B operand, T is gathered from the
//    tensor in LDS as the A operand, 16-row blocks of outputs times 4-deep slices of
//    sources, only the blocks that hold a term with |n| + |m| <= p;
//  * the tile's outputs are added into the window's LDS expansions (LDS atomics), and the
//    window writes them out once.
#include "expand_impl.h"

namespace hfmm {

constexpr int kMfWin = 64;         // sinks per window (local expansions resident in LDS)
constexpr int kMfSort = 2048;      // pairs sorted at a time (a window's pairs in chunks)
constexpr int kMfBatch = 16;       // tiles whose tensors one wave builds at a time
constexpr int kMfMaxLevel = 15;    // R components fit 17 bits below this level

typedef float v4f __attribute__((ext_vector_type(4)));

// Which M2L pairs the matrix-core kernel takes: both cells on one level, at most 15.
__device__ __forceinline__ bool mf_eligible(int4 a, int4 b)
{
    const int la = xln_level(a.x);
    return la == xln_level(b.x) && la <= kMfMaxLevel;
}

// ---------------------------------------------------------------------------
// Contraction plan for order P: 16-row output blocks (outputs ordered by degree), each
// needing source coefficients m with |m| <= P - (lowest degree in the block), taken 4 at a
// time.  Per product q: its row block, its slice, and for every lane the index of the
// tensor entry it supplies (n + m), or NC (a zero) where |n| + |m| > P or out of range.
template <int P> constexpr int mf_rows() { return (ncoef(P) + 15) / 16; }
template <int P> constexpr int mf_steps(int rt)
{
    Tab<P> T{};
    const int d0 = T.d[16 * rt];
    return (ncoef(P - d0) + 3) / 4;
}
template <int P> constexpr int mf_products()
{
    int q = 0;
    for (int rt = 0; rt < mf_rows<P>(); ++rt) q += mf_steps<P>(rt);
    return q;
}

// Row block and slice of each product (compile-time: they index register arrays).
template <int P> struct MfSteps {
    static constexpr int NC = ncoef(P), NRT = mf_rows<P>(), NQ = mf_products<P>(), NS0 = (NC + 3) / 4;
    short rt[NQ], s[NQ];
    constexpr MfSteps() : rt(), s()
    {
        int q = 0;
        for (int r = 0; r < NRT; ++r)
            for (int st = 0; st < mf_steps<P>(r); ++st) {
                rt[q] = (short)r;
                s[q] = (short)st;
                ++q;
            }
    }
};

// The tensor index each lane supplies to each product (read once per wave at run time).
template <int P> struct MfAidx {
    static constexpr int NC = ncoef(P), NRT = mf_rows<P>(), NQ = mf_products<P>();
    short a[NQ][64];
    constexpr MfAidx() : a()
    {
        Tab<P> T{};
        int q = 0;
        for (int r = 0; r < NRT; ++r)
            for (int st = 0; st < mf_steps<P>(r); ++st) {
                for (int l = 0; l < 64; ++l) {
                    const int n = 16 * r + l % 16, m = 4 * st + l / 16;
                    short v = (short)NC;
                    if (n < NC && m < NC && T.d[n] + T.d[m] <= P)
                        v = (short)midx(T.x[n] + T.x[m], T.y[n] + T.y[m], T.z[n] + T.z[m]);
                    a[q][l] = v;
                }
                ++q;
            }
    }
};

template <int P> __device__ const MfAidx<P> g_mf_aidx{};

// sort key: level (4 bits) and R + 2^16 per axis (18 bits each); unused slots sort last
__device__ __forceinline__ uint64_t mf_key(int level, int rx, int ry, int rz)
{
    return (uint64_t)level << 54 | (uint64_t)(rx + 65536) << 36 | (uint64_t)(ry + 65536) << 18 | (uint64_t)(rz + 65536);
}
__device__ __forceinline__ void mf_unkey(uint64_t k, int &level, int &rx, int &ry, int &rz)
{
    level = (int)(k >> 54);
    rx = (int)((k >> 36) & 0x3ffff) - 65536;
    ry = (int)((k >> 18) & 0x3ffff) - 65536;
    rz = (int)(k & 0x3ffff) - 65536;
}

// LDS ordering between the lanes of one wave (the waves of the workgroup run different
// tile counts, so a workgroup barrier cannot be used there).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int P> struct MfShared {
    static constexpr int NC = ncoef(P);
    float L[kMfWin][NC];                       // the window's local expansions
    uint64_t key[kMfSort];
    unsigned short idx[kMfSort];               // chunk position of the sorted pair
    unsigned char pj[kMfSort];                 // window sink of the pair (by chunk position)
    uint32_t pit[kMfSort];                     // list entry of the pair (by chunk position)
    unsigned short tstart[kMfSort];
    unsigned char tcnt[kMfSort];
    float D[4][kMfBatch][NC + 1];              // per wave: tensors of a batch of tiles (+ a zero)
    int sink[kMfWin];
    int poff[kMfWin + 1];
    int ntile;
};

template <int P>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_m2l_mfma(
    const Cell *__restrict__ cells, const int4 *__restrict__ cellc, const int *__restrict__ sinks,
    const int *__restrict__ nsink_dev, const int *__restrict__ offe, const int *__restrict__ ne,
    const uint32_t *__restrict__ csr, const float *__restrict__ M, float *__restrict__ L, double box, Split sp)
{
    constexpr int NC = ncoef(P), NRT = MfSteps<P>::NRT, NQ = MfSteps<P>::NQ, NS0 = MfSteps<P>::NS0;
    constexpr MfSteps<P> cs{};
    __shared__ MfShared<P> sh;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int nsink = *nsink_dev;
    const int w0 = blockIdx.x * kMfWin;
    if (w0 >= nsink) return;
    const int nsw = min(kMfWin, nsink - w0);

    // the window's sinks and the offsets of their pairs (contiguous in the CSR array)
    if (wv == 0) {
        const int A = lane < nsw ? sinks[w0 + lane] : -1;
        const int c = A >= 0 ? ne[A] : 0;
        const int incl = wave_incl_sum(c);
        sh.sink[lane] = A;
        sh.poff[lane] = incl - c;
        if (lane == 63) sh.poff[kMfWin] = incl;
    }
    for (int k = tid; k < kMfWin * NC; k += 256) (&sh.L[0][0])[k] = 0.0f;
    // this lane's tensor index of every product (loop invariant), two per register
    int apk[(NQ + 1) / 2];
#pragma unroll
    for (int q = 0; q < NQ; q += 2) {
        int v = g_mf_aidx<P>.a[q][lane];
        if (q + 1 < NQ) v |= (int)g_mf_aidx<P>.a[q + 1][lane] << 16;
        apk[q / 2] = v;
    }
    __syncthreads();
    const int npair = sh.poff[kMfWin];
    const int64_t base = offe[sh.sink[0]];

    for (int cb = 0; cb < npair; cb += kMfSort) {
        const int cnt = min(kMfSort, npair - cb);
        // keys of the chunk's pairs
        for (int q = tid; q < kMfSort; q += 256) {
            uint64_t key = ~0ull;
            if (q < cnt) {
                const int p = cb + q;
                int lo = 0, hi = nsw - 1;  // sink j of window pair p: largest j with poff[j] <= p
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (sh.poff[mid] <= p) lo = mid;
                    else hi = mid - 1;
                }
                const uint32_t it = csr[base + p];
                const int4 ga = cellc[sh.sink[lo]], gb = cellc[it >> 5];
                const int s = (int)(it & 31), lev = xln_level(ga.x), img = 1 << lev;
                const int rx = xln_ix(ga.x) - xln_ix(gb.x) - (s / 9 - 1) * img;
                const int ry = ga.y - gb.y - ((s / 3) % 3 - 1) * img;
                const int rz = ga.z - gb.z - (s % 3 - 1) * img;
                key = mf_key(lev, rx, ry, rz);
                sh.pj[q] = (unsigned char)lo;
                sh.pit[q] = it;
            }
            sh.key[q] = key;
            sh.idx[q] = (unsigned short)q;
        }
        __syncthreads();
        // bitonic sort of the chunk by key (unused slots carry the largest key)
        for (int k = 2; k <= kMfSort; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int i = tid; i < kMfSort; i += 256) {
                    const int pr = i ^ j;
                    if (pr > i) {
                        const uint64_t a = sh.key[i], b = sh.key[pr];
                        const bool up = (i & k) == 0;
                        if ((a > b) == up) {
                            sh.key[i] = b;
                            sh.key[pr] = a;
                            const unsigned short t = sh.idx[i];
                            sh.idx[i] = sh.idx[pr];
                            sh.idx[pr] = t;
                        }
                    }
                }
                __syncthreads();
            }
        }
        // tiles: runs of equal keys cut into pieces of up to 16 (wave 0, 64 keys a step)
        if (wv == 0) {
            int nt = 0, runstart = 0;
            for (int i0 = 0; i0 < cnt; i0 += 64) {
                const int i = i0 + lane;
                const bool v = i < cnt;
                const bool rs = v && (i == 0 || sh.key[i] != sh.key[i - 1]);
                const uint64_t rsm = __ballot(rs);
                // start of the run holding i: the last run start at or below this lane
                const uint64_t upto = rsm & ((lane == 63) ? ~0ull : ((2ull << lane) - 1ull));
                const int my_rs = upto ? i0 + 63 - __builtin_clzll(upto) : runstart;
                const bool ts = v && ((i - my_rs) & 15) == 0;
                const uint64_t tsm = __ballot(ts);
                const int rank = __popcll(tsm & ((1ull << lane) - 1ull));
                if (ts) sh.tstart[nt + rank] = (unsigned short)i;
                nt += __popcll(tsm);
                runstart = __builtin_amdgcn_readlane(my_rs, 63);
            }
            // tile sizes: to the next tile start, at most 16
            for (int t = lane; t < nt; t += 64) {
                const int st = sh.tstart[t], en = t + 1 < nt ? sh.tstart[t + 1] : cnt;
                sh.tcnt[t] = (unsigned char)min(16, en - st);
            }
            if (lane == 0) sh.ntile = nt;
        }
        __syncthreads();
        const int ntile = sh.ntile;
        for (int tb = wv * kMfBatch; tb < ntile; tb += 4 * kMfBatch) {
            const int nb = min(kMfBatch, ntile - tb);
            // derivative tensors of the batch: one lane per tile
            if (lane < nb) {
                int lev, rx, ry, rz;
                mf_unkey(sh.key[sh.tstart[tb + lane]], lev, rx, ry, rz);
                const float hA = (float)ldexp(box, -lev);
                float f[P + 1], D[NC];
                const float Rx = (float)rx, Ry = (float)ry, Rz = (float)rz;
                prefactors<P, float>(Rx * Rx + Ry * Ry + Rz * Rz, (float)(sp.scale / (double)hA), sp.kind, f);
                dtensor<P, float>(Rx, Ry, Rz, f, D);
#pragma unroll
                for (int k = 0; k < NC; ++k) sh.D[wv][lane][k] = D[k];
                sh.D[wv][lane][NC] = 0.0f;
            }
            wave_lds_sync();
            for (int t = 0; t < nb; ++t) {
                const int st = sh.tstart[tb + t], nc = sh.tcnt[tb + t];
                const int col = lane & 15, kq = lane >> 4;
                const bool has = col < nc;
                const int q = has ? sh.idx[st + col] : 0;
                const uint32_t it = has ? sh.pit[q] : 0u;
                const int j = has ? sh.pj[q] : 0;
                const float *Mb = M + (size_t)(it >> 5) * NC;
                // B operand: this lane's column (source) and coefficient m = 4 s + kq of slice s
                float bv[NS0];
#pragma unroll
                for (int s = 0; s < NS0; ++s) {
                    const int m = 4 * s + kq;
                    bv[s] = (has && m < NC) ? Mb[m] : 0.0f;
                }
                v4f acc[NRT];
#pragma unroll
                for (int r = 0; r < NRT; ++r) acc[r] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
                const float *Dt = &sh.D[wv][t][0];
#pragma unroll
                for (int q2 = 0; q2 < NQ; ++q2) {
                    const int ai = (apk[q2 / 2] >> (16 * (q2 & 1))) & 0xffff;
                    acc[cs.rt[q2]] = __builtin_amdgcn_mfma_f32_16x16x4f32(Dt[ai], bv[cs.s[q2]], acc[cs.rt[q2]], 0, 0, 0);
                }
                // output (row 16 r + 4 kq + i, column col) -> local expansion n of sink j
                if (has) {
#pragma unroll
                    for (int r = 0; r < NRT; ++r)
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int n = 16 * r + 4 * kq + i;
                            if (n < NC) atomicAdd(&sh.L[j][n], acc[r][i]);
                        }
                }
            }
            wave_lds_sync();  // the batch's tensors are read before the next batch overwrites them
        }
        __syncthreads();  // the chunk's buffers are free again
    }
    // the window's expansions, written once (the pairs of other kinds are added after)
    for (int k = tid; k < nsw * NC; k += 256) {
        const int j = k / NC, n = k - j * NC;
        L[(size_t)sh.sink[j] * NC + n] = sh.L[j][n];
    }
}

// ---------------------------------------------------------------------------
// List preparation.  A wave takes 64 cells; per cell, its M2L chunks 64 entries at a time.

// ne[c]: entries of cell c for the matrix-core kernel; no[c]: the others.
__global__ __launch_bounds__(64) void k_m2l_classify(const int4 *__restrict__ cellc, int ncell,
                                                     const int *__restrict__ head, const int *__restrict__ cnt,
                                                     const uint32_t *__restrict__ items, const int *__restrict__ next,
                                                     int *__restrict__ ne, int *__restrict__ no)
{
    const int lane = threadIdx.x;
    for (int A0 = blockIdx.x * 64; A0 < ncell; A0 += gridDim.x * 64) {
        const int A = A0 + lane;
        const int nl = A < ncell ? cnt[A] : 0;
        const int hd = nl > 0 ? head[A] : 0;
        int mine = 0;
        for (int j = 0; j < 64; ++j) {
            const int nj = __shfl(nl, j, 64);
            if (nj == 0) continue;
            const int4 ga = cellc[A0 + j];
            int chunk = __shfl(hd, j, 64), e = 0;
            for (int e0 = 0; e0 < nj; e0 += kChunk) {
                if (e0 > 0) chunk = next[chunk];
                const bool v = e0 + lane < nj;
                const bool el = v && mf_eligible(ga, cellc[items[(size_t)chunk * kChunk + lane] >> 5]);
                e += __popcll(__ballot(el));
            }
            if (lane == j) mine = e;
        }
        if (A < ncell) {
            ne[A] = mine;
            no[A] = nl - mine;
        }
    }
}

// Eligible entries -> csr[offe[c] ..] (list entries), the others -> other[offn[c] ..]
// as (sink, entry) pairs for the lane-per-pair kernel.  Also the compacted sink list.
__global__ __launch_bounds__(64) void k_m2l_split(const int4 *__restrict__ cellc, int ncell,
                                                  const int *__restrict__ head, const int *__restrict__ cnt,
                                                  const uint32_t *__restrict__ items, const int *__restrict__ next,
                                                  const int *__restrict__ ne, const int *__restrict__ offe,
                                                  const int *__restrict__ offn, const int *__restrict__ spos,
                                                  uint32_t *__restrict__ csr, int2 *__restrict__ other,
                                                  int *__restrict__ sinks)
{
    const int lane = threadIdx.x;
    const uint64_t lt = (1ull << lane) - 1ull;
    for (int A0 = blockIdx.x * 64; A0 < ncell; A0 += gridDim.x * 64) {
        const int A = A0 + lane;
        const int nl = A < ncell ? cnt[A] : 0;
        const int hd = nl > 0 ? head[A] : 0;
        if (A < ncell && ne[A] > 0) sinks[spos[A]] = A;
        const int oe = A < ncell ? offe[A] : 0, on = A < ncell ? offn[A] : 0;
        for (int j = 0; j < 64; ++j) {
            const int nj = __shfl(nl, j, 64);
            if (nj == 0) continue;
            const int4 ga = cellc[A0 + j];
            int pe = __shfl(oe, j, 64), pn = __shfl(on, j, 64);
            int chunk = __shfl(hd, j, 64);
            for (int e0 = 0; e0 < nj; e0 += kChunk) {
                if (e0 > 0) chunk = next[chunk];
                const bool v = e0 + lane < nj;
                const uint32_t it = v ? items[(size_t)chunk * kChunk + lane] : 0u;
                const bool el = v && mf_eligible(ga, cellc[it >> 5]);
                const uint64_t em = __ballot(el), om = __ballot(v && !el);
                if (el) csr[pe + __popcll(em & lt)] = it;
                if (v && !el) other[pn + __popcll(om & lt)] = make_int2(A0 + j, (int)it);
                pe += __popcll(em);
                pn += __popcll(om);
            }
        }
    }
}

__global__ void k_flag_positive(const int *__restrict__ v, int n, int *__restrict__ flag)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = v[i] > 0;
}

// ---------------------------------------------------------------------------
// host side

template <int P> static int launch_mfma(fmm_tree *t, Split sp, int nwin, hipStream_t st)
{
    const int4 *cc = ptr<int4>(t->cellc);
    int *cnt3 = ptr<int>(t->mf_tot);
    k_m2l_mfma<P><<<nwin, 256, 0, st>>>(ptr<Cell>(t->cells), cc, ptr<int>(t->mf_sinks), cnt3 + 2, ptr<int>(t->mf_offe),
                                        ptr<int>(t->mf_ne), ptr<uint32_t>(t->mf_csr), ptr<float>(t->Mc),
                                        ptr<float>(t->Lc), t->box, sp);
    return hip_check(hipGetLastError(), "m2l mfma");
}

// Plain FP32 M2L of order P with the matrix-core kernel for same-level pairs.  L is
// zeroed by the caller.  Splits the M2L list; returns the number of remaining pairs (in
// t->m2l_pairs as (sink, entry)) for the lane-per-pair kernel through *n_other.
int m2l_mfma_split_and_run(fmm_tree *t, int p, Split sp, int64_t *n_other, hipStream_t st)
{
    const int ncell = t->ncell;
    const int64_t np = t->n_m2l;
    if (np > 0x7fffffff) return set_error(FMM_ERR_ARG, "too many M2L pairs (%lld)", (long long)np);
    int rc = grow(t->mf_ne, (size_t)ncell * 4 + 64) | grow(t->mf_no, (size_t)ncell * 4 + 64) |
             grow(t->mf_offe, (size_t)ncell * 4 + 64) | grow(t->mf_offn, (size_t)ncell * 4 + 64) |
             grow(t->mf_spos, (size_t)ncell * 4 + 64) | grow(t->mf_sinks, (size_t)ncell * 4 + 64) |
             grow(t->mf_tot, 64) | grow(t->mf_csr, (size_t)np * 4 + 64) | grow(t->m2l_pairs, (size_t)np * 8 + 64);
    if (rc) return rc;
    const int *head = ptr<int>(t->lhead), *cnt = ptr<int>(t->lcnt);
    const uint32_t *items = ptr<uint32_t>(t->litems[0]);
    const int *next = ptr<int>(t->lnext[0]);
    const int4 *cc = ptr<int4>(t->cellc);
    const int nw = (ncell + 63) / 64, g = nw < 16384 ? nw : 16384;
    int *tot = ptr<int>(t->mf_tot);  // [0] eligible pairs, [1] other pairs, [2] sinks with eligible pairs
    k_m2l_classify<<<g, 64, 0, st>>>(cc, ncell, head, cnt, items, next, ptr<int>(t->mf_ne), ptr<int>(t->mf_no));
    if ((rc = scan_exclusive(ptr<int>(t->mf_ne), ptr<int>(t->mf_offe), ncell, tot, st, t->scan_tmp))) return rc;
    if ((rc = scan_exclusive(ptr<int>(t->mf_no), ptr<int>(t->mf_offn), ncell, tot + 1, st, t->scan_tmp))) return rc;
    // compacted list of the sinks with eligible pairs, in cell order
    k_flag_positive<<<(ncell + 255) / 256, 256, 0, st>>>(ptr<int>(t->mf_ne), ncell, ptr<int>(t->mf_no));
    if ((rc = scan_exclusive(ptr<int>(t->mf_no), ptr<int>(t->mf_spos), ncell, tot + 2, st, t->scan_tmp))) return rc;
    k_m2l_split<<<g, 64, 0, st>>>(cc, ncell, head, cnt, items, next, ptr<int>(t->mf_ne), ptr<int>(t->mf_offe),
                                  ptr<int>(t->mf_offn), ptr<int>(t->mf_spos), ptr<uint32_t>(t->mf_csr),
                                  ptr<int2>(t->m2l_pairs), ptr<int>(t->mf_sinks));
    if ((rc = hip_check(hipGetLastError(), "m2l split"))) return rc;
    // sizes for the grids: read back, except while being recorded (the eager evaluation
    // of the same tree found the same sizes)
    if (!t->capturing) {
        if ((rc = hip_check(hipMemcpyAsync(t->host, tot, 3 * sizeof(int), hipMemcpyDeviceToHost, st), "m2l sizes")) ||
            (rc = hip_check(hipStreamSynchronize(st), "m2l sizes")))
            return rc;
        t->mf_n_other = t->host[1];
        t->mf_nsink = t->host[2];
    }
    const int nwin = (t->mf_nsink + kMfWin - 1) / kMfWin;
    *n_other = t->mf_n_other;
    if (nwin == 0) return 0;
    switch (p) {
    case 4: return launch_mfma<4>(t, sp, nwin, st);
    case 5: return launch_mfma<5>(t, sp, nwin, st);
    case 6: return launch_mfma<6>(t, sp, nwin, st);
    case 7: return launch_mfma<7>(t, sp, nwin, st);
    case 8: return launch_mfma<8>(t, sp, nwin, st);
    }
    return set_error(FMM_ERR_ARG, "matrix-core M2L compiled for orders 4..8 (p = %d)", p);
}

}  // namespace hfmm
