// Triangular solves with the multifrontal factor (gfx950).
//
// Right-hand sides inside the library are row-major: Y[i * k + c] holds
// column c of pivot row i.  Every front f (m rows, p pivots, first pivot f0)
// has a row-major m x k work block w at W + woff[f] * k.  The factorization
// kept the inverse of every 64 x 64 diagonal block (padded with the
// identity), so a block step is a product, not a substitution:
//   forward  (y = L^-1 b):   z_b = L_bb^-1 w_b,  w_rows_below -= L_rows_below,b z_b
//   backward (x = L^-T y):   v = y_pivots - L_update,:^T x_update, then from the last
//                            block down: x_b = L_bb^-T v_b,  v_a -= L_b,a^T x_b (a < b).
// Fronts with few rows run one workgroup per front for the whole sweep
// ("fused"); larger fronts run one launch per 64-column block with the rows
// (forward) or column blocks (backward) spread over workgroups.  With 64
// right-hand sides at a time the block products run on the matrix cores.
// Summation order is fixed everywhere, so results are deterministic.

namespace wcs {
namespace dev {

template <typename T> struct SolveArgs {
    const int64_t *front_off;
    const int32_t *mfront, *pfront, *first;
    const int64_t *woff;
    const int32_t *child_ptr, *child_list;
    const int64_t *rptr;
    const int32_t *rel, *rows;
    const int64_t *dscr_off;
    const T *fronts, *dinv;
    T *W, *Y;
    int k;
};

constexpr int SB = 64;          // block size of the solves (= panel width of the factorization)
constexpr int SROWS = THREADS;  // rows per workgroup in a forward block step

// ---- shared pieces (all threads of the workgroup call them)

// w = [Y(pivots); 0] + sum over children of their update rows
template <typename T>
__device__ void fwd_assemble(const SolveArgs<T> &a, int f)
{
    int m = a.mfront[f], p = a.pfront[f], k = a.k;
    T *w = a.W + a.woff[f] * k;
    const T *y = a.Y + (int64_t)a.first[f] * k;
    int64_t mk = (int64_t)m * k, pk = (int64_t)p * k;
    for (int64_t i = threadIdx.x; i < mk; i += blockDim.x) w[i] = i < pk ? y[i] : (T)0;
    __syncthreads();
    for (int q = a.child_ptr[f]; q < a.child_ptr[f + 1]; q++) {
        int c = a.child_list[q];
        int mc = a.mfront[c], pc = a.pfront[c];
        const T *wc = a.W + a.woff[c] * k + (int64_t)pc * k;
        const int32_t *rl = a.rel + a.rptr[c] + pc;
        int64_t nu = (int64_t)(mc - pc) * k;
        for (int64_t i = threadIdx.x; i < nu; i += blockDim.x) {
            int r = (int)(i / k), cc = (int)(i % k);
            w[(int64_t)rl[r] * k + cc] += wc[i];
        }
        __syncthreads();
    }
}

// ---- matrix-core forms for 64 right-hand sides at a time

// Zs = op(Linv) * Ss (64 x 64 each); wave w produces output rows [16w, 16w+16)
template <typename T>
__device__ void blk_mfma(T (*Ds)[SB + 1], T (*Ss)[64], T (*Zs)[64])
{
    typedef typename Mfma<T>::V V;
    int tid = threadIdx.x, wave = tid / 64, lane = tid % 64, kq = lane / 16, ln = lane % 16;
    V acc[4];
#pragma unroll
    for (int cb = 0; cb < 4; cb++)
#pragma unroll
        for (int e = 0; e < 4; e++) acc[cb][e] = 0;
#pragma unroll
    for (int kk = 0; kk < SB; kk += 4) {
        T av = Ds[kk + kq][wave * 16 + ln];          // op(Linv)(row, j) = Ds[j][row]
#pragma unroll
        for (int cb = 0; cb < 4; cb++) acc[cb] = Mfma<T>::mma(av, Ss[kk + kq][cb * 16 + ln], acc[cb]);
    }
#pragma unroll
    for (int cb = 0; cb < 4; cb++)
#pragma unroll
        for (int e = 0; e < 4; e++) Zs[wave * 16 + Mfma<T>::row(kq, e)][cb * 16 + ln] = acc[cb][e];
}

// rows [r0, r1) of w:  w[r][c0 + n] -= sum_j L(r, kb + j) Zs[j][n]; waves take 64-row slabs
template <typename T>
__device__ void fwd_rows_mfma(const T *__restrict__ L, int ld, int kb, int nbk, T *__restrict__ w, int k, int c0,
                              int r0, int r1, T (*Zs)[64])
{
    typedef typename Mfma<T>::V V;
    int tid = threadIdx.x, wave = tid / 64, lane = tid % 64, kq = lane / 16, ln = lane % 16;
    int nw = blockDim.x / 64;
    for (int s0 = r0 + wave * 64; s0 < r1; s0 += nw * 64) {
        V acc[4][4];
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int j = 0; j < 4; j++)
#pragma unroll
                for (int e = 0; e < 4; e++) acc[i][j][e] = 0;
        T av[SB / 4][4];
#pragma unroll
        for (int ks = 0; ks < SB / 4; ks++) {
            int j = ks * 4 + kq;
#pragma unroll
            for (int rb = 0; rb < 4; rb++) {
                int r = s0 + rb * 16 + ln;
                av[ks][rb] = (r < r1 && j < nbk) ? L[(int64_t)(kb + j) * ld + r] : (T)0;
            }
        }
#pragma unroll
        for (int ks = 0; ks < SB / 4; ks++) {
            T bv[4];
#pragma unroll
            for (int cb = 0; cb < 4; cb++) bv[cb] = Zs[ks * 4 + kq][cb * 16 + ln];
#pragma unroll
            for (int rb = 0; rb < 4; rb++)
#pragma unroll
                for (int cb = 0; cb < 4; cb++) acc[rb][cb] = Mfma<T>::mma(av[ks][rb], bv[cb], acc[rb][cb]);
        }
#pragma unroll
        for (int rb = 0; rb < 4; rb++)
#pragma unroll
            for (int e = 0; e < 4; e++) {
                int r = s0 + rb * 16 + Mfma<T>::row(kq, e);
                if (r >= r1) continue;
                T *wr = w + (int64_t)r * k + c0;
#pragma unroll
                for (int cb = 0; cb < 4; cb++) {
                    int n = cb * 16 + ln;
                    if (c0 + n < k) wr[n] -= acc[rb][cb][e];
                }
            }
    }
}

// v[c][c0 + n] -= sum_{r in [r0, r1)} L(r, a + c) X[r][n]  (c < na, n < 64);
// wave w owns output rows c in [16w, 16w+16)
template <typename T, typename XR>
__device__ void bwd_cols_mfma(const T *__restrict__ L, int ld, int a, int na, int r0, int r1, XR xrow, int k, int c0,
                              T *__restrict__ v, T (*Ls)[SB + 1], T (*Xs)[64])
{
    typedef typename Mfma<T>::V V;
    int tid = threadIdx.x, wave = tid / 64, lane = tid % 64, kq = lane / 16, ln = lane % 16;
    // v may have just been written by other waves: order those writes before
    // the read-modify-write below even when there are no rows to sum over
    __syncthreads();
    if (r0 >= r1) return;
    V acc[4];
#pragma unroll
    for (int cb = 0; cb < 4; cb++)
#pragma unroll
        for (int e = 0; e < 4; e++) acc[cb][e] = 0;
    for (int rb = r0; rb < r1; rb += SB) {
        int nr = min(SB, r1 - rb);
        __syncthreads();
        for (int i = tid; i < SB * SB; i += blockDim.x) {
            int cc = i / SB, rr = i % SB;
            Ls[cc][rr] = (cc < na && rr < nr) ? L[(int64_t)(a + cc) * ld + rb + rr] : (T)0;
        }
        for (int i = tid; i < SB * 64; i += blockDim.x) {
            int rr = i / 64, cc = i % 64;
            Xs[rr][cc] = (rr < nr && c0 + cc < k) ? xrow(rb + rr)[c0 + cc] : (T)0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < SB; kk += 4) {
            T av = Ls[wave * 16 + ln][kk + kq];
#pragma unroll
            for (int cb = 0; cb < 4; cb++) acc[cb] = Mfma<T>::mma(av, Xs[kk + kq][cb * 16 + ln], acc[cb]);
        }
    }
#pragma unroll
    for (int e = 0; e < 4; e++) {
        int c = wave * 16 + Mfma<T>::row(kq, e);
        if (c >= na) continue;
#pragma unroll
        for (int cb = 0; cb < 4; cb++) {
            int n = cb * 16 + ln;
            if (c0 + n < k) v[(int64_t)c * k + c0 + n] -= acc[cb][e];
        }
    }
    __syncthreads();
}

// Zs[i][c] = sum_j Linv(i, j) * src_j[c] for the block starting at pivot kb
// (src rows given by a row pointer of stride k).  Stages L^-1 and the block
// rows in LDS.  For the transposed form Zs = Linv^T src set trans = true.
template <typename T, int KT>
__device__ void block_apply(const T *__restrict__ Dinv, const T *__restrict__ src, int k, int c0, int nbk,
                            bool trans, T (*Ds)[SB + 1], T (*Ss)[KT], T (*Zs)[KT])
{
    for (int i = threadIdx.x; i < SB * SB; i += blockDim.x) {
        int c = i / SB, r = i % SB;
        T v = Dinv[i];                 // column-major: Linv(r, c)
        if (trans) Ds[r][c] = v; else Ds[c][r] = v;   // Ds[j][i] holds the factor applied to src_j for output i
    }
    for (int i = threadIdx.x; i < SB * KT; i += blockDim.x) {
        int r = i / KT, c = i % KT;
        Ss[r][c] = (r < nbk && c0 + c < k) ? src[(int64_t)r * k + c0 + c] : (T)0;
    }
    __syncthreads();
    if constexpr (KT == 64) {
        blk_mfma<T>(Ds, Ss, Zs);
    } else {
        for (int i = threadIdx.x; i < SB * KT; i += blockDim.x) {
            int r = i / KT, c = i % KT;
            T s = 0;
#pragma unroll 8
            for (int j = 0; j < SB; j++) s += Ds[j][r] * Ss[j][c];
            Zs[r][c] = s;
        }
    }
    __syncthreads();
}

// rows [r0, r1) of w:  w[r][c] -= sum_j L(r, kb + j) Zs[j][c], one thread per row
template <typename T, int KT>
__device__ void fwd_rows(const T *__restrict__ L, int ld, int kb, int nbk, T *__restrict__ w, int k, int c0, int r0,
                         int r1, T (*Zs)[KT])
{
    for (int r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
        T acc[KT];
#pragma unroll
        for (int c = 0; c < KT; c++) acc[c] = 0;
        for (int j = 0; j < nbk; j++) {
            T l = L[(int64_t)(kb + j) * ld + r];
#pragma unroll
            for (int c = 0; c < KT; c++) acc[c] += l * Zs[j][c];
        }
        T *wr = w + (int64_t)r * k + c0;
#pragma unroll
        for (int c = 0; c < KT; c++)
            if (c0 + c < k) wr[c] -= acc[c];
    }
}

// v_a[c][cc] -= sum_{r in rows} L(r, a + c) * X[r][cc] over rows [r0, r1) of the
// front; X rows come from xrow(r) (a row pointer with stride k).  Thread
// (c = tid % 64, g = tid / 64) owns columns cc = g, g + 4, ...
template <typename T, int KT, typename XR>
__device__ void bwd_cols(const T *__restrict__ L, int ld, int a, int na, int r0, int r1, XR xrow, int k, int c0,
                         T *__restrict__ v, T (*Ls)[SB + 1], T (*Xs)[KT])
{
    int tid = threadIdx.x, c = tid % SB, g = tid / SB;
    constexpr int PG = (KT + 3) / 4;
    // v may have just been written by other waves: order those writes before
    // the read-modify-write below even when there are no rows to sum over
    __syncthreads();
    if (r0 >= r1) return;
    T acc[PG];
#pragma unroll
    for (int q = 0; q < PG; q++) acc[q] = 0;
    for (int rb = r0; rb < r1; rb += SB) {
        int nr = min(SB, r1 - rb);
        __syncthreads();
        for (int i = tid; i < SB * SB; i += blockDim.x) {
            int cc = i / SB, rr = i % SB;
            Ls[cc][rr] = (cc < na && rr < nr) ? L[(int64_t)(a + cc) * ld + rb + rr] : (T)0;
        }
        for (int i = tid; i < SB * KT; i += blockDim.x) {
            int rr = i / KT, cc = i % KT;
            Xs[rr][cc] = (rr < nr && c0 + cc < k) ? xrow(rb + rr)[c0 + cc] : (T)0;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PG; q++) {
            int cc = g + 4 * q;
            if (cc < KT) {
                T s = 0;
#pragma unroll 8
                for (int rr = 0; rr < SB; rr++) s += Ls[c][rr] * Xs[rr][cc];
                acc[q] += s;
            }
        }
    }
    if (c < na) {
#pragma unroll
        for (int q = 0; q < PG; q++) {
            int cc = g + 4 * q;
            if (cc < KT && c0 + cc < k) v[(int64_t)c * k + c0 + cc] -= acc[q];
        }
    }
    __syncthreads();
}

template <typename T, int KT>
__device__ __forceinline__ void fwd_rows_any(const T *L, int ld, int kb, int nbk, T *w, int k, int c0, int r0, int r1,
                                             T (*Zs)[KT])
{
    if constexpr (KT == 64) fwd_rows_mfma<T>(L, ld, kb, nbk, w, k, c0, r0, r1, Zs);
    else fwd_rows<T, KT>(L, ld, kb, nbk, w, k, c0, r0, r1, Zs);
}

template <typename T, int KT, typename XR>
__device__ __forceinline__ void bwd_cols_any(const T *L, int ld, int a, int na, int r0, int r1, XR xrow, int k, int c0,
                                             T *v, T (*Ls)[SB + 1], T (*Xs)[KT])
{
    if constexpr (KT == 64) bwd_cols_mfma<T>(L, ld, a, na, r0, r1, xrow, k, c0, v, Ls, Xs);
    else bwd_cols<T, KT>(L, ld, a, na, r0, r1, xrow, k, c0, v, Ls, Xs);
}

template <typename T, int KT> struct SolveLds {
    T Ds[SB][SB + 1];
    T Ss[SB][KT];
    T Zs[SB][KT];
};

// ---- forward

template <typename T, int KT>
__global__ __launch_bounds__(THREADS) void k_fwd_fused(const int32_t *__restrict__ flist, SolveArgs<T> a)
{
    __shared__ SolveLds<T, KT> sh;
    int f = flist[blockIdx.x];
    fwd_assemble(a, f);
    int m = a.mfront[f], p = a.pfront[f], k = a.k, f0 = a.first[f];
    const T *L = a.fronts + a.front_off[f];
    T *w = a.W + a.woff[f] * k;
    for (int c0 = 0; c0 < k; c0 += KT) {
        for (int kb = 0; kb < p; kb += SB) {
            int nbk = min(SB, p - kb);
            __syncthreads();
            block_apply<T, KT>(a.dinv + a.dscr_off[f] + (int64_t)(kb / SB) * SB * SB, w + (int64_t)kb * k, k, c0,
                               nbk, false, sh.Ds, sh.Ss, sh.Zs);
            for (int i = threadIdx.x; i < nbk * KT; i += blockDim.x) {
                int r = i / KT, c = i % KT;
                if (c0 + c < k) a.Y[(int64_t)(f0 + kb + r) * k + c0 + c] = sh.Zs[r][c];
            }
            fwd_rows_any<T, KT>(L, front_ld(m), kb, nbk, w, k, c0, kb + nbk, m, sh.Zs);
        }
    }
}

// task = (front, row slab of SROWS rows): w rows of the slab = [Y(pivots); 0]
// plus the update rows of every child that land in the slab.  The index map
// of a child is increasing, so those rows are one contiguous run found by
// binary search; children are visited in a fixed order (deterministic).
template <typename T>
__global__ __launch_bounds__(THREADS) void k_fwd_assemble(const int2 *__restrict__ tasks, SolveArgs<T> a)
{
    int2 t = tasks[blockIdx.x];
    int f = t.x;
    int m = a.mfront[f], p = a.pfront[f], k = a.k;
    int r0 = t.y * SROWS, r1 = min(m, r0 + SROWS);
    T *w = a.W + a.woff[f] * k;
    const T *y = a.Y + (int64_t)a.first[f] * k;
    for (int64_t i = (int64_t)r0 * k + threadIdx.x; i < (int64_t)r1 * k; i += blockDim.x)
        w[i] = i < (int64_t)p * k ? y[i] : (T)0;
    __syncthreads();
    for (int q = a.child_ptr[f]; q < a.child_ptr[f + 1]; q++) {
        int c = a.child_list[q];
        int mc = a.mfront[c], pc = a.pfront[c];
        const int32_t *rl = a.rel + a.rptr[c] + pc;
        int nu = mc - pc;
        int lo = 0, hi = nu;
        while (lo < hi) { int md = (lo + hi) / 2; if (rl[md] < r0) lo = md + 1; else hi = md; }
        int t0 = lo;
        hi = nu;
        while (lo < hi) { int md = (lo + hi) / 2; if (rl[md] < r1) lo = md + 1; else hi = md; }
        int t1 = lo;
        const T *wc = a.W + a.woff[c] * k + (int64_t)pc * k;
        for (int64_t i = (int64_t)t0 * k + threadIdx.x; i < (int64_t)t1 * k; i += blockDim.x) {
            int r = (int)(i / k), cc = (int)(i % k);
            w[(int64_t)rl[r] * k + cc] += wc[i];
        }
        __syncthreads();
    }
}

// task = (front, row slab) for block kb; slab 0 also stores z_b into Y.  The
// block rows w_b are only read in this launch (z goes to Y), so the
// workgroups of one launch never race.
template <typename T, int KT>
__global__ __launch_bounds__(THREADS) void k_fwd_step(const int2 *__restrict__ tasks, int kb, SolveArgs<T> a)
{
    __shared__ SolveLds<T, KT> sh;
    int2 t = tasks[blockIdx.x];
    int f = t.x;
    int m = a.mfront[f], p = a.pfront[f], k = a.k, f0 = a.first[f];
    int nbk = min(SB, p - kb);
    const T *L = a.fronts + a.front_off[f];
    T *w = a.W + a.woff[f] * k;
    int r0 = kb + nbk + t.y * SROWS, r1 = min(m, r0 + SROWS);
    for (int c0 = 0; c0 < k; c0 += KT) {
        __syncthreads();
        block_apply<T, KT>(a.dinv + a.dscr_off[f] + (int64_t)(kb / SB) * SB * SB, w + (int64_t)kb * k, k, c0, nbk,
                           false, sh.Ds, sh.Ss, sh.Zs);
        if (t.y == 0)
            for (int i = threadIdx.x; i < nbk * KT; i += blockDim.x) {
                int r = i / KT, c = i % KT;
                if (c0 + c < k) a.Y[(int64_t)(f0 + kb + r) * k + c0 + c] = sh.Zs[r][c];
            }
        if (r0 < r1) fwd_rows_any<T, KT>(L, front_ld(m), kb, nbk, w, k, c0, r0, r1, sh.Zs);
    }
}

// ---- backward

template <typename T, int KT> struct BwdLds {
    T Ds[SB][SB + 1];
    T Ss[SB][KT];
    T Zs[SB][KT];
    T Ls[SB][SB + 1];
};

// v_a = Y(pivots of block a) - L(update rows, block a)^T x(update rows), into w rows [a, a+na)
template <typename T, int KT>
__device__ void bwd_below(const SolveArgs<T> &a, int f, int ab, T (*Ls)[SB + 1], T (*Xs)[KT])
{
    int m = a.mfront[f], p = a.pfront[f], k = a.k, f0 = a.first[f];
    int na = min(SB, p - ab);
    const T *L = a.fronts + a.front_off[f];
    T *w = a.W + a.woff[f] * k;
    for (int64_t i = threadIdx.x; i < (int64_t)na * k; i += blockDim.x)
        w[(int64_t)ab * k + i] = a.Y[(int64_t)(f0 + ab) * k + i];
    const int32_t *rw = a.rows + a.rptr[f];
    const T *Y = a.Y;
    auto xrow = [&](int r) { return Y + (int64_t)rw[r] * k; };
    for (int c0 = 0; c0 < k; c0 += KT)
        bwd_cols_any<T, KT>(L, front_ld(m), ab, na, p, m, xrow, k, c0, w + (int64_t)ab * k, Ls, Xs);
}

template <typename T, int KT>
__global__ __launch_bounds__(THREADS) void k_bwd_fused(const int32_t *__restrict__ flist, SolveArgs<T> a)
{
    __shared__ BwdLds<T, KT> sh;
    int f = flist[blockIdx.x];
    int m = a.mfront[f], p = a.pfront[f], k = a.k, f0 = a.first[f];
    (void)m;
    const T *L = a.fronts + a.front_off[f];
    T *w = a.W + a.woff[f] * k;
    for (int ab = 0; ab < p; ab += SB) bwd_below<T, KT>(a, f, ab, sh.Ls, sh.Ss);
    int nblk = (p + SB - 1) / SB;
    for (int b = nblk - 1; b >= 0; b--) {
        int kb = b * SB, nbk = min(SB, p - kb);
        for (int c0 = 0; c0 < k; c0 += KT) {
            __syncthreads();
            block_apply<T, KT>(a.dinv + a.dscr_off[f] + (int64_t)b * SB * SB, w + (int64_t)kb * k, k, c0, nbk, true,
                               sh.Ds, sh.Ss, sh.Zs);
            for (int i = threadIdx.x; i < nbk * KT; i += blockDim.x) {
                int r = i / KT, c = i % KT;
                if (c0 + c < k) a.Y[(int64_t)(f0 + kb + r) * k + c0 + c] = sh.Zs[r][c];
            }
            // v_a -= L(block b rows, block a cols)^T x_b for a < b
            for (int ab = 0; ab < kb; ab += SB) {
                T(*Zs)[KT] = sh.Zs;
                auto xrow = [&](int r) { return &Zs[r - kb][0] - c0; };
                bwd_cols_any<T, KT>(L, front_ld(a.mfront[f]), ab, SB, kb, kb + nbk, xrow, k, c0, w + (int64_t)ab * k, sh.Ls,
                                    sh.Ss);
            }
        }
    }
}

// task = (front, column block a): v_a = y_a - L(update rows, a)^T x(update rows)
template <typename T, int KT>
__global__ __launch_bounds__(THREADS) void k_bwd_below(const int2 *__restrict__ tasks, SolveArgs<T> a)
{
    __shared__ BwdLds<T, KT> sh;
    int2 t = tasks[blockIdx.x];
    bwd_below<T, KT>(a, t.x, t.y * SB, sh.Ls, sh.Ss);
}

// task = (front, column block a) for block b: x_b = L_bb^-T v_b (every
// workgroup); a == b stores x_b into Y, a < b updates v_a.  v_b is only read.
template <typename T, int KT>
__global__ __launch_bounds__(THREADS) void k_bwd_step(const int2 *__restrict__ tasks, int b, SolveArgs<T> a)
{
    __shared__ BwdLds<T, KT> sh;
    int2 t = tasks[blockIdx.x];
    int f = t.x;
    int p = a.pfront[f], k = a.k, f0 = a.first[f];
    int kb = b * SB, nbk = min(SB, p - kb);
    const T *L = a.fronts + a.front_off[f];
    T *w = a.W + a.woff[f] * k;
    for (int c0 = 0; c0 < k; c0 += KT) {
        __syncthreads();
        block_apply<T, KT>(a.dinv + a.dscr_off[f] + (int64_t)b * SB * SB, w + (int64_t)kb * k, k, c0, nbk, true,
                           sh.Ds, sh.Ss, sh.Zs);
        if (t.y == b) {
            for (int i = threadIdx.x; i < nbk * KT; i += blockDim.x) {
                int r = i / KT, c = i % KT;
                if (c0 + c < k) a.Y[(int64_t)(f0 + kb + r) * k + c0 + c] = sh.Zs[r][c];
            }
        } else {
            T(*Zs)[KT] = sh.Zs;
            auto xrow = [&](int r) { return &Zs[r - kb][0] - c0; };
            bwd_cols_any<T, KT>(L, front_ld(a.mfront[f]), t.y * SB, SB, kb, kb + nbk, xrow, k, c0, w + (int64_t)t.y * SB * k,
                                sh.Ls, sh.Ss);
        }
    }
}

}  // namespace dev
}  // namespace wcs
