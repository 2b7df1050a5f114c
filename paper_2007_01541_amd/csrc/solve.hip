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
// ("fused").  Larger fronts go super-block by super-block (SS = 256 pivots):
// one workgroup per front solves the (at most four) 64-blocks of the
// super-block in sequence, then one wide launch applies the whole super-block
// to every row below it (forward) or to every earlier column block (backward)
// with K = 256.  With 64 right-hand sides at a time the block products run on
// the matrix cores.  Summation order is fixed everywhere, so results are
// deterministic.

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
    const int64_t *xoff;        // per front: element offset of its super-block inverses (-1: none)
    const T *xinv;
    T *W, *Y;
    T *part;                    // partial products of the split backward update-row sums
    int k;
};

// dst[i] -= val[i] for the N elements with ok[i]; every load is issued before
// any store (a masked-off element reads dst[0] of the caller's block, which
// is in bounds, and is not written), so the round trips to memory overlap
// instead of being serialised element by element.
template <int N, typename T, typename OffFn, typename ValFn>
__device__ __forceinline__ void sub_batch(T *__restrict__ base, OffFn off, ValFn val)
{
    T cur[N];
    int64_t o[N];
#pragma unroll
    for (int i = 0; i < N; i++) {
        o[i] = off(i);
        cur[i] = base[o[i] >= 0 ? o[i] : 0];
    }
#pragma unroll
    for (int i = 0; i < N; i++)
        if (o[i] >= 0) base[o[i]] = cur[i] - val(i);
}

constexpr int SB = 64;          // block size of the solves (= panel width of the factorization)
constexpr int SS = 4 * SB;      // super-block of the large-front sweeps
constexpr int SROWS = 64;       // rows per workgroup in a forward assembly launch

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
            sub_batch<16>(
                w,
                [&](int i) -> int64_t {
                    int e = i / 4, cb = i % 4;
                    int r = s0 + rb * 16 + Mfma<T>::row(kq, e), n = cb * 16 + ln;
                    return (r < r1 && c0 + n < k) ? (int64_t)r * k + c0 + n : -1;
                },
                [&](int i) { return acc[rb][i % 4][i / 4]; });
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
    sub_batch<16>(
        v,
        [&](int i) -> int64_t {
            int e = i / 4, cb = i % 4;
            int c = wave * 16 + Mfma<T>::row(kq, e), n = cb * 16 + ln;
            return (c < na && c0 + n < k) ? (int64_t)c * k + c0 + n : -1;
        },
        [&](int i) { return acc[i % 4][i / 4]; });
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
        sub_batch<KT>(
            w, [&](int c) -> int64_t { return c0 + c < k ? (int64_t)r * k + c0 + c : -1; },
            [&](int c) { return acc[c]; });
    }
}

// v_a[c][cc] -= sum_{r in rows} L(r, a + c) * X[r][cc] over rows [r0, r1) of the
// front; X rows come from xrow(r) (a row pointer with stride k).  The four
// waves take a quarter of the rows each, lane = column c (each lane walks its
// column of L, contiguous; the X row is broadcast); their partial sums meet
// in Ls (reused, 4 x 64 x KT elements) and are added in wave order.  All
// threads of the workgroup call it.
template <typename T, int KT, typename XR>
__device__ void bwd_cols(const T *__restrict__ L, int ld, int a, int na, int r0, int r1, XR xrow, int k, int c0,
                         T *__restrict__ v, T (*Ls)[SB + 1], T (*)[KT])
{
    static_assert(4 * SB * KT <= SB * (SB + 1), "partial sums must fit the staging array");
    int tid = threadIdx.x, wave = tid / SB, lane = tid % SB;
    // v may have just been written by other waves: order those writes before
    // the read-modify-write below even when there are no rows to sum over
    __syncthreads();
    if (r0 >= r1) return;
    int chunk = (r1 - r0 + 3) / 4, rb = r0 + wave * chunk, re = min(r1, rb + chunk);
    T acc[KT];
#pragma unroll
    for (int c = 0; c < KT; c++) acc[c] = 0;
    if (lane < na) {
        const T *lc = L + (int64_t)(a + lane) * ld;
        // UR rows at a time: their row pointers (an index load for update rows),
        // then every value, are in flight before the products
        constexpr int UR = KT <= 4 ? 16 : 4;
        for (int rg = rb; rg < re; rg += UR) {
            const T *xr[UR];
            T lv[UR], xv[UR][KT];
#pragma unroll
            for (int u = 0; u < UR; u++) xr[u] = rg + u < re ? xrow(rg + u) + c0 : nullptr;
#pragma unroll
            for (int u = 0; u < UR; u++) {
                lv[u] = xr[u] ? lc[rg + u] : (T)0;
#pragma unroll
                for (int c = 0; c < KT; c++) xv[u][c] = (xr[u] && c0 + c < k) ? xr[u][c] : (T)0;
            }
#pragma unroll
            for (int u = 0; u < UR; u++)
#pragma unroll
                for (int c = 0; c < KT; c++) acc[c] += lv[u] * xv[u][c];
        }
    }
    T *part = &Ls[0][0];
#pragma unroll
    for (int c = 0; c < KT; c++) part[(wave * SB + lane) * KT + c] = acc[c];
    __syncthreads();
    for (int e = tid; e < SB * KT; e += blockDim.x) {
        int c = e / KT, cc = e % KT;
        if (c < na && c0 + cc < k)
            v[(int64_t)c * k + c0 + cc] -= (part[c * KT + cc] + part[(SB + c) * KT + cc]) +
                                          (part[(2 * SB + c) * KT + cc] + part[(3 * SB + c) * KT + cc]);
    }
    __syncthreads();
}

// The same, staged through LDS 64 rows at a time (all threads load): for rows
// reached through an index (the update rows of a front), whose loads would
// otherwise chain.  v_a[c][cc] -= sum_{r in rows} L(r, a + c) * X[r][cc] over
// rows [r0, r1); X rows come from xrow(r) (a row pointer with stride k).  Thread
// (c = tid % 64, g = tid / 64) owns columns cc = g, g + 4, ...
template <typename T, int KT, typename XR>
__device__ void bwd_cols_staged(const T *__restrict__ L, int ld, int a, int na, int r0, int r1, XR xrow, int k, int c0,
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
    sub_batch<PG>(
        v,
        [&](int q) -> int64_t {
            int cc = g + 4 * q;
            return (c < na && cc < KT && c0 + cc < k) ? (int64_t)c * k + c0 + cc : -1;
        },
        [&](int q) { return acc[q]; });
    __syncthreads();
}

// The same for at most four right-hand sides (KT = 4), as a transposed
// matrix-vector product: lane = row (the four waves take 64 rows each per
// round of 256), so each of the 64 column loads of a lane is coalesced
// across the wave and all are in flight together; the 64 products of a lane
// are summed over the wave by a butterfly (at step h a lane keeps the half of
// its columns on its side of bit h and adds the partner's copy of them), which
// leaves column c's sum in lane c; the four waves' sums meet in Ls (reused)
// and are added in wave order (ASSIGN: v_a[c][cc] = the sum instead).  All
// threads of the workgroup call it.
template <typename T, int KT, typename XR, bool ASSIGN = false>
__device__ void bwd_cols_lanes(const T *__restrict__ L, int ld, int a, int na, int r0, int r1, XR xrow, int k,
                               int c0, T *__restrict__ v, T (*Ls)[SB + 1])
{
    static_assert(KT <= 4 && 4 * SB * KT <= SB * (SB + 1), "few right-hand sides only");
    int tid = threadIdx.x, wave = tid / SB, lane = tid % SB;
    __syncthreads();            // as in bwd_cols: writes of v by other waves come first
    if (r0 >= r1) return;
    T tot[KT];
#pragma unroll
    for (int cc = 0; cc < KT; cc++) tot[cc] = 0;
    for (int rb = r0 + wave * SB; rb < r1; rb += 4 * SB) {
        int r = rb + lane;
        bool ok = r < r1;
        T xv[KT];
        const T *xr = ok ? xrow(r) + c0 : nullptr;
#pragma unroll
        for (int cc = 0; cc < KT; cc++) xv[cc] = (ok && c0 + cc < k) ? xr[cc] : (T)0;
        T lv[SB];
#pragma unroll
        for (int c = 0; c < SB; c++) lv[c] = (ok && c < na) ? L[(int64_t)(a + c) * ld + r] : (T)0;
#pragma unroll
        for (int cc = 0; cc < KT; cc++) {
            if (c0 + cc >= k) break;
            T pr[SB];
#pragma unroll
            for (int c = 0; c < SB; c++) pr[c] = lv[c] * xv[cc];
#pragma unroll
            for (int h = SB / 2; h >= 1; h >>= 1) {
                bool up = (lane & h) != 0;
#pragma unroll
                for (int i = 0; i < h; i++) {
                    T give = up ? pr[i] : pr[i + h], keep = up ? pr[i + h] : pr[i];
                    pr[i] = keep + __shfl_xor(give, h, SB);
                }
            }
            tot[cc] += pr[0];       // column `lane`, summed over the wave's rows
        }
    }
    T *part = &Ls[0][0];
#pragma unroll
    for (int cc = 0; cc < KT; cc++) part[(wave * SB + lane) * KT + cc] = tot[cc];
    __syncthreads();
    for (int e = tid; e < SB * KT; e += blockDim.x) {
        int c = e / KT, cc = e % KT;
        if (c < na && c0 + cc < k) {
            T sum = (part[c * KT + cc] + part[(SB + c) * KT + cc]) +
                    (part[(2 * SB + c) * KT + cc] + part[(3 * SB + c) * KT + cc]);
            if constexpr (ASSIGN) v[(int64_t)c * k + c0 + cc] = sum;
            else v[(int64_t)c * k + c0 + cc] -= sum;
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

// First i in [lo, hi) with rl[i] >= key (hi if none), rl increasing; called
// by every lane of a wave alike.  Each round the 64 lanes probe evenly spaced
// entries and a ballot counts those below key, shrinking the range 64-fold:
// a few dependent loads instead of one per halving.
__device__ __forceinline__ int wave_lower_bound(const int32_t *__restrict__ rl, int lo, int hi, int key)
{
    const int lane = threadIdx.x % 64;
    while (hi > lo) {
        const int span = hi - lo;
        const int step = span <= 64 ? 1 : (span + 63) / 64;
        const int pos = lo + lane * step;
        const int cnt = __popcll(__ballot(pos < hi && rl[pos] < key));
        if (span <= 64 || cnt == 0) return lo + (span <= 64 ? cnt : 0);
        const int base = lo;
        lo = base + (cnt - 1) * step + 1;      // rl[lo - 1] < key
        hi = min(hi, base + cnt * step);      // rl[hi] >= key, or hi unchanged
    }
    return lo;
}

// task = (front, row slab of SROWS rows): w rows of the slab = [Y(pivots); 0]
// plus the update rows of every child that land in the slab.  The index map
// of a child is increasing, so those rows are one contiguous run found by a
// wave-parallel search; children are visited in a fixed order (deterministic).
// With k a multiple of 4 every thread moves groups of four columns of a row
// (vector accesses); loads of a round are issued before its stores.
template <typename T>
__global__ __launch_bounds__(THREADS) void k_fwd_assemble(const int2 *__restrict__ tasks, SolveArgs<T> a)
{
    typedef typename Vec4<T>::type V4;
    int2 t = tasks[blockIdx.x];
    int f = t.x;
    int m = a.mfront[f], p = a.pfront[f], k = a.k;
    int r0 = t.y * SROWS, r1 = min(m, r0 + SROWS);
    T *w = a.W + a.woff[f] * k;
    const T *y = a.Y + (int64_t)a.first[f] * k;
    const bool quad = (k & 3) == 0;
    const int g = quad ? 4 : 1, ng = k / g;     // groups of g columns per row
    for (int i = threadIdx.x; i < (r1 - r0) * ng; i += blockDim.x) {
        int r = r0 + i / ng, c = (i % ng) * g;
        int64_t o = (int64_t)r * k + c;
        if (quad)
            *reinterpret_cast<V4 *>(w + o) = r < p ? *reinterpret_cast<const V4 *>(y + o) : V4{0, 0, 0, 0};
        else
            w[o] = r < p ? y[o] : (T)0;
    }
    __syncthreads();
    for (int q = a.child_ptr[f]; q < a.child_ptr[f + 1]; q++) {
        int c = a.child_list[q];
        int mc = a.mfront[c], pc = a.pfront[c];
        const int32_t *rl = a.rel + a.rptr[c] + pc;
        int nu = mc - pc;
        const int t0 = wave_lower_bound(rl, 0, nu, r0);
        const int t1 = wave_lower_bound(rl, t0, nu, r1);
        const T *wc = a.W + a.woff[c] * k + (int64_t)pc * k;
        int tot = (t1 - t0) * ng;
        constexpr int B = 2;   // groups per thread per round
        for (int i0 = threadIdx.x; i0 < tot; i0 += B * blockDim.x) {
            int64_t so[B], dof[B];
#pragma unroll
            for (int b = 0; b < B; b++) {
                int i = i0 + b * blockDim.x;
                bool ok = i < tot;
                int r = t0 + (ok ? i / ng : 0), cc = ok ? (i % ng) * g : 0;
                so[b] = (int64_t)r * k + cc;
                dof[b] = ok ? (int64_t)rl[r] * k + cc : -1;
            }
            if (quad) {
                V4 uv[B], dv[B];
#pragma unroll
                for (int b = 0; b < B; b++) {
                    bool ok = dof[b] >= 0;
                    uv[b] = ok ? *reinterpret_cast<const V4 *>(wc + so[b]) : V4{0, 0, 0, 0};
                    dv[b] = ok ? *reinterpret_cast<const V4 *>(w + dof[b]) : V4{0, 0, 0, 0};
                }
#pragma unroll
                for (int b = 0; b < B; b++)
                    if (dof[b] >= 0) {
                        V4 v = dv[b];
                        v.x += uv[b].x;
                        v.y += uv[b].y;
                        v.z += uv[b].z;
                        v.w += uv[b].w;
                        *reinterpret_cast<V4 *>(w + dof[b]) = v;
                    }
            } else {
                T uv[B], dv[B];
#pragma unroll
                for (int b = 0; b < B; b++) {
                    bool ok = dof[b] >= 0;
                    uv[b] = ok ? wc[so[b]] : (T)0;
                    dv[b] = ok ? w[dof[b]] : (T)0;
                }
#pragma unroll
                for (int b = 0; b < B; b++)
                    if (dof[b] >= 0) w[dof[b]] = dv[b] + uv[b];
            }
        }
        __syncthreads();
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
        if constexpr (KT == 64) bwd_cols_any<T, KT>(L, front_ld(m), ab, na, p, m, xrow, k, c0, w + (int64_t)ab * k, Ls, Xs);
        else bwd_cols_staged<T, KT>(L, front_ld(m), ab, na, p, m, xrow, k, c0, w + (int64_t)ab * k, Ls, Xs);   // indexed rows
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


// ---- 64 x 64 tiles for 64 right-hand sides: each wave takes a slice of the
// contraction and multiplies straight from global memory (no LDS staging, no
// workgroup barrier inside the loop); the four partial tiles are added
// through LDS at the end.  Within a group of 16 k values, lane kq of a
// 16x16x4 product supplies k = kg + 4 kq + j in product j (j = 0..3), so a
// lane's four k values are consecutive in memory; the order of summation is
// fixed, so results are deterministic.

// acc[x][y] += sum over k in [kb, ke) of fa(16 x + ln, k) fb(k, 16 y + ln)
// (fa / fb return 0 outside their ranges)
template <typename T, typename FA, typename FB>
__device__ __forceinline__ void wave_mm(typename Mfma<T>::V (&acc)[4][4], int kb, int ke, FA fa, FB fb)
{
    const int lane = threadIdx.x % 64, kq = lane / 16, ln = lane % 16;
    for (int kg = kb; kg < ke; kg += 16) {
        T av[4][4], bv[4][4];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            int k = kg + 4 * kq + j;
            bool ok = k < ke;
#pragma unroll
            for (int x = 0; x < 4; x++) av[j][x] = ok ? fa(16 * x + ln, k) : (T)0;
#pragma unroll
            for (int y = 0; y < 4; y++) bv[j][y] = ok ? fb(k, 16 * y + ln) : (T)0;
        }
#pragma unroll
        for (int j = 0; j < 4; j++)
#pragma unroll
            for (int x = 0; x < 4; x++)
#pragma unroll
                for (int y = 0; y < 4; y++) acc[x][y] = Mfma<T>::mma(av[j][x], bv[j][y], acc[x][y]);
    }
}

// Sums the four waves' tiles: out(r, c, v) for every (r, c) of the 64 x 64
// tile, called by 16 elements per thread in two halves of 32 columns; red is
// LDS of 4 * 64 * 32 elements.  at(x, y, e) gives the tile position (r, c)
// of accumulator element e of acc[x][y] in this lane.  All threads of the
// workgroup call it.
template <typename T, typename At, typename Out>
__device__ __forceinline__ void reduce4m(typename Mfma<T>::V (&acc)[4][4], T *red, At at, Out out)
{
    const int tid = threadIdx.x, wave = tid / 64;
#pragma unroll
    for (int h = 0; h < 2; h++) {
        __syncthreads();
#pragma unroll
        for (int x = 0; x < 4; x++)
#pragma unroll
            for (int y = 0; y < 4; y++)
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    int2 rc = at(x, y, e);
                    if ((rc.y >> 5) == h) red[(wave * 64 + rc.x) * 32 + (rc.y & 31)] = acc[x][y][e];
                }
        __syncthreads();
        T v[8];
        int rr[8], cc[8];
#pragma unroll
        for (int q = 0; q < 8; q++) {
            int idx = tid + 256 * q;            // 0 .. 2047 over 64 rows x 32 columns
            rr[q] = idx / 32;
            cc[q] = idx % 32;
            v[q] = red[(0 * 64 + rr[q]) * 32 + cc[q]] + red[(1 * 64 + rr[q]) * 32 + cc[q]] +
                   red[(2 * 64 + rr[q]) * 32 + cc[q]] + red[(3 * 64 + rr[q]) * 32 + cc[q]];
        }
        out(rr, cc, v, 32 * h);
    }
}

// the layout of wave_mm: element e of acc[x][y] is (16 x + row(kq, e), 16 y + ln)
template <typename T, typename Out>
__device__ __forceinline__ void reduce4(typename Mfma<T>::V (&acc)[4][4], T *red, Out out)
{
    const int lane = threadIdx.x % 64, kq = lane / 16, ln = lane % 16;
    reduce4m<T>(acc, red, [&](int x, int y, int e) { return make_int2(16 * x + Mfma<T>::row(kq, e), 16 * y + ln); },
                out);
}

// ---- quad forms of the 64 x 64 wave product: one vector load of four
// consecutive elements per lane and operand feeds four 16x16x4 products.

template <typename V4> __device__ __forceinline__ auto q_at(const V4 &v, int i)
{
    return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
}

// acc[x][y] += sum over k in [kb, ke) of A(4 i + x, k) B(k, 4 j + y) for the
// product's row i and column j: qa(t, k) returns A rows 4t..4t+3 of column k,
// qb(k, t) B columns 4t..4t+3 of row k (each a 16- or 32-byte vector).  Lane
// kq of a product supplies k = kg + 4 u + kq in the u-th product of a group
// (4 U values of k).  Element e of acc[x][y] is (4 row(kq, e) + x, 4 ln + y).
template <typename T, typename QA, typename QB>
__device__ __forceinline__ void wave_mm_q(typename Mfma<T>::V (&acc)[4][4], int kb, int ke, QA qa, QB qb)
{
    typedef typename Vec4<T>::type V4;
    constexpr int U = sizeof(T) == 4 ? 4 : 2;    // products per group (FP64 quads take twice the registers)
    const int lane = threadIdx.x % 64, kq = lane / 16, ln = lane % 16;
    for (int kg = kb; kg < ke; kg += 4 * U) {
        V4 av[U], bv[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            int k = kg + 4 * u + kq;
            bool ok = k < ke;
            av[u] = ok ? qa(ln, k) : V4{0, 0, 0, 0};
            bv[u] = ok ? qb(k, ln) : V4{0, 0, 0, 0};
        }
#pragma unroll
        for (int u = 0; u < U; u++)
#pragma unroll
            for (int x = 0; x < 4; x++)
#pragma unroll
                for (int y = 0; y < 4; y++) acc[x][y] = Mfma<T>::mma(q_at(av[u], x), q_at(bv[u], y), acc[x][y]);
    }
}

// acc[x][y] += sum over k in [max(lo, kb), ke) of A(16 x + i, k) B(k, 4 j + y):
// ka(i, k4) returns A(i, k4..k4+3) (four consecutive k of row i, k4 a
// multiple of 4 relative to kb), qb(k, t) B columns 4t..4t+3 of row k.  Lane
// kq supplies k = kg + 4 kq + s in the s-th product of a group of 16, so its
// four k are one load of A.  Element e of acc[x][y] is (16 x + row(kq, e), 4 ln + y).
template <typename T, typename KA, typename QB>
__device__ __forceinline__ void wave_mm_kq(typename Mfma<T>::V (&acc)[4][4], int lo, int kb, int ke, KA ka, QB qb)
{
    typedef typename Vec4<T>::type V4;
    const int lane = threadIdx.x % 64, kq = lane / 16, ln = lane % 16;
    for (int kg = kb; kg < ke; kg += 16) {
        int k4 = kg + 4 * kq;
        V4 av[4], bv[4];
        bool any = k4 < ke;
#pragma unroll
        for (int x = 0; x < 4; x++) {
            av[x] = any ? ka(16 * x + ln, k4) : V4{0, 0, 0, 0};
            if (k4 < lo || k4 + 3 >= ke) {      // the ends of the range
                if (k4 < lo || k4 >= ke) av[x].x = 0;
                if (k4 + 1 < lo || k4 + 1 >= ke) av[x].y = 0;
                if (k4 + 2 < lo || k4 + 2 >= ke) av[x].z = 0;
                if (k4 + 3 < lo || k4 + 3 >= ke) av[x].w = 0;
            }
        }
#pragma unroll
        for (int s2 = 0; s2 < 4; s2++) {
            int k = k4 + s2;
            bv[s2] = (k >= lo && k < ke) ? qb(k, ln) : V4{0, 0, 0, 0};
        }
#pragma unroll
        for (int s2 = 0; s2 < 4; s2++)
#pragma unroll
            for (int x = 0; x < 4; x++)
#pragma unroll
                for (int y = 0; y < 4; y++)
                    acc[x][y] = Mfma<T>::mma(q_at(av[x], s2), q_at(bv[s2], y), acc[x][y]);
    }
}

template <typename T> struct MmLds {
    T red[4 * 64 * 32];
};

// ---- super-block sweeps of large fronts
//
// X_S = L_SS^-1 of every diagonal super-block S = [s0, s1) of a large front is
// built once per factorization (k_build_xinv): column-major SS x SS at
// xinv + xoff[f] + (s0 / SS) SS^2, element (r, c) at c SS + r, lower block
// triangle filled (64-blocks X_ij, i >= j).  A super-step is then two wide
// launches: forward z_S = X_S w_S, then w_r -= L(r, S) z_S for every row
// below; backward x_S = X_S^T v_S, then v_a -= L(S, a)^T x_S for every
// column block before S.

// acc (+)= op(D) S over a 64-deep product staged in LDS: D[j][i] is the
// factor applied to S row j for output row i.  Matrix cores for 64
// right-hand sides (wave w owns output rows [16w, 16w+16)); otherwise each
// thread owns outputs t, t + 256, ... of the 64 x KT block.
template <typename T, int KT> struct BlkAcc {
    static constexpr int NQ = KT == 64 ? 4 : (SB * KT + THREADS - 1) / THREADS;
    typename Mfma<T>::V v[4];
    T f[NQ];
    __device__ void zero()
    {
#pragma unroll
        for (int q = 0; q < 4; q++)
#pragma unroll
            for (int e = 0; e < 4; e++) v[q][e] = 0;
#pragma unroll
        for (int q = 0; q < NQ; q++) f[q] = 0;
    }
    __device__ void add(T (*D)[SB + 1], T (*S)[KT])
    {
        if constexpr (KT == 64) {
            int tid = threadIdx.x, wave = tid / 64, lane = tid % 64, kq = lane / 16, ln = lane % 16;
#pragma unroll
            for (int kk = 0; kk < SB; kk += 4) {
                T av = D[kk + kq][wave * 16 + ln];
#pragma unroll
                for (int cb = 0; cb < 4; cb++) v[cb] = Mfma<T>::mma(av, S[kk + kq][cb * 16 + ln], v[cb]);
            }
        } else {
#pragma unroll
            for (int q = 0; q < NQ; q++) {
                int idx = threadIdx.x + q * THREADS;
                if (idx < SB * KT) {
                    int r = idx / KT, c = idx % KT;
                    T s = 0;
#pragma unroll 8
                    for (int j = 0; j < SB; j++) s += D[j][r] * S[j][c];
                    f[q] += s;
                }
            }
        }
    }
    // out(r, c) for r < nr, c0 + c < k: fn(r, c, value)
    template <typename Fn> __device__ void store(int nr, int k, int c0, Fn fn)
    {
        if constexpr (KT == 64) {
            int tid = threadIdx.x, wave = tid / 64, lane = tid % 64, kq = lane / 16, ln = lane % 16;
#pragma unroll
            for (int cb = 0; cb < 4; cb++)
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    int r = wave * 16 + Mfma<T>::row(kq, e), c = cb * 16 + ln;
                    if (r < nr && c0 + c < k) fn(r, c, v[cb][e]);
                }
        } else {
#pragma unroll
            for (int q = 0; q < NQ; q++) {
                int idx = threadIdx.x + q * THREADS;
                if (idx < SB * KT) {
                    int r = idx / KT, c = idx % KT;
                    if (r < nr && c0 + c < k) fn(r, c, f[q]);
                }
            }
        }
    }
};

// forward, task = (front, block i of the super-block at s0): z_i = sum_{j <= i} X_ij w_j -> Y
template <typename T, int KT>
__global__ __launch_bounds__(THREADS, sizeof(T) == 4 ? 2 : 1) void k_fwd_sz(const int2 *__restrict__ tasks, int s0, SolveArgs<T> a)
{
    int2 t = tasks[blockIdx.x];
    int f = t.x, ib = t.y;
    int p = a.pfront[f], k = a.k, f0 = a.first[f];
    int s1 = min(p, s0 + SS);
    int i0 = s0 + ib * SB, ni = min(SB, s1 - i0);
    const T *X = a.xinv + a.xoff[f] + (int64_t)(s0 / SS) * SS * SS;
    const T *w = a.W + a.woff[f] * k;
    if constexpr (KT == 64) {
        // wave jb adds X_ij w_j for its block j <= i
        typedef typename Vec4<T>::type V4;
        __shared__ MmLds<T> mm;
        int wave = threadIdx.x / 64, lane = threadIdx.x % 64, kq = lane / 16, ln = lane % 16;
        bool quad = (k & 3) == 0;
        for (int c0 = 0; c0 < k; c0 += 64) {
            typename Mfma<T>::V acc[4][4];
#pragma unroll
            for (int x = 0; x < 4; x++)
#pragma unroll
                for (int y = 0; y < 4; y++)
#pragma unroll
                    for (int e = 0; e < 4; e++) acc[x][y][e] = 0;
            if (wave <= ib) {
                int j0 = s0 + wave * SB, nj = min(SB, s1 - j0);
                if (quad)   // rows of X_ij in quads (X is column-major, rows inside the super-block)
                    wave_mm_q<T>(
                        acc, 0, nj,
                        [&](int q, int kk) {
                            return *reinterpret_cast<const V4 *>(X + (int64_t)(j0 - s0 + kk) * SS + (i0 - s0) + 4 * q);
                        },
                        [&](int kk, int q) {
                            int c = c0 + 4 * q;
                            return c < k ? *reinterpret_cast<const V4 *>(w + (int64_t)(j0 + kk) * k + c)
                                         : V4{0, 0, 0, 0};
                        });
                else
                    wave_mm<T>(
                        acc, 0, nj,
                        [&](int r, int kk) { return r < ni ? X[(int64_t)(j0 - s0 + kk) * SS + (i0 - s0 + r)] : (T)0; },
                        [&](int kk, int c) { return c0 + c < k ? w[(int64_t)(j0 + kk) * k + c0 + c] : (T)0; });
            }
            auto put = [&](int *rr, int *cc, T *v, int cb) {
#pragma unroll
                for (int q = 0; q < 8; q++) {
                    int r = rr[q], c = cb + cc[q];
                    if (r < ni && c0 + c < k) a.Y[(int64_t)(f0 + i0 + r) * k + c0 + c] = v[q];
                }
            };
            if (quad)
                reduce4m<T>(
                    acc, mm.red,
                    [&](int x, int y, int e) { return make_int2(4 * Mfma<T>::row(kq, e) + x, 4 * ln + y); }, put);
            else
                reduce4<T>(acc, mm.red, put);
        }
        return;
    }
    // KT < 64: wave q adds X_iq w_q for its block q <= i, lane = output row
    // (coalesced down the columns of X, w rows broadcast); the four partial
    // sums meet in LDS and are added in wave order
    __shared__ T part[4 * SB * KT];
    int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    for (int c0 = 0; c0 < k; c0 += KT) {
        T acc[KT];
#pragma unroll
        for (int c = 0; c < KT; c++) acc[c] = 0;
        if (wave <= ib) {
            int j0 = s0 + wave * SB, nj = min(SB, s1 - j0);
            const T *xc = X + (int64_t)(j0 - s0) * SS + (i0 - s0) + lane;   // X(i0 + lane, j0 + j) at xc[j SS]
            // UJ columns at a time, every load issued before the products
            constexpr int UJ = KT <= 4 ? 16 : 4;
            for (int jg = 0; jg < nj; jg += UJ) {
                T xv[UJ], wv[UJ][KT];
#pragma unroll
                for (int u = 0; u < UJ; u++) {
                    int j = jg + u;
                    bool ok = j < nj;
                    xv[u] = ok ? xc[(int64_t)j * SS] : (T)0;
#pragma unroll
                    for (int c = 0; c < KT; c++)
                        wv[u][c] = (ok && c0 + c < k) ? w[(int64_t)(j0 + j) * k + c0 + c] : (T)0;
                }
#pragma unroll
                for (int u = 0; u < UJ; u++)
#pragma unroll
                    for (int c = 0; c < KT; c++) acc[c] += xv[u] * wv[u][c];
            }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < KT; c++) part[(wave * SB + lane) * KT + c] = acc[c];
        __syncthreads();
        for (int e = threadIdx.x; e < SB * KT; e += THREADS) {
            int r = e / KT, c = e % KT;
            if (r < ni && c0 + c < k)
                a.Y[(int64_t)(f0 + i0 + r) * k + c0 + c] =
                    (part[r * KT + c] + part[(SB + r) * KT + c]) + (part[(2 * SB + r) * KT + c] + part[(3 * SB + r) * KT + c]);
        }
    }
}

// forward, task = (front, 64-row tile of the rows below s1): w_r -= sum over
// the blocks b of the super-block of L(r, b) z_b (z from Y).  Tiles start at
// s1 rounded down to a multiple of 4 (aligned vector loads of L); rows before
// s1 are not written.
template <typename T, int KT>
__global__ __launch_bounds__(THREADS, sizeof(T) == 4 ? 3 : 1) void k_fwd_srows(const int2 *__restrict__ tasks, int s0, SolveArgs<T> a)
{
    int2 t = tasks[blockIdx.x];
    int f = t.x;
    int m = a.mfront[f], p = a.pfront[f], k = a.k, f0 = a.first[f], ld = front_ld(m);
    int s1 = min(p, s0 + SS);
    int r0 = (s1 & ~3) + t.y * SB, r1 = min(m, r0 + SB);
    const T *L = a.fronts + a.front_off[f];
    T *w = a.W + a.woff[f] * k;
    for (int c0 = 0; c0 < k; c0 += KT) {
        if constexpr (KT == 64) {
            // wave q takes the pivot columns [s0 + 64 q, s0 + 64 q + 64) of the super-block
            typedef typename Vec4<T>::type V4;
            __shared__ MmLds<T> mm;
            int wave = threadIdx.x / 64, lane = threadIdx.x % 64, kq = lane / 16, ln = lane % 16;
            bool quad = (k & 3) == 0;   // rows of Y are then vector-aligned
            constexpr int kc = SB;
            typename Mfma<T>::V acc[4][4];
#pragma unroll
            for (int x = 0; x < 4; x++)
#pragma unroll
                for (int y = 0; y < 4; y++)
#pragma unroll
                    for (int e = 0; e < 4; e++) acc[x][y][e] = 0;
            int kb = s0 + wave * kc;
            if (kb < s1) {
                if (quad)
                    wave_mm_q<T>(
                        acc, kb, min(s1, kb + kc),
                        [&](int q, int kk) {
                            int r = r0 + 4 * q;
                            return r < r1 ? *reinterpret_cast<const V4 *>(L + (int64_t)kk * ld + r) : V4{0, 0, 0, 0};
                        },
                        [&](int kk, int q) {
                            int c = c0 + 4 * q;
                            return c < k ? *reinterpret_cast<const V4 *>(a.Y + (int64_t)(f0 + kk) * k + c)
                                         : V4{0, 0, 0, 0};
                        });
                else
                    wave_mm<T>(
                        acc, kb, min(s1, kb + kc),
                        [&](int r, int kk) { return r0 + r < r1 ? L[(int64_t)kk * ld + r0 + r] : (T)0; },
                        [&](int kk, int c) { return c0 + c < k ? a.Y[(int64_t)(f0 + kk) * k + c0 + c] : (T)0; });
            }
            auto out = [&](int *rr, int *cc, T *v, int cb) {
                sub_batch<8>(
                    w,
                    [&](int q) -> int64_t {
                        int r = r0 + rr[q], c = cb + cc[q];
                        return (r >= s1 && r < r1 && c0 + c < k) ? (int64_t)r * k + c0 + c : -1;
                    },
                    [&](int q) { return v[q]; });
            };
            if (quad)
                reduce4m<T>(
                    acc, mm.red,
                    [&](int x, int y, int e) { return make_int2(4 * Mfma<T>::row(kq, e) + x, 4 * ln + y); }, out);
            else
                reduce4<T>(acc, mm.red, out);
        } else {
            // wave q takes the pivot block [s0 + 64 q, s0 + 64 q + 64), lane = row of the
            // tile; z of the whole super-block is staged once, the four partial sums
            // meet in LDS (the same array, after a barrier) and w is updated once
            __shared__ T buf[SS * KT];          // Zs[j][c] = buf[j KT + c]; then part[q][row][c]
            int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
            __syncthreads();
            for (int e = threadIdx.x; e < SS * KT; e += THREADS) {
                int j = e / KT, c = e % KT;
                buf[e] = (s0 + j < s1 && c0 + c < k) ? a.Y[(int64_t)(f0 + s0 + j) * k + c0 + c] : (T)0;
            }
            __syncthreads();
            T acc[KT];
#pragma unroll
            for (int c = 0; c < KT; c++) acc[c] = 0;
            int r = r0 + lane, kb = s0 + wave * SB, ke = min(s1, kb + SB);
            if (r >= s1 && r < r1) {
                constexpr int UJ = 16;      // loads of 16 columns in flight before their products
                for (int jg = kb; jg < ke; jg += UJ) {
                    T lv[UJ];
#pragma unroll
                    for (int u = 0; u < UJ; u++) lv[u] = jg + u < ke ? L[(int64_t)(jg + u) * ld + r] : (T)0;
#pragma unroll
                    for (int u = 0; u < UJ; u++)
                        if (jg + u < ke)
#pragma unroll
                            for (int c = 0; c < KT; c++) acc[c] += lv[u] * buf[(jg + u - s0) * KT + c];
                }
            }
            __syncthreads();
#pragma unroll
            for (int c = 0; c < KT; c++) buf[(wave * SB + lane) * KT + c] = acc[c];
            __syncthreads();
            for (int e = threadIdx.x; e < SB * KT; e += THREADS) {
                int rr = e / KT, c = e % KT, rw = r0 + rr;
                if (rw >= s1 && rw < r1 && c0 + c < k)
                    w[(int64_t)rw * k + c0 + c] -= (buf[rr * KT + c] + buf[(SB + rr) * KT + c]) +
                                                    (buf[(2 * SB + rr) * KT + c] + buf[(3 * SB + rr) * KT + c]);
            }
        }
    }
}

// forward rows when the super-block is a single 64-column block (every front
// of at most 64 pivots, as at the leaves) and k is a multiple of 4: each wave
// takes one task (front, 64-row tile) and the whole contraction, and updates
// its rows of w itself (no reduction between waves, no barrier)
template <typename T>
__global__ __launch_bounds__(THREADS, sizeof(T) == 4 ? 3 : 1) void k_fwd_srows1(const int2 *__restrict__ tasks, int ntasks, int s0,
                                                           SolveArgs<T> a)
{
    typedef typename Vec4<T>::type V4;
    int ti = blockIdx.x * (THREADS / 64) + threadIdx.x / 64;
    if (ti >= ntasks) return;
    int2 t = tasks[ti];
    int f = t.x;
    int m = a.mfront[f], p = a.pfront[f], k = a.k, f0 = a.first[f], ld = front_ld(m);
    int s1 = min(p, s0 + SB);
    int r0 = (s1 & ~3) + t.y * SB, r1 = min(m, r0 + SB);
    const T *L = a.fronts + a.front_off[f];
    T *w = a.W + a.woff[f] * k;
    const int lane = threadIdx.x % 64, kq = lane / 16, ln = lane % 16;
    for (int c0 = 0; c0 < k; c0 += 64) {
        typename Mfma<T>::V acc[4][4];
#pragma unroll
        for (int x = 0; x < 4; x++)
#pragma unroll
            for (int y = 0; y < 4; y++)
#pragma unroll
                for (int e = 0; e < 4; e++) acc[x][y][e] = 0;
        wave_mm_q<T>(
            acc, s0, s1,
            [&](int q, int kk) {
                int r = r0 + 4 * q;
                return r < r1 ? *reinterpret_cast<const V4 *>(L + (int64_t)kk * ld + r) : V4{0, 0, 0, 0};
            },
            [&](int kk, int q) {
                int c = c0 + 4 * q;
                return c < k ? *reinterpret_cast<const V4 *>(a.Y + (int64_t)(f0 + kk) * k + c) : V4{0, 0, 0, 0};
            });
        // rows 4 row(kq, e) + x of the tile, columns c0 + 4 ln .. + 3: one vector each
#pragma unroll
        for (int xh = 0; xh < 4; xh += 2) {
            T *dst[2][4];
            V4 cur[2][4];
#pragma unroll
            for (int x = 0; x < 2; x++)
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    int r = r0 + 4 * Mfma<T>::row(kq, e) + xh + x, c = c0 + 4 * ln;
                    dst[x][e] = (r >= s1 && r < r1 && c < k) ? w + (int64_t)r * k + c : nullptr;
                    cur[x][e] = dst[x][e] ? *reinterpret_cast<const V4 *>(dst[x][e]) : V4{0, 0, 0, 0};
                }
#pragma unroll
            for (int x = 0; x < 2; x++)
#pragma unroll
                for (int e = 0; e < 4; e++)
                    if (dst[x][e]) {
                        V4 v = cur[x][e];
                        v.x -= acc[xh + x][0][e];
                        v.y -= acc[xh + x][1][e];
                        v.z -= acc[xh + x][2][e];
                        v.w -= acc[xh + x][3][e];
                        *reinterpret_cast<V4 *>(dst[x][e]) = v;
                    }
        }
    }
}

// backward, task = (front, block j of the super-block at s0): x_j = sum_{i >= j} X_ij^T v_i -> Y
template <typename T, int KT>
__global__ __launch_bounds__(THREADS, sizeof(T) == 4 ? 2 : 1) void k_bwd_sx(const int2 *__restrict__ tasks, int s0, SolveArgs<T> a)
{
    int2 t = tasks[blockIdx.x];
    int f = t.x, jb = t.y;
    int p = a.pfront[f], k = a.k, f0 = a.first[f];
    int s1 = min(p, s0 + SS);
    int nblk = (s1 - s0 + SB - 1) / SB;
    int j0 = s0 + jb * SB, nj = min(SB, s1 - j0);
    const T *X = a.xinv + a.xoff[f] + (int64_t)(s0 / SS) * SS * SS;
    const T *w = a.W + a.woff[f] * k;
    if constexpr (KT == 64) {
        // wave q adds X_ij^T v_i for block i = j + q
        typedef typename Vec4<T>::type V4;
        __shared__ MmLds<T> mm;
        int wave = threadIdx.x / 64, lane = threadIdx.x % 64, kq = lane / 16, ln = lane % 16;
        bool quad = (k & 3) == 0;
        for (int c0 = 0; c0 < k; c0 += 64) {
            typename Mfma<T>::V acc[4][4];
#pragma unroll
            for (int x = 0; x < 4; x++)
#pragma unroll
                for (int y = 0; y < 4; y++)
#pragma unroll
                    for (int e = 0; e < 4; e++) acc[x][y][e] = 0;
            int ib = jb + wave;
            if (ib < nblk) {
                int i0 = s0 + ib * SB, ni = min(SB, s1 - i0);
                if (quad)   // X_ij^T: the contraction runs down a column of X (four per load)
                    wave_mm_kq<T>(
                        acc, 0, 0, ni,
                        [&](int r, int k4) {
                            return r < nj ? *reinterpret_cast<const V4 *>(X + (int64_t)(j0 - s0 + r) * SS + (i0 - s0) + k4)
                                          : V4{0, 0, 0, 0};
                        },
                        [&](int kk, int q) {
                            int c = c0 + 4 * q;
                            return c < k ? *reinterpret_cast<const V4 *>(w + (int64_t)(i0 + kk) * k + c)
                                         : V4{0, 0, 0, 0};
                        });
                else
                    wave_mm<T>(
                        acc, 0, ni,
                        [&](int r, int kk) { return r < nj ? X[(int64_t)(j0 - s0 + r) * SS + (i0 - s0 + kk)] : (T)0; },
                        [&](int kk, int c) { return c0 + c < k ? w[(int64_t)(i0 + kk) * k + c0 + c] : (T)0; });
            }
            auto put = [&](int *rr, int *cc, T *v, int cb) {
#pragma unroll
                for (int q = 0; q < 8; q++) {
                    int r = rr[q], c = cb + cc[q];
                    if (r < nj && c0 + c < k) a.Y[(int64_t)(f0 + j0 + r) * k + c0 + c] = v[q];
                }
            };
            if (quad)
                reduce4m<T>(
                    acc, mm.red,
                    [&](int x, int y, int e) { return make_int2(16 * x + Mfma<T>::row(kq, e), 4 * ln + y); }, put);
            else
                reduce4<T>(acc, mm.red, put);
        }
        return;
    }
    if constexpr (KT <= 4) {
        // x_j = sum over the rows of the blocks i >= j of X(row, j0 + r) v(row):
        // a transposed product over the super-block's rows (lane = row)
        __shared__ T Lt[SB][SB + 1];
        auto vrow = [&](int r) { return w + (int64_t)(s0 + r) * k; };
        for (int c0 = 0; c0 < k; c0 += KT)
            bwd_cols_lanes<T, KT, decltype(vrow), true>(X, SS, j0 - s0, nj, j0 - s0, s1 - s0, vrow, k, c0,
                                                        a.Y + (int64_t)(f0 + j0) * k, Lt);
        return;
    }
    // KT < 64: wave q adds X_ij^T v_i for block i = j + q, lane = output row r
    // (each lane walks column j0 + r of X, contiguous); partial sums meet in
    // LDS and are added in wave order
    __shared__ T part[4 * SB * KT];
    int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    for (int c0 = 0; c0 < k; c0 += KT) {
        T acc[KT];
#pragma unroll
        for (int c = 0; c < KT; c++) acc[c] = 0;
        int ib = jb + wave;
        if (ib < nblk) {
            int i0 = s0 + ib * SB, ni = min(SB, s1 - i0);
            const T *xc = X + (int64_t)(j0 - s0 + lane) * SS + (i0 - s0);   // X(i0 + kk, j0 + lane) at xc[kk]
            constexpr int UK = KT <= 4 ? 16 : 4;     // loads of UK rows in flight before their products
            for (int kg = 0; kg < ni; kg += UK) {
                T xv[UK], wv[UK][KT];
#pragma unroll
                for (int u = 0; u < UK; u++) {
                    bool ok = kg + u < ni;
                    xv[u] = ok ? xc[kg + u] : (T)0;
#pragma unroll
                    for (int c = 0; c < KT; c++)
                        wv[u][c] = (ok && c0 + c < k) ? w[(int64_t)(i0 + kg + u) * k + c0 + c] : (T)0;
                }
#pragma unroll
                for (int u = 0; u < UK; u++)
#pragma unroll
                    for (int c = 0; c < KT; c++) acc[c] += xv[u] * wv[u][c];
            }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < KT; c++) part[(wave * SB + lane) * KT + c] = acc[c];
        __syncthreads();
        for (int e = threadIdx.x; e < SB * KT; e += THREADS) {
            int r = e / KT, c = e % KT;
            if (r < nj && c0 + c < k)
                a.Y[(int64_t)(f0 + j0 + r) * k + c0 + c] =
                    (part[r * KT + c] + part[(SB + r) * KT + c]) + (part[(2 * SB + r) * KT + c] + part[(3 * SB + r) * KT + c]);
        }
    }
}

// backward, task = (front, column block a) with 64 a < s0: v_a -= L([s0, s1), a)^T x_[s0, s1)
// (x read from Y); each workgroup owns its block a
template <typename T, int KT>
__global__ __launch_bounds__(THREADS, sizeof(T) == 4 ? 2 : 1) void k_bwd_scols(const int2 *__restrict__ tasks, int s0, SolveArgs<T> a)
{
    int2 t = tasks[blockIdx.x];
    int f = t.x;
    int m = a.mfront[f], p = a.pfront[f], k = a.k, f0 = a.first[f];
    int s1 = min(p, s0 + SS);
    int ab = t.y * SB;
    const T *L = a.fronts + a.front_off[f];
    T *w = a.W + a.woff[f] * k;
    const T *Y = a.Y;
    if constexpr (KT == 64) {
        // out^T(n, c) = sum_r x_r[n] L(r, ab + c); wave q takes the rows [s0 + 64 q, s0 + 64 q + 64)
        typedef typename Vec4<T>::type V4;
        __shared__ MmLds<T> mm;
        int wave = threadIdx.x / 64, lane = threadIdx.x % 64, kq = lane / 16, ln = lane % 16, ld = front_ld(m);
        bool quad = (k & 3) == 0;
        constexpr int kc = SB;
        for (int c0 = 0; c0 < k; c0 += 64) {
            typename Mfma<T>::V acc[4][4];
#pragma unroll
            for (int x = 0; x < 4; x++)
#pragma unroll
                for (int y = 0; y < 4; y++)
#pragma unroll
                    for (int e = 0; e < 4; e++) acc[x][y][e] = 0;
            int rb = s0 + wave * kc;
            if (rb < s1) {
                if (quad)   // product rows: the block's columns c (four rows r per load of L)
                    wave_mm_kq<T>(
                        acc, rb, rb, min(s1, rb + kc),
                        [&](int c, int r4) { return *reinterpret_cast<const V4 *>(L + (int64_t)(ab + c) * ld + r4); },
                        [&](int r, int q) {
                            int n = c0 + 4 * q;
                            return n < k ? *reinterpret_cast<const V4 *>(Y + (int64_t)(f0 + r) * k + n)
                                         : V4{0, 0, 0, 0};
                        });
                else
                    wave_mm<T>(
                        acc, rb, min(s1, rb + kc),
                        [&](int n, int r) { return c0 + n < k ? Y[(int64_t)(f0 + r) * k + c0 + n] : (T)0; },
                        [&](int r, int c) { return L[(int64_t)(ab + c) * ld + r]; });
            }
            T *v = w + (int64_t)ab * k;
            if (quad)   // tile (c, n): consecutive threads update consecutive n
                reduce4m<T>(
                    acc, mm.red,
                    [&](int x, int y, int e) { return make_int2(16 * x + Mfma<T>::row(kq, e), 4 * ln + y); },
                    [&](int *rr, int *cc, T *val, int cb) {
                        sub_batch<8>(
                            v,
                            [&](int q) -> int64_t {
                                int c = rr[q], n = cb + cc[q];
                                return c0 + n < k ? (int64_t)c * k + c0 + n : -1;
                            },
                            [&](int q) { return val[q]; });
                    });
            else
                reduce4<T>(acc, mm.red, [&](int *rr, int *cc, T *val, int cb) {
                    sub_batch<8>(
                        v,
                        [&](int q) -> int64_t {
                            int n = rr[q], c = cb + cc[q];
                            return c0 + n < k ? (int64_t)c * k + c0 + n : -1;
                        },
                        [&](int q) { return val[q]; });
                });
        }
        return;
    }
    __shared__ BwdLds<T, KT> sh;
    auto xrow = [&](int r) { return Y + (int64_t)(f0 + r) * k; };
    for (int c0 = 0; c0 < k; c0 += KT)
        if constexpr (KT <= 4)
            bwd_cols_lanes<T, KT>(L, front_ld(m), ab, SB, s0, s1, xrow, k, c0, w + (int64_t)ab * k, sh.Ls);
        else
            bwd_cols_any<T, KT>(L, front_ld(m), ab, SB, s0, s1, xrow, k, c0, w + (int64_t)ab * k, sh.Ls, sh.Ss);
}

// backward update rows, split: task = (front, column block a, first row, slot):
// part[slot] = -L(rows [r0, r0 + BELOW_ROWS) of the update part, a)^T x(rows)
constexpr int BELOW_ROWS = 256;
template <typename T, int KT>
__global__ __launch_bounds__(THREADS) void k_bwd_below_part(const int4 *__restrict__ tasks, SolveArgs<T> a)
{
    int4 t = tasks[blockIdx.x];
    int f = t.x, ab = t.y * SB, r0 = t.z;
    int m = a.mfront[f], p = a.pfront[f], k = a.k;
    int na = min(SB, p - ab), r1 = min(m, r0 + BELOW_ROWS);
    const T *L = a.fronts + a.front_off[f];
    T *out = a.part + (int64_t)t.w * SB * k;
    const int32_t *rw = a.rows + a.rptr[f];
    const T *Y = a.Y;
    if constexpr (KT == 64) {
        // part^T(n, c) = -sum_r x(rows[r])[n] L(r, ab + c) over the rows r >= p of
        // the slab (it starts at a multiple of 4); wave q takes a quarter of them
        typedef typename Vec4<T>::type V4;
        __shared__ MmLds<T> mm;
        constexpr int RW = BELOW_ROWS / 4;
        int wave = threadIdx.x / 64, lane = threadIdx.x % 64, kq = lane / 16, ln = lane % 16, ld = front_ld(m);
        bool quad = (k & 3) == 0;
        for (int c0 = 0; c0 < k; c0 += 64) {
            typename Mfma<T>::V acc[4][4];
#pragma unroll
            for (int x = 0; x < 4; x++)
#pragma unroll
                for (int y = 0; y < 4; y++)
#pragma unroll
                    for (int e = 0; e < 4; e++) acc[x][y][e] = 0;
            int rb = r0 + wave * RW;
            if (rb < r1) {
                if (quad)   // product rows: pivot columns c (four rows r per load); columns: right-hand sides
                    wave_mm_kq<T>(
                        acc, p, rb, min(r1, rb + RW),
                        [&](int c, int r4) {
                            return c < na ? *reinterpret_cast<const V4 *>(L + (int64_t)(ab + c) * ld + r4)
                                          : V4{0, 0, 0, 0};
                        },
                        [&](int r, int q) {
                            int n = c0 + 4 * q;
                            return n < k ? *reinterpret_cast<const V4 *>(Y + (int64_t)rw[r] * k + n) : V4{0, 0, 0, 0};
                        });
                else
                    wave_mm<T>(
                        acc, max(rb, p), min(r1, rb + RW),
                        [&](int n, int r) { return c0 + n < k ? Y[(int64_t)rw[r] * k + c0 + n] : (T)0; },
                        [&](int r, int c) { return c < na ? L[(int64_t)(ab + c) * ld + r] : (T)0; });
            }
            if (quad)   // tile (c, n): consecutive threads write consecutive n
                reduce4m<T>(
                    acc, mm.red,
                    [&](int x, int y, int e) { return make_int2(16 * x + Mfma<T>::row(kq, e), 4 * ln + y); },
                    [&](int *rr, int *cc, T *val, int cb) {
#pragma unroll
                        for (int q = 0; q < 8; q++) {
                            int c = rr[q], n = cb + cc[q];
                            if (c0 + n < k) out[(int64_t)c * k + c0 + n] = -val[q];
                        }
                    });
            else
                reduce4<T>(acc, mm.red, [&](int *rr, int *cc, T *val, int cb) {
#pragma unroll
                    for (int q = 0; q < 8; q++) {
                        int n = rr[q], c = cb + cc[q];
                        if (c0 + n < k) out[(int64_t)c * k + c0 + n] = -val[q];
                    }
                });
        }
        return;
    }
    __shared__ BwdLds<T, KT> sh;
    for (int64_t i = threadIdx.x; i < (int64_t)SB * k; i += blockDim.x) out[i] = (T)0;
    auto xrow = [&](int r) { return Y + (int64_t)rw[r] * k; };
    for (int c0 = 0; c0 < k; c0 += KT)
        if constexpr (KT <= 4)
            bwd_cols_lanes<T, KT>(L, front_ld(m), ab, na, max(r0, p), r1, xrow, k, c0, out, sh.Ls);
        else if constexpr (sizeof(T) == 4)   // measured: staged 64 rows at a time is faster in FP32, not in FP64
            bwd_cols_staged<T, KT>(L, front_ld(m), ab, na, max(r0, p), r1, xrow, k, c0, out, sh.Ls, sh.Ss);
        else
            bwd_cols_any<T, KT>(L, front_ld(m), ab, na, max(r0, p), r1, xrow, k, c0, out, sh.Ls, sh.Ss);
}

// task = (front, column block a, first slot, slots): v_a = y_a + sum of the partial blocks (in slot order)
template <typename T>
__global__ __launch_bounds__(THREADS) void k_bwd_below_sum(const int4 *__restrict__ tasks, SolveArgs<T> a)
{
    int4 t = tasks[blockIdx.x];
    int f = t.x, ab = t.y * SB;
    int p = a.pfront[f], k = a.k, f0 = a.first[f];
    int na = min(SB, p - ab);
    T *w = a.W + a.woff[f] * k + (int64_t)ab * k;
    const T *y = a.Y + (int64_t)(f0 + ab) * k;
    int64_t tot = (int64_t)na * k;
    if ((k & 3) == 0) {     // four consecutive elements per thread (vector accesses)
        typedef typename Vec4<T>::type V4;
        for (int64_t i = 4 * (int64_t)threadIdx.x; i < tot; i += 4 * (int64_t)blockDim.x) {
            V4 s = *reinterpret_cast<const V4 *>(y + i);
            for (int q = 0; q < t.w; q++) {
                V4 v = *reinterpret_cast<const V4 *>(a.part + (int64_t)(t.z + q) * SB * k + i);
                s.x += v.x;
                s.y += v.y;
                s.z += v.z;
                s.w += v.w;
            }
            *reinterpret_cast<V4 *>(w + i) = s;
        }
        return;
    }
    for (int64_t i = threadIdx.x; i < tot; i += blockDim.x) {
        T s = y[i];
        for (int q = 0; q < t.w; q++) s += a.part[(int64_t)(t.z + q) * SB * k + i];
        w[i] = s;
    }
}

// ---- super-block inverses (after the factorization)
// ---- products with the factor itself (Y row-major n x k in pivot order)
//
// L^T Y: task = (front, column block a).  Output row first + ab + c is
// sum over the front's rows r >= ab + c of L(r, ab + c) Yin(rows[r]); every
// pivot row belongs to exactly one front, so no two tasks write a row.  The
// front's rows [ab, m) are split over the four waves in multiples of 16.
template <typename T>
__global__ __launch_bounds__(THREADS, sizeof(T) == 4 ? 3 : 2) void k_apply_lt(const int2 *__restrict__ tasks, SolveArgs<T> a,
                                                      const T *__restrict__ Yin, T *__restrict__ Yout)
{
    __shared__ MmLds<T> mm;
    int2 t = tasks[blockIdx.x];
    int f = t.x, ab = t.y * SB;
    int m = a.mfront[f], p = a.pfront[f], k = a.k, ld = front_ld(m);
    int na = min(SB, p - ab), first = a.first[f];
    const T *L = a.fronts + a.front_off[f];
    const int32_t *rw = a.rows + a.rptr[f];
    int wave = threadIdx.x / 64;
    int per = ((m - ab + 63) / 64) * 16;
    int rb = ab + wave * per, re = min(m, rb + per);
    for (int c0 = 0; c0 < k; c0 += 64) {
        typename Mfma<T>::V acc[4][4];
#pragma unroll
        for (int x = 0; x < 4; x++)
#pragma unroll
            for (int y = 0; y < 4; y++)
#pragma unroll
                for (int e = 0; e < 4; e++) acc[x][y][e] = 0;
        if (rb < re)
            wave_mm<T>(
                acc, rb, re,
                [&](int c, int r) { return (c < na && r >= ab + c) ? L[(int64_t)(ab + c) * ld + r] : (T)0; },
                [&](int r, int col) { return c0 + col < k ? Yin[(int64_t)rw[r] * k + c0 + col] : (T)0; });
        reduce4<T>(acc, mm.red, [&](int *rr, int *cc, T *val, int cb) {
#pragma unroll
            for (int q = 0; q < 8; q++) {
                int c = rr[q], col = cb + cc[q];
                if (c < na && c0 + col < k) Yout[(int64_t)(first + ab + c) * k + c0 + col] = val[q];
            }
        });
    }
}

// L Y, first pass: task = (front, 64-row tile).  W row woff[f] + r of the
// front's own row block gets sum over its pivot columns c <= r of
// L(r, c) Yin(first + c); k_apply_gather then adds up, for every row of Y,
// the W rows of all fronts that hold it.
template <typename T>
__global__ __launch_bounds__(THREADS, sizeof(T) == 4 ? 3 : 2) void k_apply_l(const int2 *__restrict__ tasks, SolveArgs<T> a,
                                                     const T *__restrict__ Yin, T *__restrict__ W)
{
    __shared__ MmLds<T> mm;
    int2 t = tasks[blockIdx.x];
    int f = t.x, r0 = t.y * SB;
    int m = a.mfront[f], p = a.pfront[f], k = a.k, ld = front_ld(m);
    int nr = min(SB, m - r0), first = a.first[f];
    int kend = min(p, r0 + SB);   // columns c <= r < r0 + SB
    const T *L = a.fronts + a.front_off[f];
    T *out = W + a.woff[f] * k;
    int wave = threadIdx.x / 64;
    int per = ((kend + 63) / 64) * 16;
    int cb0 = wave * per, ce = min(kend, cb0 + per);
    for (int c0 = 0; c0 < k; c0 += 64) {
        typename Mfma<T>::V acc[4][4];
#pragma unroll
        for (int x = 0; x < 4; x++)
#pragma unroll
            for (int y = 0; y < 4; y++)
#pragma unroll
                for (int e = 0; e < 4; e++) acc[x][y][e] = 0;
        if (cb0 < ce)
            wave_mm<T>(
                acc, cb0, ce,
                [&](int rr, int c) { return (rr < nr && c <= r0 + rr) ? L[(int64_t)c * ld + r0 + rr] : (T)0; },
                [&](int c, int col) { return c0 + col < k ? Yin[(int64_t)(first + c) * k + c0 + col] : (T)0; });
        reduce4<T>(acc, mm.red, [&](int *rr, int *cc, T *val, int cb) {
#pragma unroll
            for (int q = 0; q < 8; q++) {
                int r = rr[q], col = cb + cc[q];
                if (r < nr && c0 + col < k) out[(int64_t)(r0 + r) * k + c0 + col] = val[q];
            }
        });
    }
}

// L Y, second pass: Y(i) = sum of the W rows glist[gptr[i] .. gptr[i+1]) (in
// that fixed order: fronts ascending), i.e. every front's contribution to row i
template <typename T>
__global__ void k_apply_gather(const int64_t *__restrict__ gptr, const int64_t *__restrict__ glist, int n, int k,
                               const T *__restrict__ W, T *__restrict__ Y)
{
    int64_t total = (int64_t)n * k;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        int i = (int)(idx / k), c = (int)(idx % k);
        T s = 0;
        for (int64_t q = gptr[i]; q < gptr[i + 1]; q++) s += W[glist[q] * k + c];
        Y[idx] = s;
    }
}

// task = (front, super-block index si, column block jb): X_jj = L_jj^-1 (the
// stored 64-block inverse), then for i > j: X_ij = -L_ii^-1 sum_{j <= q < i} L_iq X_qj.
// Rows and columns past the end of the super-block are zero.
template <typename T>
__global__ __launch_bounds__(THREADS) void k_build_xinv(const int4 *__restrict__ tasks, const int64_t *__restrict__ front_off,
                                                        const int32_t *__restrict__ mfront,
                                                        const int32_t *__restrict__ pfront,
                                                        const int64_t *__restrict__ dscr_off,
                                                        const int64_t *__restrict__ xoff, const T *__restrict__ fronts,
                                                        const T *__restrict__ dinv, T *__restrict__ xinv)
{
    __shared__ T D[SB][SB + 1];
    __shared__ T S[SB][64];
    int4 t = tasks[blockIdx.x];
    int f = t.x, s0 = t.y * SS, jb = t.z;
    int m = mfront[f], p = pfront[f], ld = front_ld(m);
    int s1 = min(p, s0 + SS);
    int nblk = (s1 - s0 + SB - 1) / SB;
    int j0 = s0 + jb * SB, nj = min(SB, s1 - j0);
    const T *L = fronts + front_off[f];
    T *X = xinv + xoff[f] + (int64_t)t.y * SS * SS;
    auto Xat = [&](int ib, int r, int c) -> T & { return X[(int64_t)(jb * SB + c) * SS + ib * SB + r]; };
    // X_jj: the stored inverse of block j (column-major 64 x 64, identity-padded)
    const T *Dj = dinv + dscr_off[f] + (int64_t)(j0 / SB) * SB * SB;
    for (int e = threadIdx.x; e < SB * SB; e += THREADS) {
        int c = e / SB, r = e % SB;
        Xat(jb, r, c) = (r < nj && c < nj) ? Dj[e] : (T)0;
    }
    for (int ib = jb + 1; ib < nblk; ib++) {
        int i0 = s0 + ib * SB, ni = min(SB, s1 - i0);
        BlkAcc<T, 64> acc;
        acc.zero();
        // T_i = sum_q L_iq X_qj
        for (int qb = jb; qb < ib; qb++) {
            int q0 = s0 + qb * SB, nq = min(SB, s1 - q0);
            __syncthreads();
            for (int e = threadIdx.x; e < SB * SB; e += THREADS) {
                int q = e / SB, i = e % SB;            // L(i0 + i, q0 + q) applied to X row q for output row i
                D[q][i] = (i < ni && q < nq) ? L[(int64_t)(q0 + q) * ld + i0 + i] : (T)0;
            }
            for (int e = threadIdx.x; e < SB * 64; e += THREADS) {
                int q = e / 64, c = e % 64;
                S[q][c] = Xat(qb, q, c);
            }
            __syncthreads();
            acc.add(D, S);
        }
        __syncthreads();
        acc.store(SB, 64, 0, [&](int r, int c, T val) { S[r][c] = val; });
        // X_ij = -L_ii^-1 T_i
        const T *Di = dinv + dscr_off[f] + (int64_t)(i0 / SB) * SB * SB;
        for (int e = threadIdx.x; e < SB * SB; e += THREADS) {
            int c = e / SB, r = e % SB;                 // Linv(r, c) applied to T row c for output row r
            D[c][r] = Di[e];
        }
        __syncthreads();
        BlkAcc<T, 64> res;
        res.zero();
        res.add(D, S);
        __syncthreads();
        res.store(SB, 64, 0, [&](int r, int c, T val) { Xat(ib, r, c) = (r < ni && c < nj) ? -val : (T)0; });
        __syncthreads();
    }
}

}  // namespace dev
}  // namespace wcs
