// Device kernels of the multifrontal sparse Cholesky (gfx950).
//
// Storage: every front (amalgamated supernode) s owns an m x m column-major
// buffer at front_off[s]; its first p columns become the factor panel
// [L11; L21] and its trailing (m-p) x (m-p) lower triangle the update
// (Schur complement) matrix that is added into the parent front.
//
// Dense steps inside a front are blocked right-looking Cholesky with panel
// width NB: factor the NB x NB diagonal block, solve the rows below it
// against that block, then subtract the panel's outer product from the
// trailing lower triangle on the matrix cores (16x16x4 MFMA).
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wcs {
namespace dev {

constexpr int NB = 64;        // panel width
constexpr int TS = 64;        // trailing-update tile (TS x TS per workgroup)
constexpr int TR = 64;        // rows per triangular-solve tile
constexpr int EA_COLS = 8;    // update-matrix columns per extend-add task
constexpr int THREADS = 256;

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
// Operand layout of both 16x16x4 forms: lane l supplies A(l%16, l/16) and
// B(l/16, l%16).  The accumulator layout differs: element e of lane l holds
// C(4*(l/16) + e, l%16) for f32 and C(4*e + l/16, l%16) for f64.
template <> struct Mfma<float> {
    typedef floatx4 V;
    static __device__ __forceinline__ int row(int kq, int e) { return 4 * kq + e; }
    static __device__ __forceinline__ V mma(float a, float b, V c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <> struct Mfma<double> {
    typedef doublex4 V;
    static __device__ __forceinline__ int row(int kq, int e) { return 4 * e + kq; }
    static __device__ __forceinline__ V mma(double a, double b, V c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

// ---------------------------------------------------------------- utilities

template <typename T>
__global__ void k_fill(T *__restrict__ p, int64_t n, T v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

// fronts[amap[e]] = values[e]: the stored entries of A into their fronts
template <typename T>
__global__ void k_scatter(const double *__restrict__ values, const int64_t *__restrict__ amap, int64_t nnz,
                          T *__restrict__ fronts)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < nnz; i += stride) fronts[amap[i]] = (T)values[i];
}

// ---------------------------------------------------------------- extend-add
// task = (child front, first update column).  The child's update matrix
// U = F_c[p_c:m_c, p_c:m_c] (lower) is added into its parent front through
// rel (positions of the child's update rows in the parent's row list).  All
// tasks of one launch have distinct parents, so the adds do not race.
template <typename T>
__global__ void k_extend_add(const int2 *__restrict__ tasks, const int64_t *__restrict__ front_off,
                             const int32_t *__restrict__ mfront, const int32_t *__restrict__ pfront,
                             const int32_t *__restrict__ sparent, const int64_t *__restrict__ rptr,
                             const int32_t *__restrict__ rel, T *__restrict__ fronts)
{
    int2 t = tasks[blockIdx.x];
    int c = t.x;
    int mc = mfront[c], pc = pfront[c];
    int nu = mc - pc;
    int par = sparent[c];
    int mp = mfront[par];
    const T *U = fronts + front_off[c] + (int64_t)pc * mc + pc;
    T *Fp = fronts + front_off[par];
    const int32_t *rl = rel + rptr[c] + pc;
    int c1 = min(t.y + EA_COLS, nu);
    for (int col = t.y; col < c1; col++) {
        int pcol = rl[col];
        const T *u = U + (int64_t)col * mc;
        T *dst = Fp + (int64_t)pcol * mp;
        for (int r = col + threadIdx.x; r < nu; r += blockDim.x) dst[rl[r]] += u[r];
    }
}

// ---------------------------------------------------------------- panel
// task = (front, tile).  Every workgroup factors the diagonal block
// F[k0:k0+nb, k0:k0+nb] in LDS (in precision TD); tile 0 writes it back, tile
// t >= 1 solves rows [k0+nb+(t-1)*TR, ...) of the panel: X = B * L_kk^-T.
// A non-positive (or NaN) pivot is reported through atomicMin on *bad (in
// global pivot numbering) and replaced by 1 so the rest stays finite.
template <typename T, typename TD>
__global__ __launch_bounds__(THREADS) void k_panel(const int2 *__restrict__ tasks, int k0,
                                                   const int64_t *__restrict__ front_off,
                                                   const int32_t *__restrict__ mfront,
                                                   const int32_t *__restrict__ pfront,
                                                   const int32_t *__restrict__ first, T *__restrict__ fronts,
                                                   int32_t *__restrict__ bad)
{
    __shared__ TD D[NB][NB + 1];     // D[c][r] = L(k0+r, k0+c)
    __shared__ TD X[NB][TR + 1];     // X[c][r] = panel(row r of tile, column c)
    int2 t = tasks[blockIdx.x];
    int f = t.x;
    int m = mfront[f], p = pfront[f];
    int nb = min(NB, p - k0);
    T *F = fronts + front_off[f];
    int tid = threadIdx.x;
    for (int idx = tid; idx < NB * NB; idx += THREADS) {
        int c = idx / NB, r = idx % NB;
        TD v = 0;
        if (c < nb && r < nb && r >= c) v = (TD)F[(int64_t)(k0 + c) * m + k0 + r];
        D[c][r] = v;
    }
    __syncthreads();
    for (int j = 0; j < nb; j++) {
        if (tid == 0) {
            TD d = D[j][j];
            if (!(d > (TD)0)) {
                atomicMin(bad, first[f] + k0 + j);
                d = (TD)1;
            }
            D[j][j] = sqrt(d);
        }
        __syncthreads();
        TD djj = D[j][j];
        for (int r = j + 1 + tid; r < nb; r += THREADS) D[j][r] /= djj;
        __syncthreads();
        int w = nb - j - 1;
        for (int idx = tid; idx < w * w; idx += THREADS) {
            int c = j + 1 + idx / w, r = j + 1 + idx % w;
            if (r >= c) D[c][r] -= D[j][r] * D[j][c];
        }
        __syncthreads();
    }
    if (t.y == 0) {
        for (int idx = tid; idx < nb * nb; idx += THREADS) {
            int c = idx / nb, r = idx % nb;
            if (r >= c) F[(int64_t)(k0 + c) * m + k0 + r] = (T)D[c][r];
        }
        return;
    }
    int r0 = k0 + nb + (t.y - 1) * TR;
    int nr = min(TR, m - r0);
    for (int idx = tid; idx < NB * TR; idx += THREADS) {
        int c = idx / TR, r = idx % TR;
        X[c][r] = (c < nb && r < nr) ? (TD)F[(int64_t)(k0 + c) * m + r0 + r] : (TD)0;
    }
    __syncthreads();
    // X := X * L^-T, column by column: x_c = (b_c - sum_{t<c} x_t L(c,t)) / L(c,c)
    for (int c = 0; c < nb; c++) {
        if (tid < TR) X[c][tid] /= D[c][c];
        __syncthreads();
        int w = nb - c - 1;
        for (int idx = tid; idx < w * TR; idx += THREADS) {
            int cc = c + 1 + idx / TR, r = idx % TR;
            X[cc][r] -= X[c][r] * D[c][cc];
        }
        __syncthreads();
    }
    for (int idx = tid; idx < nb * TR; idx += THREADS) {
        int c = idx / TR, r = idx % TR;
        if (r < nr) F[(int64_t)(k0 + c) * m + r0 + r] = (T)X[c][r];
    }
}

// ---------------------------------------------------------------- trailing update
// task = (front, ti, tj): C = F[i0:i0+TS, j0:j0+TS] -= A * B^T with
// A = F[i0:, k0:k0+nb], B = F[j0:, k0:k0+nb], i0 = k0+nb+ti*TS, j0 = k0+nb+tj*TS.
// Four waves, each a 32 x 32 quarter of the tile as 2 x 2 MFMA 16x16 blocks.
template <typename T>
__global__ __launch_bounds__(THREADS) void k_syrk(const int4 *__restrict__ tasks, int k0,
                                                  const int64_t *__restrict__ front_off,
                                                  const int32_t *__restrict__ mfront,
                                                  const int32_t *__restrict__ pfront, T *__restrict__ fronts)
{
    __shared__ T As[NB][TS + 4];
    __shared__ T Bs[NB][TS + 4];
    int4 t = tasks[blockIdx.x];
    int f = t.x;
    int m = mfront[f], p = pfront[f];
    int nb = min(NB, p - k0);
    int i0 = k0 + nb + t.y * TS, j0 = k0 + nb + t.z * TS;
    T *F = fronts + front_off[f];
    int tid = threadIdx.x;
    for (int idx = tid; idx < NB * TS; idx += THREADS) {
        int k = idx / TS, r = idx % TS;
        bool ok = k < nb;
        As[k][r] = (ok && i0 + r < m) ? F[(int64_t)(k0 + k) * m + i0 + r] : (T)0;
        Bs[k][r] = (ok && j0 + r < m) ? F[(int64_t)(k0 + k) * m + j0 + r] : (T)0;
    }
    __syncthreads();
    int wave = tid / 64, lane = tid % 64;
    int wr = (wave / 2) * 32, wc = (wave % 2) * 32;
    typedef typename Mfma<T>::V V;
    V acc[2][2];
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++)
            for (int e = 0; e < 4; e++) acc[a][b][e] = 0;
    int kq = lane / 16, ln = lane % 16;
    int kmax = (nb + 3) & ~3;
    for (int kk = 0; kk < kmax; kk += 4) {
        T a0 = As[kk + kq][wr + ln], a1 = As[kk + kq][wr + 16 + ln];
        T b0 = Bs[kk + kq][wc + ln], b1 = Bs[kk + kq][wc + 16 + ln];
        acc[0][0] = Mfma<T>::mma(a0, b0, acc[0][0]);
        acc[0][1] = Mfma<T>::mma(a0, b1, acc[0][1]);
        acc[1][0] = Mfma<T>::mma(a1, b0, acc[1][0]);
        acc[1][1] = Mfma<T>::mma(a1, b1, acc[1][1]);
    }
    bool diag = t.y == t.z;
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++) {
            int col = wc + b * 16 + ln;
            if (j0 + col >= m) continue;
            for (int e = 0; e < 4; e++) {
                int row = wr + a * 16 + Mfma<T>::row(kq, e);
                if (i0 + row >= m || (diag && row < col)) continue;
                F[(int64_t)(j0 + col) * m + i0 + row] -= acc[a][b][e];
            }
        }
}

// ---------------------------------------------------------------- solves
// Right-hand sides inside the library are row-major: Y[i * k + c] holds
// column c of pivot row i.  One workgroup per front; lane groups cover
// (rhs, row) pairs.

// gather Y = P B (cast to T)  /  scatter X = P^T Y (cast back)
template <typename T>
__global__ void k_perm_in(const double *__restrict__ B, int64_t ld, const int32_t *__restrict__ perm, int n,
                          int k, T *__restrict__ Y, const double *__restrict__ colscale)
{
    int64_t total = (int64_t)n * k;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        int i = (int)(idx / k), c = (int)(idx % k);
        double v = B[(int64_t)c * ld + perm[i]];
        if (colscale) v *= colscale[c];
        Y[idx] = (T)v;
    }
}

template <typename T>
__global__ void k_perm_out(const T *__restrict__ Y, const int32_t *__restrict__ perm, int n, int k,
                           double *__restrict__ X, int64_t ld, const double *__restrict__ colscale, int accumulate)
{
    int64_t total = (int64_t)n * k;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        int i = (int)(idx / k), c = (int)(idx % k);
        double v = (double)Y[idx];
        if (colscale) v /= colscale[c];
        double *dst = X + (int64_t)c * ld + perm[i];
        if (accumulate) *dst += v;
        else *dst = v;
    }
}

// Plain copies between a caller column-major block and the internal
// row-major layout without permutation (used by the half solves).
template <typename T>
__global__ void k_rows_in(const double *__restrict__ B, int64_t ld, int n, int k, T *__restrict__ Y)
{
    int64_t total = (int64_t)n * k;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        int i = (int)(idx / k), c = (int)(idx % k);
        Y[idx] = (T)B[(int64_t)c * ld + i];
    }
}

template <typename T>
__global__ void k_rows_out(const T *__restrict__ Y, int n, int k, double *__restrict__ X, int64_t ld)
{
    int64_t total = (int64_t)n * k;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        int i = (int)(idx / k), c = (int)(idx % k);
        X[(int64_t)c * ld + i] = (double)Y[idx];
    }
}

// Forward substitution of one front (multifrontal): W = [Y(pivots); 0] plus
// the children's update vectors, then W[0:p] := L11^-1 W[0:p] and
// W[p:m] -= L21 W[0:p]; the pivots' part goes back to Y, W[p:m] stays for
// the parent.
template <typename T>
__global__ __launch_bounds__(THREADS) void k_fwd_front(const int32_t *__restrict__ flist,
                                                       const int64_t *__restrict__ front_off,
                                                       const int32_t *__restrict__ mfront,
                                                       const int32_t *__restrict__ pfront,
                                                       const int32_t *__restrict__ first,
                                                       const int64_t *__restrict__ woff,
                                                       const int32_t *__restrict__ child_ptr,
                                                       const int32_t *__restrict__ child_list,
                                                       const int64_t *__restrict__ rptr,
                                                       const int32_t *__restrict__ rel,
                                                       const T *__restrict__ fronts, T *__restrict__ W,
                                                       T *__restrict__ Y, int k)
{
    int f = flist[blockIdx.x];
    int m = mfront[f], p = pfront[f], f0 = first[f];
    const T *L = fronts + front_off[f];
    T *w = W + woff[f] * k;
    int tid = threadIdx.x;
    int64_t mk = (int64_t)m * k, pk = (int64_t)p * k;
    for (int64_t idx = tid; idx < mk; idx += THREADS) w[idx] = idx < pk ? Y[(int64_t)f0 * k + idx] : (T)0;
    __syncthreads();
    for (int q = child_ptr[f]; q < child_ptr[f + 1]; q++) {
        int c = child_list[q];
        int mc = mfront[c], pc = pfront[c];
        const T *wc = W + woff[c] * k + (int64_t)pc * k;
        const int32_t *rl = rel + rptr[c] + pc;
        int64_t nu = (int64_t)(mc - pc) * k;
        for (int64_t idx = tid; idx < nu; idx += THREADS) {
            int r = (int)(idx / k), cc = (int)(idx % k);
            w[(int64_t)rl[r] * k + cc] += wc[idx];
        }
        __syncthreads();
    }
    for (int j = 0; j < p; j++) {
        const T *col = L + (int64_t)j * m;
        T ljj = col[j];
        // every thread reads w[j] before anyone overwrites it: scale in registers
        int64_t n_upd = (int64_t)(m - j - 1) * k;
        for (int64_t idx = tid; idx < n_upd; idx += THREADS) {
            int r = j + 1 + (int)(idx / k), cc = (int)(idx % k);
            w[(int64_t)r * k + cc] -= col[r] * (w[(int64_t)j * k + cc] / ljj);
        }
        __syncthreads();
        for (int cc = tid; cc < k; cc += THREADS) w[(int64_t)j * k + cc] /= ljj;
        __syncthreads();
    }
    for (int64_t idx = tid; idx < pk; idx += THREADS) Y[(int64_t)f0 * k + idx] = w[idx];
}

// Backward substitution of one front: x_j = (y_j - sum_{i>j} L(i,j) x_i) / L(j,j)
// for the pivots j from last to first, with x of the update rows already
// final (they belong to ancestor fronts).  Reads and writes Y in place.
template <typename T>
__global__ __launch_bounds__(THREADS) void k_bwd_front(const int32_t *__restrict__ flist,
                                                       const int64_t *__restrict__ front_off,
                                                       const int32_t *__restrict__ mfront,
                                                       const int32_t *__restrict__ pfront,
                                                       const int32_t *__restrict__ first,
                                                       const int64_t *__restrict__ woff,
                                                       const int64_t *__restrict__ rptr,
                                                       const int32_t *__restrict__ rows,
                                                       const T *__restrict__ fronts, T *__restrict__ W,
                                                       T *__restrict__ Y, int k)
{
    __shared__ double red[THREADS];
    int f = flist[blockIdx.x];
    int m = mfront[f], p = pfront[f], f0 = first[f];
    const T *L = fronts + front_off[f];
    T *x = W + woff[f] * k;                 // local copy of x over the front's rows
    const int32_t *rw = rows + rptr[f];
    int tid = threadIdx.x;
    int64_t mk = (int64_t)m * k;
    for (int64_t idx = tid; idx < mk; idx += THREADS) {
        int r = (int)(idx / k), cc = (int)(idx % k);
        x[idx] = Y[(int64_t)rw[r] * k + cc];
    }
    __syncthreads();
    // lane groups: g = tid / k handles rows g, g + G, ...; cc = tid % k
    int kk = k < THREADS ? k : THREADS;
    int G = THREADS / kk;
    for (int j = p - 1; j >= 0; j--) {
        const T *col = L + (int64_t)j * m;
        for (int c0 = 0; c0 < k; c0 += kk) {
            int cc = c0 + tid % kk;
            int g = tid / kk;
            double s = 0;
            if (g < G && cc < k)
                for (int r = j + 1 + g; r < m; r += G) s += (double)col[r] * (double)x[(int64_t)r * k + cc];
            red[tid] = s;
            __syncthreads();
            if (tid < kk && c0 + tid < k) {
                double tot = 0;
                for (int gg = 0; gg < G; gg++) tot += red[gg * kk + tid];
                int c = c0 + tid;
                T v = (T)(((double)x[(int64_t)j * k + c] - tot) / (double)col[j]);
                x[(int64_t)j * k + c] = v;
            }
            __syncthreads();
        }
    }
    int64_t pk = (int64_t)p * k;
    for (int64_t idx = tid; idx < pk; idx += THREADS) Y[(int64_t)f0 * k + idx] = x[idx];
}

// ---------------------------------------------------------------- A * X (FP64)
// Full symmetric CSR in the original order; values expanded from the stored
// lower entries by k_expand_values.
__global__ void k_expand_values(const double *__restrict__ values, const int64_t *__restrict__ src, int64_t nnz,
                                double *__restrict__ out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nnz; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = values[src[i]];
}

// R = B - A X  (or Y = A X when B is null), column-major n x k with ld.
// One wave per row; lanes split the row's entries (k columns one after another).
__global__ void k_spmv_colmajor(const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                const double *__restrict__ v, int n, int k, const double *__restrict__ X,
                                const double *__restrict__ B, double *__restrict__ R, int64_t ld)
{
    int wave = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64);
    int lane = threadIdx.x % 64;
    if (wave >= n) return;
    int64_t a = rp[wave], b = rp[wave + 1];
    for (int c = 0; c < k; c++) {
        const double *x = X + (int64_t)c * ld;
        double s = 0;
        for (int64_t q = a + lane; q < b; q += 64) s += v[q] * x[ci[q]];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
        if (lane == 0) {
            int64_t o = (int64_t)c * ld + wave;
            R[o] = B ? B[o] - s : s;
        }
    }
}

// Row-major variant for many right-hand sides: one wave per row, lanes over
// the k columns (k <= 64 per pass), X and R row-major (ld = k).
__global__ void k_spmm_rowmajor(const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                const double *__restrict__ v, int n, int k, const double *__restrict__ X,
                                const double *__restrict__ B, double *__restrict__ R)
{
    int wave = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64);
    int lane = threadIdx.x % 64;
    if (wave >= n) return;
    int64_t a = rp[wave], b = rp[wave + 1];
    for (int c0 = 0; c0 < k; c0 += 64) {
        int c = c0 + lane;
        if (c >= k) break;
        double s = 0;
        for (int64_t q = a; q < b; q++) s += v[q] * X[(int64_t)ci[q] * k + c];
        int64_t o = (int64_t)wave * k + c;
        R[o] = B ? B[o] - s : s;
    }
}

// per-column sum of squares of a column-major block (k columns, ld) -> out[c]
__global__ void k_colnorm2(const double *__restrict__ A, int n, int k, int64_t ld, double *__restrict__ out)
{
    __shared__ double red[THREADS];
    int c = blockIdx.x;
    const double *a = A + (int64_t)c * ld;
    double s = 0;
    for (int i = threadIdx.x; i < n; i += THREADS) s += a[i] * a[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = THREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = red[0];
}

// per-column max |a| of a column-major block
__global__ void k_colamax(const double *__restrict__ A, int n, int k, int64_t ld, double *__restrict__ out)
{
    __shared__ double red[THREADS];
    int c = blockIdx.x;
    const double *a = A + (int64_t)c * ld;
    double s = 0;
    for (int i = threadIdx.x; i < n; i += THREADS) s = fmax(s, fabs(a[i]));
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = THREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = red[0];
}

// scale[c] = amax[c] > 0 ? 1 / amax[c] : 1
__global__ void k_inv_scale(const double *__restrict__ amax, int k, double *__restrict__ scale)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < k) scale[c] = amax[c] > 0 ? 1.0 / amax[c] : 1.0;
}

// ---------------------------------------------------------------- gradient
// gA[e] for stored entry e = (i, j): -(lam_i x_j + lam_j x_i), or -lam_i x_i on the diagonal
__global__ void k_grad_pattern(const int32_t *__restrict__ rowind, const int32_t *__restrict__ colof, int64_t nnz,
                               const double *__restrict__ lam, const double *__restrict__ x,
                               double *__restrict__ gA)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
        int i = rowind[e], j = colof[e];
        gA[e] = i == j ? -lam[i] * x[i] : -(lam[i] * x[j] + lam[j] * x[i]);
    }
}

}  // namespace dev
}  // namespace wcs
