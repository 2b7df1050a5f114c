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
#include "common.h"

namespace wcs {
namespace dev {

template <typename T>
__global__ void k_fill(T *__restrict__ p, int64_t n, T v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

// zero the lower triangle of the pivot columns [c0, c0 + ZCOLS) of a front
// (task = (front, c0)), one wave per column.  The update-matrix columns are
// not zeroed: the front's first trailing update assigns them.
constexpr int ZCOLS = 16;
template <typename T>
__global__ void k_zero_lower(const int2 *__restrict__ tasks, const int64_t *__restrict__ front_off,
                             const int32_t *__restrict__ mfront, const int32_t *__restrict__ pfront,
                             T *__restrict__ fronts)
{
    int2 t = tasks[blockIdx.x];
    int m = mfront[t.x], ld = front_ld(m);
    T *F = fronts + front_off[t.x];
    int c1 = min(t.y + ZCOLS, pfront[t.x]);
    // 16-byte stores over the aligned groups of VEC rows that hold rows >= c (the
    // column starts are 32-byte aligned; a group may reach into the upper
    // triangle or the padding rows, which are zeroed as well: harmless)
    constexpr int VEC = 16 / (int)sizeof(T);
    typedef typename std::conditional<sizeof(T) == 4, float4, double2>::type V;
    int g1 = (m + VEC - 1) / VEC;
    for (int c = t.y + (int)threadIdx.x / 64; c < c1; c += (int)blockDim.x / 64) {
        V *col = reinterpret_cast<V *>(F + (int64_t)c * ld);
        for (int g = c / VEC + (int)threadIdx.x % 64; g < g1; g += 64) col[g] = V{};
    }
}

// fronts[amap[e]] = values[e]: the stored entries of A into their fronts
template <typename T>
__global__ void k_scatter(const double *__restrict__ values, const int64_t *__restrict__ amap, int64_t nnz,
                          T *__restrict__ fronts)
{
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    constexpr int B = 4;   // loads of B entries before their stores
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i0 < nnz; i0 += B * stride) {
        int64_t dst[B];
        T v[B];
#pragma unroll
        for (int b = 0; b < B; b++) {
            int64_t i = i0 + b * stride;
            dst[b] = i < nnz ? amap[i] : -1;
            v[b] = i < nnz ? (T)values[i] : (T)0;
        }
#pragma unroll
        for (int b = 0; b < B; b++)
            if (dst[b] >= 0) fronts[dst[b]] = v[b];
    }
}

// LU fronts: the stored entry e = (r, c), r >= c, carries A[r][c] (lower) and
// A[c][r] (upper); amap[e] is the position of (max, min) of their pivot
// indices, so the L fronts (lower triangle of P A P^T) take A[r][c] when r
// comes after c in pivot order and A[c][r] otherwise, the U^T fronts the other.
__global__ void k_scatter_lu(const double *__restrict__ lower, const double *__restrict__ upper,
                             const int64_t *__restrict__ amap, const int32_t *__restrict__ rowind,
                             const int32_t *__restrict__ colof, const int32_t *__restrict__ iperm, int64_t nnz,
                             double *__restrict__ FL, double *__restrict__ FU)
{
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nnz; i += stride) {
        int64_t dst = amap[i];
        double lo = lower[i], up = upper[i];
        bool flip = iperm[rowind[i]] < iperm[colof[i]];
        FL[dst] = flip ? up : lo;
        FU[dst] = flip ? lo : up;
    }
}

// ---------------------------------------------------------------- extend-add
// task = (child front, first update column).  The child's update matrix
// U = F_c[p_c:m_c, p_c:m_c] (lower) is added into its parent front through
// rel (positions of the child's update rows in the parent's row list).  All
// tasks of one launch have distinct parents, so the adds do not race.
// The update columns split in two: the first split[c] land in the parent's
// pivot columns and are added before the parent is factored (split given:
// columns below split[c] only); the rest land in the parent's own update
// matrix and are added after the parent's trailing updates (split null).
template <typename T>
__global__ __launch_bounds__(256) void k_extend_add(const int2 *__restrict__ tasks, const int64_t *__restrict__ front_off,
                                                    const int32_t *__restrict__ mfront, const int32_t *__restrict__ pfront,
                                                    const int32_t *__restrict__ sparent, const int64_t *__restrict__ rptr,
                                                    const int32_t *__restrict__ rel, const int32_t *__restrict__ split,
                                                    T *__restrict__ fronts)
{
    int2 t = tasks[blockIdx.x];
    int c = t.x;
    int mc = mfront[c], pc = pfront[c];
    int nu = mc - pc;
    int cend = split ? split[c] : nu;
    int par = sparent[c];
    int mp = mfront[par];
    int ldc = front_ld(mc), ldp = front_ld(mp);
    const T *U = fronts + front_off[c] + (int64_t)pc * ldc + pc;
    T *Fp = fronts + front_off[par];
    const int32_t *rl = rel + rptr[c] + pc;
    const int c0 = t.y, nc = min(EA_COLS, cend - c0);
    // each thread keeps its rows for all EA_COLS columns of the task: the row
    // positions are read once, and the loads of every column are in flight
    // together before the adds (one wait for the child, one for the parent)
    int64_t pcol[EA_COLS];
#pragma unroll
    for (int j = 0; j < EA_COLS; j++) pcol[j] = (int64_t)rl[c0 + min(j, nc - 1)] * ldp;
    constexpr int RB = 2;   // rows per thread per round
    for (int r0 = c0 + (int)threadIdx.x; r0 < nu; r0 += RB * (int)blockDim.x) {
        int pr[RB];
        T uv[RB][EA_COLS], dv[RB][EA_COLS];
#pragma unroll
        for (int i = 0; i < RB; i++) {
            int r = r0 + i * (int)blockDim.x;
            pr[i] = r < nu ? rl[r] : 0;
#pragma unroll
            for (int j = 0; j < EA_COLS; j++) {
                bool ok = r < nu && j < nc && r >= c0 + j;
                uv[i][j] = ok ? U[(int64_t)(c0 + j) * ldc + r] : (T)0;
            }
        }
#pragma unroll
        for (int i = 0; i < RB; i++)
#pragma unroll
            for (int j = 0; j < EA_COLS; j++) {
                int r = r0 + i * (int)blockDim.x;
                bool ok = r < nu && j < nc && r >= c0 + j;
                dv[i][j] = Fp[ok ? pcol[j] + pr[i] : 0];
            }
#pragma unroll
        for (int i = 0; i < RB; i++)
#pragma unroll
            for (int j = 0; j < EA_COLS; j++) {
                int r = r0 + i * (int)blockDim.x;
                if (r < nu && j < nc && r >= c0 + j) Fp[pcol[j] + pr[i]] = dv[i][j] + uv[i][j];
            }
    }
}

// ---------------------------------------------------------------- panel
// Broadcast of lane v (a compile-time constant after unrolling) of each row of
// 16 lanes to its row: a DPP row_newbcast move, which stays in the vector
// unit (no round trip through a scalar register, as v_readlane takes).
template <int V>
__device__ __forceinline__ int row_bcast_i(int x)
{
    return __builtin_amdgcn_mov_dpp(x, 0x150 + V, 0xF, 0xF, true);
}
template <int V>
__device__ __forceinline__ float row_bcast_t(float x)
{
    return __int_as_float(row_bcast_i<V>(__float_as_int(x)));
}
template <int V>
__device__ __forceinline__ double row_bcast_t(double x)
{
    return __hiloint2double(row_bcast_i<V>(__double2hiint(x)), row_bcast_i<V>(__double2loint(x)));
}
template <typename T>
__device__ __forceinline__ T row_bcast(T x, int v)
{
    switch (v) {
    case 0: return row_bcast_t<0>(x);
    case 1: return row_bcast_t<1>(x);
    case 2: return row_bcast_t<2>(x);
    case 3: return row_bcast_t<3>(x);
    case 4: return row_bcast_t<4>(x);
    case 5: return row_bcast_t<5>(x);
    case 6: return row_bcast_t<6>(x);
    case 7: return row_bcast_t<7>(x);
    case 8: return row_bcast_t<8>(x);
    case 9: return row_bcast_t<9>(x);
    case 10: return row_bcast_t<10>(x);
    case 11: return row_bcast_t<11>(x);
    case 12: return row_bcast_t<12>(x);
    case 13: return row_bcast_t<13>(x);
    case 14: return row_bcast_t<14>(x);
    default: return row_bcast_t<15>(x);
    }
}

// 1 / sqrt(d) to working precision: the hardware estimate refined by Newton
// steps r <- r (3 - d r^2) / 2 (two for FP64, one for FP32), so that a pivot
// costs one square-root estimate and multiplications instead of a correctly
// rounded square root and divisions.
__device__ __forceinline__ double rsqrt_refined(double d)
{
    double r = __builtin_amdgcn_rsq(d);
    r = r * (1.5 - 0.5 * d * r * r);
    r = r * (1.5 - 0.5 * d * r * r);
    return r;
}
__device__ __forceinline__ float rsqrt_refined(float d)
{
    float r = __builtin_amdgcn_rsqf(d);
    return r * (1.5f - 0.5f * d * r * r);
}

// 16 x 16 x 16 product on one wave: acc += X * Y with X(r, k) = fx(r, k),
// Y(k, n) = fy(k, n); the caller maps acc element e of lane l to
// C(Mfma<TD>::row(l/16, e), l%16).
template <typename TD, typename FX, typename FY>
__device__ __forceinline__ typename Mfma<TD>::V mm16(typename Mfma<TD>::V acc, FX fx, FY fy)
{
    int lane = threadIdx.x % 64, kq = lane / 16, ln = lane % 16;
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) acc = Mfma<TD>::mma(fx(ln, kk + kq), fy(kk + kq, ln), acc);
    return acc;
}

// Broadcast of lane `src` (wave-uniform) of x to every lane, through a scalar
// register (v_readlane).
__device__ __forceinline__ double lane_bcast(double x, int src)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), src),
                            __builtin_amdgcn_readlane(__double2loint(x), src));
}
__device__ __forceinline__ float lane_bcast(float x, int src)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), src));
}

// Factorization of one NB x NB diagonal block held in LDS by all four waves
// of a workgroup.  A: column-major (A[c][r] = block(r, c)), lower part
// meaningful, upper part zero, padded past the block's nb columns with the
// identity; on return it holds the factor L (upper part zero).  Iv receives
// the inverses of the four 16 x 16 diagonal sub-blocks of L (Iv[b][c][r] =
// L_bb^-1(r, c), upper parts zero), Rd the reciprocal pivots.  The caller synchronises the workgroup after
// filling A; the helper ends synchronised, after which waves 1..3 run
// slab(c) for c = 0..3 (work of the caller that needs L and the inverses).
// Right-looking by 16-column blocks: wave 0 factors the block's columns for
// all rows at once, one lane per row holding the 16 columns in registers
// (pivot l_jj = sqrt(a_jj), column l_rj = a_rj / l_jj, then the block's later
// columns a_rc -= l_rj l_cj, with a_jj and l_cj broadcast from their lanes),
// so the pivot chain of the block is 16 short steps; the rows and columns
// after the block are then updated by the panel's 16 x 16 x 16 matrix-core
// products, spread over the four waves.  Last, wave w inverts diagonal
// sub-block w by forward substitution (lane c forms column c).
// A non-positive (or NaN) pivot is reported through atomicMin on *bad (pivot
// number piv0 + column, if report) and replaced by 1 so the rest stays finite.
// 1 / sqrt(d) for a pivot of the diagonal-block factorization: the hardware
// estimate (relative error below 2^-24 in FP64) and one Newton step, which
// leaves a few units in the last place (FP64: about 1e-15 relative; FP32: the
// estimate refined once as well).
template <typename TD> __device__ __forceinline__ TD rsqrt_pivot(TD d)
{
    TD r = sizeof(TD) == 8 ? (TD)__builtin_amdgcn_rsq((double)d) : (TD)__builtin_amdgcn_rsqf((float)d);
    return r * ((TD)1.5 - (TD)0.5 * d * r * r);
}

// the inverses of the four 16 x 16 diagonal sub-blocks of a diagonal block:
// DiagInv<TD>[b][c][r] = L_bb^-1(r, c) (rows padded to 17: lane c's column
// writes fall in distinct banks)
template <typename TD> using DiagInv = TD[NB / 16][16][17];

template <typename TD, typename Slab>
__device__ __forceinline__ void factor_diag_block(TD (&A)[NB][NB + 1], DiagInv<TD> &Iv, TD (&Rd)[NB], int nb,
                                                  bool report, int32_t *bad, int32_t piv0, Slab slab)
{
    typedef typename Mfma<TD>::V VD;
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int kq = lane / 16, ln = lane % 16;
    // A(ib.., jb..) -= L_i L_j^T with the 16 x 16 blocks L of column block kb
    auto syrk_pair = [&](int kb, int ib, int jb) {
        VD acc = {0, 0, 0, 0};
        acc = mm16<TD>(acc, [&](int r, int k) { return A[kb + k][ib + r]; },
                       [&](int k, int n) { return A[kb + k][jb + n]; });
#pragma unroll
        for (int e = 0; e < 4; e++) A[jb + ln][ib + Mfma<TD>::row(kq, e)] -= acc[e];
    };
    // inverse of diagonal sub-block kb: lane c < 16 solves L y = e_c column by
    // column, each y entry taken out of all later right-hand sides at once;
    // the next column of L is read from LDS while the current one is applied
    auto invert = [&](int kb) {
        if (lane < 16) {
            const int c = lane;
            TD y[16], s2[16], rd[16], cur[16], nxt[16];
#pragma unroll
            for (int rr = 0; rr < 16; rr++) {
                s2[rr] = (rr == c) ? (TD)1 : (TD)0;
                rd[rr] = Rd[kb + rr];
                cur[rr] = A[kb][kb + rr];
            }
#pragma unroll
            for (int rr = 0; rr < 16; rr++) {
                if (rr + 1 < 16)
#pragma unroll
                    for (int q = rr + 2; q < 16; q++) nxt[q] = A[kb + rr + 1][kb + q];
                y[rr] = s2[rr] * rd[rr];
#pragma unroll
                for (int q = rr + 1; q < 16; q++) s2[q] -= cur[q] * y[rr];
#pragma unroll
                for (int q = rr + 2; q < 16; q++) cur[q] = nxt[q];
            }
#pragma unroll
            for (int rr = 0; rr < 16; rr++) Iv[kb / 16][c][rr] = y[rr];
        }
    };
    // wave 0: the 16 columns of block kb for all 64 rows (lane = row), two
    // pivots at a time: l_j = a_j / sqrt(a_jj), l_{j+1} = (a_{j+1} - l_j
    // l_{j+1,j}) / sqrt(a_{j+1,j+1} - l_{j+1,j}^2), then the block's later
    // columns a_v -= l_j l_vj + l_{j+1} l_v,j+1; pivot values broadcast from
    // their lanes.  A non-positive pivot is replaced by 1 and the first one
    // reported after the block.
    auto pivots = [&](auto bc_) {
        constexpr int kb = 16 * decltype(bc_)::value;
        TD a[16];
#pragma unroll
        for (int u = 0; u < 16; u++) a[u] = A[kb + u][lane];
        int first_bad = INT32_MAX;
        TD rd_own = 0;
#pragma unroll
        for (int u = 0; u < 16; u += 2) {
            const int j = kb + u;
            TD d0 = lane_bcast(a[u], j);
            TD d01 = lane_bcast(a[u], j + 1);
            TD d1 = lane_bcast(a[u + 1], j + 1);
            if (!(d0 > (TD)0)) {
                first_bad = min(first_bad, j);
                d0 = (TD)1;
            }
            TD r0 = rsqrt_pivot(d0);
            TD l10 = d01 * r0;
            TD e1 = d1 - l10 * l10;
            if (!(e1 > (TD)0)) {
                first_bad = min(first_bad, j + 1);
                e1 = (TD)1;
            }
            TD r1 = rsqrt_pivot(e1);
            TD l0 = (lane == j) ? d0 * r0 : a[u] * r0;
            TD l1 = (lane == j + 1) ? e1 * r1 : (a[u + 1] - l0 * l10) * r1;
            rd_own = (lane == j) ? r0 : (lane == j + 1 ? r1 : rd_own);
            a[u] = l0;
            a[u + 1] = l1;
#pragma unroll
            for (int v = u + 2; v < 16; v++)
                a[v] -= l0 * lane_bcast(l0, kb + v) + l1 * lane_bcast(l1, kb + v);
        }
#pragma unroll
        for (int u = 0; u < 16; u++) A[kb + u][lane] = (lane >= kb + u) ? a[u] : (TD)0;
        if (lane >= kb && lane < kb + 16) Rd[lane] = rd_own;
        if (report && first_bad < nb && lane == 0) atomicMin(bad, piv0 + first_bad);
    };
    // Right-looking over the four column blocks with the next block's updates
    // first: after block b's pivots, waves 1..3 update the column block b + 1
    // (its block pairs), then wave 0 factors it while the others apply block
    // b's remaining pairs and invert block b.
    if (wave == 0) pivots(std::integral_constant<int, 0>());
    __syncthreads();
    static_for<0, NB / 16, 1>([&](auto bc_) {
        constexpr int b = decltype(bc_)::value, kb = 16 * b;
        if constexpr (kb + 16 < NB) {
            // pairs (ib, kb + 16): the next column block, one per wave 1..3
            if (wave > 0 && kb + 16 * wave < NB) syrk_pair(kb, kb + 16 * wave, kb + 16);
            __syncthreads();
            if (wave == 0) {
                pivots(std::integral_constant<int, b + 1>());
            } else {
                int q = 0;
#pragma unroll
                for (int ib = kb + 32; ib < NB; ib += 16)
#pragma unroll
                    for (int jb = kb + 32; jb <= ib; jb += 16)
                        if (q++ % 3 == wave - 1) syrk_pair(kb, ib, jb);
                if (wave == 3 - (b % 3)) invert(kb);
            }
            __syncthreads();
        } else {
            if (wave == 0) invert(kb);   // the last block
            __syncthreads();
        }
    });
    if (wave != 0) static_for<0, NB / 16, 1>([&](auto cc) { slab(cc); });
}

// The factored block (rounded to T, full NB x NB column-major, padding and
// upper part included) and the inverses of its 16 x 16 diagonal sub-blocks
// (rounded to T, zero elsewhere) to global memory; wave w writes columns
// 16 w .. 16 w + 15 (after factor_diag_block: A and Iv complete).
template <typename T, typename TD>
__device__ __forceinline__ void store_diag_block(const TD (&A)[NB][NB + 1], const DiagInv<TD> &Iv, T *D, T *Dinv)
{
    const int r = threadIdx.x % 64, cb = 16 * (threadIdx.x / 64);
    T lv[16];
#pragma unroll
    for (int c = 0; c < 16; c++) lv[c] = (T)A[cb + c][r];
#pragma unroll
    for (int c = 0; c < 16; c++) D[(cb + c) * NB + r] = lv[c];
    if (Dinv) {
#pragma unroll
        for (int c = 0; c < 16; c++) lv[c] = r / 16 == cb / 16 ? (T)Iv[cb / 16][c][r % 16] : (T)0;
#pragma unroll
        for (int c = 0; c < 16; c++) Dinv[(cb + c) * NB + r] = lv[c];
    }
}

// task = (front, tile).  Every workgroup factors the diagonal block
// A = F[k0:k0+nb, k0:k0+nb] (still unfactored in the front), padded to
// NB x NB with the identity (factor_diag_block).  Waves 1..3 own 64-row
// slabs of the panel below the block (rows [k0+nb+t*TRW, +TRW)) and solve
// X L^T = B by 16-column blocks, X_c = (B_c - sum_{j<c} X_j L_cj^T) L_cc^-T,
// as matrix-core products, each block as soon as its diagonal sub-block is
// inverted, while wave 0 factors the next one.  They work on transposed
// blocks (X_c^T = L_cc^-1 (B_c^T - L_cj X_j^T)), so a product's accumulator
// is the next product's B operand: the contraction index of step s in lane
// group q is Mfma<T>::row(q, s), the row an accumulator element holds.
// Tile 0 writes the factored block to `dscr` (the front must keep the
// unfactored block readable for the other workgroups of this launch, and a
// later launch copies it into place; another one inverts it for the solves).
constexpr int TRW = THREADS - 64;   // panel rows per workgroup (waves 1..3)

template <typename T, typename TD>
__global__ __launch_bounds__(THREADS, sizeof(T) == 4 ? 2 : 1) void k_panel(const int2 *__restrict__ tasks, int k0,
                                                   const int64_t *__restrict__ front_off,
                                                   const int32_t *__restrict__ mfront,
                                                   const int32_t *__restrict__ pfront,
                                                   const int32_t *__restrict__ first,
                                                   const int64_t *__restrict__ dscr_off, T *__restrict__ fronts,
                                                   T *__restrict__ dscr, int32_t *__restrict__ bad)
{
    __shared__ TD A[NB][NB + 1];     // column-major: A[c][r] = block(r, c); becomes L
    __shared__ DiagInv<TD> Iv;       // inverses of the 16 x 16 diagonal sub-blocks
    __shared__ TD Rd[NB];            // 1 / L(r, r)
    int2 t = tasks[blockIdx.x];
    int f = t.x;
    int m = mfront[f], p = pfront[f], ld = front_ld(m);
    int nb = min(NB, p - k0);
    T *F = fronts + front_off[f];
    int tid = threadIdx.x;
    int wave = tid / 64, lane = tid % 64;
    int kq = lane / 16, ln = lane % 16;
    int row0 = k0 + nb + t.y * TRW + (wave - 1) * 64;
    typedef typename Mfma<T>::V V;
    // waves 1..3: xs[c][rb] holds the transposed 16 x 16 block (rows
    // row0 + 16 rb.., panel columns 16 c..) of B, later of X: element e of
    // lane (kq, ln) is column 16 c + Mfma<T>::row(kq, e) of row row0 + 16 rb + ln
    V xs[NB / 16][4];
    const bool slab = wave > 0 && row0 < m;
    if (wave == 0) {
        // every load unconditional (clamped into the block) so all 64 are in
        // flight at once; the select afterwards pads with the identity
        const int r = lane;
        const int rc = min(r, nb - 1);
        T raw[NB];
#pragma unroll
        for (int c = 0; c < NB; c++) raw[c] = F[(int64_t)(k0 + min(c, nb - 1)) * ld + k0 + rc];
#pragma unroll
        for (int c = 0; c < NB; c++) A[c][r] = (r < nb && c < nb && c <= r) ? (TD)raw[c] : (c == r ? (TD)1 : (TD)0);
    } else if (row0 < m) {
#pragma unroll
        for (int c = 0; c < NB / 16; c++)
#pragma unroll
            for (int rb = 0; rb < 4; rb++)
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    int row = row0 + rb * 16 + ln, k = c * 16 + Mfma<T>::row(kq, e);
                    xs[c][rb][e] = (row < m && k < nb) ? F[(int64_t)(k0 + k) * ld + row] : (T)0;
                }
    }
    // slab block c: X_c^T = L_cc^-1 (B_c^T - sum_{j<c} L_cj X_j^T), then stored
    auto slab_block = [&](auto cc) {
        constexpr int c = decltype(cc)::value;
        const int kb = 16 * c;
#pragma unroll
        for (int rb = 0; rb < 4; rb++) {
            V acc = xs[c][rb];
#pragma unroll
            for (int j = 0; j < c; j++)
#pragma unroll
                for (int st = 0; st < 4; st++)
                    acc = Mfma<T>::mma(-(T)A[16 * j + Mfma<T>::row(kq, st)][kb + ln], xs[j][rb][st], acc);
            V x = {0, 0, 0, 0};
#pragma unroll
            for (int st = 0; st < 4; st++)
                x = Mfma<T>::mma((T)Iv[c][Mfma<T>::row(kq, st)][ln], acc[st], x);
            xs[c][rb] = x;
            int row = row0 + rb * 16 + ln;
            if (row < m)
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    int n = kb + Mfma<T>::row(kq, e);
                    if (n < nb) F[(int64_t)(k0 + n) * ld + row] = x[e];
                }
        }
    };
    __syncthreads();
    factor_diag_block<TD>(A, Iv, Rd, nb, t.y == 0, bad, first[f] + k0, [&](auto cc) {
        if (slab) slab_block(cc);
    });
    // tile 0: the factored block to the scratch
    if (t.y == 0) store_diag_block<T, TD>(A, Iv, dscr + dscr_off[f] + (int64_t)(k0 / NB) * NB * NB, (T *)nullptr);
}

// ---------------------------------------------------------------- fused panel steps
// Large fronts (p at or above a threshold) are factored by a different
// schedule of the same arithmetic: the diagonal block of every panel is
// factored once, one step ahead, and each panel's triangular solve is fused
// with the update of the rest of its outer block.  Per outer block [K0, kend):
//   k_diag_factor   D_K0 (the block's first diagonal block), once per front;
//   k_step, k0 = K0, K0 + NB, ...: rows below D_k solved against L_kk, the
//                   outer block's later columns updated by the panel, and the
//                   next diagonal block D_{k+1} factored as soon as its last
//                   update lands (by the workgroup that applies it);
// then the trailing updates with the whole outer block, as for other fronts.
// The factored diagonal block sits in the diagonal-block scratch (as the
// panel kernel leaves it) and the inverses of its 16 x 16 diagonal
// sub-blocks in the block's slot of the inverses (replaced by the full block
// inverse once the level is done): the step kernel solves with exactly the
// values the panel kernel uses, so both schedules give the same factor bit
// for bit.

// task = front; factors the diagonal block of pivot columns [k0, k0 + nb) from
// the front (all of its updates applied) into the scratch and the inverse slot.
template <typename T, typename TD>
__global__ __launch_bounds__(THREADS) void k_diag_factor(const int32_t *__restrict__ tasks, int k0,
                                                         const int64_t *__restrict__ front_off,
                                                         const int32_t *__restrict__ mfront,
                                                         const int32_t *__restrict__ pfront,
                                                         const int32_t *__restrict__ first,
                                                         const int64_t *__restrict__ dscr_off,
                                                         const T *__restrict__ fronts, T *__restrict__ dscr,
                                                         T *__restrict__ dinv, int32_t *__restrict__ bad)
{
    __shared__ TD A[NB][NB + 1];
    __shared__ DiagInv<TD> Iv;
    __shared__ TD Rd[NB];
    const int f = tasks[blockIdx.x];
    const int m = mfront[f], p = pfront[f], ld = front_ld(m);
    const int nb = min(NB, p - k0);
    const T *F = fronts + front_off[f];
    // thread (wave, lane) loads row lane of columns wave + 4 i: every load in
    // flight at once (addresses clamped into the block, padding selected after)
    const int r = threadIdx.x % 64, c0 = threadIdx.x / 64;
    T raw[NB / 4];
#pragma unroll
    for (int i = 0; i < NB / 4; i++)
        raw[i] = F[(int64_t)(k0 + min(c0 + 4 * i, nb - 1)) * ld + k0 + min(r, nb - 1)];
#pragma unroll
    for (int i = 0; i < NB / 4; i++) {
        const int c = c0 + 4 * i;
        A[c][r] = (r < nb && c < nb && c <= r) ? (TD)raw[i] : (c == r ? (TD)1 : (TD)0);
    }
    __syncthreads();
    factor_diag_block<TD>(A, Iv, Rd, nb, true, bad, first[f] + k0, [](auto) {});
    const int64_t o = dscr_off[f] + (int64_t)(k0 / NB) * NB * NB;
    store_diag_block<T, TD>(A, Iv, dscr + o, dinv + o);
}

// Task flags of k_step (int4 w); task z = -2 marks a pure copy task whose
// w is the end of its row range.
constexpr int STEP_WRITE = 1;    // write the tile's panel rows X_i
constexpr int STEP_DIAG = 2;     // the tile is the next diagonal block: factor it
constexpr int STEP_DIRECT = 4;   // X_i to its place (else to the transposed position)
constexpr int STEP_COPY = 8;     // move the deferred panels [K0, k0) of the tile's rows into place
constexpr int STEP_COPY_ONLY = -2;

// Panel rows written to the transposed position F[R * ld + C] (R > C: the
// front's upper triangle, never part of L) are moved to F[C * ld + R]: rows
// [r0, r1), columns [c0, c1) (whole panels starting at multiples of NB from
// c0), each panel only for its rows below its diagonal block (R >= panel + NB).
template <typename T>
__device__ __forceinline__ void move_deferred(T *F, int ld, int m, int r0, int r1, int c0, int c1,
                                              T (*tile)[NB + 1])
{
    r1 = min(r1, m);
    for (int cb = c0; cb < c1; cb += NB) {
        const int rs = max(r0, cb + NB);
        for (int rb = rs; rb < r1; rb += NB) {
            const int nr = min(NB, r1 - rb), nc = min(NB, c1 - cb);
            // thread (wave, lane): element lane of rows / columns wave + 4 i, all loads in flight
            const int a = threadIdx.x % 64, b0 = threadIdx.x / 64;
            T v[NB / 4];
#pragma unroll
            for (int i = 0; i < NB / 4; i++)
                v[i] = F[(int64_t)(rb + min(b0 + 4 * i, nr - 1)) * ld + cb + min(a, nc - 1)];
            __syncthreads();
#pragma unroll
            for (int i = 0; i < NB / 4; i++) tile[b0 + 4 * i][a] = v[i];
            __syncthreads();
#pragma unroll
            for (int i = 0; i < NB / 4; i++) {
                const int c = b0 + 4 * i;
                if (a < nr && c < nc) F[(int64_t)(cb + c) * ld + rb + a] = tile[a][c];
            }
        }
    }
}

// One panel step (see above): panel k = pivot columns [k0, k0 + nb) of the
// outer block [K0, min(K0 + nbo, p)).  Task (front, i0, j0, w) owns the
// 64-row tile [i0, i0 + 64) of the rows below D_k (i0 = k0 + nb + 64 t):
//  - X_i = A_i L_kk^-T by 16-column block forward substitution on the matrix
//    cores (the panel kernel's slab solve, from the stored L_kk and
//    sub-block inverses), wave w taking rows 16 w.. of the tile;
//  - j0 >= 0: X_j likewise for rows [j0, j0 + 64) of the panel (the update's
//    B rows), then C(i0.., j0..) -= X_i X_j^T on the lower part of the
//    64 x 64 tile, K = nb, accumulated in the order of the update kernels
//    (wave w: tile columns 16 w.., four interleaved row blocks);
//  - STEP_DIAG (i0 = j0 = k0 + nb): the updated tile is D_{k+1}; it is
//    factored at once and stored like D_k;
//  - STEP_WRITE: X_i goes to the front.  While strips of the outer block
//    follow, other workgroups of the launch still read the panel's unfactored
//    rows, so it goes to the transposed position; the outer block's last step
//    (no strips) writes in place and moves the deferred panels (STEP_COPY,
//    and copy-only tasks for the rows above its own).
template <typename T, typename TD>
__global__ __launch_bounds__(THREADS, 2) void k_step(const int4 *__restrict__ tasks, int k0, int K0, int nbo,
                                                     const int64_t *__restrict__ front_off,
                                                     const int32_t *__restrict__ mfront,
                                                     const int32_t *__restrict__ pfront,
                                                     const int32_t *__restrict__ first,
                                                     const int64_t *__restrict__ dscr_off, T *__restrict__ fronts,
                                                     T *__restrict__ dscr, T *__restrict__ dinv,
                                                     int32_t *__restrict__ bad)
{
    typedef typename Mfma<T>::V V;
    typedef typename Vec4<T>::type V4;
    constexpr int LSZ = NB * (NB + 1);
    // L_kk and the sub-block inverses: rows of LST elements, so that the solve's
    // operand reads (lane group kq reading row 4 kq + s in FP32, row 4 s + kq
    // in FP64) of the four lane groups fall in distinct banks
    constexpr int LST = sizeof(T) == 4 ? NB + 4 : NB + 16;
    // X_i, X_j (k-major): FP64 rows padded to 80 elements; FP32 rows unpadded
    // with columns swizzled by xcol, which keeps the row-block stores (rows
    // 4 kq + e) and the update's reads (rows kk + kq) both free of conflicts
    constexpr int XLD = sizeof(T) == 4 ? NB : NB + 16;
    constexpr size_t PH1 = 2 * (size_t)NB * LST * sizeof(T);            // L_kk, sub-block inverses
    constexpr size_t PH2 = 2 * (size_t)NB * XLD * sizeof(T);            // X_i, X_j
    constexpr size_t PH3 = ((size_t)LSZ + sizeof(DiagInv<TD>) / sizeof(TD) + NB) * sizeof(TD);   // D_{k+1} being factored
    constexpr size_t PH = PH1 > PH2 ? (PH1 > PH3 ? PH1 : PH3) : (PH2 > PH3 ? PH2 : PH3);
    __shared__ __align__(16) char smem[PH];
    T(*Ls)[LST] = reinterpret_cast<T(*)[LST]>(smem);
    T(*Ivs)[LST] = reinterpret_cast<T(*)[LST]>(smem + (size_t)NB * LST * sizeof(T));
    T(*Lt)[NB + 1] = reinterpret_cast<T(*)[NB + 1]>(smem);   // transpose tile of the deferred-panel moves
    T(*XA)[XLD] = reinterpret_cast<T(*)[XLD]>(smem);
    T(*XB)[XLD] = reinterpret_cast<T(*)[XLD]>(smem + (size_t)NB * XLD * sizeof(T));
    auto xcol = [](int k, int c) { return sizeof(T) == 4 ? c ^ ((((k >> 2) ^ k) & 3) << 4) : c; };
    const int4 t = tasks[blockIdx.x];
    const int f = t.x, i0 = t.y, j0 = t.z, w = t.w;
    const int m = mfront[f], p = pfront[f], ld = front_ld(m);
    const int nb = min(NB, p - k0);
    const int kend = min(K0 + nbo, p);
    T *F = fronts + front_off[f];
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    const int kq = lane / 16, ln = lane % 16;
    if (j0 == STEP_COPY_ONLY) {
        move_deferred<T>(F, ld, m, i0, w, K0, k0, Lt);
        return;
    }
    const int64_t ok = dscr_off[f] + (int64_t)(k0 / NB) * NB * NB;
    {
        // thread (wave, lane): row lane of columns wave + 4 i, all loads in
        // flight; the solve reads only the 16 x 16 blocks of L_kk below its
        // diagonal blocks and the diagonal blocks' inverses, so only those
        // are fetched (whole 64-byte lines of a column each)
        T lv[NB / 4], iv[NB / 4];
#pragma unroll
        for (int i = 0; i < NB / 4; i++) {
            const int c = wave + 4 * i;
            lv[i] = lane >= 16 * (c / 16 + 1) ? dscr[ok + c * NB + lane] : (T)0;
            iv[i] = lane / 16 == c / 16 ? dinv[ok + c * NB + lane] : (T)0;
        }
#pragma unroll
        for (int i = 0; i < NB / 4; i++) {
            Ls[wave + 4 * i][lane] = lv[i];
            Ivs[wave + 4 * i][lane] = iv[i];
        }
    }
    // xs[c][h]: transposed 16 x 16 block (rows 16 wave.. of the tile, panel
    // columns 16 c..) of A_i (h = 0) or A_j (h = 1), later of X: element e of
    // lane (kq, ln) is column 16 c + Mfma<T>::row(kq, e) of row 16 wave + ln.
    // A tile on the diagonal (i0 = j0) has X_j = X_i: solved once.
    const bool two = j0 >= 0, dtile = j0 == i0;
    V xs[NB / 16][2];
#pragma unroll
    for (int h = 0; h < 2; h++) {
        const int row = (h ? j0 : i0) + 16 * wave + ln;
        const bool rok = (h == 0 || (two && !dtile)) && row < m;
#pragma unroll
        for (int c = 0; c < NB / 16; c++)
#pragma unroll
            for (int e = 0; e < 4; e++) {
                int k = 16 * c + Mfma<T>::row(kq, e);
                xs[c][h][e] = (rok && k < nb) ? F[(int64_t)(k0 + k) * ld + row] : (T)0;
            }
    }
    // the tile's earlier values, read now (they do not depend on the solve):
    // element x of quad cq[e] is row r0(e) + x of column cl(e) (wave w's
    // columns j0 + 16 w ..): FP64 r0 = i0 + 4 Mfma<T>::row(kq, e), cl = j0 +
    // 16 w + ln, the accumulator's own layout, whose four lane groups cover
    // 16 consecutive rows; FP32 (coalesced order, see the epilogue) r0 = i0 +
    // 4 (lane % 16), cl = j0 + 16 w + 4 e + lane / 16.  A quad reaching past
    // the stored lower part is read element by element (masked elements read
    // as 0 and are not stored)
    constexpr bool colepi = sizeof(T) == 4;
    const int jend = min(j0 + NB, kend);
    auto qrow = [&](int e) { return i0 + 4 * (colepi ? lane % 16 : Mfma<T>::row(kq, e)); };
    auto qcol = [&](int e) { return j0 + 16 * wave + (colepi ? 4 * e + lane / 16 : ln); };
    V4 cq[4];
    if (two) {
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const int r0 = qrow(e), col = qcol(e);
            const T *q = F + (int64_t)col * ld + r0;
            if (col < jend && r0 >= col && r0 + 3 < m) {
                cq[e] = *reinterpret_cast<const V4 *>(q);
            } else {
                T v[4];
#pragma unroll
                for (int x = 0; x < 4; x++) {
                    const int r = r0 + x;
                    v[x] = (col < jend && r >= col && r < m) ? q[x] : (T)0;
                }
                cq[e].x = v[0];
                cq[e].y = v[1];
                cq[e].z = v[2];
                cq[e].w = v[3];
            }
        }
    }
    __syncthreads();
    static_for<0, NB / 16, 1>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        const int kb = 16 * c;
#pragma unroll
        for (int h = 0; h < 2; h++) {
            if (h == 1 && (!two || dtile)) break;
            V acc = xs[c][h];
#pragma unroll
            for (int j = 0; j < c; j++)
#pragma unroll
                for (int st = 0; st < 4; st++)
                    acc = Mfma<T>::mma(-Ls[16 * j + Mfma<T>::row(kq, st)][kb + ln], xs[j][h][st], acc);
            V x = {0, 0, 0, 0};
#pragma unroll
            for (int st = 0; st < 4; st++) x = Mfma<T>::mma(Ivs[kb + Mfma<T>::row(kq, st)][kb + ln], acc[st], x);
            xs[c][h] = x;
        }
    });
    // FP32, panel rows to the transposed position: straight from the
    // registers, where a lane holds four consecutive columns 16 c + 4 kq.. of
    // its row (one 16-byte store each)
    constexpr bool reg_park = sizeof(T) == 4;
    if (reg_park && (w & STEP_WRITE) && !(w & STEP_DIRECT)) {
        const int row = i0 + 16 * wave + ln;
        if (row < m) {
            T *q = F + (int64_t)row * ld + k0;
#pragma unroll
            for (int c = 0; c < NB / 16; c++) {
                const int kb = 16 * c + 4 * kq;
                if (kb + 3 < nb) {
                    V4 o;
                    o.x = xs[c][0][0];
                    o.y = xs[c][0][1];
                    o.z = xs[c][0][2];
                    o.w = xs[c][0][3];
                    *reinterpret_cast<V4 *>(q + kb) = o;
                } else {
#pragma unroll
                    for (int x = 0; x < 4; x++)
                        if (kb + x < nb) q[kb + x] = xs[c][0][x];
                }
            }
        }
    }
    __syncthreads();   // L_kk and the inverses are no longer read (X_i, X_j take their place)
#pragma unroll
    for (int c = 0; c < NB / 16; c++)
#pragma unroll
        for (int e = 0; e < 4; e++) {
            int k = 16 * c + Mfma<T>::row(kq, e);
            XA[k][xcol(k, 16 * wave + ln)] = xs[c][0][e];
            if (two) XB[k][xcol(k, 16 * wave + ln)] = xs[c][dtile ? 0 : 1][e];
        }
    __syncthreads();
    if (w & STEP_WRITE) {
        if (w & STEP_DIRECT) {
            for (int e = tid; e < NB * NB; e += THREADS) {
                int k = e / NB, r = e % NB;
                if (k < nb && i0 + r < m) F[(int64_t)(k0 + k) * ld + i0 + r] = XA[k][xcol(k, r)];
            }
        } else if (!reg_park) {
            for (int e = tid; e < NB * NB; e += THREADS) {
                int r = e / NB, k = e % NB;
                if (k < nb && i0 + r < m) F[(int64_t)(i0 + r) * ld + k0 + k] = XA[k][xcol(k, r)];
            }
        }
    }
    if (two) {
        V acc[4];
#pragma unroll
        for (int x = 0; x < 4; x++) acc[x] = V{0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < NB; kk += 4) {
            V4 a4 = *reinterpret_cast<const V4 *>(&XA[kk + kq][xcol(kk + kq, 4 * ln)]);
            T b = XB[kk + kq][xcol(kk + kq, 16 * wave + ln)];
            acc[0] = Mfma<T>::mma(a4.x, b, acc[0]);
            acc[1] = Mfma<T>::mma(a4.y, b, acc[1]);
            acc[2] = Mfma<T>::mma(a4.z, b, acc[2]);
            acc[3] = Mfma<T>::mma(a4.w, b, acc[3]);
        }
        // element e of acc[x] is C(row 4 Mfma<T>::row(kq, e) + x, column 16 wave + ln) of the tile:
        // rows come in aligned quads (i0 is a multiple of 4).  FP32: a lane's
        // quads (rows 16 kq + 4 e, e = 0..3) would be stored as 16-byte
        // pieces of 64 cache lines per instruction; they go through LDS
        // (quad rq of the wave's column cl at cl * 64 + 4 (rq ^ cl): distinct
        // banks both ways) and come back as the quads of four whole columns
        T av[4][4];
        if constexpr (colepi) {
            __syncthreads();   // every wave is done with X_i, X_j
            T *Q = reinterpret_cast<T *>(smem) + wave * 16 * 64;
#pragma unroll
            for (int e = 0; e < 4; e++) {
                V4 v;
                v.x = acc[0][e];
                v.y = acc[1][e];
                v.z = acc[2][e];
                v.w = acc[3][e];
                *reinterpret_cast<V4 *>(Q + ln * 64 + 4 * ((4 * kq + e) ^ ln)) = v;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int cl = 4 * e + lane / 16, rq = lane % 16;
                const V4 v = *reinterpret_cast<const V4 *>(Q + cl * 64 + 4 * (rq ^ cl));
                av[e][0] = v.x;
                av[e][1] = v.y;
                av[e][2] = v.z;
                av[e][3] = v.w;
            }
        } else {
#pragma unroll
            for (int e = 0; e < 4; e++)
#pragma unroll
                for (int x = 0; x < 4; x++) av[e][x] = acc[x][e];
        }
        T nv[4][4];
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const int r0 = qrow(e), col = qcol(e);
            T *q = F + (int64_t)col * ld + r0;
            nv[e][0] = cq[e].x - av[e][0];
            nv[e][1] = cq[e].y - av[e][1];
            nv[e][2] = cq[e].z - av[e][2];
            nv[e][3] = cq[e].w - av[e][3];
            if (col < jend && r0 >= col && r0 + 3 < m) {
                V4 o;
                o.x = nv[e][0];
                o.y = nv[e][1];
                o.z = nv[e][2];
                o.w = nv[e][3];
                *reinterpret_cast<V4 *>(q) = o;
            } else {
#pragma unroll
                for (int x = 0; x < 4; x++) {
                    const int r = r0 + x;
                    if (col < jend && r >= col && r < m) q[x] = nv[e][x];
                    else nv[e][x] = 0;
                }
            }
        }
        if (w & STEP_DIAG) {
            // D_{k+1} = the updated tile (i0 = j0 = k0 + nb): factor it now
            TD(*A)[NB + 1] = reinterpret_cast<TD(*)[NB + 1]>(smem);
            DiagInv<TD> &Iv = *reinterpret_cast<DiagInv<TD> *>(smem + (size_t)LSZ * sizeof(TD));
            TD *Rd = reinterpret_cast<TD *>(smem + (size_t)LSZ * sizeof(TD) + sizeof(DiagInv<TD>));
            const int nb2 = min(NB, p - j0);
            __syncthreads();   // X_i, X_j no longer read
            // the lanes' 16 elements each cover the tile once: the block's
            // lower part, the identity past nb2, zero elsewhere
#pragma unroll
            for (int e = 0; e < 4; e++)
#pragma unroll
                for (int x = 0; x < 4; x++) {
                    const int c = qcol(e) - j0, r = qrow(e) - i0 + x;
                    A[c][r] = (r < nb2 && c < nb2 && c <= r) ? (TD)nv[e][x] : (c == r && r >= nb2) ? (TD)1 : (TD)0;
                }
            __syncthreads();
            factor_diag_block<TD>(*reinterpret_cast<TD(*)[NB][NB + 1]>(A), Iv, *reinterpret_cast<TD(*)[NB]>(Rd), nb2,
                                  true, bad, first[f] + j0, [](auto) {});
            const int64_t o2 = dscr_off[f] + (int64_t)(j0 / NB) * NB * NB;
            store_diag_block<T, TD>(*reinterpret_cast<TD(*)[NB][NB + 1]>(A), Iv, dscr + o2, dinv + o2);
        }
    }
    if (w & STEP_COPY) move_deferred<T>(F, ld, m, i0, i0 + NB, K0, k0, Lt);
}

// Every factored NB x NB diagonal block of a level's fronts (task = (front,
// block)), from its copy in dscr: copied into the lower triangle of its place
// in the front, and inverted in FP64 and rounded to T into dinv (column major,
// same offsets).  One wave per block; lane c forms column c of L^-1 by forward
// substitution, right-looking (15 and more independent updates per step).
// The triangular solves use these; nothing in the factorization reads them,
// so each level's blocks are handled beside the levels above it, off the
// panel chain.
template <typename T>
__global__ __launch_bounds__(64) void k_diag_inv(const int2 *__restrict__ tasks,
                                                 const int64_t *__restrict__ dscr_off, const T *__restrict__ dscr,
                                                 T *__restrict__ dinv, const int64_t *__restrict__ front_off,
                                                 const int32_t *__restrict__ mfront,
                                                 const int32_t *__restrict__ pfront, T *__restrict__ fronts)
{
    __shared__ double L[NB][NB + 1];   // column-major: L[c][r] = L(r, c)
    int2 t = tasks[blockIdx.x];
    int64_t o = dscr_off[t.x] + (int64_t)t.y * NB * NB;
    const T *D = dscr + o;
    const int c = threadIdx.x;
    {
        // lane c loads row c of every column (all loads in flight)
        T v[NB];
#pragma unroll
        for (int j = 0; j < NB; j++) v[j] = D[j * NB + c];
        const int k0 = t.y * NB, nb = min(NB, pfront[t.x] - k0), ld = front_ld(mfront[t.x]);
        T *F = fronts + front_off[t.x] + (int64_t)k0 * ld + k0;
#pragma unroll
        for (int j = 0; j < NB; j++)
            if (c < nb && c >= j) F[(int64_t)j * ld + c] = v[j];
#pragma unroll
        for (int j = 0; j < NB; j++) L[j][c] = (double)v[j];
    }
    __syncthreads();
    double y[NB];
#pragma unroll
    for (int r = 0; r < NB; r++) y[r] = (r == c) ? 1.0 : 0.0;
#pragma unroll
    for (int r = 0; r < NB; r++) {
        y[r] = y[r] / L[r][r];
#pragma unroll
        for (int q = r + 1; q < NB; q++) y[q] -= L[r][q] * y[r];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < NB; r++) L[c][r] = y[r];
    __syncthreads();
    for (int i = c; i < NB * NB; i += 64) dinv[o + i] = (T)L[i / NB][i % NB];
}

// ---------------------------------------------------------------- leaf fronts
// Persistent factorization of the leaf fronts (no children) of one or many
// assembly trees in a single launch: every workgroup takes the next front
// from a queue (fronts listed largest first; *counter starts at 0 and is
// advanced atomically) until the queue is empty, so every workgroup exits.
// The front's pivot columns (m x p, zeroed and filled with A beforehand) are
// staged in LDS, column-major with leading dimension sld (= 16 mod 32, so the
// four k-columns a wave reads per matrix-core step fall in distinct bank
// halves), and factored by right-looking column steps (l_jj = sqrt(a_jj),
// l_ij = a_ij / l_jj below it, then the later pivot columns updated by the
// rank-one product; each element by one thread in a fixed order).  The
// factored panel goes back to the front and its diagonal block to the
// diagonal-block scratch (as the panel kernel's block, identity-padded);
// then the update matrix C = -L21 L21^T (lower triangle; a leaf has no
// children, so it is assigned) is formed on the matrix cores straight from
// the LDS copy, 64 x 64 tiles spread over the waves.  Fronts that fit:
// p <= NB and sld * p <= LeafCfg<T>::ELEMS (the plan routes the others to the
// level-synchronous kernels, which run beside this launch).  A non-positive pivot is reported as in the
// panel kernel.
// LDS of the staged panel: FP32 80 KB (two workgroups per compute unit),
// FP64 156 KB (one); either holds the pivot columns of nearly every leaf
// front of the benchmark matrices
template <typename T> struct LeafCfg {
    static constexpr int BYTES = sizeof(T) == 4 ? 81920 - 64 : 159744 - 64;
    static constexpr int ELEMS = BYTES / (int)sizeof(T);
    static constexpr int PER_CU = sizeof(T) == 4 ? 2 : 1;
};
__host__ __device__ inline int leaf_sld(int m) { return ((m + 15) / 32) * 32 + 16; }

template <typename T>
__global__ __launch_bounds__(THREADS, LeafCfg<T>::PER_CU) void k_leaf(const int32_t *__restrict__ queue, int nq,
                                                     int32_t *__restrict__ counter,
                                                     const int64_t *__restrict__ front_off,
                                                     const int32_t *__restrict__ mfront,
                                                     const int32_t *__restrict__ pfront,
                                                     const int32_t *__restrict__ first,
                                                     const int64_t *__restrict__ dscr_off, T *__restrict__ fronts,
                                                     T *__restrict__ dscr, int32_t *__restrict__ bad)
{
    __shared__ __align__(16) T S[LeafCfg<T>::ELEMS];
    __shared__ int s_task;
    typedef typename Mfma<T>::V V;
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    const int kq = lane / 16, ln = lane % 16;
    for (;;) {
        if (tid == 0) s_task = atomicAdd(counter, 1);
        __syncthreads();
        const int q = s_task;
        __syncthreads();                  // every thread has read s_task (and the last front's LDS use is over)
        if (q >= nq) break;
        const int f = queue[q];
        const int m = mfront[f], p = pfront[f], ld = front_ld(m), sld = leaf_sld(m);
        T *F = fronts + front_off[f];
        for (int c = 0; c < p; c++)
            for (int r = c + tid; r < m; r += THREADS) S[c * sld + r] = F[(int64_t)c * ld + r];
        for (int j = 0; j < p; j++) {
            __syncthreads();              // column j is final
            T d = S[j * sld + j];
            if (!(d > (T)0)) {
                if (tid == 0) atomicMin(bad, first[f] + j);
                d = (T)1;
            }
            const T rp = rsqrt_refined(d);
            __syncthreads();              // every thread has read the pivot
            for (int i = j + tid; i < m; i += THREADS) S[j * sld + i] = i == j ? d * rp : S[j * sld + i] * rp;
            __syncthreads();
            for (int c = j + 1; c < p; c++) {
                const T lc = S[j * sld + c];
                for (int i = c + tid; i < m; i += THREADS) S[c * sld + i] -= S[j * sld + i] * lc;
            }
        }
        __syncthreads();
        for (int c = 0; c < p; c++)
            for (int r = c + tid; r < m; r += THREADS) F[(int64_t)c * ld + r] = S[c * sld + r];
        T *D = dscr + dscr_off[f];
        for (int e = tid; e < NB * NB; e += THREADS) {
            int c = e / NB, r = e % NB;
            D[e] = (r < p && c < p && r >= c) ? S[c * sld + r] : (r == c ? (T)1 : (T)0);
        }
        // update matrix, 64 x 64 tiles of the lower triangle from row and column
        // p rounded down to 4 (earlier rows and columns masked), round robin
        // over the waves.  The A operand takes the tile rows in the order that
        // leaves each lane the results of four consecutive rows of one column
        // (MFMA row 4e + q of the FP64 form holds row 4q + e; the FP32 form
        // already does), so each quad goes out as one 16- or 32-byte store.
        const int p4 = p & ~3, nu = m - p4, nt = (nu + 63) / 64;
        const int arow = sizeof(T) == 8 ? 4 * (ln % 4) + ln / 4 : ln;
        int tile = 0;
        for (int bj = 0; bj < nt; bj++)
            for (int bi = bj; bi < nt; bi++, tile++) {
                if (tile % (THREADS / 64) != wave) continue;
                const int i0 = p4 + 64 * bi, j0 = p4 + 64 * bj;
                V acc[4][4];
#pragma unroll
                for (int x = 0; x < 4; x++)
#pragma unroll
                    for (int y = 0; y < 4; y++)
#pragma unroll
                        for (int e = 0; e < 4; e++) acc[x][y][e] = 0;
                for (int kc = 0; kc < p; kc += 4) {
                    const int k = kc + kq;
                    T av[4], bv[4];
#pragma unroll
                    for (int x = 0; x < 4; x++) {
                        int ra = i0 + 16 * x + arow, rb = j0 + 16 * x + ln;
                        av[x] = (k < p && ra < m) ? S[k * sld + ra] : (T)0;
                        bv[x] = (k < p && rb < m) ? S[k * sld + rb] : (T)0;
                    }
#pragma unroll
                    for (int x = 0; x < 4; x++)
#pragma unroll
                        for (int y = 0; y < 4; y++) acc[x][y] = Mfma<T>::mma(av[x], bv[y], acc[x][y]);
                }
                typedef typename Vec4<T>::type V4;
#pragma unroll
                for (int x = 0; x < 4; x++)
#pragma unroll
                    for (int y = 0; y < 4; y++) {
                        const int r0 = i0 + 16 * x + 4 * kq, col = j0 + 16 * y + ln;
                        if (col < p || col >= m) continue;
                        if (r0 >= col && r0 + 3 < m) {
                            V4 v;
                            v.x = -acc[x][y][0];
                            v.y = -acc[x][y][1];
                            v.z = -acc[x][y][2];
                            v.w = -acc[x][y][3];
                            *reinterpret_cast<V4 *>(F + (int64_t)col * ld + r0) = v;
                        } else {
#pragma unroll
                            for (int e = 0; e < 4; e++)
                                if (r0 + e < m && r0 + e >= col) F[(int64_t)col * ld + r0 + e] = -acc[x][y][e];
                        }
                    }
            }
    }
}

// ---------------------------------------------------------------- LU panel
// LU without pivoting of a front with a symmetric pattern (the nonsymmetric
// matrices of Section 5.1): two buffers with the same layout as the Cholesky
// fronts, FL holding the lower triangle (L and the lower half of the update
// matrix) and FU the upper triangle transposed (U^T and the transposed upper
// half), so that every trailing update is C -= A B^T on a lower triangle:
// FL -= L21 (U12^T)^T and FU -= U12^T L21^T.
//
// task = (front, tile), k0 = the panel's first column.  Every workgroup
// assembles the panel's diagonal block A11 (lower part from FL, strict upper
// from FU, padded to NB x NB with the identity) and factors it as L11 U11
// (Doolittle: unit lower L11, FP64) by 16-column blocks: wave 0 eliminates a
// block's columns for all 64 rows at once (lane = row, pivot row values
// broadcast from the pivot's lane), wave 1 forms the block rows of U to its
// right (U12 = L_bb^-1 A12, a column per lane), waves 2 and 3 invert the
// block's 16 x 16 diagonal parts of L and U, and the rest of the block is
// updated by the 16 x 16 x 16 matrix-core products L21 U12.  The TRW rows of
// the workgroup below the block are then solved by 16-column block
// substitution on the matrix cores: L21 = A21 U11^-1 in FL (X U11 = A21) and
// U12^T = A12^T L11^-T in FU (X L11^T = A12^T), wave w taking 48 rows.  Tile
// 0 writes the factored block to the diagonal-block scratch of both factors
// (L11 with its unit diagonal, U11^T), which a later launch copies into
// place, as for the Cholesky panel.  A zero or non-finite pivot is reported
// through atomicMin on *bad (global pivot numbering) and replaced by 1.
template <typename T>
__global__ __launch_bounds__(THREADS, 1) void k_lu_panel(const int2 *__restrict__ tasks, int k0,
                                                         const int64_t *__restrict__ front_off,
                                                         const int32_t *__restrict__ mfront,
                                                         const int32_t *__restrict__ pfront,
                                                         const int32_t *__restrict__ first,
                                                         const int64_t *__restrict__ dscr_off, T *__restrict__ FL,
                                                         T *__restrict__ FU, T *__restrict__ dscrL,
                                                         T *__restrict__ dscrU, int32_t *__restrict__ bad)
{
    static_assert(sizeof(T) == 8, "the LU factors are FP64");
    typedef typename Mfma<double>::V VD;
    __shared__ double A[NB][NB + 1];     // column-major: A[c][r] = block(r, c); becomes L11 \ U11
    __shared__ double Li[NB][NB + 1];    // inverses of the 16 x 16 diagonal blocks of L11, Li[c][r] = (r, c)
    __shared__ double Ui[NB][NB + 1];    // ... and of U11
    const int2 t = tasks[blockIdx.x];
    const int f = t.x;
    const int m = mfront[f], p = pfront[f], ld = front_ld(m);
    const int nb = min(NB, p - k0);
    T *L = FL + front_off[f];
    T *U = FU + front_off[f];
    const int tid = threadIdx.x;
    const int wave = tid / 64, lane = tid % 64, kq = lane / 16, ln = lane % 16;
    {
        // thread (wave, lane): row lane of columns wave + 4 i, every load in flight
        // (addresses clamped into the block): L below the diagonal, U^T above it
        const int r = lane, c0 = wave, rc = min(r, nb - 1);
        T lv[NB / 4], uv[NB / 4];
#pragma unroll
        for (int i = 0; i < NB / 4; i++) {
            const int cc = min(c0 + 4 * i, nb - 1);
            lv[i] = L[(int64_t)(k0 + cc) * ld + k0 + rc];
            uv[i] = U[(int64_t)(k0 + rc) * ld + k0 + cc];
        }
#pragma unroll
        for (int i = 0; i < NB / 4; i++) {
            const int c = c0 + 4 * i;
            double v = r == c ? 1.0 : 0.0;
            if (r < nb && c < nb) v = r >= c ? (double)lv[i] : (double)uv[i];
            A[c][r] = v;
            Li[c][r] = 0.0;
            Ui[c][r] = 0.0;
        }
    }
    __syncthreads();
    static_for<0, NB / 16, 1>([&](auto bc_) {
        constexpr int kb = 16 * decltype(bc_)::value;
        if (wave == 0) {
            // the block's 16 columns, all rows: pivot d = a_jj, l_rj = a_rj / d
            // below it, a_rv -= l_rj u_jv for the block's later columns
            double a[16];
#pragma unroll
            for (int u = 0; u < 16; u++) a[u] = A[kb + u][lane];
            int first_bad = INT32_MAX;
#pragma unroll
            for (int u = 0; u < 16; u++) {
                const int j = kb + u;
                double d = lane_bcast(a[u], j);
                if (!(d != 0.0 && fabs(d) <= __builtin_huge_val())) {
                    first_bad = min(first_bad, j);
                    d = 1.0;
                    if (lane == j) a[u] = 1.0;
                }
                const double l = a[u] * (1.0 / d);
                const bool below = lane > j;
                if (below) a[u] = l;
#pragma unroll
                for (int v = u + 1; v < 16; v++) {
                    const double ujv = lane_bcast(a[v], j);
                    if (below) a[v] -= l * ujv;
                }
            }
#pragma unroll
            for (int u = 0; u < 16; u++) A[kb + u][lane] = a[u];
            if (t.y == 0 && first_bad < nb && lane == 0) atomicMin(bad, first[f] + k0 + first_bad);
        }
        __syncthreads();
        if (wave == 1) {
            // rows of U to the right of the block: U12 = L_bb^-1 A12, column kb + 16 + lane
            const int col = kb + 16 + lane;
            if (col < NB) {
                double x[16];
#pragma unroll
                for (int tt = 0; tt < 16; tt++) x[tt] = A[col][kb + tt];
#pragma unroll
                for (int tt = 0; tt < 16; tt++)
#pragma unroll
                    for (int q = tt + 1; q < 16; q++) x[q] -= A[kb + tt][kb + q] * x[tt];
#pragma unroll
                for (int tt = 0; tt < 16; tt++) A[col][kb + tt] = x[tt];
            }
        } else if (wave == 2 && lane < 16) {
            // column c of L_bb^-1 (unit diagonal)
            const int c = lane;
            double y[16];
#pragma unroll
            for (int r = 0; r < 16; r++) y[r] = r == c ? 1.0 : 0.0;
#pragma unroll
            for (int tt = 0; tt < 16; tt++)
#pragma unroll
                for (int q = tt + 1; q < 16; q++) y[q] -= A[kb + tt][kb + q] * y[tt];
#pragma unroll
            for (int r = 0; r < 16; r++) Li[kb + c][kb + r] = y[r];
        } else if (wave == 3 && lane < 16) {
            // column c of U_bb^-1, from the last row up
            const int c = lane;
            double y[16];
#pragma unroll
            for (int r = 0; r < 16; r++) y[r] = r == c ? 1.0 : 0.0;
#pragma unroll
            for (int tt = 15; tt >= 0; tt--) {
                y[tt] /= A[kb + tt][kb + tt];
#pragma unroll
                for (int r = 0; r < tt; r++) y[r] -= A[kb + tt][kb + r] * y[tt];
            }
#pragma unroll
            for (int r = 0; r < 16; r++) Ui[kb + c][kb + r] = y[r];
        }
        __syncthreads();
        if constexpr (kb + 16 < NB) {
            // the rest of the block: A22 -= L21 U12, block pairs round-robin over the waves
            int q = 0;
#pragma unroll
            for (int ib = kb + 16; ib < NB; ib += 16)
#pragma unroll
                for (int jb = kb + 16; jb < NB; jb += 16)
                    if (q++ % 4 == wave) {
                        VD acc = {0, 0, 0, 0};
                        acc = mm16<double>(acc, [&](int r, int k) { return A[kb + k][ib + r]; },
                                           [&](int k, int n) { return A[jb + n][kb + k]; });
#pragma unroll
                        for (int e = 0; e < 4; e++) A[jb + ln][ib + Mfma<double>::row(kq, e)] -= acc[e];
                    }
            __syncthreads();
        }
    });
    if (t.y == 0) {
        T *DL = dscrL + dscr_off[f] + (int64_t)(k0 / NB) * NB * NB;
        T *DU = dscrU + dscr_off[f] + (int64_t)(k0 / NB) * NB * NB;
        for (int e = tid; e < NB * NB; e += THREADS) {
            int c = e / NB, r = e % NB;
            DL[e] = (T)(r > c ? A[c][r] : (r == c ? 1.0 : 0.0));
            DU[e] = (T)(r >= c ? A[r][c] : 0.0);        // U11^T: (r, c) = u(c, r)
        }
    }
    // the rows below the block by 16-column block substitution on transposed
    // 16 x 16 blocks (as the Cholesky panel's slab): xs[c][rb] element e of
    // lane (kq, ln) is column 16 c + Mfma::row(kq, e) of row row0 + 16 rb + ln
    constexpr int RB = TRW / 64;     // 16-row blocks per wave
    const int row0 = k0 + nb + t.y * TRW + wave * 16 * RB;
#pragma unroll
    for (int side = 0; side < 2; side++) {
        // side 0: X U11 = A21 in FL; side 1: X L11^T = A12^T in FU
        T *X = side ? U : L;
        VD xs[NB / 16][RB];
#pragma unroll
        for (int c = 0; c < NB / 16; c++)
#pragma unroll
            for (int rb = 0; rb < RB; rb++)
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    const int row = row0 + 16 * rb + ln, k = 16 * c + Mfma<double>::row(kq, e);
                    xs[c][rb][e] = (row < m && k < nb) ? (double)X[(int64_t)(k0 + k) * ld + row] : 0.0;
                }
        static_for<0, NB / 16, 1>([&](auto cc) {
            constexpr int c = decltype(cc)::value;
            constexpr int kb = 16 * c;
#pragma unroll
            for (int rb = 0; rb < RB; rb++) {
                VD acc = xs[c][rb];
#pragma unroll
                for (int j = 0; j < c; j++)
#pragma unroll
                    for (int st = 0; st < 4; st++) {
                        const int kk = 16 * j + Mfma<double>::row(kq, st);
                        // side 0: (U^T)_cj(ln, kk) = U(kk, kb + ln); side 1: L_cj(ln, kk) = L(kb + ln, kk)
                        const double mv = side ? A[kk][kb + ln] : A[kb + ln][kk];
                        acc = Mfma<double>::mma(-mv, xs[j][rb][st], acc);
                    }
                VD x = {0, 0, 0, 0};
#pragma unroll
                for (int st = 0; st < 4; st++) {
                    const int kk = kb + Mfma<double>::row(kq, st);
                    // side 0: (U_cc^-1)^T(ln, kk); side 1: L_cc^-1(ln, kk)
                    const double dv = side ? Li[kk][kb + ln] : Ui[kb + ln][kk];
                    x = Mfma<double>::mma(dv, acc[st], x);
                }
                xs[c][rb] = x;
                const int row = row0 + 16 * rb + ln;
                if (row < m)
#pragma unroll
                    for (int e = 0; e < 4; e++) {
                        const int n = kb + Mfma<double>::row(kq, e);
                        if (n < nb) X[(int64_t)(k0 + n) * ld + row] = (T)x[e];
                    }
            }
        });
    }
}

}  // namespace dev
}  // namespace wcs

#include "update.h"

namespace wcs {
namespace dev {

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
// X[:, c] += a[:, c] (lda > 0) or a (lda == 0: one vector for every column);
// column-major n x k with leading dimension ld
__global__ void k_add_cols(double *__restrict__ X, int64_t ld, int n, int k, const double *__restrict__ a,
                           int64_t lda)
{
    int64_t nk = (int64_t)n * k, stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nk; i += stride) {
        int64_t c = i / n, r = i % n;
        X[c * ld + r] += a[c * lda + r];
    }
}

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

// ---------------------------------------------------------------- A * X (FP64)
// Full symmetric CSR in the original order; values expanded from the stored
// lower entries by k_expand_values.
// Each thread takes eight grid-strided entries per pass, their source indices
// and then their gathered values all in flight before the stores, so that a
// small grid (one that leaves most of the chip to another stream) still keeps
// enough loads outstanding.
__global__ void k_expand_values(const double *__restrict__ values, const int64_t *__restrict__ src, int64_t nnz,
                                double *__restrict__ out)
{
    constexpr int U = 8;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + (U - 1) * stride < nnz; i += U * stride) {
        int64_t s[U];
        double v[U];
#pragma unroll
        for (int u = 0; u < U; u++) s[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
        for (int u = 0; u < U; u++) v[u] = values[s[u]];
#pragma unroll
        for (int u = 0; u < U; u++) __builtin_nontemporal_store(v[u], out + i + u * stride);
    }
    for (; i < nnz; i += stride) out[i] = values[src[i]];
}

// R = B - A X (or Y = A X when B is null).  Element (row i, column c) of X,
// B and R sits at i * sx + c * sc (row-major: sx = k, sc = 1; column-major:
// sx = 1, sc = ld).  Narrow form: one wave per row, lanes split the row's
// entries, one pass per column.  Wide form: one wave per row, lanes are the
// columns (up to 64 per pass), so every matrix entry is read once per pass.
__global__ void k_spmv_narrow(const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                              const double *__restrict__ v, int n, int k, const double *__restrict__ X,
                              const double *__restrict__ B, double *__restrict__ R, int64_t sx, int64_t sc)
{
    int row = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64);
    int lane = threadIdx.x % 64;
    if (row >= n) return;
    int64_t a = rp[row], b = rp[row + 1];
    for (int c = 0; c < k; c++) {
        const double *x = X + (int64_t)c * sc;
        double s = 0;
        for (int64_t q = a + lane; q < b; q += 64) s += v[q] * x[(int64_t)ci[q] * sx];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
        if (lane == 0) {
            int64_t o = (int64_t)row * sx + (int64_t)c * sc;
            R[o] = B ? B[o] - s : s;
        }
    }
}

// One column (k = 1), element i at i * sx: one wave per work item (as in the
// vector form below); a lane takes the entries lane, lane + 64, ... four at a
// time, issuing the index, value and X loads of all four before the products
// (four partial sums, fixed order).
__global__ __launch_bounds__(256) void k_spmv_one(const int4 *__restrict__ items, int nitems,
                                                  const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                  const double *__restrict__ v, const double *__restrict__ X,
                                                  int64_t sx, const double *__restrict__ B, double *__restrict__ R,
                                                  double *__restrict__ P)
{
    int it = blockIdx.x * 4 + (int)threadIdx.x / 64, lane = threadIdx.x % 64;
    if (it >= nitems) return;
    int4 w4 = items[it];
    int row = w4.x;
    int64_t a = rp[row] + w4.y, b = rp[row] + w4.z;
    double s[4] = {0, 0, 0, 0};
    for (int64_t q0 = a + lane; q0 < b; q0 += 256) {
        int c[4];
        double w[4], x[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            int64_t q = q0 + 64 * u;
            bool ok = q < b;
            c[u] = ok ? __builtin_nontemporal_load(ci + q) : 0;
            w[u] = ok ? __builtin_nontemporal_load(v + q) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; u++) x[u] = X[(int64_t)c[u] * sx];
#pragma unroll
        for (int u = 0; u < 4; u++) s[u] += w[u] * x[u];
    }
    double t = (s[0] + s[1]) + (s[2] + s[3]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) t += __shfl_down(t, off, 64);
    if (lane == 0) {
        if (w4.w >= 0) {
            P[w4.w] = t;
        } else {
            int64_t o = (int64_t)row * sx;
            R[o] = B ? B[o] - t : t;
        }
    }
}

// Wide form for row-major X (k columns, leading dimension k): one wave per
// row, lanes are the columns (64 per pass).  Each wave loads 64 (column,
// value) pairs at once with non-temporal loads (the matrix is streamed once
// and should not evict X from the caches) and broadcasts them, keeping eight
// gathers of X rows in flight.  Rows go to XCDs in contiguous ranges (block b
// runs on XCD b % 8), so rows of one subtree of the dissection share an L2.
__global__ __launch_bounds__(256) void k_spmv_wide(const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                   const double *__restrict__ v, int n, int k,
                                                   const double *__restrict__ X, const double *__restrict__ B,
                                                   double *__restrict__ R)
{
    int nrb = (n + 3) / 4;
    int per = (nrb + 7) / 8;
    int rb = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (rb >= nrb) return;
    int row = rb * 4 + (int)threadIdx.x / 64;
    int lane = threadIdx.x % 64;
    if (row >= n) return;
    int64_t a = rp[row], b = rp[row + 1];
    for (int c0 = 0; c0 < k; c0 += 64) {
        int c = c0 + lane;
        bool on = c < k;
        const double *xc = X + (on ? c : 0);
        double s0 = 0, s1 = 0;
        for (int64_t q0 = a; q0 < b; q0 += 64) {
            int cnt = (int)min((int64_t)64, b - q0);
            int myc = lane < cnt ? __builtin_nontemporal_load(ci + q0 + lane) : 0;
            double myv = lane < cnt ? __builtin_nontemporal_load(v + q0 + lane) : 0.0;
            int t = 0;
            for (; t + 8 <= cnt; t += 8) {
                double x[8], w[8];
#pragma unroll
                for (int u = 0; u < 8; u++) {
                    x[u] = xc[(int64_t)__shfl(myc, t + u) * k];
                    w[u] = __shfl(myv, t + u);
                }
#pragma unroll
                for (int u = 0; u < 8; u += 2) {
                    s0 += w[u] * x[u];
                    s1 += w[u + 1] * x[u + 1];
                }
            }
            for (; t < cnt; t++) s0 += __shfl(myv, t) * xc[(int64_t)__shfl(myc, t) * k];
        }
        if (on) {
            int64_t o = (int64_t)row * k + c;
            R[o] = B ? B[o] - (s0 + s1) : (s0 + s1);
        }
    }
}

// Vector form for row-major X with k = EL * LPE columns (EL = 4, LPE = 1, 2,
// 4, 8, 16): a group of LPE lanes takes one matrix entry and EL columns per
// lane (two 8-byte (FP32 X) or 16-byte (FP64 X) loads of the X row), so one
// wave instruction gathers the X rows of 64 / LPE entries at once.  Products
// and sums are FP64 whatever the type of X.  Partial sums of the lane groups
// are added with shuffles (fixed order).  Output R = B - mul[c] (A X), or R =
// A X when B is null (null mul means 1); B may be R itself (each element is
// read and written by one lane).  Rows longer than SPMV_CHUNK entries come in
// several work items that leave partial sums for k_spmv_long_sum (a single
// wave would otherwise walk a row of all N entries alone, after everything
// else).
constexpr int SPMV_CHUNK = 4096;
constexpr int SPMV_GROUP = 3;   // rows of one column pattern per work item (k_spmv_grp)
template <typename TX> struct SpmvVec;
template <> struct SpmvVec<double> {
    using V = double2;
    static constexpr int EL = 4;
    __device__ static double at(const V &x, int j) { return j == 0 ? x.x : x.y; }
};
// FP32 rows: four columns per lane, two 8-byte halves (the FP64 sums of a
// group's rows then fit the register budget of three waves per SIMD)
struct SpmvVecF4 {
    using V = float2;
    static constexpr int EL = 4;
    __device__ static double at(const V &x, int j) { return (double)(j == 0 ? x.x : x.y); }
};

// The product by groups of up to SPMV_GROUP rows with one column pattern
// (g = group rows, -1 past its end): every gathered X row serves
// every row of the group, whose values are read side by side, so a pattern
// shared by three rows (the wavelets of a cell) costs a third of the
// gathers.  Item (group, first entry, chunks of a split group or -1, partial
// slot): a chunk of a split group leaves row r's partial sums in slot
// slot + r * chunks (for k_spmv_long_sum); otherwise R is written as above.
template <int LPE, typename TX, typename SV = SpmvVec<TX>>
__global__ __launch_bounds__(256) void k_spmv_grp(const int4 *__restrict__ items, int nitems,
                                                  const int4 *__restrict__ groups, const int64_t *__restrict__ rp,
                                                  const int32_t *__restrict__ ci, const double *__restrict__ v,
                                                  const TX *__restrict__ X, const double *B,
                                                  const double *__restrict__ mul, double *R, double *__restrict__ P)
{
    using V = typename SV::V;
    constexpr int G = SPMV_GROUP;
    constexpr int EL = SV::EL, H = EL / 2, K = EL * LPE, EPI = 64 / LPE;
    constexpr int U = EPI >= 16 ? 1 : 16 / EPI;   // about 16 entries in flight per wave
    int it = blockIdx.x * 4 + (int)threadIdx.x / 64, lane = threadIdx.x % 64;
    if (it >= nitems) return;
    const int4 w4 = items[it];
    const int4 g4 = groups[w4.x];
    static_assert(G >= 2 && G <= 4, "a group is one int4 of rows");
    const int rows[4] = {g4.x, g4.y, g4.z, g4.w};
    int ng = 1;
#pragma unroll
    for (int g = 1; g < G; g++) ng += rows[g] >= 0;
    const int64_t len = rp[rows[0] + 1] - rp[rows[0]];
    const int64_t a = w4.y, b = min(len, a + (int64_t)SPMV_CHUNK);
    int64_t base[G];
#pragma unroll
    for (int g = 0; g < G; g++) base[g] = g < ng ? rp[rows[g]] : rp[rows[0]];
    int q = lane / LPE, ql = lane % LPE;
    const V *xc = reinterpret_cast<const V *>(X) + 2 * ql;   // a row is 2 LPE vectors V
    double s[G][EL];
#pragma unroll
    for (int g = 0; g < G; g++)
#pragma unroll
        for (int j = 0; j < EL; j++) s[g][j] = 0;
    for (int64_t q0 = a; q0 < b; q0 += 64) {
        int cnt = (int)min((int64_t)64, b - q0);
        int myc = lane < cnt ? __builtin_nontemporal_load(ci + base[0] + q0 + lane) : 0;
        double myv[G];
#pragma unroll
        for (int g = 0; g < G; g++)
            myv[g] = lane < cnt && g < ng ? __builtin_nontemporal_load(v + base[g] + q0 + lane) : 0.0;
        int t = 0;
        for (; t + U * EPI <= cnt; t += U * EPI) {
            V x0[U], x1[U];
            double w[U][G];
#pragma unroll
            for (int u = 0; u < U; u++) {
                int e = t + EPI * u + q;
                const V *pr = xc + (int64_t)__shfl(myc, e) * (2 * LPE);
                x0[u] = pr[0];
                x1[u] = pr[1];
#pragma unroll
                for (int g = 0; g < G; g++) w[u][g] = __shfl(myv[g], e);
            }
#pragma unroll
            for (int u = 0; u < U; u++)
#pragma unroll
                for (int j = 0; j < H; j++) {
                    const double x0j = SV::at(x0[u], j), x1j = SV::at(x1[u], j);
#pragma unroll
                    for (int g = 0; g < G; g++) {
                        s[g][j] += w[u][g] * x0j;
                        s[g][H + j] += w[u][g] * x1j;
                    }
                }
        }
        for (; t < cnt; t += EPI) {
            int e = t + q;
            bool ok = e < cnt;
            int cc = __shfl(myc, ok ? e : t);
            double ww[G];
#pragma unroll
            for (int g = 0; g < G; g++) ww[g] = __shfl(myv[g], ok ? e : t);
            if (ok) {
                const V *pr = xc + (int64_t)cc * (2 * LPE);
                V a0 = pr[0], a1 = pr[1];
#pragma unroll
                for (int j = 0; j < H; j++)
#pragma unroll
                    for (int g = 0; g < G; g++) {
                        s[g][j] += ww[g] * SV::at(a0, j);
                        s[g][H + j] += ww[g] * SV::at(a1, j);
                    }
            }
        }
    }
#pragma unroll
    for (int off = 32; off >= LPE; off >>= 1)
#pragma unroll
        for (int g = 0; g < G; g++)
#pragma unroll
            for (int j = 0; j < EL; j++) s[g][j] += __shfl_down(s[g][j], off, 64);
    if (q == 0) {
#pragma unroll
        for (int g = 0; g < G; g++) {
            if (g >= ng) break;
            if (w4.z >= 0) {      // a chunk of a split group: its partial sums
#pragma unroll
                for (int j = 0; j < EL; j++) P[(int64_t)(w4.w + g * w4.z) * K + EL * ql + j] = s[g][j];
                continue;
            }
            int64_t o = (int64_t)rows[g] * K + EL * ql;
#pragma unroll
            for (int j = 0; j < EL; j++) {
                double r = s[g][j];
                if (mul) r *= mul[EL * ql + j];
                R[o + j] = B ? B[o + j] - r : r;
            }
        }
    }
}

// Long rows: R = B - mul[c] (sum of the row's chunk partials in slot order),
// element (row, c) at row * sx + c; one workgroup per long row (row, first
// slot, slots), threads over the k columns.
__global__ void k_spmv_long_sum(const int4 *__restrict__ rows, int k, int64_t sx, const double *__restrict__ P,
                                const double *B, const double *__restrict__ mul, double *R)
{
    int4 t = rows[blockIdx.x];
    for (int c = threadIdx.x; c < k; c += blockDim.x) {
        double s = 0;
        for (int q = 0; q < t.z; q++) s += P[(int64_t)(t.y + q) * k + c];
        if (mul) s *= mul[c];
        int64_t o = (int64_t)t.x * sx + c;
        R[o] = B ? B[o] - s : s;
    }
}

// The same two permutations through LDS for k >= 4: a workgroup moves a tile
// of 64 caller rows j (original order) by 64 columns, reading and writing
// both layouts with consecutive threads on consecutive addresses (caller side:
// consecutive j of a column; pivot side: consecutive columns of a row, the row
// of j at iperm[j]).
// Xp[iperm[j] * k + c] = X[c * ld + j]
__global__ __launch_bounds__(256) void k_gather_rows_t(const double *__restrict__ X, int64_t ld,
                                                       const int32_t *__restrict__ iperm, int n, int k,
                                                       double *__restrict__ Xp)
{
    __shared__ double T[64][65];
    int j0 = blockIdx.x * 64, c0 = blockIdx.y * 64;
    int nj = min(64, n - j0), nc = min(64, k - c0);
    for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) {
        int c = e / 64, jj = e % 64;
        if (jj < nj && c < nc) T[jj][c] = X[(int64_t)(c0 + c) * ld + j0 + jj];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) {
        int jj = e / 64, c = e % 64;
        if (jj < nj && c < nc) Xp[(int64_t)iperm[j0 + jj] * k + c0 + c] = T[jj][c];
    }
}

// X[c * ld + j] = Xp[iperm[j] * k + c]
__global__ __launch_bounds__(256) void k_scatter_rows_t(const double *__restrict__ Xp,
                                                        const int32_t *__restrict__ iperm, int n, int k,
                                                        double *__restrict__ X, int64_t ld)
{
    __shared__ double T[64][65];
    int j0 = blockIdx.x * 64, c0 = blockIdx.y * 64;
    int nj = min(64, n - j0), nc = min(64, k - c0);
    for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) {
        int jj = e / 64, c = e % 64;
        if (jj < nj && c < nc) T[jj][c] = Xp[(int64_t)iperm[j0 + jj] * k + c0 + c];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) {
        int c = e / 64, jj = e % 64;
        if (jj < nj && c < nc) X[(int64_t)(c0 + c) * ld + j0 + jj] = T[jj][c];
    }
}

// Xp[i * k + c] = X[perm[i] + c * ld]  (caller column-major -> row-major pivot order)
__global__ void k_gather_rows(const double *__restrict__ X, int64_t ld, const int32_t *__restrict__ perm, int n, int k,
                              double *__restrict__ Xp)
{
    int64_t total = (int64_t)n * k;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        int i = (int)(idx / k), c = (int)(idx % k);
        Xp[idx] = X[(int64_t)c * ld + perm[i]];
    }
}

// X[perm[i] + c * ld] = Xp[i * k + c]
__global__ void k_scatter_rows(const double *__restrict__ Xp, const int32_t *__restrict__ perm, int n, int k,
                               double *__restrict__ X, int64_t ld)
{
    int64_t total = (int64_t)n * k;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        int i = (int)(idx / k), c = (int)(idx % k);
        X[(int64_t)c * ld + perm[i]] = Xp[idx];
    }
}

// Y = (T)(R * scale[c])  (same row-major layout).  The grid stride is
// rounded down to a multiple of k, so that every thread stays on one column
// (no division per element; fewer than k threads idle).
template <typename T>
__global__ void k_cast_scaled(const double *__restrict__ R, int64_t total, int k, const double *__restrict__ scale,
                              T *__restrict__ Y)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x / k * k;
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= stride) return;
    const double s = scale ? scale[idx % k] : 1.0;
    for (; idx < total; idx += stride) Y[idx] = (T)(R[idx] * s);
}

// X (+)= Y / scale[c], scale a power of two (the product with its inverse is
// the same number); one column per thread as above
template <typename T>
__global__ void k_add_unscaled(const T *__restrict__ Y, int64_t total, int k, const double *__restrict__ scale,
                               int accumulate, double *__restrict__ X)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x / k * k;
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= stride) return;
    const double inv = scale ? 1.0 / scale[idx % k] : 1.0;
    for (; idx < total; idx += stride) {
        const double y = (double)Y[idx] * inv;
        X[idx] = accumulate ? X[idx] + y : y;
    }
}

// Column reductions of a row-major n x k array, per segment of rows: op 0 sum
// of squares, op 1 max |a|.  seg_ptr (nseg + 1 row offsets) splits the rows
// into independent blocks; null means one segment [0, n).  Each segment gets
// gridDim.x / nseg blocks, each reducing a fixed contiguous row range; the
// final pass adds the partials in block order, so the result is deterministic.
__global__ void k_colred_part(const double *__restrict__ A, int n, int k, int op, const int32_t *__restrict__ seg_ptr,
                              int nseg, double *__restrict__ part)
{
    __shared__ double red[THREADS];
    int bps = gridDim.x / nseg;
    int sg = blockIdx.x / bps, sub = blockIdx.x % bps;
    int64_t s0 = seg_ptr ? seg_ptr[sg] : 0, s1 = seg_ptr ? seg_ptr[sg + 1] : n;
    int64_t r0 = s0 + (s1 - s0) * sub / bps, r1 = s0 + (s1 - s0) * (sub + 1) / bps;
    int kc = k < THREADS ? k : THREADS;
    int groups = THREADS / kc;
    for (int c0 = 0; c0 < k; c0 += kc) {
        int c = c0 + threadIdx.x % kc, g = threadIdx.x / kc;
        double s = 0;
        // unrolled so that eight loads are in flight ahead of the (ordered) sum
        if (g < groups && c < k)
#pragma unroll 8
            for (int64_t r = r0 + g; r < r1; r += groups) {
                double x = A[r * k + c];
                s = op == 0 ? s + x * x : fmax(s, fabs(x));
            }
        red[threadIdx.x] = s;
        __syncthreads();
        if ((int)threadIdx.x < kc && c < k) {
            double t = 0;
            for (int gg = 0; gg < groups; gg++) {
                double x = red[gg * kc + threadIdx.x];
                t = op == 0 ? t + x : fmax(t, x);
            }
            part[(int64_t)blockIdx.x * k + c] = t;
        }
        __syncthreads();
    }
}

// out[sg * k + c] = reduction over the bps partials of segment sg (grid: one block per segment)
// Final pass (one workgroup of THREADS per segment): the partials of a column
// are split over THREADS / k threads (strided), whose sums are then combined
// in thread order; fixed order throughout.
__global__ __launch_bounds__(THREADS) void k_colred_final(const double *__restrict__ part, int bps, int k, int op,
                                                          double *__restrict__ out)
{
    __shared__ double red[THREADS];
    int sg = blockIdx.x;
    int kc = k < THREADS ? k : THREADS, groups = THREADS / kc;
    for (int c0 = 0; c0 < k; c0 += kc) {
        int c = c0 + (int)threadIdx.x % kc, g = (int)threadIdx.x / kc;
        double t = 0;
        if (g < groups && c < k) {
#pragma unroll 8
            for (int b = g; b < bps; b += groups) {
                double x = part[((int64_t)sg * bps + b) * k + c];
                t = op == 0 ? t + x : fmax(t, x);
            }
        }
        red[threadIdx.x] = t;
        __syncthreads();
        if ((int)threadIdx.x < kc && c < k) {
            double u = 0;
            for (int gg = 0; gg < groups; gg++) {
                double x = red[gg * kc + threadIdx.x];
                u = op == 0 ? u + x : fmax(u, x);
            }
            out[(int64_t)sg * k + c] = u;
        }
        __syncthreads();
    }
}

// Column scale of the residual before its FP32 cast: scale[c] = 2^-e with
// 2^e <= amax[c] < 2^(e+1) (1 for a zero or non-finite column); amax[c] is
// overwritten with 2^e = 1 / scale[c]
__global__ void k_inv_scale(double *__restrict__ amax, int k, double *__restrict__ scale)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= k) return;
    double m = amax[c];
    int e = m > 0 && m <= 1.7976931348623157e308 ? ilogb(m) : 0;
    scale[c] = ldexp(1.0, -e);     // a power of two: m * scale in [1, 2), and unscaling is exact
    amax[c] = ldexp(1.0, e);       // its inverse, for the residual update
}

// ---------------------------------------------------------------- theta scheme
// Time stepping of G u' = L u + f with the theta scheme (Section 5, eq:theta)
// in an L2-orthonormal wavelet basis (G = I) and L = -K, K the symmetric
// positive definite operator matrix: A = I + theta dt K is factored once.

// A = I + c K on the stored lower pattern, c = theta dt (entry e at (rowind[e], colof[e]))
__global__ void k_theta_matrix(const int32_t *__restrict__ rowind, const int32_t *__restrict__ colof, int64_t nnz,
                               const double *K, double c, double *A)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x)
        A[e] = c * K[e] + (rowind[e] == colof[e] ? 1.0 : 0.0);
}

// Right-hand side of one step in pivot order from AU = A u:
// (I - (1 - theta) dt K) u = (u - (1 - theta) A u) / theta, plus the forcing
// dt ((1 - theta) f_i + theta f_{i+1}) read through the permutation
__global__ void k_theta_rhs(const double *__restrict__ U, const double *__restrict__ AU,
                            const double *__restrict__ F0, const double *__restrict__ F1,
                            const int32_t *__restrict__ perm, int n, double theta, double dt, double *__restrict__ B)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int o = perm[i];
        B[i] = (U[i] - (1.0 - theta) * AU[i]) / theta + dt * ((1.0 - theta) * F0[o] + theta * F1[o]);
    }
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
