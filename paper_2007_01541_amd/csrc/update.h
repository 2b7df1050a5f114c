// Trailing-update kernels of the blocked Cholesky and LU factorizations:
// C -= A B^T on 128 x 128 (or 64 x 64) tiles of a front on the matrix cores.
#pragma once
#include "common.h"

namespace wcs {
namespace dev {

// ---------------------------------------------------------------- trailing update
// C(row, col) -= acc[x][y][e] on the lower part (row >= col, row < m,
// col < jend) for the 64 elements of a lane, rows from rowf(x, e) and columns
// from colf(y).  All loads of a half (x in {0,1}, then {2,3}) are issued
// before any store, a masked-off element loading a harmless in-bounds word
// (F[0]) that is never stored, so the round trips to memory overlap instead
// of being serialised element by element.

template <typename T, typename V, typename RowFn, typename ColFn>
__device__ __forceinline__ void tile_sub(T *__restrict__ F, int ld, int m, int jbeg, int jend, int pa,
                                         const V (&acc)[4][4],
                                         RowFn rowf, ColFn colf)
{
    // columns >= pa hold no earlier value (update matrix before its first
    // update): they are assigned -acc instead of updated, and not read
#pragma unroll
    for (int h = 0; h < 4; h += 2) {
        T cv[2][4][4];
#pragma unroll
        for (int x = 0; x < 2; x++)
#pragma unroll
            for (int y = 0; y < 4; y++)
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    int row = rowf(h + x, e), col = colf(y);
                    bool ok = col >= jbeg && col < jend && row < m && row >= col && col < pa;
                    cv[x][y][e] = F[ok ? (int64_t)col * ld + row : 0];
                }
#pragma unroll
        for (int x = 0; x < 2; x++)
#pragma unroll
            for (int y = 0; y < 4; y++)
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    int row = rowf(h + x, e), col = colf(y);
                    if (col >= jbeg && col < jend && row < m && row >= col)
                        F[(int64_t)col * ld + row] = col < pa ? cv[x][y][e] - acc[h + x][y][e] : -acc[h + x][y][e];
                }
    }
}

// The same update for a tile whose accumulators come in quads of consecutive
// rows: av(q, y, t) belongs to row rowq(q) + t (t = 0..3) and column colf(y),
// q, y = 0..3.  With the quad's first row a multiple of 4 (aligned) and all
// four rows inside the stored lower part, the quad is read and written as one
// 16-byte (FP32) or 32-byte (FP64) access; other quads element by element.
// In two halves (q = h, h + 1 for h = 0, 2): load(h) reads a half's earlier
// values, store(h, av) writes the half; a kernel may issue load(0) early (the
// object holds no reference to the accumulators, which stay in registers).
template <typename T, typename RowFn, typename ColFn>
struct QuadEpilogue {
    T *F;
    int ld, m, jbeg, jend, pa;
    bool aligned;
    RowFn rowq;
    ColFn colf;
    __device__ __forceinline__ bool full(int r0, int c) const
    {
        return aligned && c >= jbeg && c < jend && r0 >= c && r0 + 3 < m;
    }
    __device__ __forceinline__ void load(int h, T (&cv)[2][4][4]) const
    {
        typedef typename Vec4<T>::type V4;
#pragma unroll
        for (int e2 = 0; e2 < 2; e2++)
#pragma unroll
            for (int y = 0; y < 4; y++) {
                int r0 = rowq(h + e2), c = colf(y);
                if (full(r0, c)) {
                    V4 v = *reinterpret_cast<const V4 *>(F + (c < pa ? (int64_t)c * ld + r0 : 0));
                    cv[e2][y][0] = v.x;
                    cv[e2][y][1] = v.y;
                    cv[e2][y][2] = v.z;
                    cv[e2][y][3] = v.w;
                } else {
#pragma unroll
                    for (int x = 0; x < 4; x++) {
                        int r = r0 + x;
                        bool ok = c >= jbeg && c < jend && r < m && r >= c && c < pa;
                        cv[e2][y][x] = F[ok ? (int64_t)c * ld + r : 0];
                    }
                }
            }
    }
    template <typename AccFn>
    __device__ __forceinline__ void store(int h, const T (&cv)[2][4][4], AccFn av) const
    {
        typedef typename Vec4<T>::type V4;
#pragma unroll
        for (int e2 = 0; e2 < 2; e2++)
#pragma unroll
            for (int y = 0; y < 4; y++) {
                int r0 = rowq(h + e2), c = colf(y);
                T o[4];
#pragma unroll
                for (int x = 0; x < 4; x++) o[x] = c < pa ? cv[e2][y][x] - av(h + e2, y, x) : -av(h + e2, y, x);
                if (full(r0, c)) {
                    V4 v;
                    v.x = o[0];
                    v.y = o[1];
                    v.z = o[2];
                    v.w = o[3];
                    *reinterpret_cast<V4 *>(F + (int64_t)c * ld + r0) = v;
                } else {
#pragma unroll
                    for (int x = 0; x < 4; x++) {
                        int r = r0 + x;
                        if (c >= jbeg && c < jend && r < m && r >= c) F[(int64_t)c * ld + r] = o[x];
                    }
                }
            }
    }
};
template <typename T, typename RowFn, typename ColFn>
__device__ __forceinline__ QuadEpilogue<T, RowFn, ColFn> quad_epilogue(T *F, int ld, int m, int jbeg, int jend,
                                                                       int pa, bool aligned, RowFn rowq, ColFn colf)
{
    return QuadEpilogue<T, RowFn, ColFn>{F, ld, m, jbeg, jend, pa, aligned, rowq, colf};
}
template <typename T, typename AccFn, typename RowFn, typename ColFn>
__device__ __forceinline__ void tile_sub_quads(T *__restrict__ F, int ld, int m, int jbeg, int jend, int pa,
                                               bool aligned, AccFn av, RowFn rowq, ColFn colf)
{
    auto q = quad_epilogue<T>(F, ld, m, jbeg, jend, pa, aligned, rowq, colf);
#pragma unroll
    for (int h = 0; h < 4; h += 2) {
        T cv[2][4][4];
        q.load(h, cv);
        q.store(h, cv, av);
    }
}



// task = (front, i0, j0, jend): C = F[i0:i0+UT, j0:min(j0+UT, jend)] -= A B^T
// on the lower part (row >= column), with A = F[i0:, ka:ka+K], B = F[j0:, ka:ka+K]
// and K = min(kw, p - ka) for the front's p.  B is read bdelta elements away
// from F (0 for Cholesky; the LU fronts read it from the other factor's
// buffer, whose fronts sit at the same offsets).  The first outer block's update
// (ka = 0) assigns C = -A B^T in the update-matrix columns (>= p), which are
// not zeroed beforehand.  Tiles are TW x TW (128 or 64):
// one wave per 64 x 64 quarter (4 x 4 MFMA 16x16 blocks each); K advances in
// chunks of KC staged through double-buffered LDS.  The 64 x 64 variant gives
// four times as many workgroups for the same front, which pays on mid-size
// fronts; the autotuner picks the tile per level.
constexpr int UT = 128;

// A trailing-update task with its front's descriptors, so that one 32-byte
// (scalar) load gives the workgroup everything it needs:
// a = (front offset low, high 32 bits, m, p), b = (i0, j0, jend, jbeg): the
// tile's columns are [max(j0, jbeg), min(j0 + TW, jend)); j0 is rounded down
// to a multiple of 4 so that the rows of the tile come in aligned quads.
struct UpdTask {
    int4 a, b;
};

template <typename T> struct UpdCfg;
template <> struct UpdCfg<float> { static constexpr int KC = 32; };
template <> struct UpdCfg<double> { static constexpr int KC = 16; };

// LDS position of logical tile row r (0..UT-1) in "fragment order": within
// each 64-row wave block, row q*16 + l goes to l*4 + q, so the four operands a
// lane needs for its four 16-row MFMA blocks are adjacent (one 16-byte read
// for FP32, two for FP64).
__device__ __forceinline__ int frag_pos(int r) { return (r & ~63) + (r & 15) * 4 + ((r >> 4) & 3); }

template <typename T, int TW>
__device__ __forceinline__ void update_tile(const UpdTask t, int ka, int kw, T *__restrict__ fronts, int64_t bdelta)
{
    constexpr int KC = UpdCfg<T>::KC;
    constexpr int NTH = TW * TW / 64;          // one wave per 64 x 64 quarter
    constexpr int LD = TW + (sizeof(T) == 4 ? 4 : 2);
    __shared__ __align__(16) T As[2][KC][LD];
    __shared__ __align__(16) T Bs[2][KC][LD];
    constexpr int KSTEP = NTH / TW;            // k rows covered by one pass of the block
    constexpr int PER = KC / KSTEP;            // elements of each operand per thread per chunk
    int i0 = t.b.x, j0 = t.b.y, jend = t.b.z, jbeg = t.b.w;
    int m = t.a.z, p = t.a.w, ld = front_ld(m);
    int K = min(kw, p - ka);
    const int64_t foff = (int64_t)(((uint64_t)(uint32_t)t.a.y << 32) | (uint32_t)t.a.x);
    const T *F0 = fronts + foff;
    T *F = fronts + foff;
    int tid = threadIdx.x;
    int wave = tid / 64, lane = tid % 64;
    int wr = (wave / (TW / 64)) * 64, wc = (wave % (TW / 64)) * 64;
    int kq = lane / 16, ln = lane % 16;
    bool active = (i0 + wr + 63 >= j0 + wc) && (j0 + wc < jend) && (i0 + wr < m);
    // staging: thread loads tile row r for k = k_first + KSTEP*q
    const int r = tid % TW, k_first = tid / TW;
    const int rpos = frag_pos(r);
    const bool arow = i0 + r < m, brow = j0 + r < m;
    const T *pa = F0 + (int64_t)(ka + k_first) * ld + i0 + r;
    const T *pb = F0 + bdelta + (int64_t)(ka + k_first) * ld + j0 + r;
    const int64_t kstride = (int64_t)KSTEP * ld;
    T ra[PER], rb[PER];
    auto gload = [&](int kc) {
        const T *qa = pa + (int64_t)kc * ld, *qb = pb + (int64_t)kc * ld;
#pragma unroll
        for (int q = 0; q < PER; q++) {
            bool kok = kc + k_first + q * KSTEP < K;
            ra[q] = (kok && arow) ? qa[q * kstride] : (T)0;
            rb[q] = (kok && brow) ? qb[q * kstride] : (T)0;
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int q = 0; q < PER; q++) {
            As[buf][k_first + q * KSTEP][rpos] = ra[q];
            Bs[buf][k_first + q * KSTEP][rpos] = rb[q];
        }
    };
    typedef typename Mfma<T>::V V;
    typedef typename Vec4<T>::type V4;
    V acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++)
#pragma unroll
            for (int e = 0; e < 4; e++) acc[i][j][e] = 0;
    int nchunk = (K + KC - 1) / KC;
    gload(0);
    sstore(0);
    __syncthreads();
    auto body = [&](int c) __attribute__((always_inline)) {
        int buf = c & 1;
        if (c + 1 < nchunk) gload((c + 1) * KC);
        if (active) {
#pragma unroll
            for (int kk = 0; kk < KC; kk += 4) {
                V4 a4 = *reinterpret_cast<const V4 *>(&As[buf][kk + kq][wr + ln * 4]);
                V4 b4 = *reinterpret_cast<const V4 *>(&Bs[buf][kk + kq][wc + ln * 4]);
                T av[4] = {a4.x, a4.y, a4.z, a4.w};
                T bv[4] = {b4.x, b4.y, b4.z, b4.w};
#pragma unroll
                for (int x = 0; x < 4; x++)
#pragma unroll
                    for (int y = 0; y < 4; y++) acc[x][y] = Mfma<T>::mma(av[x], bv[y], acc[x][y]);
            }
        }
        if (c + 1 < nchunk) sstore(buf ^ 1);
        __syncthreads();
    };
    // FP32 128-tiles: the tile's earlier values are read while the last
    // chunk's products run (quads over e: accumulator element e is row 4 kq + e)
    constexpr bool quads = sizeof(T) == 4 && TW == 128;
    auto epi = quad_epilogue<T>(F, ld, m, jbeg, jend, ka == 0 ? p : m, (i0 & 3) == 0,
                                [=](int x) { return i0 + wr + x * 16 + 4 * kq; },
                                [=](int y) { return j0 + wc + y * 16 + ln; });
    T c0v[2][4][4], c1v[2][4][4];
    for (int c = 0; c + 1 < nchunk; c++) body(c);
    if constexpr (quads)
        if (active) {
            epi.load(0, c0v);
            epi.load(2, c1v);
        }
    body(nchunk - 1);
    if (!active) return;
    if constexpr (quads) {
        auto av = [&](int q, int y, int t) { return acc[q][y][t]; };
        epi.store(0, c0v, av);
        epi.store(2, c1v, av);
    } else if constexpr (sizeof(T) == 4)
        tile_sub_quads<T>(F, ld, m, jbeg, jend, ka == 0 ? p : m, (i0 & 3) == 0,
                          [&](int q, int y, int t) { return acc[q][y][t]; },
                          [&](int x) { return i0 + wr + x * 16 + 4 * kq; },
                          [&](int y) { return j0 + wc + y * 16 + ln; });
    else
        tile_sub<T>(F, ld, m, jbeg, jend, ka == 0 ? p : m, acc,
                    [&](int x, int e) { return i0 + wr + x * 16 + Mfma<T>::row(kq, e); },
                    [&](int y) { return j0 + wc + y * 16 + ln; });
}

// FP32 epilogue of the streamed kernel in coalesced order.  Its accumulator
// layout gives lane (kq, ln) the row quads wr + 16 kq + 4 e (e = 0..3) of
// columns wc + 4 ln + y, so storing from the registers would touch 64 cache
// lines with 16 bytes each per instruction (measured: 2.3 TB/s against 5.3
// TB/s for whole columns).  Each wave passes its 64 x 64 quadrant through
// LDS instead, in two halves of 32 columns (8 KB per wave, in stage memory
// the products no longer read), and every store then covers four whole
// 64-row columns: lane L the rows wr + 4 (L % 16) .. + 3 of column 4 s + L / 16
// of the half.  Quads are swizzled in LDS (quad rq of local column cl at
// cl * 64 + 4 (rq ^ (cl / 4 % 16))) so that both the quad writes and the
// column reads hit distinct banks.  load(h, cv) reads half h's earlier values
// (update columns only; a kernel may issue it early), store(h, cv, acc, Q)
// writes the half.
struct ColumnEpilogue {
    float *F;
    int ld, m, jbeg, jend, pa, r00, c00;   // r00, c00: the quadrant's first row and column
    bool aligned;
    __device__ __forceinline__ static int qpos(int cl, int rq) { return cl * 64 + 4 * (rq ^ ((cl >> 2) & 15)); }
    __device__ __forceinline__ bool full(int r0, int c) const
    {
        return aligned && c >= jbeg && c < jend && r0 >= c && r0 + 3 < m;
    }
    __device__ __forceinline__ void load(int h, float (&cv)[8][4]) const
    {
        const int lane = threadIdx.x % 64, r0 = r00 + 4 * (lane % 16);
#pragma unroll
        for (int s = 0; s < 8; s++) {
            const int c = c00 + 32 * h + 4 * s + lane / 16;
            if (full(r0, c)) {
                float4 v = *reinterpret_cast<const float4 *>(F + (c < pa ? (int64_t)c * ld + r0 : 0));
                cv[s][0] = v.x;
                cv[s][1] = v.y;
                cv[s][2] = v.z;
                cv[s][3] = v.w;
            } else {
#pragma unroll
                for (int x = 0; x < 4; x++) {
                    const int r = r0 + x;
                    const bool ok = c >= jbeg && c < jend && r < m && r >= c && c < pa;
                    cv[s][x] = F[ok ? (int64_t)c * ld + r : 0];
                }
            }
        }
    }
    template <typename Acc>
    __device__ __forceinline__ void store(int h, const float (&cv)[8][4], const Acc &acc, float *Q) const
    {
        const int lane = threadIdx.x % 64, kq = lane / 16, ln = lane % 16;
        // the half's quads into LDS: lanes whose columns 4 ln + y fall in it
        if (ln / 8 == h) {
#pragma unroll
            for (int y = 0; y < 4; y++)
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    float4 v = make_float4(acc[0][y][e], acc[1][y][e], acc[2][y][e], acc[3][y][e]);
                    *reinterpret_cast<float4 *>(Q + qpos(4 * (ln % 8) + y, 4 * kq + e)) = v;
                }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int rq = lane % 16, r0 = r00 + 4 * rq;
#pragma unroll
        for (int s = 0; s < 8; s++) {
            const int cl = 4 * s + lane / 16, c = c00 + 32 * h + cl;
            const float4 a = *reinterpret_cast<const float4 *>(Q + qpos(cl, rq));
            const float av[4] = {a.x, a.y, a.z, a.w};
            float o[4];
#pragma unroll
            for (int x = 0; x < 4; x++) o[x] = c < pa ? cv[s][x] - av[x] : -av[x];
            if (full(r0, c)) {
                *reinterpret_cast<float4 *>(F + (int64_t)c * ld + r0) = make_float4(o[0], o[1], o[2], o[3]);
            } else {
#pragma unroll
                for (int x = 0; x < 4; x++) {
                    const int r = r0 + x;
                    if (c >= jbeg && c < jend && r < m && r >= c) F[(int64_t)c * ld + r] = o[x];
                }
            }
        }
        // the next half reuses Q: its reads above are done before its writes
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
};

// Trailing update, streamed form.  Same task and result as k_update<T, 128>,
// but the operand chunks go from global memory straight into LDS through the
// load unit's LDS path (global_load_lds, 16 bytes per lane), with NS chunks in
// flight, so no registers hold staged data and the load latency is covered by
// NS - 1 chunks of matrix-core work.  One DMA instruction fills a contiguous
// 1 KB run of LDS in lane order, so the LDS tile keeps the natural row order
// (rows contiguous for each k) and the MFMA blocks of a wave take interleaved
// rows instead: block x of a wave covers the rows wr + 4 i + x (i = 0..15), so
// the four A operands of a lane (x = 0..3) are the four consecutive rows
// wr + 4 ln + {0..3}, one 16-byte LDS read; the same for B and the columns.
// Rows past the front are clamped to its last row (their products land in
// rows that are never stored); k past K is clamped to the last valid column
// and masked to zero in the last chunk.  The fronts buffer must be followed
// by at least 16 bytes of other workspace memory (it is).
template <typename T> struct DmaCfg;
template <> struct DmaCfg<float> { static constexpr int KC = 16; };
template <> struct DmaCfg<double> { static constexpr int KC = 8; };

typedef __attribute__((address_space(3))) void lds_void_t;

// wait until at most N vector-memory operations of this wave are outstanding
template <int N> __device__ __forceinline__ void wait_vmcnt()
{
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

// workgroup barrier without a memory fence: the fence of __syncthreads would
// wait for every LDS transfer in flight; the streaming loop below waits for
// exactly the chunk it needs instead.  The empty asm statements keep the
// compiler from moving memory operations across the barrier.
__device__ __forceinline__ void barrier_nofence()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// One global -> LDS transfer of 16 bytes per lane (global_load_lds_dwordx4):
// lane l's 16 bytes from g land at LDS byte address lds + 16 l, lds being
// wave-uniform.  Issued from inline assembly so that the compiler does not
// treat it as an LDS write it must wait for before every LDS read; the
// caller orders it with explicit vmcnt waits and barriers.  M0 (the LDS base
// register of the transfer) is restored before the statement ends.
__device__ __forceinline__ void dma_to_lds16(const void *g, uint32_t lds)
{
    uint32_t saved;
    asm volatile("s_mov_b32 %0, m0\n\ts_mov_b32 m0, %2\n\tglobal_load_lds_dwordx4 %1, off\n\ts_mov_b32 m0, %0"
                 : "=&s"(saved)
                 : "v"(g), "s"(lds)
                 : "memory");
}

// NS = 4 stages (64 KB of LDS, two workgroups per compute unit) or 3 (48 KB,
// three in FP32; FP64 stays at two, its registers would spill at three): the
// deeper pipeline pays on long contractions, the third workgroup on short
// ones; the autotuner picks per level.  The launch bound keeps the
// accumulators within the register budget of that many waves.
template <typename T, int NS, int KC>
__device__ __forceinline__ void update_tile_dma(const UpdTask t, int ka, int kw, T *__restrict__ fronts,
                                                int64_t bdelta)
{
    static_assert(NS >= 2 && NS <= 4, "the stage arrays below hold two to four stages");
    constexpr int VEC = 16 / (int)sizeof(T);       // elements per lane per DMA instruction
    constexpr int LPR = 128 / VEC;                 // lanes per 128-element k row
    constexpr int RPI = 64 / LPR;                  // k rows per DMA instruction (f32 2, f64 1)
    constexpr int IPO = KC / RPI;                  // DMA instructions per operand per chunk
    constexpr int IPW = 2 * IPO / 4;               // ... per wave
    static_assert(IPW * 4 == 2 * IPO, "chunk must split evenly over the waves");
    // one array per stage: distinct objects, so the compiler can tell a read
    // of one stage from a transfer into another
    __shared__ __align__(16) T S0[2][KC][128];
    __shared__ __align__(16) T S1[2][KC][128];
    __shared__ __align__(16) T S2[2][NS >= 3 ? KC : 1][128];   // unused with two stages
    __shared__ __align__(16) T S3[2][NS == 4 ? KC : 1][128];   // unused with fewer than four
    auto stage = [&](auto st_) -> T(*)[KC][128] {
        constexpr int st = decltype(st_)::value;
        if constexpr (st == 0) return S0;
        else if constexpr (st == 1) return S1;
        else if constexpr (st == 2) return reinterpret_cast<T(*)[KC][128]>(&S2[0][0][0]);   // (three or more)
        else return reinterpret_cast<T(*)[KC][128]>(&S3[0][0][0]);   // (four stages only)
    };
    int i0 = t.b.x, j0 = t.b.y, jend = t.b.z, jbeg = t.b.w;
    int m = t.a.z, p = t.a.w, ld = front_ld(m);
    int K = min(kw, p - ka);
    T *F = fronts + (int64_t)(((uint64_t)(uint32_t)t.a.y << 32) | (uint32_t)t.a.x);
    int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    int wr = (wave / 2) * 64, wc = (wave % 2) * 64;
    int kq = lane / 16, ln = lane % 16;
    bool active = (i0 + wr + 63 >= j0 + wc) && (j0 + wc < jend) && (i0 + wr < m);
    typedef __attribute__((address_space(3))) T *lds_t;
    // this lane's part of every DMA instruction of the wave: k row in the chunk and tile row
    const int lrow = (lane % LPR) * VEC, lk = lane / LPR;
    // tile origins need not be multiples of VEC, so a lane's VEC rows may run
    // up to VEC - 1 elements past the end of a column (into the next column or
    // the next buffer of the workspace: in bounds); those rows are never stored
    const int rowA = min(i0 + lrow, m - 1), rowB = min(j0 + lrow, m - 1);
    auto issue = [&](auto st_, int c) {
        T(*Sx)[KC][128] = stage(st_);
#pragma unroll
        for (int s = 0; s < IPW; s++) {
            int q = wave + 4 * s, op = q / IPO, qq = q % IPO;
            int kr = qq * RPI;
            int kg = min(c * KC + kr + lk, K - 1);
            const T *g = F + (op ? bdelta : 0) + (int64_t)(ka + kg) * ld + (op ? rowB : rowA);
            uint32_t dst = (uint32_t)(uintptr_t)(lds_t)&Sx[op][kr][0];
            dma_to_lds16((const void *)g, __builtin_amdgcn_readfirstlane(dst));
        }
    };
    typedef typename Mfma<T>::V V;
    typedef typename Vec4<T>::type V4;
    V acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++)
#pragma unroll
            for (int e = 0; e < 4; e++) acc[i][j][e] = 0;
    auto compute = [&](auto st_, int kleft) {
        T(*Sx)[KC][128] = stage(st_);
#pragma unroll
        for (int kk = 0; kk < KC; kk += 4) {
            V4 a4 = *reinterpret_cast<const V4 *>(&Sx[0][kk + kq][wr + 4 * ln]);
            V4 b4 = *reinterpret_cast<const V4 *>(&Sx[1][kk + kq][wc + 4 * ln]);
            bool kv = kk + kq < kleft;
            T av[4] = {kv ? a4.x : (T)0, kv ? a4.y : (T)0, kv ? a4.z : (T)0, kv ? a4.w : (T)0};
            T bv[4] = {b4.x, b4.y, b4.z, b4.w};
#pragma unroll
            for (int x = 0; x < 4; x++)
#pragma unroll
                for (int y = 0; y < 4; y++) acc[x][y] = Mfma<T>::mma(av[x], bv[y], acc[x][y]);
        }
    };
    const int nchunk = (K + KC - 1) / KC;
    // epilogue; in FP32 the first half of the tile's earlier values is read
    // while the last chunk's products run (workgroups of one launch tend to
    // reach their epilogues together, and their C traffic would otherwise
    // leave the matrix cores idle)
    auto epi = quad_epilogue<T>(F, ld, m, jbeg, jend, ka == 0 ? p : m, (i0 & 3) == 0,
                                [=](int e) { return i0 + wr + 4 * Mfma<T>::row(kq, e); },
                                [=](int y) { return j0 + wc + 4 * ln + y; });
    constexpr bool early = sizeof(T) == 4;
    constexpr bool early2 = early && NS != 3;   // both halves where the registers allow (two waves per SIMD)
    constexpr bool colepi = sizeof(T) == 4;     // FP32: the coalesced epilogue through LDS
    T c0v[2][4][4], c1v[2][4][4];
    ColumnEpilogue cepi{reinterpret_cast<float *>(F), ld, m, jbeg, jend, ka == 0 ? p : m, i0 + wr, j0 + wc,
                        (i0 & 3) == 0};
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;
    // chunk c lives in stage c % NS
    auto step = [&](auto st_, auto nx_, int c) {
        if (c >= nchunk) return;
        int after = min(NS - 2, nchunk - 1 - c);   // chunks this wave issued after chunk c
        if (after >= 2) wait_vmcnt<2 * IPW>();
        else if (after == 1) wait_vmcnt<IPW>();
        else wait_vmcnt<0>();
        barrier_nofence();                          // chunk c visible from every wave; chunk c-1 consumed
        if (c + NS - 1 < nchunk) issue(nx_, c + NS - 1);   // refills the stage of chunk c-1
        if (active) compute(st_, K - c * KC);
    };
    issue(I0(), 0);
    if constexpr (NS >= 3)
        if (nchunk > 1) issue(I1(), 1);
    if constexpr (NS == 4)
        if (nchunk > 2) issue(I2(), 2);
    auto group = [&](int c) __attribute__((always_inline)) {
        if constexpr (NS == 2) {
            step(I0(), I1(), c);
            step(I1(), I0(), c + 1);
        } else if constexpr (NS == 4) {
            step(I0(), I3(), c);
            step(I1(), I0(), c + 1);
            step(I2(), I1(), c + 2);
            step(I3(), I2(), c + 3);
        } else {
            step(I0(), I2(), c);
            step(I1(), I0(), c + 1);
            step(I2(), I1(), c + 2);
        }
    };
    int c = 0;
    for (; c + NS < nchunk; c += NS) group(c);
    // before the last group: the early epilogue reads (younger than every
    // transfer issued so far, so the group's waits now also cover the chunks
    // still in flight: stricter, never looser)
    if constexpr (early)
        if (active) {
            if constexpr (colepi) {
                cepi.load(0, reinterpret_cast<float(&)[8][4]>(c0v));
                if constexpr (early2) cepi.load(1, reinterpret_cast<float(&)[8][4]>(c1v));
            } else {
                epi.load(0, c0v);
                if constexpr (early2) epi.load(2, c1v);
            }
        }
    group(c);
    wait_vmcnt<0>();   // no transfer may land in LDS after the workgroup ends
    if constexpr (colepi) {
        // every wave is past its last products: the stage memory becomes the
        // epilogue's (8 KB per wave); each wave passes this barrier once per
        // tile, as it does every chunk barrier
        barrier_nofence();
        if (!active) return;
        float *Q = reinterpret_cast<float *>(wave < 2 ? &S0[0][0][0] : &S1[0][0][0]) + (wave & 1) * 2048;
        if constexpr (!early) cepi.load(0, reinterpret_cast<float(&)[8][4]>(c0v));
        cepi.store(0, reinterpret_cast<float(&)[8][4]>(c0v), acc, Q);
        if constexpr (!early2) cepi.load(1, reinterpret_cast<float(&)[8][4]>(c1v));
        cepi.store(1, reinterpret_cast<float(&)[8][4]>(c1v), acc, Q);
    } else {
        if (!active) return;
        auto av = [&](int q, int y, int t) { return acc[t][y][q]; };
        if constexpr (!early) epi.load(0, c0v);
        epi.store(0, c0v, av);
        if constexpr (!early2) epi.load(2, c1v);
        epi.store(2, c1v, av);
    }
}

// The trailing-update kernels: workgroup b takes tasks b, b + grid, ... (a
// launch may use fewer workgroups than tasks: the look-ahead updates on the
// side stream do, so that the panel-step kernels on the main stream always
// find room on the compute units).
template <typename T, int TW>
__global__ __launch_bounds__(TW * TW / 64, 2) void k_update(const UpdTask *__restrict__ tasks, int ntask, int ka,
                                                            int kw, T *__restrict__ fronts, int64_t bdelta)
{
    for (int i = blockIdx.x; i < ntask; i += gridDim.x) {
        if (i != (int)blockIdx.x) __syncthreads();   // the previous tile's LDS reads are done
        update_tile<T, TW>(tasks[i], ka, kw, fronts, bdelta);
    }
}

template <typename T, int NS, int KC = DmaCfg<T>::KC>
__global__ __launch_bounds__(256, (NS == 3 && sizeof(T) == 4) ? 3 : 2) void k_update_dma(
    const UpdTask *__restrict__ tasks, int ntask, int ka, int kw, T *__restrict__ fronts, int64_t bdelta)
{
    for (int i = blockIdx.x; i < ntask; i += gridDim.x) {
        if (i != (int)blockIdx.x) __syncthreads();   // the previous tile's LDS reads are done
        update_tile_dma<T, NS, KC>(tasks[i], ka, kw, fronts, bdelta);
    }
}

}  // namespace dev
}  // namespace wcs
