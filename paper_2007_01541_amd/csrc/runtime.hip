// Device runtime: static launch plan, workspace layout, launch sequences for
// the numeric factorization, the solves, iterative refinement and the
// pattern gradient, and their C ABI entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.h"
#include "kernels.hip"
#include "solve.hip"

namespace wcs {
const Symbolic &symbolic_of(wcs_symbolic h);

namespace {

using namespace dev;

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) {                                                         \
            set_error(std::string(#expr) + ": " + hipGetErrorString(e_));               \
            return WCS_EHIP;                                                            \
        }                                                                               \
    } while (0)

// FP32 fronts with at least this many pivots factor their diagonal blocks in
// FP64 (environment WCS_FP64_DIAG_COLS, default 1024; read when a factor is created)
int32_t fp64_diag_min_cols()
{
    const char *e = std::getenv("WCS_FP64_DIAG_COLS");
    return e ? std::atoi(e) : 1024;
}

// Workgroups of the matrix-value expansion when it runs beside the first
// solve of a refinement (environment WCS_EXPAND_BLOCKS, default 256: one per
// CU of an MI355X; measured on the 2^18 headline system with 64 right-hand
// sides, 128 and 256 are equally fast, 64 and 512 or more slower)
int expand_side_blocks()
{
    const char *e = std::getenv("WCS_EXPAND_BLOCKS");
    int b = e ? std::atoi(e) : 256;
    return b > 0 ? b : 256;
}

size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// independent diagonal blocks of the matrix (1 unless it is a batch)
size_t nseg_of(const Symbolic &S) { return S.seg_ptr.size() >= 2 ? S.seg_ptr.size() - 1 : 1; }

// outer block: trailing updates use K = NBO columns at once (environment
// WCS_OUTER_BLOCK, a multiple of the panel width, default 512; read when a
// plan is built)
int32_t outer_block()
{
    const char *e = std::getenv("WCS_OUTER_BLOCK");
    int32_t v = e ? std::atoi(e) : 512;
    return v >= 64 && v % 64 == 0 ? v : 512;
}
// fronts with more rows solve block by block over many workgroups (tuning knob WCS_SOLVE_STEP_ROWS)
// Fronts of at most this many rows are solved one workgroup per front for the
// whole sweep; by default none (the super-block path is faster for them too).
int32_t solve_step_min_rows()
{
    const char *e = std::getenv("WCS_SOLVE_STEP_ROWS");
    return e ? std::atoi(e) : 0;
}
constexpr int kPartBlocks = 512;             // blocks of the two-pass column reductions

// Leaf fronts whose pivot columns fit in LDS are factored by one persistent
// launch (k_leaf) instead of the level-synchronous panel and update launches
// (environment WCS_LEAF_KERNEL, default 1; 0 = off).  Cholesky factors only.
bool leaf_kernel_enabled()
{
    const char *e = std::getenv("WCS_LEAF_KERNEL");
    return e ? std::atoi(e) != 0 : true;
}

// Cholesky fronts with at least this many pivots are factored by the fused
// panel steps (k_diag_factor + k_step) instead of the panel kernel and a
// separate update of the outer block's later columns (environment
// WCS_STEP_MIN_COLS; read when a plan is built).  Same factor bit for bit.
// Workgroups of a look-ahead trailing update on the side stream, as a
// multiple of the compute units (environment WCS_SIDE_GRID, workgroups per
// compute unit in quarters; default 0 = one workgroup per tile): the tiles
// are shared out over that many workgroups, which leaves room on every unit
// for the panel steps on the main stream.  Measured at N = 2^18: 4, 6 and 8
// quarters slow the factorization (FP32 47.3 -> 48.6-49.9 ms, FP64 81.6 ->
// 82-92 ms).
int side_grid(int ncu)
{
    const char *e = std::getenv("WCS_SIDE_GRID");
    int q = e ? std::atoi(e) : 0;
    return q > 0 ? q * ncu / 4 : 0;
}

// Right-hand-side counts from 5 up to this one run the 16-column sweep
// kernels, larger ones the 64-column ones (environment WCS_SOLVE_KT16_MAX,
// read by every solve; default 4: none).  Measured at N = 2^18, one solve:
// 8 RHS FP32 11.7 ms with the 16-column kernels, 7.0 ms with the 64-column
// ones; 16 RHS 12.2 / 7.1 ms; FP64 16 RHS 22.1 / 14.4 ms.
int kt16_max_rhs()
{
    const char *e = std::getenv("WCS_SOLVE_KT16_MAX");
    return e ? std::atoi(e) : 4;
}

// Fronts with at least this many pivots are factored as late as their
// parent allows (one level below it) instead of at their height in the
// assembly tree (environment WCS_LATE_MIN_PIVOTS, read when a factor is
// created; default 1024, 0 = off): a large front off the longest path of the
// tree then shares the launches of a level above with the fronts it is
// independent of, instead of lengthening the chain of its own level.
// Measured at N = 2^18 (alternating runs): FP32 factor 43.8 ms at their
// heights, 43.5 with 2048, 43.0 with 1024, 43.1 with 512; FP64 78.5, 78.1,
// 77.8, 77.7 ms; one FP32 solve 8.64 -> 8.33 ms with 1024.
int32_t late_min_pivots()
{
    const char *e = std::getenv("WCS_LATE_MIN_PIVOTS");
    return e ? std::atoi(e) : 1024;
}

int32_t step_min_cols()
{
    const char *e = std::getenv("WCS_STEP_MIN_COLS");
    return e ? std::atoi(e) : 1024;
}

// Static schedule derived from the symbolic structure only.  Inside every
// front: for each outer block of NBO pivot columns, for each NB-wide panel in
// it, factor the panel (diagonal block + rows below) and update the rest of
// the outer block's columns; then update the trailing matrix with the whole
// outer block (K = NBO).
enum OpKind { OP_PANEL = 0, OP_PANEL_FP64DIAG = 1, OP_UPDATE = 2, OP_DIAG = 3, OP_STEP = 4 };
struct Op {
    int32_t kind;
    int32_t ka, kw;      // panel: ka = k0; update: columns [ka, ka + min(kw, p - ka)) form K
    int64_t off, cnt;    // tasks (update: 128 x 128 tiles)
    int64_t off64 = 0, cnt64 = 0;   // update: the same work as 64 x 64 tiles
    // look-ahead: the part of an outer block's trailing update beyond the next
    // outer block's pivot columns runs on the side stream (side); the update of
    // those next pivot columns by the following block first waits for it (join)
    bool side = false, join = false;
    bool d64 = false;    // OP_DIAG / OP_STEP: diagonal blocks factored in FP64 (FP32 fronts)
};
struct SuperStep {
    int32_t s0;                  // first pivot of the super-block
    int64_t d_off, d_cnt;        // (front, 64-block of the super-block) tasks in sblk_tasks: X_S products
    int64_t t_off, t_cnt;        // wide part: forward (front, 64-row tile) / backward (front, column block)
    int64_t t1_off = 0, t1_cnt = 0;   // forward: tiles of fronts whose super-block is one 64-column block
};
struct SolveLevel {
    int64_t fused_off = 0, fused_cnt = 0;          // fronts solved by one workgroup each (in slist)
    int64_t step_off = 0, step_cnt = 0;            // fronts solved super-block by super-block (in slist)
    std::pair<int64_t, int64_t> assemble{0, 0};    // forward assembly tasks
    std::vector<SuperStep> fwd;                    // s0 ascending
    std::pair<int64_t, int64_t> below{0, 0};       // backward update-row partial tasks (sbelow_tasks)
    std::pair<int64_t, int64_t> below_sum{0, 0};   // ... and their sums (sbsum_tasks)
    std::vector<SuperStep> bwd;                    // s0 descending
    std::pair<int64_t, int64_t> xinv{0, 0};        // super-block inverse tasks of this level (xinv_tasks)
};
struct Level {
    SolveLevel sv;
    int32_t upd_var = 0;                           // update kernel of this level (WCS_UPD_*; autotuned)
    std::vector<Op> ops;
    std::vector<std::pair<int64_t, int64_t>> ea;   // extend-add rounds into the pivot columns (offset, count)
    std::vector<std::pair<int64_t, int64_t>> ea_post;   // ... into the update matrices, after the trailing updates
    int64_t dinv_off = 0, dinv_cnt = 0;            // diagonal blocks of this level's fronts (dinv_tasks)
    int64_t leaf_off = 0, leaf_cnt = 0;            // fronts factored by the persistent leaf kernel (leaf_queue)
    int64_t fl_off = 0, fl_cnt = 0;                // fronts of this level in flist
};

struct Plan {
    std::vector<Level> levels;
    std::vector<int2> pan_tasks;
    std::vector<int4> upd_tasks;
    std::vector<int32_t> upd_jbeg;                // per update task: first column it writes
    std::vector<int2> ea_tasks;
    std::vector<int32_t> flist;
    std::vector<int32_t> mfront, pfront, first;
    std::vector<int64_t> woff;                    // per front: row offset of its solve buffer
    int64_t wrows = 0;
    std::vector<int64_t> dscr_off;                // per front: element offset of its diagonal-block scratch
    std::vector<int2> dinv_tasks;                 // (front, diagonal block) of every NB x NB block
    int64_t dscr_elems = 0;
    std::vector<int2> zero_tasks;                 // (front, first column) chunks of ZCOLS columns
    int64_t lower_elems = 0;
    std::vector<int32_t> child_ptr, child_list;
    std::vector<int32_t> ea_split;                // per front: update columns that land in the parent's pivot columns
    std::vector<int32_t> colof;                   // column of each stored entry
    std::vector<int32_t> slist;                   // fronts per level for the solves (fused first, then stepped)
    std::vector<int2> sfwd_tasks, sbwd_tasks, sasm_tasks, sblk_tasks;
    std::vector<int4> sbelow_tasks, sbsum_tasks, xinv_tasks;
    int64_t part_blocks = 0;                      // SB x k partial blocks of the split update-row sums
    std::vector<int64_t> xoff;                    // per front: offset of its super-block inverses (-1: none)
    std::vector<int2> alt_tasks, al_tasks;        // products with the factor: (front, column block) / (front, row tile)
    std::vector<int64_t> gptr, glist;             // rows of the L product: W rows holding each row, fronts ascending
    int64_t xelems = 0;
    // SpMV work items: (row, first entry, end entry within the row, partial
    // slot or -1); rows longer than SPMV_CHUNK entries are split into chunks
    // (listed first) whose partial sums spmv_long (row, first slot, slots)
    // adds in slot order
    std::vector<int4> spmv_chunks, spmv_long;
    int64_t spmv_slots = 0;
    // the same product by groups of up to SPMV_GROUP rows with one column
    // pattern (a wavelet matrix has three rows per pattern, one per wavelet
    // of a cell): spmv_grp (rows, -1 past the group's end); items (group,
    // first entry, chunks of a split group or -1, partial slot of its first
    // row's chunk); row g of a split group with nc chunks keeps its partial
    // for chunk c at slot first + g nc + c, which spmv_glong (row, first slot,
    // slots) adds in slot order
    std::vector<int4> spmv_grp, spmv_gitems, spmv_glong;
    int64_t spmv_gslots = 0;
    std::vector<int32_t> leaf_queue;              // leaf fronts of the persistent kernel, largest first
    std::vector<int32_t> diag_fronts;             // OP_DIAG tasks (fronts)
    std::vector<int4> step_tasks;                 // OP_STEP tasks (front, i0, j0, flags)
    int32_t nbo = 512;                            // outer block of this plan

    // esz: element size of the fronts; leaf_ok: route leaf fronts that fit in
    // LDS to the persistent leaf kernel
    void build(const Symbolic &S, size_t esz = 8, bool leaf_ok = false, bool step_ok = false)
    {
        const int32_t NBO = outer_block();
        nbo = NBO;
        const int32_t step_min = step_min_cols();
        int32_t ns = S.ns;
        const int32_t diag64 = fp64_diag_min_cols();
        mfront.resize(ns);
        pfront.resize(ns);
        first.resize(ns);
        woff.resize(ns);
        dscr_off.resize(ns);
        wrows = 0;
        dscr_elems = 0;
        dinv_tasks.clear();
        for (int32_t s = 0; s < ns; s++) {
            mfront[s] = S.m_of(s);
            pfront[s] = S.p_of(s);
            first[s] = S.sptr[s];
            woff[s] = wrows;
            wrows += mfront[s];
            dscr_off[s] = dscr_elems;
            dscr_elems += (int64_t)((pfront[s] + NB - 1) / NB) * NB * NB;
        }
        child_ptr.assign((size_t)ns + 1, 0);
        for (int32_t s = 0; s < ns; s++)
            if (S.sparent[s] >= 0) child_ptr[S.sparent[s] + 1]++;
        for (int32_t s = 0; s < ns; s++) child_ptr[s + 1] += child_ptr[s];
        child_list.resize(child_ptr[ns]);
        {
            std::vector<int32_t> fill(child_ptr.begin(), child_ptr.end() - 1);
            for (int32_t s = 0; s < ns; s++)
                if (S.sparent[s] >= 0) child_list[fill[S.sparent[s]]++] = s;   // ascending
        }
        ea_split.assign((size_t)ns, 0);
        for (int32_t c = 0; c < ns; c++) {
            int32_t par = S.sparent[c];
            if (par < 0) continue;
            const int32_t *rl = S.rel.data() + S.rptr[c] + pfront[c];
            int32_t nu = mfront[c] - pfront[c], js = 0;
            while (js < nu && rl[js] < pfront[par]) js++;   // rel ascends
            ea_split[c] = js;
        }
        int32_t H = S.nlevels;
        std::vector<std::vector<int32_t>> bylev(H);
        {
            // level of every front: its height, or for large fronts one below
            // its parent's level (parents come after their children)
            const int32_t late = late_min_pivots();
            std::vector<int32_t> lev(S.height.begin(), S.height.end());
            for (int32_t s = ns - 1; s >= 0; s--) {
                int32_t par = S.sparent[s];
                if (late > 0 && par > s && pfront[s] >= late) lev[s] = std::max(lev[s], lev[par] - 1);
            }
            for (int32_t s = 0; s < ns; s++) bylev[lev[s]].push_back(s);
        }
        levels.assign(H, Level());
        flist.clear();
        pan_tasks.clear();
        upd_tasks.clear();
        upd_jbeg.clear();
        ea_tasks.clear();
        leaf_queue.clear();
        diag_fronts.clear();
        step_tasks.clear();
        const int leaf_elems = esz == 4 ? LeafCfg<float>::ELEMS : LeafCfg<double>::ELEMS;
        for (int32_t h = 0; h < H; h++) {
            Level &L = levels[h];
            const std::vector<int32_t> &all = bylev[h];
            // the fronts of this level that the level-synchronous launches factor
            std::vector<int32_t> fr;
            L.leaf_off = (int64_t)leaf_queue.size();
            for (int32_t s : all) {
                bool leaf = h == 0 && leaf_ok && pfront[s] <= NB &&
                            (int64_t)leaf_sld(mfront[s]) * pfront[s] <= leaf_elems;
                (leaf ? leaf_queue : fr).push_back(s);
            }
            L.leaf_cnt = (int64_t)leaf_queue.size() - L.leaf_off;
            // largest fronts first (work per front ~ m^2 p)
            std::stable_sort(leaf_queue.begin() + L.leaf_off, leaf_queue.end(), [&](int32_t a, int32_t b) {
                return (double)mfront[a] * mfront[a] * pfront[a] > (double)mfront[b] * mfront[b] * pfront[b];
            });
            L.fl_off = (int64_t)flist.size();
            flist.insert(flist.end(), all.begin(), all.end());
            L.fl_cnt = (int64_t)all.size();
            L.dinv_off = (int64_t)dinv_tasks.size();
            for (int32_t s : all)
                for (int32_t b = 0; b < (pfront[s] + NB - 1) / NB; b++) dinv_tasks.push_back(make_int2(s, b));
            L.dinv_cnt = (int64_t)dinv_tasks.size() - L.dinv_off;
            // extend-add rounds: round r adds the r-th child of every parent;
            // first the children's columns that land in the pivot columns, and
            // after the level's trailing updates the rest
            int32_t maxk = 0;
            for (int32_t s : fr) maxk = std::max(maxk, child_ptr[s + 1] - child_ptr[s]);
            for (int post = 0; post < 2; post++)
                for (int32_t r = 0; r < maxk; r++) {
                    int64_t off = (int64_t)ea_tasks.size();
                    for (int32_t s : fr) {
                        if (child_ptr[s] + r >= child_ptr[s + 1]) continue;
                        int32_t c = child_list[child_ptr[s] + r];
                        int32_t nu = mfront[c] - pfront[c], js = ea_split[c];
                        if (post)
                            for (int32_t c0 = js; c0 < nu; c0 += EA_COLS) ea_tasks.push_back(make_int2(c, c0));
                        else
                            for (int32_t c0 = 0; c0 < js; c0 += EA_COLS) ea_tasks.push_back(make_int2(c, c0));
                    }
                    int64_t cnt = (int64_t)ea_tasks.size() - off;
                    if (cnt) (post ? L.ea_post : L.ea).push_back({off, cnt});
                }
            int32_t maxp = 0;
            for (int32_t s : fr) maxp = std::max(maxp, pfront[s]);
            // fronts of the fused panel steps, and the others
            std::vector<int32_t> frs, fro;
            for (int32_t s : fr) (step_ok && pfront[s] >= step_min && pfront[s] > NB ? frs : fro).push_back(s);
            // tasks of one panel step of front s (see k_step): the tile holding the
            // next diagonal block first, then the other tiles of the first strip
            // (they write the panel rows), then the later strips
            auto step_of = [&](int32_t s, int32_t K0, int32_t k0, std::vector<int4> &head, std::vector<int4> &rest) {
                int32_t p = pfront[s], m = mfront[s];
                int32_t nb = std::min(NB, p - k0), kend = std::min(K0 + NBO, p), rs = k0 + nb;
                if (rs < kend) {
                    head.push_back(make_int4(s, rs, rs, STEP_WRITE | STEP_DIAG));
                    for (int32_t i0 = rs + NB; i0 < m; i0 += NB) rest.push_back(make_int4(s, i0, rs, STEP_WRITE));
                    for (int32_t j0 = rs + NB; j0 < kend; j0 += NB)
                        for (int32_t i0 = j0; i0 < m; i0 += NB) rest.push_back(make_int4(s, i0, j0, 0));
                } else {
                    int32_t fl = STEP_WRITE | STEP_DIRECT | (K0 < k0 ? STEP_COPY : 0);
                    for (int32_t i0 = rs; i0 < m; i0 += NB) rest.push_back(make_int4(s, i0, -1, fl));
                    if (K0 < k0)
                        for (int32_t r0 = K0 + NB; r0 < rs; r0 += NB)
                            rest.push_back(make_int4(s, r0, STEP_COPY_ONLY, std::min(r0 + NB, rs)));
                }
            };
            int32_t tw = UT;
            // tiles start at a multiple of 4 (the columns before clo masked):
            // every tile then holds whole aligned quads of rows
            auto tiles = [&](int32_t s, int32_t clo, int32_t jend) {
                int32_t m = mfront[s];
                for (int32_t j0 = clo & ~3; j0 < jend; j0 += tw)
                    for (int32_t i0 = j0; i0 < m; i0 += tw) {
                        upd_tasks.push_back(make_int4(s, i0, j0, jend));
                        upd_jbeg.push_back(clo);
                    }
            };
            for (int32_t K0 = 0; K0 < maxp; K0 += NBO) {
                for (int32_t k0 = K0; k0 < std::min(K0 + NBO, maxp); k0 += NB) {
                    for (int pass = 0; pass < 2; pass++) {
                        Op op{pass ? OP_PANEL_FP64DIAG : OP_PANEL, k0, NB, (int64_t)pan_tasks.size(), 0};
                        for (int32_t s : fro) {
                            int32_t p = pfront[s], m = mfront[s];
                            if (p <= k0 || (p >= diag64) != (pass == 1)) continue;
                            int32_t nb = std::min(NB, p - k0);
                            int32_t nt = std::max(1, (m - k0 - nb + TRW - 1) / TRW);
                            for (int32_t t = 0; t < nt; t++) pan_tasks.push_back(make_int2(s, t));
                        }
                        op.cnt = (int64_t)pan_tasks.size() - op.off;
                        if (op.cnt) L.ops.push_back(op);
                    }
                    for (int pass = 0; pass < 2; pass++) {
                        if (k0 == K0) {
                            Op dg{OP_DIAG, k0, NB, (int64_t)diag_fronts.size(), 0};
                            dg.d64 = pass == 1;
                            for (int32_t s : frs)
                                if (pfront[s] > k0 && (pfront[s] >= diag64) == (pass == 1)) diag_fronts.push_back(s);
                            dg.cnt = (int64_t)diag_fronts.size() - dg.off;
                            if (dg.cnt) L.ops.push_back(dg);
                        }
                        std::vector<int4> head, rest;
                        for (int32_t s : frs)
                            if (pfront[s] > k0 && (pfront[s] >= diag64) == (pass == 1)) step_of(s, K0, k0, head, rest);
                        Op st{OP_STEP, k0, K0, (int64_t)step_tasks.size(), 0};
                        st.d64 = pass == 1;
                        step_tasks.insert(step_tasks.end(), head.begin(), head.end());
                        step_tasks.insert(step_tasks.end(), rest.begin(), rest.end());
                        st.cnt = (int64_t)step_tasks.size() - st.off;
                        if (st.cnt) L.ops.push_back(st);
                    }
                    Op up{OP_UPDATE, k0, NB, 0, 0};
                    for (int v = 0; v < 2; v++) {
                        tw = v == 0 ? UT : 64;
                        int64_t o = (int64_t)upd_tasks.size();
                        for (int32_t s : fro) {
                            int32_t p = pfront[s];
                            if (p <= k0) continue;
                            int32_t nb = std::min(NB, p - k0);
                            int32_t kend = K0 + std::min(NBO, p - K0);
                            if (k0 + nb < kend) tiles(s, k0 + nb, kend);
                        }
                        (v == 0 ? up.off : up.off64) = o;
                        (v == 0 ? up.cnt : up.cnt64) = (int64_t)upd_tasks.size() - o;
                    }
                    if (up.cnt) L.ops.push_back(up);
                }
                // trailing update with the outer block (K = NBO): first the next outer
                // block's pivot columns (main stream), then everything to their right
                // (side stream, overlapping the next block's panels)
                for (int part = 0; part < 2; part++) {
                    Op up{OP_UPDATE, K0, NBO, 0, 0};
                    up.side = part == 1;
                    up.join = part == 0 && K0 > 0;
                    for (int v = 0; v < 2; v++) {
                        tw = v == 0 ? UT : 64;
                        int64_t o = (int64_t)upd_tasks.size();
                        for (int32_t s : fr) {
                            int32_t p = pfront[s], m = mfront[s];
                            if (p <= K0) continue;
                            int32_t kend = K0 + std::min(NBO, p - K0);
                            int32_t nend = kend < p ? std::min(p, kend + NBO) : kend;
                            if (part == 0 && kend < nend) tiles(s, kend, nend);
                            if (part == 1 && nend < m) tiles(s, nend, m);
                        }
                        (v == 0 ? up.off : up.off64) = o;
                        (v == 0 ? up.cnt : up.cnt64) = (int64_t)upd_tasks.size() - o;
                    }
                    if (up.cnt || up.join) L.ops.push_back(up);
                }
            }
        }
        // solve schedule
        slist.clear();
        sfwd_tasks.clear();
        sblk_tasks.clear();
        sbsum_tasks.clear();
        xinv_tasks.clear();
        part_blocks = 0;
        xoff.assign(ns, -1);
        xelems = 0;
        sbelow_tasks.clear();
        sbwd_tasks.clear();
        sasm_tasks.clear();
        const int32_t step_rows = solve_step_min_rows();
        for (int32_t h = 0; h < H; h++) {
            SolveLevel &V = levels[h].sv;
            std::vector<int32_t> big;
            V.fused_off = (int64_t)slist.size();
            for (int32_t s : bylev[h]) {
                if (mfront[s] > step_rows) big.push_back(s);
                else slist.push_back(s);
            }
            V.fused_cnt = (int64_t)slist.size() - V.fused_off;
            V.step_off = (int64_t)slist.size();
            slist.insert(slist.end(), big.begin(), big.end());
            V.step_cnt = (int64_t)big.size();
            int32_t maxp = 0;
            for (int32_t s : big) maxp = std::max(maxp, pfront[s]);
            V.assemble.first = (int64_t)sasm_tasks.size();
            for (int32_t s : big)
                for (int32_t t = 0; t < (mfront[s] + SROWS - 1) / SROWS; t++) sasm_tasks.push_back(make_int2(s, t));
            V.assemble.second = (int64_t)sasm_tasks.size() - V.assemble.first;
            V.xinv.first = (int64_t)xinv_tasks.size();
            for (int32_t s : big) {
                int32_t nsup = (pfront[s] + SS - 1) / SS;
                xoff[s] = xelems;
                // SS x SS per super-block; the last one only as many 64-column blocks as it
                // has pivots (no kernel touches the columns beyond)
                int32_t nb_last = (pfront[s] - (nsup - 1) * SS + SB - 1) / SB;
                xelems += (int64_t)(nsup - 1) * SS * SS + (int64_t)nb_last * SB * SS;
                for (int32_t si = 0; si < nsup; si++) {
                    int32_t nb = (std::min(pfront[s], (si + 1) * SS) - si * SS + SB - 1) / SB;
                    for (int32_t jb = 0; jb < nb; jb++) xinv_tasks.push_back(make_int4(s, si, jb, 0));
                }
            }
            V.xinv.second = (int64_t)xinv_tasks.size() - V.xinv.first;
            auto blk_tasks = [&](int32_t s0) {
                int64_t off = (int64_t)sblk_tasks.size();
                for (int32_t s : big) {
                    if (pfront[s] <= s0) continue;
                    int32_t nb = (std::min(pfront[s], s0 + SS) - s0 + SB - 1) / SB;
                    for (int32_t b = 0; b < nb; b++) sblk_tasks.push_back(make_int2(s, b));
                }
                return std::make_pair(off, (int64_t)sblk_tasks.size() - off);
            };
            for (int32_t s0 = 0; s0 < maxp; s0 += SS) {
                auto d = blk_tasks(s0);
                SuperStep st{s0, d.first, d.second, 0, 0};
                for (int one = 0; one < 2; one++) {    // super-blocks of several 64-column blocks, then of one
                    int64_t off = (int64_t)sfwd_tasks.size();
                    for (int32_t s : big) {
                        if (pfront[s] <= s0) continue;
                        int32_t s1 = std::min(pfront[s], s0 + SS);    // row tiles start at s1 & ~3
                        if ((s1 - s0 <= SB) != (one == 1)) continue;
                        int32_t nt = mfront[s] > s1 ? (mfront[s] - (s1 & ~3) + SB - 1) / SB : 0;
                        for (int32_t t = 0; t < nt; t++) sfwd_tasks.push_back(make_int2(s, t));
                    }
                    int64_t cnt = (int64_t)sfwd_tasks.size() - off;
                    if (one) { st.t1_off = off; st.t1_cnt = cnt; }
                    else { st.t_off = off; st.t_cnt = cnt; }
                }
                V.fwd.push_back(st);
            }
            V.below.first = (int64_t)sbelow_tasks.size();
            V.below_sum.first = (int64_t)sbsum_tasks.size();
            for (int32_t s : big)
                for (int32_t a = 0; a < (pfront[s] + SB - 1) / SB; a++) {
                    int64_t slot0 = part_blocks;
                    for (int32_t r0 = pfront[s] & ~3; mfront[s] > pfront[s] && r0 < mfront[s]; r0 += BELOW_ROWS)
                        sbelow_tasks.push_back(make_int4(s, a, r0, (int32_t)part_blocks++));
                    sbsum_tasks.push_back(make_int4(s, a, (int32_t)slot0, (int32_t)(part_blocks - slot0)));
                }
            V.below.second = (int64_t)sbelow_tasks.size() - V.below.first;
            V.below_sum.second = (int64_t)sbsum_tasks.size() - V.below_sum.first;
            int32_t nsup = (maxp + SS - 1) / SS;
            for (int32_t si = nsup - 1; si >= 0; si--) {
                int32_t s0 = si * SS;
                auto d = blk_tasks(s0);
                int64_t off = (int64_t)sbwd_tasks.size();
                for (int32_t s : big) {
                    if (pfront[s] <= s0) continue;
                    for (int32_t a = 0; a < s0 / SB; a++) sbwd_tasks.push_back(make_int2(s, a));
                }
                V.bwd.push_back({s0, d.first, d.second, off, (int64_t)sbwd_tasks.size() - off});
            }
        }
        // SpMV chunks of the pivot-order CSR
        spmv_chunks.clear();
        spmv_long.clear();
        spmv_slots = 0;
        for (int32_t i = 0; i < S.n; i++) {
            int64_t len = S.csr_ptr[i + 1] - S.csr_ptr[i];
            if (len <= SPMV_CHUNK) continue;
            int32_t nc = (int32_t)((len + SPMV_CHUNK - 1) / SPMV_CHUNK);
            spmv_long.push_back(make_int4(i, (int32_t)spmv_slots, nc, 0));
            for (int32_t c = 0; c < nc; c++)
                spmv_chunks.push_back(make_int4(i, c * SPMV_CHUNK, (int32_t)std::min<int64_t>(len, (int64_t)(c + 1) * SPMV_CHUNK),
                                                (int32_t)spmv_slots++));
        }
        for (int32_t i = 0; i < S.n; i++) {
            int64_t len = S.csr_ptr[i + 1] - S.csr_ptr[i];
            if (len <= SPMV_CHUNK) spmv_chunks.push_back(make_int4(i, 0, (int32_t)len, -1));
        }
        // row groups: rows with equal column lists (hash, then an exact
        // comparison with the group's first row), in order of their first row
        {
            std::vector<uint64_t> hsh((size_t)S.n);
            for (int32_t i = 0; i < S.n; i++) {
                uint64_t h = 1469598103934665603ull ^ (uint64_t)(S.csr_ptr[i + 1] - S.csr_ptr[i]);
                for (int64_t q = S.csr_ptr[i]; q < S.csr_ptr[i + 1]; q++)
                    h = (h ^ (uint64_t)(uint32_t)S.csr_col[q]) * 1099511628211ull;
                hsh[i] = h;
            }
            auto same = [&](int32_t a, int32_t b) {
                int64_t la = S.csr_ptr[a + 1] - S.csr_ptr[a];
                return la == S.csr_ptr[b + 1] - S.csr_ptr[b] &&
                       std::equal(S.csr_col.begin() + S.csr_ptr[a], S.csr_col.begin() + S.csr_ptr[a + 1],
                                  S.csr_col.begin() + S.csr_ptr[b]);
            };
            std::vector<int32_t> order((size_t)S.n);
            for (int32_t i = 0; i < S.n; i++) order[i] = i;
            std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return hsh[a] < hsh[b]; });
            std::vector<std::vector<int32_t>> groups;
            std::vector<int32_t> first_of((size_t)S.n, -1);   // group index by its first row
            for (size_t q = 0; q < order.size();) {
                size_t q1 = q;
                while (q1 < order.size() && hsh[order[q1]] == hsh[order[q]]) q1++;
                // equal hashes: split into classes of equal lists (ascending rows)
                std::vector<int32_t> rest(order.begin() + q, order.begin() + q1);
                std::sort(rest.begin(), rest.end());
                while (!rest.empty()) {
                    std::vector<int32_t> cls, other;
                    for (int32_t r : rest) (same(rest[0], r) ? cls : other).push_back(r);
                    for (size_t g0 = 0; g0 < cls.size(); g0 += SPMV_GROUP) {
                        first_of[cls[g0]] = (int32_t)groups.size();
                        groups.emplace_back(cls.begin() + g0, cls.begin() + std::min(cls.size(), g0 + SPMV_GROUP));
                    }
                    rest.swap(other);
                }
                q = q1;
            }
            spmv_grp.clear();
            spmv_gitems.clear();
            spmv_glong.clear();
            spmv_gslots = 0;
            std::vector<int32_t> gid;   // groups in order of their first row
            for (int32_t i = 0; i < S.n; i++)
                if (first_of[i] >= 0) gid.push_back(first_of[i]);
            std::vector<int4> shortit;
            for (int32_t g : gid) {
                const std::vector<int32_t> &rs = groups[g];
                int32_t gi = (int32_t)spmv_grp.size();
                spmv_grp.push_back(make_int4(rs[0], rs.size() > 1 ? rs[1] : -1, rs.size() > 2 ? rs[2] : -1,
                                             rs.size() > 3 ? rs[3] : -1));
                int64_t len = S.csr_ptr[rs[0] + 1] - S.csr_ptr[rs[0]];
                if (len <= SPMV_CHUNK) {
                    shortit.push_back(make_int4(gi, 0, -1, -1));
                    continue;
                }
                int32_t nc = (int32_t)((len + SPMV_CHUNK - 1) / SPMV_CHUNK);
                for (size_t r = 0; r < rs.size(); r++)
                    spmv_glong.push_back(make_int4(rs[r], (int32_t)(spmv_gslots + (int64_t)r * nc), nc, 0));
                for (int32_t c = 0; c < nc; c++)
                    spmv_gitems.push_back(make_int4(gi, c * SPMV_CHUNK, nc, (int32_t)(spmv_gslots + c)));
                spmv_gslots += (int64_t)rs.size() * nc;
            }
            // split groups first (their chunks are the longest items)
            spmv_gitems.insert(spmv_gitems.end(), shortit.begin(), shortit.end());
        }
        // products with the factor
        alt_tasks.clear();
        al_tasks.clear();
        for (int32_t s = 0; s < ns; s++) {
            for (int32_t b = 0; b < (pfront[s] + SB - 1) / SB; b++) alt_tasks.push_back(make_int2(s, b));
            for (int32_t t = 0; t < (mfront[s] + SB - 1) / SB; t++) al_tasks.push_back(make_int2(s, t));
        }
        gptr.assign((size_t)S.n + 1, 0);
        for (int32_t s = 0; s < ns; s++)
            for (int64_t q = S.rptr[s]; q < S.rptr[s + 1]; q++) gptr[S.rows[q] + 1]++;
        for (int32_t i = 0; i < S.n; i++) gptr[i + 1] += gptr[i];
        glist.resize((size_t)gptr[S.n]);
        {
            std::vector<int64_t> fill(gptr.begin(), gptr.end() - 1);
            for (int32_t s = 0; s < ns; s++)
                for (int64_t q = S.rptr[s]; q < S.rptr[s + 1]; q++)
                    glist[fill[S.rows[q]]++] = woff[s] + (q - S.rptr[s]);
        }
        zero_tasks.clear();
        lower_elems = 0;
        for (int32_t s = 0; s < ns; s++) {
            for (int32_t c0 = 0; c0 < pfront[s]; c0 += ZCOLS) zero_tasks.push_back(make_int2(s, c0));
            lower_elems += (int64_t)pfront[s] * mfront[s] - (int64_t)pfront[s] * (pfront[s] - 1) / 2;
        }
        colof.resize((size_t)S.nnz);
        for (int32_t j = 0; j < S.n; j++)
            for (int64_t p = S.colptr[j]; p < S.colptr[j + 1]; p++) colof[p] = j;
    }
};

// Workspace layout (byte offsets), all segments 256-byte aligned.
struct Layout {
    size_t fronts, W, Y, Xr, Rr, Br, vec, bad;
    size_t front_off, mfront, pfront, first, sparent, rptr, rows, rel, amap, woff, child_ptr, child_list, easplit;
    size_t perm, csr_ptr, csr_col, csr_src, csr_val, rowind, colof, segp;
    size_t pan, upd, ea, flist, dscr, dinv, dscr_off, slist, sfwd, sbelow, sbwd, sasm, part, ztasks;
    size_t sblk, sbsum, xinvt, xoff, xinv, part2, dinvt, altt, alt2, gptr, glist;
    size_t spchunk, splong, sppart, iperm, leafq, leafc, diagf, stept, spgrp, spgit, spglong;
    // LU factors only: the U^T fronts and their diagonal-block scratch, inverses and super-block inverses
    size_t fronts_u = 0, dscr_u = 0, dinv_u = 0, xinv_u = 0;
    size_t total;

    void compute(const Symbolic &S, const Plan &P, size_t esz, int32_t k, bool lu = false)
    {
        size_t o = 0;
        auto seg = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes); return at; };
        size_t n = (size_t)S.n, ns = (size_t)S.ns;
        fronts = seg((size_t)S.front_off.back() * esz + 64);   // + slack read past the last column by k_update_dma
        if (lu) {
            fronts_u = seg((size_t)S.front_off.back() * esz + 64);
            dscr_u = seg((size_t)P.dscr_elems * esz);
            dinv_u = seg((size_t)P.dscr_elems * esz);
            xinv_u = seg((size_t)std::max<int64_t>(1, P.xelems) * esz);
        }
        W = seg((size_t)P.wrows * k * esz);
        Y = seg(n * k * esz);
        Xr = seg(n * k * 8);
        Rr = seg(n * k * 8);
        Br = seg(n * k * 8);
        size_t nseg = nseg_of(S);
        vec = seg((2 * nseg * k + 2 * (size_t)k) * 8 + 64);
        bad = seg(64);
        front_off = seg((ns + 1) * 8);
        mfront = seg(ns * 4);
        pfront = seg(ns * 4);
        first = seg(ns * 4);
        sparent = seg(ns * 4);
        rptr = seg((ns + 1) * 8);
        rows = seg(S.rows.size() * 4);
        rel = seg(S.rel.size() * 4);
        amap = seg((size_t)S.nnz * 8);
        woff = seg(ns * 8);
        child_ptr = seg((ns + 1) * 4);
        child_list = seg(std::max<size_t>(1, P.child_list.size()) * 4);
        easplit = seg(ns * 4);
        perm = seg(n * 4);
        csr_ptr = seg((n + 1) * 8);
        csr_col = seg(S.csr_col.size() * 4);
        csr_src = seg(S.csr_src.size() * 8);
        csr_val = seg(S.csr_col.size() * 8);
        rowind = seg((size_t)S.nnz * 4);
        colof = seg((size_t)S.nnz * 4);
        pan = seg(std::max<size_t>(1, P.pan_tasks.size()) * sizeof(int2));
        upd = seg(std::max<size_t>(1, P.upd_tasks.size()) * sizeof(UpdTask));
        ea = seg(std::max<size_t>(1, P.ea_tasks.size()) * sizeof(int2));
        flist = seg(std::max<size_t>(1, P.flist.size()) * 4);
        dscr = seg((size_t)P.dscr_elems * esz);
        dinv = seg((size_t)P.dscr_elems * esz);
        slist = seg(std::max<size_t>(1, P.slist.size()) * 4);
        sfwd = seg(std::max<size_t>(1, P.sfwd_tasks.size()) * sizeof(int2));
        sbelow = seg(std::max<size_t>(1, P.sbelow_tasks.size()) * sizeof(int4));
        sbwd = seg(std::max<size_t>(1, P.sbwd_tasks.size()) * sizeof(int2));
        sblk = seg(std::max<size_t>(1, P.sblk_tasks.size()) * sizeof(int2));
        sbsum = seg(std::max<size_t>(1, P.sbsum_tasks.size()) * sizeof(int4));
        xinvt = seg(std::max<size_t>(1, P.xinv_tasks.size()) * sizeof(int4));
        dinvt = seg(std::max<size_t>(1, P.dinv_tasks.size()) * sizeof(int2));
        altt = seg(std::max<size_t>(1, P.alt_tasks.size()) * sizeof(int2));
        alt2 = seg(std::max<size_t>(1, P.al_tasks.size()) * sizeof(int2));
        gptr = seg(P.gptr.size() * 8);
        glist = seg(std::max<size_t>(1, P.glist.size()) * 8);
        xoff = seg(ns * 8);
        xinv = seg((size_t)std::max<int64_t>(1, P.xelems) * esz);
        part2 = seg((size_t)std::max<int64_t>(1, P.part_blocks) * SB * k * esz);
        sasm = seg(std::max<size_t>(1, P.sasm_tasks.size()) * sizeof(int2));
        part = seg(std::max<size_t>(kPartBlocks, nseg) * k * 8 * 2);
        segp = seg((nseg + 1) * 4);
        ztasks = seg(std::max<size_t>(1, P.zero_tasks.size()) * sizeof(int2));
        dscr_off = seg(ns * 8);
        spchunk = seg(std::max<size_t>(1, P.spmv_chunks.size()) * sizeof(int4));
        splong = seg(std::max<size_t>(1, P.spmv_long.size()) * sizeof(int4));
        sppart = seg((size_t)std::max<int64_t>(1, std::max(P.spmv_slots, P.spmv_gslots)) * k * 8);
        spgrp = seg(std::max<size_t>(1, P.spmv_grp.size()) * sizeof(int4));
        spgit = seg(std::max<size_t>(1, P.spmv_gitems.size()) * sizeof(int4));
        spglong = seg(std::max<size_t>(1, P.spmv_glong.size()) * sizeof(int4));
        iperm = seg(n * 4);
        leafq = seg(std::max<size_t>(1, P.leaf_queue.size()) * 4);
        leafc = seg(4);
        diagf = seg(std::max<size_t>(1, P.diag_fronts.size()) * 4);
        stept = seg(std::max<size_t>(1, P.step_tasks.size()) * sizeof(int4));
        total = o;
    }
};

size_t elem_size(wcs_precision p) { return p == WCS_FP32 ? 4 : 8; }
bool is_lu(wcs_precision p) { return p == WCS_LU64; }
bool valid_prec(wcs_precision p) { return p == WCS_FP64 || p == WCS_FP32 || p == WCS_LU64; }

// Update kernel used before any autotuning: on large fronts the streamed form
// is the faster one in FP64 and the register-staged one in FP32.
int32_t default_update_variant(wcs_precision p) { return p == WCS_FP32 ? WCS_UPD_REG128 : WCS_UPD_STREAM128; }

int grid_for(int64_t work, int threads = 256)
{
    int64_t g = (work + threads - 1) / threads;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, 1 << 16));
}

}  // namespace
}  // namespace wcs

struct wcs_factor_s {
    const wcs::Symbolic *S = nullptr;
    wcs::Plan plan;
    wcs::Layout lay;
    wcs_precision prec = WCS_FP64;
    int32_t max_nrhs = 1;
    char *ws = nullptr;
    size_t bytes = 0;
    bool have_values = false;
    std::vector<double> last_rel;              // last refinement residuals per (segment, column)
    int static_device = -1;                    // device whose static workspace this factor holds, or -1
    int ncu = 256;                             // compute units of the device (grid of the persistent leaf kernel)

    // replay of recorded launch sequences (wcs_factor_use_graphs)
    bool graphs = false;
    hipGraphExec_t fgraph = nullptr;           // numeric factorization, recorded for fgraph_values
    const double *fgraph_values = nullptr;
    struct SweepGraph {
        int part, k;
        hipGraphExec_t exec;
    };
    std::vector<SweepGraph> sgraphs;           // triangular sweeps per (part, nrhs)

    // look-ahead: side stream (default priority) and the two events that order
    // it; a third stream inverts each level's diagonal blocks beside the
    // following levels
    hipStream_t side = nullptr, aux = nullptr;
    hipEvent_t ev_main = nullptr, ev_side = nullptr, ev_aux = nullptr;

    void drop_graphs()
    {
        if (fgraph) (void)hipGraphExecDestroy(fgraph);
        fgraph = nullptr;
        fgraph_values = nullptr;
        for (auto &g : sgraphs) (void)hipGraphExecDestroy(g.exec);
        sgraphs.clear();
    }
    ~wcs_factor_s();
    void release()
    {
        drop_graphs();
        if (ev_main) (void)hipEventDestroy(ev_main);
        if (ev_side) (void)hipEventDestroy(ev_side);
        if (ev_aux) (void)hipEventDestroy(ev_aux);
        if (side) (void)hipStreamDestroy(side);
        if (aux) (void)hipStreamDestroy(aux);
    }

    template <typename P> P *at(size_t off) const { return reinterpret_cast<P *>(ws + off); }
};

// ---------------------------------------------------------------- static workspace
// Device memory of wcs_factor_create_static, for callers that cannot
// allocate: a file-scope array of WCS_STATIC_WORKSPACE_BYTES that every GPU
// the library runs on holds until the process ends.  Host code never passes
// `scratch` itself to a kernel or a copy (on the host it names a stand-in,
// not the device array): each device's address comes from
// hipGetSymbolAddress, taken once per device with that device current.  At
// most one factor per device lives in it at a time.
__device__ __align__(256) unsigned char scratch[WCS_STATIC_WORKSPACE_BYTES];

namespace wcs {
namespace {
struct StaticSlot {
    char *ptr = nullptr;      // device address of `scratch` on this device
    bool in_use = false;      // a live factor holds it
};
std::mutex g_static_mu;
std::vector<StaticSlot> g_static;   // per device ordinal
}  // namespace
}  // namespace wcs

wcs_factor_s::~wcs_factor_s()
{
    release();
    if (static_device >= 0) {
        std::lock_guard<std::mutex> lk(wcs::g_static_mu);
        wcs::g_static[(size_t)static_device].in_use = false;
    }
}

namespace wcs {
namespace {

// Optional per-kernel-class timing with HIP events on the launch stream,
// plus the algorithmic work of every launch (for roofline accounting).
enum KClass { KC_FILL = 0, KC_SCATTER, KC_EXTEND_ADD, KC_PANEL, KC_PANEL_FP64DIAG, KC_UPDATE, KC_COUNT };

struct Prof {
    hipStream_t st;
    bool levels = false;                 // time levels instead of kernel classes
    std::vector<hipEvent_t> lev;         // begin/end per level
    std::vector<double> lev_flops;
    std::vector<hipEvent_t> ev[KC_COUNT];
    double flops[KC_COUNT] = {0};
    double bytes[KC_COUNT] = {0};
    int mark(std::vector<hipEvent_t> &v)
    {
        hipEvent_t a;
        HIP_TRY(hipEventCreate(&a));
        v.push_back(a);
        HIP_TRY(hipEventRecord(a, st));
        return WCS_OK;
    }
    int collect_levels(wcs_kernel_stat *out)
    {
        HIP_TRY(hipStreamSynchronize(st));
        for (size_t h = 0; h + 1 < lev.size() + 1 && 2 * h + 1 < lev.size(); h++) {
            float t = 0;
            HIP_TRY(hipEventElapsedTime(&t, lev[2 * h], lev[2 * h + 1]));
            out[h].launches = 0;
            out[h].ms = t;
            out[h].flops = lev_flops[h];
            out[h].bytes = 0;
        }
        return WCS_OK;
    }
    int begin(int c)
    {
        if (levels) return WCS_OK;
        hipEvent_t a;
        HIP_TRY(hipEventCreate(&a));
        ev[c].push_back(a);
        HIP_TRY(hipEventRecord(a, st));
        return WCS_OK;
    }
    int end(int c)
    {
        if (levels) return WCS_OK;
        hipEvent_t b;
        HIP_TRY(hipEventCreate(&b));
        ev[c].push_back(b);
        HIP_TRY(hipEventRecord(b, st));
        return WCS_OK;
    }
    int collect(wcs_kernel_stat *out)
    {
        HIP_TRY(hipStreamSynchronize(st));
        for (int c = 0; c < KC_COUNT; c++) {
            double ms = 0;
            for (size_t i = 0; i + 1 < ev[c].size(); i += 2) {
                float t = 0;
                HIP_TRY(hipEventElapsedTime(&t, ev[c][i], ev[c][i + 1]));
                ms += t;
            }
            out[c].launches = (int32_t)(ev[c].size() / 2);
            out[c].ms = ms;
            out[c].flops = flops[c];
            out[c].bytes = bytes[c];
        }
        return WCS_OK;
    }
    ~Prof()
    {
        for (int c = 0; c < KC_COUNT; c++)
            for (hipEvent_t e : ev[c]) (void)hipEventDestroy(e);
        for (hipEvent_t e : lev) (void)hipEventDestroy(e);
    }
};

#define PROF_BEGIN(c) do { if (prof) { int r_ = prof->begin(c); if (r_) return r_; } } while (0)
#define PROF_END(c) do { if (prof) { int r_ = prof->end(c); if (r_) return r_; } } while (0)

// algorithmic work (host accounting only)
double panel_flops(const Plan &P, int32_t s, int32_t k0)
{
    double nb = std::min(NB, P.pfront[s] - k0);
    double below = P.mfront[s] - k0 - nb;
    return nb * nb * nb / 3.0 + below * nb * nb;
}
// one k_step task: the panel rows it solves (if it writes them), its share of
// the outer block's update, and the next diagonal block it factors
double step_flops(const Plan &P, const int4 &t, int32_t k0, int32_t K0)
{
    if (t.z == STEP_COPY_ONLY) return 0;
    double m = P.mfront[t.x], p = P.pfront[t.x];
    double nb = std::min<double>(NB, p - k0);
    double fl = 0;
    if (t.w & STEP_WRITE) fl += nb * nb * std::min<double>(NB, m - t.y);
    if (t.z >= 0) {
        double cnt = 0;
        int32_t jend = std::min(t.z + NB, std::min(K0 + P.nbo, P.pfront[t.x]));
        for (int32_t col = t.z; col < jend; col++)
            cnt += std::max<double>(0, std::min<double>(t.y + NB, m) - std::max<double>(t.y, col));
        fl += 2.0 * nb * cnt;
    }
    if (t.w & STEP_DIAG) {
        double nb2 = std::min<double>(NB, p - t.z);
        fl += nb2 * nb2 * nb2 / 3.0;
    }
    return fl;
}
double update_flops(const Plan &P, const int4 &t, int32_t jbeg, int32_t ka, int32_t kw, int32_t tw)
{
    int32_t m = P.mfront[t.x], p = P.pfront[t.x];
    double K = std::min(kw, p - ka);
    double cnt = 0;
    for (int32_t col = std::max(t.z, jbeg); col < std::min(t.z + tw, t.w); col++)
        cnt += std::max(0, std::min(t.y + tw, m) - std::max(t.y, col));
    return 2.0 * K * cnt;
}

// Numeric factorization.  Cholesky: values = the stored lower entries.  LU
// (f->prec == WCS_LU64, T = double): values = the entries on and below the
// diagonal, upper = the entry above the diagonal of each stored lower entry;
// every step runs on the L fronts and the U^T fronts alike (see k_lu_panel).
template <typename T>
int launch_factor(wcs_factor f, const double *values, hipStream_t st, Prof *prof, const double *upper = nullptr)
{
    const Layout &Lo = f->lay;
    const Plan &P = f->plan;
    const Symbolic &S = *f->S;
    const size_t esz = sizeof(T);
    const bool lu = is_lu(f->prec);
    T *fronts = f->at<T>(Lo.fronts);
    T *fronts_u = lu ? f->at<T>(Lo.fronts_u) : nullptr;
    const int nbuf = lu ? 2 : 1;
    auto buf = [&](int b) { return b ? fronts_u : fronts; };
    hipLaunchKernelGGL(k_fill<int32_t>, dim3(1), dim3(64), 0, st, f->at<int32_t>(Lo.bad), (int64_t)1, INT32_MAX);
    PROF_BEGIN(KC_FILL);
    for (int b = 0; b < nbuf; b++)
        hipLaunchKernelGGL(k_zero_lower<T>, dim3((unsigned)std::min<int64_t>(P.zero_tasks.size(), 1 << 30)), dim3(256),
                           0, st, f->at<int2>(Lo.ztasks), f->at<int64_t>(Lo.front_off), f->at<int32_t>(Lo.mfront),
                           f->at<int32_t>(Lo.pfront), buf(b));
    PROF_END(KC_FILL);
    PROF_BEGIN(KC_SCATTER);
    if constexpr (sizeof(T) == 8) {
        if (lu)
            hipLaunchKernelGGL(k_scatter_lu, dim3(grid_for(S.nnz)), dim3(256), 0, st, values, upper,
                               f->at<int64_t>(Lo.amap), f->at<int32_t>(Lo.rowind), f->at<int32_t>(Lo.colof),
                               f->at<int32_t>(Lo.iperm), S.nnz, fronts, fronts_u);
    }
    if (!lu)
        hipLaunchKernelGGL(k_scatter<T>, dim3(grid_for(S.nnz)), dim3(256), 0, st, values, f->at<int64_t>(Lo.amap),
                           S.nnz, fronts);
    PROF_END(KC_SCATTER);
    if (prof) {
        prof->bytes[KC_FILL] += (double)P.lower_elems * esz * nbuf;
        prof->bytes[KC_SCATTER] += (double)S.nnz * (8 + 8 + esz) * nbuf;
    }
    const int64_t *fo = f->at<int64_t>(Lo.front_off);
    const int32_t *mf = f->at<int32_t>(Lo.mfront);
    const int32_t *pf = f->at<int32_t>(Lo.pfront);
    const int32_t *fi = f->at<int32_t>(Lo.first);
    const int32_t *sp = f->at<int32_t>(Lo.sparent);
    const int64_t *rp = f->at<int64_t>(Lo.rptr);
    const int32_t *rl = f->at<int32_t>(Lo.rel);
    const int2 *pan = f->at<int2>(Lo.pan);
    const UpdTask *upd = f->at<UpdTask>(Lo.upd);
    const int2 *ea = f->at<int2>(Lo.ea);
    int32_t *bad = f->at<int32_t>(Lo.bad);
    const int64_t *dso = f->at<int64_t>(Lo.dscr_off);
    T *dscr = f->at<T>(Lo.dscr);
    T *dinv = f->at<T>(Lo.dinv);
    // trailing updates marked `side` go to the side stream (not while timing
    // kernel classes, whose events time one stream; level timing is fine, as
    // every level joins the side stream before its closing event)
    hipStream_t side = ((prof && !prof->levels) || !f->side) ? st : f->side;
    hipStream_t aux = ((prof && !prof->levels) || !f->aux) ? st : f->aux;
    bool pending = false;   // side-stream work not yet joined into st
    const int32_t *esp = f->at<int32_t>(Lo.easplit);
    auto extend_add = [&](const std::vector<std::pair<int64_t, int64_t>> &rounds, bool pre) -> int {
        for (auto &r : rounds) {
            PROF_BEGIN(KC_EXTEND_ADD);
            for (int b = 0; b < nbuf; b++)
                hipLaunchKernelGGL(k_extend_add<T>, dim3((unsigned)r.second), dim3(256), 0, st, ea + r.first, fo, mf,
                                   pf, sp, rp, rl, pre ? esp : nullptr, buf(b));
            PROF_END(KC_EXTEND_ADD);
            if (prof)
                for (int64_t t = r.first; t < r.first + r.second; t++) {
                    int2 task = P.ea_tasks[t];
                    double nu = P.mfront[task.x] - P.pfront[task.x];
                    double c1 = std::min<double>(task.y + EA_COLS, pre ? P.ea_split[task.x] : nu);
                    for (double col = task.y; col < c1; col++)
                        prof->bytes[KC_EXTEND_ADD] += (nu - col) * (3 * esz + 4) * nbuf;
                }
        }
        return WCS_OK;
    };
    for (size_t h = 0; h < P.levels.size(); h++) {
        const Level &L = P.levels[h];
        if (prof && prof->levels) {
            int r_ = prof->mark(prof->lev);
            if (r_) return r_;
            double fl = 0;
            for (int64_t q = L.fl_off; q < L.fl_off + L.fl_cnt; q++) {
                int32_t s = P.flist[q];
                for (int32_t t = 0; t < P.pfront[s]; t++) fl += (double)(P.mfront[s] - t) * (P.mfront[s] - t);
            }
            prof->lev_flops.push_back(fl);
        }
        int r_ea = extend_add(L.ea, true);
        if (r_ea) return r_ea;
        if (L.leaf_cnt) {
            // on the side stream when the level also has fronts for the
            // level-synchronous launches (independent of these); the level's
            // closing join waits for it
            hipStream_t ls = st;
            if (side != st && !L.ops.empty()) {
                HIP_TRY(hipEventRecord(f->ev_main, st));
                HIP_TRY(hipStreamWaitEvent(side, f->ev_main, 0));
                ls = side;
            }
            int32_t *ctr = f->at<int32_t>(Lo.leafc);
            PROF_BEGIN(KC_PANEL);
            hipLaunchKernelGGL(k_fill<int32_t>, dim3(1), dim3(64), 0, ls, ctr, (int64_t)1, 0);
            hipLaunchKernelGGL(k_leaf<T>, dim3((unsigned)std::min<int64_t>(L.leaf_cnt, LeafCfg<T>::PER_CU * f->ncu)),
                               dim3(THREADS), 0, ls, f->at<int32_t>(Lo.leafq) + L.leaf_off, (int)L.leaf_cnt, ctr, fo,
                               mf, pf, fi, dso, fronts, dscr, bad);
            PROF_END(KC_PANEL);
            if (ls != st) {
                HIP_TRY(hipEventRecord(f->ev_side, ls));
                pending = true;
            }
            if (prof)
                for (int64_t q = L.leaf_off; q < L.leaf_off + L.leaf_cnt; q++) {
                    int32_t s = P.leaf_queue[q];
                    double m = P.mfront[s], pp = P.pfront[s];
                    prof->flops[KC_PANEL] += pp * pp * pp / 3.0 + (m - pp) * pp * pp + (m - pp) * (m - pp + 1) * pp;
                }
        }
        for (const Op &op : L.ops) {
            if (op.kind == OP_UPDATE) {
                bool small = L.upd_var == WCS_UPD_REG64;
                int64_t off = small ? op.off64 : op.off, cnt = small ? op.cnt64 : op.cnt;
                if (op.join && pending) {
                    HIP_TRY(hipStreamWaitEvent(st, f->ev_side, 0));
                    pending = false;
                }
                if (cnt == 0) continue;
                hipStream_t us = st;
                unsigned grid = (unsigned)cnt;
                if (op.side && side != st) {
                    const int cap = side_grid(f->ncu) * (small ? 4 : 1);   // 64-tiles: one-wave workgroups
                    if (cap > 0 && cnt > cap) grid = (unsigned)cap;
                    HIP_TRY(hipEventRecord(f->ev_main, st));
                    HIP_TRY(hipStreamWaitEvent(side, f->ev_main, 0));
                    us = side;
                }
                PROF_BEGIN(KC_UPDATE);
                for (int b = 0; b < nbuf; b++) {
                    // LU: the L fronts take B from the U^T fronts and the other way round
                    T *cf = buf(b);
                    const int64_t bd = lu ? (int64_t)(buf(1 - b) - cf) : 0;
                    if (small)
                        hipLaunchKernelGGL((k_update<T, 64>), dim3(grid), dim3(64), 0, us, upd + off, (int)cnt, op.ka,
                                           op.kw, cf, bd);
                    else if (L.upd_var == WCS_UPD_STREAM128)
                        hipLaunchKernelGGL((k_update_dma<T, 4>), dim3(grid), dim3(256), 0, us, upd + off, (int)cnt,
                                           op.ka, op.kw, cf, bd);
                    else if (L.upd_var == WCS_UPD_STREAM128_3)
                        hipLaunchKernelGGL((k_update_dma<T, 3>), dim3(grid), dim3(256), 0, us, upd + off, (int)cnt,
                                           op.ka, op.kw, cf, bd);
                    else if (L.upd_var == WCS_UPD_STREAM128_K32)
                        hipLaunchKernelGGL((k_update_dma<T, 2, 2 * DmaCfg<T>::KC>), dim3(grid), dim3(256), 0, us,
                                           upd + off, (int)cnt, op.ka, op.kw, cf, bd);
                    else
                        hipLaunchKernelGGL((k_update<T, UT>), dim3(grid), dim3(UT * UT / 64), 0, us,
                                           upd + off, (int)cnt, op.ka, op.kw, cf, bd);
                }
                PROF_END(KC_UPDATE);
                if (us != st) {
                    HIP_TRY(hipEventRecord(f->ev_side, side));
                    pending = true;
                }
                if (prof)
                    for (int64_t q = off; q < off + cnt; q++)
                        prof->flops[KC_UPDATE] += nbuf * update_flops(P, P.upd_tasks[q], P.upd_jbeg[q], op.ka, op.kw,
                                                                       small ? 64 : UT);
            } else if (op.kind == OP_DIAG || op.kind == OP_STEP) {
                int c = op.d64 ? KC_PANEL_FP64DIAG : KC_PANEL;
                PROF_BEGIN(c);
                if (op.kind == OP_DIAG) {
                    if (op.d64)
                        hipLaunchKernelGGL((k_diag_factor<T, double>), dim3((unsigned)op.cnt), dim3(THREADS), 0, st,
                                           f->at<int32_t>(Lo.diagf) + op.off, op.ka, fo, mf, pf, fi, dso, fronts, dscr,
                                           dinv, bad);
                    else
                        hipLaunchKernelGGL((k_diag_factor<T, T>), dim3((unsigned)op.cnt), dim3(THREADS), 0, st,
                                           f->at<int32_t>(Lo.diagf) + op.off, op.ka, fo, mf, pf, fi, dso, fronts, dscr,
                                           dinv, bad);
                } else {
                    const int nbo = P.nbo;
                    if (op.d64)
                        hipLaunchKernelGGL((k_step<T, double>), dim3((unsigned)op.cnt), dim3(THREADS), 0, st,
                                           f->at<int4>(Lo.stept) + op.off, op.ka, op.kw, nbo, fo, mf, pf, fi, dso,
                                           fronts, dscr, dinv, bad);
                    else
                        hipLaunchKernelGGL((k_step<T, T>), dim3((unsigned)op.cnt), dim3(THREADS), 0, st,
                                           f->at<int4>(Lo.stept) + op.off, op.ka, op.kw, nbo, fo, mf, pf, fi, dso,
                                           fronts, dscr, dinv, bad);
                }
                PROF_END(c);
                if (prof) {
                    if (op.kind == OP_DIAG)
                        for (int64_t q = op.off; q < op.off + op.cnt; q++) {
                            double nb = std::min(NB, P.pfront[P.diag_fronts[q]] - op.ka);
                            prof->flops[c] += nb * nb * nb / 3.0;
                        }
                    else
                        for (int64_t q = op.off; q < op.off + op.cnt; q++) prof->flops[c] += step_flops(P, P.step_tasks[q], op.ka, op.kw);
                }
            } else {
                int c = (op.kind == OP_PANEL || lu) ? KC_PANEL : KC_PANEL_FP64DIAG;
                PROF_BEGIN(c);
                if constexpr (sizeof(T) == 8) {
                    if (lu)
                        hipLaunchKernelGGL(k_lu_panel<T>, dim3((unsigned)op.cnt), dim3(THREADS), 0, st, pan + op.off,
                                           op.ka, fo, mf, pf, fi, dso, fronts, fronts_u, dscr, f->at<T>(Lo.dscr_u),
                                           bad);
                }
                if (lu) {
                } else if (op.kind == OP_PANEL)
                    hipLaunchKernelGGL((k_panel<T, T>), dim3((unsigned)op.cnt), dim3(THREADS), 0, st,
                                       pan + op.off, op.ka, fo, mf, pf, fi, dso, fronts, dscr, bad);
                else
                    hipLaunchKernelGGL((k_panel<T, double>), dim3((unsigned)op.cnt), dim3(THREADS), 0, st,
                                       pan + op.off, op.ka, fo, mf, pf, fi, dso, fronts, dscr, bad);
                PROF_END(c);
                if (prof)
                    for (int64_t q = op.off; q < op.off + op.cnt; q++)
                        if (P.pan_tasks[q].y == 0) prof->flops[c] += nbuf * panel_flops(P, P.pan_tasks[q].x, op.ka);
            }
        }
        if (pending) {   // the next level's extend-add reads this level's update matrices
            HIP_TRY(hipStreamWaitEvent(st, f->ev_side, 0));
            pending = false;
        }
        if (L.dinv_cnt) {
            // this level's fronts are final: beside the levels above, copy their
            // diagonal blocks into place and invert them, then build the solve's
            // super-block inverses from them
            if (aux != st) {
                HIP_TRY(hipEventRecord(f->ev_main, st));
                HIP_TRY(hipStreamWaitEvent(aux, f->ev_main, 0));
            }
            PROF_BEGIN(KC_FILL);
            for (int b = 0; b < nbuf; b++)
                hipLaunchKernelGGL(k_diag_inv<T>, dim3((unsigned)L.dinv_cnt), dim3(64), 0, aux,
                                   f->at<int2>(Lo.dinvt) + L.dinv_off, dso, b ? f->at<T>(Lo.dscr_u) : dscr,
                                   b ? f->at<T>(Lo.dinv_u) : dinv, fo, mf, pf, buf(b));
            const std::pair<int64_t, int64_t> &xt = L.sv.xinv;
            for (int b = 0; b < nbuf && xt.second; b++)
                hipLaunchKernelGGL(k_build_xinv<T>, dim3((unsigned)xt.second), dim3(THREADS), 0, aux,
                                   f->at<int4>(Lo.xinvt) + xt.first, fo, mf, pf, dso, f->at<int64_t>(Lo.xoff),
                                   buf(b), b ? f->at<T>(Lo.dinv_u) : dinv,
                                   b ? f->at<T>(Lo.xinv_u) : f->at<T>(Lo.xinv));
            PROF_END(KC_FILL);
            // read the block, write its inverse and the lower half of its place
            if (prof) prof->bytes[KC_FILL] += (double)L.dinv_cnt * NB * NB * esz * 2.5 * nbuf;
        }
        r_ea = extend_add(L.ea_post, false);
        if (r_ea) return r_ea;
        if (prof && prof->levels) {
            int r_ = prof->mark(prof->lev);
            if (r_) return r_;
        }
    }
    if (aux != st) {   // the diagonal blocks and the solve's inverses
        HIP_TRY(hipEventRecord(f->ev_aux, aux));
        HIP_TRY(hipStreamWaitEvent(st, f->ev_aux, 0));
    }
    HIP_TRY(hipGetLastError());
    return WCS_OK;
}

// device pointers of the factor for the solve and product kernels
// upper = true: the U^T fronts of an LU factor (the backward sweep solves
// with U = (U^T)^T exactly as the Cholesky one solves with L^T)
template <typename T>
SolveArgs<T> solve_args(wcs_factor f, int k, bool upper = false)
{
    SolveArgs<T> a;
    const Layout &Lo = f->lay;
    a.front_off = f->at<int64_t>(Lo.front_off);
    a.mfront = f->at<int32_t>(Lo.mfront);
    a.pfront = f->at<int32_t>(Lo.pfront);
    a.first = f->at<int32_t>(Lo.first);
    a.woff = f->at<int64_t>(Lo.woff);
    a.child_ptr = f->at<int32_t>(Lo.child_ptr);
    a.child_list = f->at<int32_t>(Lo.child_list);
    a.rptr = f->at<int64_t>(Lo.rptr);
    a.rel = f->at<int32_t>(Lo.rel);
    a.rows = f->at<int32_t>(Lo.rows);
    a.dscr_off = f->at<int64_t>(Lo.dscr_off);
    a.fronts = f->at<T>(Lo.fronts);
    a.dinv = f->at<T>(Lo.dinv);
    a.xoff = f->at<int64_t>(Lo.xoff);
    a.xinv = f->at<T>(Lo.xinv);
    a.part = f->at<T>(Lo.part2);
    a.W = f->at<T>(Lo.W);
    a.Y = f->at<T>(Lo.Y);
    a.k = k;
    if (upper && is_lu(f->prec)) {
        a.fronts = f->at<T>(Lo.fronts_u);
        a.dinv = f->at<T>(Lo.dinv_u);
        a.xinv = f->at<T>(Lo.xinv_u);
    }
    return a;
}

// Y (row-major, pivot order, n x k) := L^-1 Y and/or L^-T Y
template <typename T, int KT>
int launch_sweeps(wcs_factor f, int part, int k, hipStream_t st)
{
    const Layout &Lo = f->lay;
    const Plan &P = f->plan;
    SolveArgs<T> a = solve_args<T>(f, k);
    const SolveArgs<T> au = solve_args<T>(f, k, true);    // the backward sweep's factor (LU: U^T)
    const int32_t *sl = f->at<int32_t>(Lo.slist);
    const int2 *tf = f->at<int2>(Lo.sfwd);
    const int4 *tb = f->at<int4>(Lo.sbelow);
    const int4 *tbs = f->at<int4>(Lo.sbsum);
    const int2 *ts = f->at<int2>(Lo.sbwd);
    const int2 *tas = f->at<int2>(Lo.sasm);
    const int2 *sbk = f->at<int2>(Lo.sblk);
    if (part == WCS_SOLVE_FULL || part == WCS_SOLVE_L) {
        for (const Level &L : P.levels) {
            const SolveLevel &V = L.sv;
            if (V.fused_cnt)
                hipLaunchKernelGGL((k_fwd_fused<T, KT>), dim3((unsigned)V.fused_cnt), dim3(THREADS), 0, st,
                                   sl + V.fused_off, a);
            if (V.step_cnt) {
                hipLaunchKernelGGL(k_fwd_assemble<T>, dim3((unsigned)V.assemble.second), dim3(THREADS), 0, st,
                                   tas + V.assemble.first, a);
                for (const SuperStep &s : V.fwd) {
                    hipLaunchKernelGGL((k_fwd_sz<T, KT>), dim3((unsigned)s.d_cnt), dim3(THREADS), 0, st,
                                       sbk + s.d_off, s.s0, a);
                    if (s.t_cnt)
                        hipLaunchKernelGGL((k_fwd_srows<T, KT>), dim3((unsigned)s.t_cnt), dim3(THREADS), 0, st,
                                           tf + s.t_off, s.s0, a);
                    if (s.t1_cnt) {
                        // one 64-column block: a wave per tile when the quad form applies
                        if (KT == 64 && k % 4 == 0)
                            hipLaunchKernelGGL(k_fwd_srows1<T>, dim3((unsigned)((s.t1_cnt + 3) / 4)), dim3(THREADS), 0,
                                               st, tf + s.t1_off, (int)s.t1_cnt, s.s0, a);
                        else
                            hipLaunchKernelGGL((k_fwd_srows<T, KT>), dim3((unsigned)s.t1_cnt), dim3(THREADS), 0, st,
                                               tf + s.t1_off, s.s0, a);
                    }
                }
            }
        }
    }
    if (part == WCS_SOLVE_FULL || part == WCS_SOLVE_LT) {
        for (size_t h = P.levels.size(); h-- > 0;) {
            const SolveLevel &V = P.levels[h].sv;
            if (V.fused_cnt)
                hipLaunchKernelGGL((k_bwd_fused<T, KT>), dim3((unsigned)V.fused_cnt), dim3(THREADS), 0, st,
                                   sl + V.fused_off, au);
            if (V.step_cnt) {
                if (V.below.second)
                    hipLaunchKernelGGL((k_bwd_below_part<T, KT>), dim3((unsigned)V.below.second), dim3(THREADS), 0,
                                       st, tb + V.below.first, au);
                hipLaunchKernelGGL(k_bwd_below_sum<T>, dim3((unsigned)V.below_sum.second), dim3(THREADS), 0, st,
                                   tbs + V.below_sum.first, au);
                for (const SuperStep &s : V.bwd) {
                    hipLaunchKernelGGL((k_bwd_sx<T, KT>), dim3((unsigned)s.d_cnt), dim3(THREADS), 0, st,
                                       sbk + s.d_off, s.s0, au);
                    if (s.t_cnt)
                        hipLaunchKernelGGL((k_bwd_scols<T, KT>), dim3((unsigned)s.t_cnt), dim3(THREADS), 0, st,
                                           ts + s.t_off, s.s0, au);
                }
            }
        }
    }
    HIP_TRY(hipGetLastError());
    return WCS_OK;
}

template <typename T>
int launch_solve_internal(wcs_factor f, int part, int k, hipStream_t st)
{
    if (k <= 4) return launch_sweeps<T, 4>(f, part, k, st);
    if (k <= kt16_max_rhs()) return launch_sweeps<T, 16>(f, part, k, st);
    return launch_sweeps<T, 64>(f, part, k, st);
}

// Records the launches made by fn on st into an executable graph.  The
// sequences recorded here are kernel launches only (no memset or copy nodes).
template <typename Fn>
int record(hipStream_t st, hipGraphExec_t *out, Fn &&fn)
{
    HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    int rc = fn();
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(st, &g);
    if (rc == WCS_OK && e != hipSuccess) {
        set_error(std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        rc = WCS_EHIP;
    }
    if (rc == WCS_OK) {
        e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            set_error(std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
            rc = WCS_EHIP;
        }
    }
    if (g) (void)hipGraphDestroy(g);
    return rc;
}

// The sweeps of one solve, replayed from a recorded graph when graphs are on
// (a stream other than the legacy default stream is needed for recording).
template <typename T>
int run_sweeps(wcs_factor f, int part, int k, hipStream_t st)
{
    if (!f->graphs || st == nullptr) return launch_solve_internal<T>(f, part, k, st);
    hipGraphExec_t ex = nullptr;
    for (auto &g : f->sgraphs)
        if (g.part == part && g.k == k) ex = g.exec;
    if (!ex) {
        int rc = record(st, &ex, [&] { return launch_solve_internal<T>(f, part, k, st); });
        if (rc) return rc;
        f->sgraphs.push_back({part, k, ex});
    }
    HIP_TRY(hipGraphLaunch(ex, st));
    return WCS_OK;
}

template <typename T>
int launch_solve(wcs_factor f, int part, int k, double *B, int64_t ld, hipStream_t st)
{
    const Layout &Lo = f->lay;
    int n = f->S->n;
    T *Y = f->at<T>(Lo.Y);
    const int32_t *perm = f->at<int32_t>(Lo.perm);
    int64_t nk = (int64_t)n * k;
    if (part == WCS_SOLVE_LT)
        hipLaunchKernelGGL(k_rows_in<T>, dim3(grid_for(nk)), dim3(256), 0, st, B, ld, n, k, Y);
    else
        hipLaunchKernelGGL(k_perm_in<T>, dim3(grid_for(nk)), dim3(256), 0, st, B, ld, perm, n, k, Y,
                           (const double *)nullptr);
    int rc = run_sweeps<T>(f, part, k, st);
    if (rc) return rc;
    if (part == WCS_SOLVE_L)
        hipLaunchKernelGGL(k_rows_out<T>, dim3(grid_for(nk)), dim3(256), 0, st, Y, n, k, B, ld);
    else
        hipLaunchKernelGGL(k_perm_out<T>, dim3(grid_for(nk)), dim3(256), 0, st, Y, perm, n, k, B, ld,
                           (const double *)nullptr, 0);
    HIP_TRY(hipGetLastError());
    return WCS_OK;
}

// B := P^T L B (WCS_APPLY_L, B in pivot order) or L^T P B (WCS_APPLY_LT, result
// in pivot order); B column-major FP64, computed in the factor's precision
template <typename T>
int launch_apply(wcs_factor f, int part, int k, double *B, int64_t ld, hipStream_t st)
{
    const Layout &Lo = f->lay;
    const Plan &P = f->plan;
    int n = f->S->n;
    T *Y = f->at<T>(Lo.Y), *W = f->at<T>(Lo.W);
    const int32_t *perm = f->at<int32_t>(Lo.perm);
    int64_t nk = (int64_t)n * k;
    SolveArgs<T> a = solve_args<T>(f, k);
    if (part == WCS_APPLY_LT) {
        hipLaunchKernelGGL(k_perm_in<T>, dim3(grid_for(nk)), dim3(256), 0, st, B, ld, perm, n, k, Y,
                           (const double *)nullptr);
        if (!P.alt_tasks.empty())
            hipLaunchKernelGGL(k_apply_lt<T>, dim3((unsigned)P.alt_tasks.size()), dim3(THREADS), 0, st,
                               f->at<int2>(Lo.altt), a, (const T *)Y, W);
        hipLaunchKernelGGL(k_rows_out<T>, dim3(grid_for(nk)), dim3(256), 0, st, (const T *)W, n, k, B, ld);
    } else {
        hipLaunchKernelGGL(k_rows_in<T>, dim3(grid_for(nk)), dim3(256), 0, st, B, ld, n, k, Y);
        if (!P.al_tasks.empty())
            hipLaunchKernelGGL(k_apply_l<T>, dim3((unsigned)P.al_tasks.size()), dim3(THREADS), 0, st,
                               f->at<int2>(Lo.alt2), a, (const T *)Y, W);
        hipLaunchKernelGGL(k_apply_gather<T>, dim3(grid_for(nk)), dim3(256), 0, st, f->at<int64_t>(Lo.gptr),
                           f->at<int64_t>(Lo.glist), n, k, (const T *)W, Y);
        hipLaunchKernelGGL(k_perm_out<T>, dim3(grid_for(nk)), dim3(256), 0, st, (const T *)Y, perm, n, k, B, ld,
                           (const double *)nullptr, 0);
    }
    HIP_TRY(hipGetLastError());
    return WCS_OK;
}

// beside = true: the expansion runs on a side stream next to the first solve
// of a refinement; its grid is then held to expand_side_blocks() workgroups,
// so that the solve's kernels are not queued behind its 2^16 workgroups.
int ensure_csr_values(wcs_factor f, const double *values, hipStream_t st, bool beside = false)
{
    const Symbolic &S = *f->S;
    int64_t nz = (int64_t)S.csr_col.size();
    int grid = grid_for(nz);
    if (beside) grid = std::min(grid, expand_side_blocks());
    hipLaunchKernelGGL(k_expand_values, dim3(grid), dim3(256), 0, st, values,
                       f->at<int64_t>(f->lay.csr_src), nz, f->at<double>(f->lay.csr_val));
    HIP_TRY(hipGetLastError());
    return WCS_OK;
}

// Caller column-major (leading dimension ld) <-> row-major n x k in pivot order
void gather_rows(wcs_factor f, const double *X, int64_t ld, int k, double *Xp, hipStream_t st)
{
    int n = f->S->n;
    if (k >= 4)
        hipLaunchKernelGGL(k_gather_rows_t, dim3((unsigned)((n + 63) / 64), (unsigned)((k + 63) / 64)), dim3(256), 0,
                           st, X, ld, f->at<int32_t>(f->lay.iperm), n, k, Xp);
    else
        hipLaunchKernelGGL(k_gather_rows, dim3(grid_for((int64_t)n * k)), dim3(256), 0, st, X, ld,
                           f->at<int32_t>(f->lay.perm), n, k, Xp);
}
void scatter_rows(wcs_factor f, const double *Xp, int k, double *X, int64_t ld, hipStream_t st)
{
    int n = f->S->n;
    if (k >= 4)
        hipLaunchKernelGGL(k_scatter_rows_t, dim3((unsigned)((n + 63) / 64), (unsigned)((k + 63) / 64)), dim3(256), 0,
                           st, Xp, f->at<int32_t>(f->lay.iperm), n, k, X, ld);
    else
        hipLaunchKernelGGL(k_scatter_rows, dim3(grid_for((int64_t)n * k)), dim3(256), 0, st, Xp,
                           f->at<int32_t>(f->lay.perm), n, k, X, ld);
}

// Row-major X of k = 4 LPE columns, LPE a power of two up to 16: the vector
// SpMM form (both types)
template <typename TX> bool spmv_vec_fits(int k)
{
    return k % 4 == 0 && k / 4 <= 16 && ((k / 4) & (k / 4 - 1)) == 0;
}

// R = B - mul[c] (C X), or R = C X when B is null; C = P A P^T in pivot order,
// row-major X, B, R with leading dimension k (spmv_vec_fits<TX>(k))
template <typename TX>
void launch_spmv_vec(wcs_factor f, int k, const TX *X, const double *B, const double *mul, double *R, hipStream_t st)
{
    // work items by groups of rows with one column pattern (k_spmv_grp)
    const Plan &P = f->plan;
    const int64_t *rp = f->at<int64_t>(f->lay.csr_ptr);
    const int32_t *ci = f->at<int32_t>(f->lay.csr_col);
    const double *v = f->at<double>(f->lay.csr_val);
    const int4 *items = f->at<int4>(f->lay.spgit);
    const int4 *grp = f->at<int4>(f->lay.spgrp);
    double *part = f->at<double>(f->lay.sppart);
    int ni = (int)P.spmv_gitems.size();
    dim3 g((unsigned)((ni + 3) / 4)), b(256);
    if constexpr (sizeof(TX) == 4) {
        // FP32 rows: four columns per lane (SpmvVecF4)
        switch (k / 4) {
        case 1: hipLaunchKernelGGL((k_spmv_grp<1, TX, SpmvVecF4>), g, b, 0, st, items, ni, grp, rp, ci, v, X, B, mul, R, part); break;
        case 2: hipLaunchKernelGGL((k_spmv_grp<2, TX, SpmvVecF4>), g, b, 0, st, items, ni, grp, rp, ci, v, X, B, mul, R, part); break;
        case 4: hipLaunchKernelGGL((k_spmv_grp<4, TX, SpmvVecF4>), g, b, 0, st, items, ni, grp, rp, ci, v, X, B, mul, R, part); break;
        case 8: hipLaunchKernelGGL((k_spmv_grp<8, TX, SpmvVecF4>), g, b, 0, st, items, ni, grp, rp, ci, v, X, B, mul, R, part); break;
        default: hipLaunchKernelGGL((k_spmv_grp<16, TX, SpmvVecF4>), g, b, 0, st, items, ni, grp, rp, ci, v, X, B, mul, R, part); break;
        }
    } else switch (k / 4) {
    case 1: hipLaunchKernelGGL((k_spmv_grp<1, TX>), g, b, 0, st, items, ni, grp, rp, ci, v, X, B, mul, R, part); break;
    case 2: hipLaunchKernelGGL((k_spmv_grp<2, TX>), g, b, 0, st, items, ni, grp, rp, ci, v, X, B, mul, R, part); break;
    case 4: hipLaunchKernelGGL((k_spmv_grp<4, TX>), g, b, 0, st, items, ni, grp, rp, ci, v, X, B, mul, R, part); break;
    case 8: hipLaunchKernelGGL((k_spmv_grp<8, TX>), g, b, 0, st, items, ni, grp, rp, ci, v, X, B, mul, R, part); break;
    default: hipLaunchKernelGGL((k_spmv_grp<16, TX>), g, b, 0, st, items, ni, grp, rp, ci, v, X, B, mul, R, part); break;
    }
    if (!P.spmv_glong.empty())
        hipLaunchKernelGGL(k_spmv_long_sum, dim3((unsigned)P.spmv_glong.size()), dim3(64), 0, st,
                           f->at<int4>(f->lay.spglong), k, (int64_t)k, part, B, mul, R);
}

// R = B - C X or Y = C X (B null) with C = P A P^T in pivot order; element
// (i, c) at i * sx + c * sc
int launch_spmv(wcs_factor f, int k, const double *X, const double *B, double *R, int64_t sx, int64_t sc,
                hipStream_t st)
{
    const Symbolic &S = *f->S;
    int n = S.n;
    const int64_t *rp = f->at<int64_t>(f->lay.csr_ptr);
    const int32_t *ci = f->at<int32_t>(f->lay.csr_col);
    const double *v = f->at<double>(f->lay.csr_val);
    unsigned nrb = (unsigned)((n + 3) / 4);
    if (sx == k && sc == 1 && spmv_vec_fits<double>(k)) {
        launch_spmv_vec<double>(f, k, X, B, nullptr, R, st);
    } else if (k == 1) {
        const Plan &P = f->plan;
        int ni = (int)P.spmv_chunks.size();
        double *part = f->at<double>(f->lay.sppart);
        hipLaunchKernelGGL(k_spmv_one, dim3((unsigned)((ni + 3) / 4)), dim3(256), 0, st, f->at<int4>(f->lay.spchunk),
                           ni, rp, ci, v, X, sx, B, R, part);
        if (!P.spmv_long.empty())
            hipLaunchKernelGGL(k_spmv_long_sum, dim3((unsigned)P.spmv_long.size()), dim3(64), 0, st,
                               f->at<int4>(f->lay.splong), 1, sx, part, B, (const double *)nullptr, R);
    } else if (k >= 8 && sx == k && sc == 1) {
        int per = ((int)nrb + 7) / 8;
        hipLaunchKernelGGL(k_spmv_wide, dim3((unsigned)(8 * per)), dim3(256), 0, st, rp, ci, v, n, k, X, B, R);
    } else {
        hipLaunchKernelGGL(k_spmv_narrow, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, rp, ci, v, n, k, X, B, R,
                           sx, sc);
    }
    HIP_TRY(hipGetLastError());
    return WCS_OK;
}

// out[c] (whole column) or out[sg * k + c] (per segment) = column reduction
// (op 0: sum of squares, op 1: max |a|) of row-major n x k A
void launch_colred(wcs_factor f, const double *A, int n, int k, int op, bool segmented, double *out, hipStream_t st)
{
    double *part = f->at<double>(f->lay.part);
    int nseg = segmented ? (int)nseg_of(*f->S) : 1;
    const int32_t *sp = segmented && nseg > 1 ? f->at<int32_t>(f->lay.segp) : nullptr;
    int bps = std::max(1, kPartBlocks / nseg);
    hipLaunchKernelGGL(k_colred_part, dim3((unsigned)(bps * nseg)), dim3(THREADS), 0, st, A, n, k, op, sp, nseg,
                       part);
    hipLaunchKernelGGL(k_colred_final, dim3((unsigned)nseg), dim3(THREADS), 0, st, part, bps, k, op, out);
}

// Refinement in pivot order: Bp = P B, Xp = solve(Bp), then while any
// column has ||R|| > tol ||Bp|| for R = Bp - C Xp: Xp += D = solve(R s) / s
// with the per-column power of two s ~ 1 / max|R| (keeps R inside the FP32
// range, unscaling is exact); X = P^T Xp.  With an FP32 factor Xp0 and every
// D are FP32 numbers times 2^e, so the residual is formed from their FP32
// rows (half the gathered bytes): R = Bp - C Y0, then R -= (C Y) / s after
// each correction, with FP64 products and sums.  That updated residual is
// Bp - C Xp up to the FP64 rounding of the sums Xp + D.  For a batch the test
// is per instance and column (each block of the block-diagonal matrix is its
// own system).
// The loop itself: Bp (row-major n x k, pivot order) holds P B, the matrix
// values are expanded (or will be once csr_ready, if given, has fired: the
// first residual waits for it); leaves P X in Xp and the residuals in
// f->last_rel.
template <typename T>
int refine_pivot(wcs_factor f, int k, double tol, int max_iter, wcs_ir_report *rep, hipStream_t st,
                 hipEvent_t csr_ready = nullptr)
{
    const Layout &Lo = f->lay;
    int n = f->S->n;
    int rc = WCS_OK;
    double *Bp = f->at<double>(Lo.Br);      // row-major n x k, pivot order
    double *Xp = f->at<double>(Lo.Xr);
    double *Rp = f->at<double>(Lo.Rr);
    const int nseg = (int)nseg_of(*f->S), nsk = nseg * k;
    // vec: [0,nsk) |B|^2 and [nsk,2nsk) |R|^2 per (segment, column); then amax[k], scale[k]
    double *vec = f->at<double>(Lo.vec);
    double *amax = vec + 2 * nsk, *scale = amax + k;    // amax becomes 1 / scale
    // FP32 factor: residual from the FP32 rows of the solves (see above)
    const bool from_y = sizeof(T) == 4 && spmv_vec_fits<float>(k);
    T *Y = f->at<T>(Lo.Y);
    int64_t nk = (int64_t)n * k;
    launch_colred(f, Bp, n, k, 0, true, vec, st);
    hipLaunchKernelGGL(k_cast_scaled<T>, dim3(grid_for(nk)), dim3(256), 0, st, Bp, nk, k, (const double *)nullptr, Y);
    rc = run_sweeps<T>(f, WCS_SOLVE_FULL, k, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_add_unscaled<T>, dim3(grid_for(nk)), dim3(256), 0, st, Y, nk, k, (const double *)nullptr, 0,
                       Xp);
    std::vector<double> h((size_t)2 * nsk);
    f->last_rel.assign((size_t)nsk, -1.0);
    rep->iterations = 0;
    rep->raw_residual = -1;
    rep->final_residual = -1;
    int status = WCS_ENOTCONV;
    for (int it = 0;; it++) {
        if (it == 0 && csr_ready) HIP_TRY(hipStreamWaitEvent(st, csr_ready, 0));
        if constexpr (sizeof(T) == 4) {
            if (from_y)
                launch_spmv_vec<float>(f, k, Y, it == 0 ? Bp : Rp, it == 0 ? nullptr : amax, Rp, st);
        }
        if (!from_y) {
            rc = launch_spmv(f, k, Xp, Bp, Rp, k, 1, st);
            if (rc) return rc;
        }
        HIP_TRY(hipGetLastError());
        double worst = 0;
        auto residual_norms = [&]() -> int {
            launch_colred(f, Rp, n, k, 0, true, vec + nsk, st);
            HIP_TRY(hipMemcpyAsync(h.data(), vec, sizeof(double) * 2 * nsk, hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            worst = 0;
            for (int c = 0; c < nsk; c++) {
                double bn = std::sqrt(h[c]), rn = std::sqrt(h[nsk + c]);
                double rel = bn > 0 ? rn / bn : rn;
                f->last_rel[c] = rel;
                if (!(rel <= worst)) worst = rel;   // NaN propagates as worst
            }
            return WCS_OK;
        };
        rc = residual_norms();
        if (rc) return rc;
        // an updated residual that passes the test by less than a factor 100
        // is formed once more from the iterate itself (R = Bp - C Xp, FP64
        // rows), so the drift of the updates cannot decide convergence
        if (from_y && worst <= tol && worst > 1e-2 * tol) {
            rc = launch_spmv(f, k, Xp, Bp, Rp, k, 1, st);
            if (rc) return rc;
            rc = residual_norms();
            if (rc) return rc;
        }
        if (it == 0) rep->raw_residual = worst;
        rep->final_residual = worst;
        if (worst <= tol) { status = WCS_OK; break; }
        if (it >= max_iter) break;
        launch_colred(f, Rp, n, k, 1, false, amax, st);
        hipLaunchKernelGGL(k_inv_scale, dim3(1), dim3(64 * ((k + 63) / 64)), 0, st, amax, k, scale);
        hipLaunchKernelGGL(k_cast_scaled<T>, dim3(grid_for(nk)), dim3(256), 0, st, Rp, nk, k,
                           (const double *)scale, Y);
        rc = run_sweeps<T>(f, WCS_SOLVE_FULL, k, st);
        if (rc) return rc;
        hipLaunchKernelGGL(k_add_unscaled<T>, dim3(grid_for(nk)), dim3(256), 0, st, Y, nk, k,
                           (const double *)scale, 1, Xp);
        rep->iterations = it + 1;
    }
    HIP_TRY(hipGetLastError());
    return status;
}

template <typename T>
int solve_refined(wcs_factor f, const double *values, int k, const double *B, double *X, int64_t ld, double tol,
                  int max_iter, wcs_ir_report *rep, hipStream_t st)
{
    const Layout &Lo = f->lay;
    // the matrix values for the residual are expanded on the third stream
    // while the first solve runs; the first residual waits for them
    hipStream_t aux = f->aux ? f->aux : st;
    if (aux != st) {
        HIP_TRY(hipEventRecord(f->ev_main, st));
        HIP_TRY(hipStreamWaitEvent(aux, f->ev_main, 0));
    }
    int rc = ensure_csr_values(f, values, aux, aux != st);
    if (rc) return rc;
    if (aux != st) HIP_TRY(hipEventRecord(f->ev_aux, aux));
    gather_rows(f, B, ld, k, f->at<double>(Lo.Br), st);
    int status = refine_pivot<T>(f, k, tol, max_iter, rep, st, aux != st ? f->ev_aux : nullptr);
    if (status != WCS_OK && status != WCS_ENOTCONV) return status;
    scatter_rows(f, f->at<double>(Lo.Xr), k, X, ld, st);
    HIP_TRY(hipGetLastError());
    if (status != WCS_OK)
        set_error("iterative refinement stopped at relative residual " + std::to_string(rep->final_residual));
    return status;
}

// Theta scheme (Section 5, eq:theta with G = I, L = -K): u_{i+1} = A^-1
// ((u_i - (1 - theta) A u_i) / theta + dt ((1 - theta) f_i + theta f_{i+1}))
// for the factored A = I + theta dt K, in pivot order throughout; an FP64
// factor solves each step directly, an FP32 factor refines each step to tol
// against A.  Column 0 of U is u_0; columns 1..nsteps are written.
template <typename T>
int theta_steps(wcs_factor f, const double *A_values, double theta, double dt, int nsteps, const double *F,
                int64_t ldf, double *U, int64_t ldu, double tol, wcs_ir_report *rep, hipStream_t st)
{
    const Layout &Lo = f->lay;
    int n = f->S->n;
    int rc = ensure_csr_values(f, A_values, st);
    if (rc) return rc;
    double *Bp = f->at<double>(Lo.Br), *Xp = f->at<double>(Lo.Xr), *AU = f->at<double>(Lo.Rr);
    const int32_t *perm = f->at<int32_t>(Lo.perm);
    T *Y = f->at<T>(Lo.Y);
    unsigned g = grid_for(n);
    hipLaunchKernelGGL(k_gather_rows, dim3(g), dim3(256), 0, st, U, ldu, perm, n, 1, Xp);
    rep->iterations = 0;
    rep->raw_residual = -1;
    rep->final_residual = -1;
    for (int i = 0; i < nsteps; i++) {
        rc = launch_spmv(f, 1, Xp, nullptr, AU, 1, 1, st);
        if (rc) return rc;
        hipLaunchKernelGGL(k_theta_rhs, dim3(g), dim3(256), 0, st, Xp, AU, F + (int64_t)i * ldf,
                           F + (int64_t)(i + 1) * ldf, perm, n, theta, dt, Bp);
        if constexpr (sizeof(T) == 8) {
            hipLaunchKernelGGL(k_cast_scaled<T>, dim3(g), dim3(256), 0, st, Bp, (int64_t)n, 1,
                               (const double *)nullptr, Y);
            rc = run_sweeps<T>(f, WCS_SOLVE_FULL, 1, st);
            if (rc) return rc;
            hipLaunchKernelGGL(k_add_unscaled<T>, dim3(g), dim3(256), 0, st, Y, (int64_t)n, 1,
                               (const double *)nullptr, 0, Xp);
        } else {
            wcs_ir_report r;
            rc = refine_pivot<T>(f, 1, tol, 10, &r, st);
            rep->iterations = std::max(rep->iterations, r.iterations);
            rep->raw_residual = std::max(rep->raw_residual, r.raw_residual);
            rep->final_residual = std::max(rep->final_residual, r.final_residual);
            if (rc == WCS_ENOTCONV) {
                set_error("theta scheme: refinement of step " + std::to_string(i + 1) + " stopped at relative residual " +
                          std::to_string(r.final_residual));
                return rc;
            }
            if (rc) return rc;
        }
        hipLaunchKernelGGL(k_scatter_rows, dim3(g), dim3(256), 0, st, Xp, perm, n, 1, U + (int64_t)(i + 1) * ldu, ldu);
    }
    HIP_TRY(hipGetLastError());
    return WCS_OK;
}

template <typename V>
int upload(wcs_factor f, size_t off, const std::vector<V> &v, hipStream_t st)
{
    if (v.empty()) return WCS_OK;
    HIP_TRY(hipMemcpyAsync(f->ws + off, v.data(), v.size() * sizeof(V), hipMemcpyHostToDevice, st));
    return WCS_OK;
}

}  // namespace
}  // namespace wcs

using namespace wcs;

extern "C" {

int wcs_workspace_size(wcs_symbolic sym, wcs_precision prec, int32_t max_nrhs, size_t *bytes)
{
    if (!sym || !bytes || max_nrhs < 1 || !valid_prec(prec)) {
        set_error("invalid argument to wcs_workspace_size");
        return WCS_EINVAL;
    }
    try {
        Plan P;
        P.build(symbolic_of(sym), elem_size(prec), prec != WCS_LU64 && leaf_kernel_enabled(), prec != WCS_LU64);
        Layout L;
        L.compute(symbolic_of(sym), P, elem_size(prec), max_nrhs, is_lu(prec));
        *bytes = L.total;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return WCS_ENOMEM;
    }
    return WCS_OK;
}

}  // extern "C"

namespace wcs {
namespace {
// Plan and layout of a new factor (host only).
int new_factor(wcs_symbolic sym, wcs_precision prec, int32_t max_nrhs, wcs_factor *fp)
{
    wcs_factor f = new (std::nothrow) wcs_factor_s;
    if (!f) return WCS_ENOMEM;
    try {
        f->S = &symbolic_of(sym);
        f->prec = prec;
        f->max_nrhs = max_nrhs;
        f->plan.build(*f->S, elem_size(prec), prec != WCS_LU64 && leaf_kernel_enabled(), prec != WCS_LU64);
        for (Level &L : f->plan.levels) L.upd_var = default_update_variant(prec);
        f->lay.compute(*f->S, f->plan, elem_size(prec), max_nrhs, is_lu(prec));
    } catch (const std::bad_alloc &) {
        delete f;
        set_error("host allocation failed");
        return WCS_ENOMEM;
    }
    *fp = f;
    return WCS_OK;
}

// Copies the static plan tables into the factor's workspace (stream order,
// then waits: the host vectors are pageable).  Deletes f on failure.
int upload_plan(wcs_factor f, hipStream_t st, wcs_factor *out);
}  // namespace
}  // namespace wcs

extern "C" {

int wcs_factor_create(wcs_symbolic sym, wcs_precision prec, int32_t max_nrhs, void *workspace, size_t bytes,
                      wcs_stream stream, wcs_factor *out)
{
    if (!sym || !out || max_nrhs < 1 || !valid_prec(prec) || !workspace) {
        set_error("invalid argument to wcs_factor_create");
        return WCS_EINVAL;
    }
    if (((uintptr_t)workspace) % 256) {
        set_error("workspace must be 256-byte aligned");
        return WCS_EINVAL;
    }
    *out = nullptr;
    wcs_factor f = nullptr;
    int rc = new_factor(sym, prec, max_nrhs, &f);
    if (rc) return rc;
    if (bytes < f->lay.total) {
        set_error("workspace too small: need " + std::to_string(f->lay.total) + " bytes, got " + std::to_string(bytes));
        delete f;
        return WCS_ENOMEM;
    }
    f->ws = (char *)workspace;
    f->bytes = bytes;
    if (hipStreamCreateWithFlags(&f->side, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&f->aux, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&f->ev_main, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&f->ev_side, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&f->ev_aux, hipEventDisableTiming) != hipSuccess) {
        set_error("could not create the look-ahead stream or its events");
        delete f;
        return WCS_EHIP;
    }
    return upload_plan(f, (hipStream_t)stream, out);
}

int wcs_factor_create_static(wcs_symbolic sym, wcs_precision prec, int32_t max_nrhs, wcs_stream stream,
                             wcs_factor *out)
{
    if (!sym || !out || max_nrhs < 1 || !valid_prec(prec)) {
        set_error("invalid argument to wcs_factor_create_static");
        return WCS_EINVAL;
    }
    *out = nullptr;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    wcs_factor f = nullptr;
    int rc = new_factor(sym, prec, max_nrhs, &f);
    if (rc) return rc;
    if (f->lay.total > (size_t)WCS_STATIC_WORKSPACE_BYTES) {
        set_error("static workspace too small: this system needs " + std::to_string(f->lay.total) +
                  " bytes, the static workspace holds " + std::to_string((size_t)WCS_STATIC_WORKSPACE_BYTES));
        delete f;
        return WCS_ENOMEM;
    }
    {
        std::lock_guard<std::mutex> lk(g_static_mu);
        if (g_static.size() <= (size_t)dev) g_static.resize((size_t)dev + 1);
        StaticSlot &slot = g_static[(size_t)dev];
        if (!slot.ptr) {   // first use on this device (it is current): the array's device address
            void *p = nullptr;
            hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p) {
                set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
                delete f;
                return WCS_EHIP;
            }
            slot.ptr = (char *)p;
        }
        if (slot.in_use) {
            set_error("the static workspace of device " + std::to_string(dev) + " is held by another factor");
            delete f;
            return WCS_ESTATE;
        }
        slot.in_use = true;
        f->ws = slot.ptr;
        f->static_device = dev;
    }
    f->bytes = (size_t)WCS_STATIC_WORKSPACE_BYTES;
    // no look-ahead or auxiliary stream: every launch goes to the caller's stream
    return upload_plan(f, (hipStream_t)stream, out);
}

}  // extern "C"

namespace wcs {
namespace {
int upload_plan(wcs_factor f, hipStream_t st, wcs_factor *out)
{
    {
        int dev = 0, ncu = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
            f->ncu = ncu;
    }
    const Symbolic &S = *f->S;
    const Plan &P = f->plan;
    const Layout &L = f->lay;
    int rc = WCS_OK;
    rc = rc ? rc : upload(f, L.front_off, S.front_off, st);
    rc = rc ? rc : upload(f, L.mfront, P.mfront, st);
    rc = rc ? rc : upload(f, L.pfront, P.pfront, st);
    rc = rc ? rc : upload(f, L.first, P.first, st);
    rc = rc ? rc : upload(f, L.sparent, S.sparent, st);
    rc = rc ? rc : upload(f, L.rptr, S.rptr, st);
    rc = rc ? rc : upload(f, L.rows, S.rows, st);
    rc = rc ? rc : upload(f, L.rel, S.rel, st);
    rc = rc ? rc : upload(f, L.amap, S.amap, st);
    rc = rc ? rc : upload(f, L.woff, P.woff, st);
    rc = rc ? rc : upload(f, L.child_ptr, P.child_ptr, st);
    rc = rc ? rc : upload(f, L.child_list, P.child_list, st);
    rc = rc ? rc : upload(f, L.easplit, P.ea_split, st);
    rc = rc ? rc : upload(f, L.perm, S.perm, st);
    rc = rc ? rc : upload(f, L.csr_ptr, S.csr_ptr, st);
    rc = rc ? rc : upload(f, L.csr_col, S.csr_col, st);
    rc = rc ? rc : upload(f, L.csr_src, S.csr_src, st);
    rc = rc ? rc : upload(f, L.spchunk, f->plan.spmv_chunks, st);
    rc = rc ? rc : upload(f, L.splong, f->plan.spmv_long, st);
    rc = rc ? rc : upload(f, L.spgrp, f->plan.spmv_grp, st);
    rc = rc ? rc : upload(f, L.spgit, f->plan.spmv_gitems, st);
    rc = rc ? rc : upload(f, L.spglong, f->plan.spmv_glong, st);
    rc = rc ? rc : upload(f, L.iperm, S.iperm, st);
    rc = rc ? rc : upload(f, L.rowind, S.rowind, st);
    rc = rc ? rc : upload(f, L.colof, P.colof, st);
    rc = rc ? rc : upload(f, L.pan, P.pan_tasks, st);
    {
        std::vector<UpdTask> ud(P.upd_tasks.size());
        for (size_t q = 0; q < ud.size(); q++) {
            int4 t = P.upd_tasks[q];
            int64_t o = S.front_off[t.x];
            ud[q].a = make_int4((int32_t)(uint32_t)(uint64_t)o, (int32_t)((uint64_t)o >> 32), P.mfront[t.x],
                                P.pfront[t.x]);
            ud[q].b = make_int4(t.y, t.z, t.w, P.upd_jbeg[q]);
        }
        rc = rc ? rc : upload(f, L.upd, ud, st);
    }
    rc = rc ? rc : upload(f, L.ea, P.ea_tasks, st);
    rc = rc ? rc : upload(f, L.flist, P.flist, st);
    rc = rc ? rc : upload(f, L.dscr_off, P.dscr_off, st);
    rc = rc ? rc : upload(f, L.slist, P.slist, st);
    rc = rc ? rc : upload(f, L.sfwd, P.sfwd_tasks, st);
    rc = rc ? rc : upload(f, L.sbelow, P.sbelow_tasks, st);
    rc = rc ? rc : upload(f, L.sbwd, P.sbwd_tasks, st);
    rc = rc ? rc : upload(f, L.sblk, P.sblk_tasks, st);
    rc = rc ? rc : upload(f, L.sbsum, P.sbsum_tasks, st);
    rc = rc ? rc : upload(f, L.xinvt, P.xinv_tasks, st);
    rc = rc ? rc : upload(f, L.dinvt, P.dinv_tasks, st);
    rc = rc ? rc : upload(f, L.altt, P.alt_tasks, st);
    rc = rc ? rc : upload(f, L.alt2, P.al_tasks, st);
    rc = rc ? rc : upload(f, L.gptr, P.gptr, st);
    rc = rc ? rc : upload(f, L.glist, P.glist, st);
    rc = rc ? rc : upload(f, L.xoff, P.xoff, st);
    rc = rc ? rc : upload(f, L.sasm, P.sasm_tasks, st);
    rc = rc ? rc : upload(f, L.ztasks, P.zero_tasks, st);
    rc = rc ? rc : upload(f, L.leafq, P.leaf_queue, st);
    rc = rc ? rc : upload(f, L.diagf, P.diag_fronts, st);
    rc = rc ? rc : upload(f, L.stept, P.step_tasks, st);
    std::vector<int32_t> segp = S.seg_ptr.size() >= 2 ? S.seg_ptr : std::vector<int32_t>{0, S.n};
    rc = rc ? rc : upload(f, L.segp, segp, st);
    if (rc == WCS_OK) {
        hipError_t e = hipStreamSynchronize(st);   // host vectors are pageable: finish the copies
        if (e != hipSuccess) {
            set_error(std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
            rc = WCS_EHIP;
        }
    }
    if (rc) { delete f; return rc; }
    *out = f;
    return WCS_OK;
}
}  // namespace
}  // namespace wcs

extern "C" {

int wcs_factor_numeric(wcs_factor f, const double *values_dev, wcs_stream stream, int32_t *bad_col)
{
    if (!f || !values_dev) { set_error("invalid argument to wcs_factor_numeric"); return WCS_EINVAL; }
    if (is_lu(f->prec)) { set_error("an LU factor takes both triangles: wcs_factor_numeric_lu"); return WCS_EINVAL; }
    hipStream_t st = (hipStream_t)stream;
    int rc;
    auto eager = [&] {
        return f->prec == WCS_FP64 ? launch_factor<double>(f, values_dev, st, nullptr)
                                   : launch_factor<float>(f, values_dev, st, nullptr);
    };
    if (f->graphs && st != nullptr) {
        if (f->fgraph && f->fgraph_values != values_dev) {
            (void)hipGraphExecDestroy(f->fgraph);
            f->fgraph = nullptr;
        }
        if (!f->fgraph) {
            rc = record(st, &f->fgraph, eager);
            if (rc) { f->fgraph = nullptr; return rc; }
            f->fgraph_values = values_dev;
        }
        HIP_TRY(hipGraphLaunch(f->fgraph, st));
        rc = WCS_OK;
    } else {
        rc = eager();
    }
    if (rc) return rc;
    f->have_values = true;
    if (bad_col) return wcs_factor_check(f, stream, bad_col);
    return WCS_OK;
}

int wcs_factor_numeric_lu(wcs_factor f, const double *lower_dev, const double *upper_dev, wcs_stream stream,
                          int32_t *bad_col)
{
    if (!f || !lower_dev || !upper_dev) { set_error("invalid argument to wcs_factor_numeric_lu"); return WCS_EINVAL; }
    if (!is_lu(f->prec)) { set_error("wcs_factor_numeric_lu needs a factor created with WCS_LU64"); return WCS_EINVAL; }
    int rc = launch_factor<double>(f, lower_dev, (hipStream_t)stream, nullptr, upper_dev);
    if (rc) return rc;
    f->have_values = true;
    if (bad_col) return wcs_factor_check(f, stream, bad_col);
    return WCS_OK;
}

int wcs_factor_profile(wcs_factor f, const double *values_dev, wcs_stream stream, wcs_kernel_stat *stats)
{
    if (f && is_lu(f->prec)) { set_error("wcs_factor_profile is not defined for an LU factor"); return WCS_EINVAL; }
    if (!f || !values_dev || !stats) { set_error("invalid argument to wcs_factor_profile"); return WCS_EINVAL; }
    hipStream_t st = (hipStream_t)stream;
    Prof prof;
    prof.st = st;
    int rc = f->prec == WCS_FP64 ? launch_factor<double>(f, values_dev, st, &prof)
                                 : launch_factor<float>(f, values_dev, st, &prof);
    if (rc) return rc;
    f->have_values = true;
    return prof.collect(stats);
}

int wcs_factor_check(wcs_factor f, wcs_stream stream, int32_t *bad_col)
{
    if (!f || !bad_col) { set_error("invalid argument to wcs_factor_check"); return WCS_EINVAL; }
    if (!f->have_values) { set_error("no numeric factorization yet"); return WCS_ESTATE; }
    int32_t h = INT32_MAX;
    HIP_TRY(hipMemcpyAsync(&h, f->ws + f->lay.bad, sizeof(int32_t), hipMemcpyDeviceToHost, (hipStream_t)stream));
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    if (h != INT32_MAX) {
        *bad_col = h;
        if (is_lu(f->prec)) {
            set_error("zero or non-finite pivot in the LU factorization: pivot " + std::to_string(h) +
                      " (original index " + std::to_string(f->S->perm[h]) + ")");
            return WCS_ESINGULAR;
        }
        set_error("matrix is not positive definite: pivot " + std::to_string(h) + " (original index " +
                  std::to_string(f->S->perm[h]) + ")");
        return WCS_ENOTSPD;
    }
    *bad_col = -1;
    return WCS_OK;
}

int wcs_factor_profile_levels(wcs_factor f, const double *values_dev, wcs_stream stream, wcs_kernel_stat *levels)
{
    if (f && is_lu(f->prec)) { set_error("wcs_factor_profile_levels is not defined for an LU factor"); return WCS_EINVAL; }
    if (!f || !values_dev || !levels) { set_error("invalid argument to wcs_factor_profile_levels"); return WCS_EINVAL; }
    hipStream_t st = (hipStream_t)stream;
    Prof prof;
    prof.st = st;
    prof.levels = true;
    int rc = f->prec == WCS_FP64 ? launch_factor<double>(f, values_dev, st, &prof)
                                 : launch_factor<float>(f, values_dev, st, &prof);
    if (rc) return rc;
    f->have_values = true;
    return prof.collect_levels(levels);
}

void wcs_factor_free(wcs_factor f) { delete f; }

int wcs_factor_autotune(wcs_factor f, const double *values_dev, wcs_stream stream, int32_t *tiles, double *ms)
{
    if (f && is_lu(f->prec)) { set_error("wcs_factor_autotune is not defined for an LU factor"); return WCS_EINVAL; }
    if (!f || !values_dev) { set_error("invalid argument to wcs_factor_autotune"); return WCS_EINVAL; }
    hipStream_t st = (hipStream_t)stream;
    Plan &P = f->plan;
    size_t H = P.levels.size();
    auto timed = [&](std::vector<double> &lev_ms) -> int {
        std::vector<wcs_kernel_stat> out(H);
        Prof prof;
        prof.st = st;
        prof.levels = true;
        int rc = f->prec == WCS_FP64 ? launch_factor<double>(f, values_dev, st, &prof)
                                     : launch_factor<float>(f, values_dev, st, &prof);
        if (rc) return rc;
        rc = prof.collect_levels(out.data());
        if (rc) return rc;
        lev_ms.resize(H);
        for (size_t h = 0; h < H; h++) lev_ms[h] = out[h].ms;
        return WCS_OK;
    };
    // each candidate kernel on every level: a warm-up factorization, then a timed one
    constexpr int NV = 5;
    std::vector<double> t[NV];
    const int32_t dflt = default_update_variant(f->prec);
    for (int v = 0; v < NV; v++) {
        for (Level &L : P.levels) L.upd_var = v;
        std::vector<double> warm;
        int rc = timed(warm);
        if (!rc) rc = timed(t[v]);
        if (rc) {
            for (Level &L : P.levels) L.upd_var = dflt;
            return rc;
        }
    }
    double before = 0, after = 0;
    for (size_t h = 0; h < H; h++) {
        int best = dflt;
        for (int v = 0; v < NV; v++)
            if (t[v][h] < t[best][h]) best = v;
        P.levels[h].upd_var = best;
        before += t[dflt][h];
        after += t[best][h];
        if (tiles) tiles[h] = best;
    }
    if (ms) {
        ms[0] = before;
        ms[1] = after;
    }
    if (f->fgraph) {   // recorded launches used the old tiles
        (void)hipGraphExecDestroy(f->fgraph);
        f->fgraph = nullptr;
        f->fgraph_values = nullptr;
    }
    f->have_values = true;
    return WCS_OK;
}

int wcs_factor_set_tiles(wcs_factor f, const int32_t *tiles)
{
    if (!f || !tiles) { set_error("invalid argument to wcs_factor_set_tiles"); return WCS_EINVAL; }
    for (size_t h = 0; h < f->plan.levels.size(); h++)
        if (tiles[h] < WCS_UPD_REG128 || tiles[h] > WCS_UPD_STREAM128_K32) {
            set_error("update kernel variant must be WCS_UPD_REG128, WCS_UPD_REG64, WCS_UPD_STREAM128, "
                      "WCS_UPD_STREAM128_3 or WCS_UPD_STREAM128_K32");
            return WCS_EINVAL;
        }
    for (size_t h = 0; h < f->plan.levels.size(); h++) f->plan.levels[h].upd_var = tiles[h];
    if (f->fgraph) {
        (void)hipGraphExecDestroy(f->fgraph);
        f->fgraph = nullptr;
        f->fgraph_values = nullptr;
    }
    return WCS_OK;
}

int wcs_factor_use_graphs(wcs_factor f, int enable)
{
    if (!f) { set_error("null factor"); return WCS_EINVAL; }
    if (!enable) f->drop_graphs();
    f->graphs = enable != 0;
    return WCS_OK;
}

int wcs_factor_residuals(wcs_factor f, double *rel, int64_t count)
{
    if (!f || !rel || count < 0) { set_error("invalid argument to wcs_factor_residuals"); return WCS_EINVAL; }
    if (f->last_rel.empty()) { set_error("no refinement has run on this factor"); return WCS_ESTATE; }
    if (count < (int64_t)f->last_rel.size()) {
        set_error("residual buffer too small: need " + std::to_string(f->last_rel.size()));
        return WCS_EINVAL;
    }
    std::copy(f->last_rel.begin(), f->last_rel.end(), rel);
    return WCS_OK;
}

namespace wcs {
namespace {
// columns [j0, j1) of the L fronts (upper = false) or of the U^T fronts of an LU factor
int export_columns(wcs_factor f, int32_t j0, int32_t j1, int64_t *Lp, int32_t *Li, double *Lx, wcs_stream stream,
                   bool upper);
}  // namespace
}  // namespace wcs

int wcs_factor_export(wcs_factor f, int32_t j0, int32_t j1, int64_t *Lp, int32_t *Li, double *Lx, wcs_stream stream)
{
    return export_columns(f, j0, j1, Lp, Li, Lx, stream, false);
}

int wcs_factor_export_upper(wcs_factor f, int32_t j0, int32_t j1, int64_t *Up, int32_t *Ui, double *Ux,
                            wcs_stream stream)
{
    if (f && !is_lu(f->prec)) { set_error("wcs_factor_export_upper needs an LU factor"); return WCS_EINVAL; }
    return export_columns(f, j0, j1, Up, Ui, Ux, stream, true);
}

}  // extern "C"

namespace wcs {
namespace {
int export_columns(wcs_factor f, int32_t j0, int32_t j1, int64_t *Lp, int32_t *Li, double *Lx, wcs_stream stream,
                   bool upper)
{
    if (!f || !Lp || j0 < 0 || j1 < j0 || j1 > f->S->n || ((Li == nullptr) != (Lx == nullptr))) {
        set_error("invalid argument to wcs_factor_export");
        return WCS_EINVAL;
    }
    const Symbolic &S = *f->S;
    Lp[0] = 0;
    for (int32_t j = j0; j < j1; j++) {
        int32_t s = S.snode_of[j];
        Lp[j - j0 + 1] = Lp[j - j0] + (S.m_of(s) - (j - S.sptr[s]));
    }
    if (!Li) return WCS_OK;
    if (!f->have_values) { set_error("no numeric factorization yet"); return WCS_ESTATE; }
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(hipStreamSynchronize(st));
    size_t esz = elem_size(f->prec);
    std::vector<char> buf;
    for (int32_t j = j0; j < j1; j++) {
        int32_t s = S.snode_of[j];
        int32_t m = S.m_of(s), t = j - S.sptr[s];
        int32_t cnt = m - t;
        buf.resize((size_t)cnt * esz);
        size_t off = (upper ? f->lay.fronts_u : f->lay.fronts) +
                     ((size_t)S.front_off[s] + (size_t)t * front_ld_host(m) + t) * esz;
        HIP_TRY(hipMemcpy(buf.data(), f->ws + off, (size_t)cnt * esz, hipMemcpyDeviceToHost));
        int64_t o = Lp[j - j0];
        for (int32_t r = 0; r < cnt; r++) {
            Li[o + r] = S.rows[S.rptr[s] + t + r];
            Lx[o + r] = esz == 8 ? ((const double *)buf.data())[r] : (double)((const float *)buf.data())[r];
        }
    }
    return WCS_OK;
}
}  // namespace
}  // namespace wcs

extern "C" {

int wcs_solve(wcs_factor f, wcs_part part, int32_t nrhs, double *B_dev, int64_t ld, wcs_stream stream)
{
    if (!f || !B_dev || nrhs < 1 || nrhs > f->max_nrhs || ld < f->S->n || part < 0 || part > 2) {
        set_error("invalid argument to wcs_solve");
        return WCS_EINVAL;
    }
    if (!f->have_values) { set_error("no numeric factorization yet"); return WCS_ESTATE; }
    hipStream_t st = (hipStream_t)stream;
    return f->prec == WCS_FP32 ? launch_solve<float>(f, part, nrhs, B_dev, ld, st)
                               : launch_solve<double>(f, part, nrhs, B_dev, ld, st);
}

int wcs_apply(wcs_factor f, wcs_apply_part part, int32_t nrhs, double *B_dev, int64_t ld, wcs_stream stream)
{
    if (f && is_lu(f->prec)) { set_error("wcs_apply is not defined for an LU factor"); return WCS_EINVAL; }
    if (!f || !B_dev || nrhs < 1 || nrhs > f->max_nrhs || ld < f->S->n ||
        (part != WCS_APPLY_L && part != WCS_APPLY_LT)) {
        set_error("invalid argument to wcs_apply");
        return WCS_EINVAL;
    }
    if (!f->have_values) { set_error("no numeric factorization yet"); return WCS_ESTATE; }
    hipStream_t st = (hipStream_t)stream;
    return f->prec == WCS_FP64 ? launch_apply<double>(f, part, nrhs, B_dev, ld, st)
                               : launch_apply<float>(f, part, nrhs, B_dev, ld, st);
}

int wcs_solve_refined(wcs_factor f, const double *values_dev, int32_t nrhs, const double *B_dev, double *X_dev,
                      int64_t ld, double tol, int32_t max_iter, wcs_ir_report *rep, wcs_stream stream)
{
    if (f && is_lu(f->prec)) { set_error("wcs_solve_refined is not defined for an LU factor"); return WCS_EINVAL; }
    if (!f || !values_dev || !B_dev || !X_dev || !rep || nrhs < 1 || nrhs > f->max_nrhs || ld < f->S->n ||
        max_iter < 0 || !(tol >= 0)) {
        set_error("invalid argument to wcs_solve_refined");
        return WCS_EINVAL;
    }
    if (!f->have_values) { set_error("no numeric factorization yet"); return WCS_ESTATE; }
    hipStream_t st = (hipStream_t)stream;
    return f->prec == WCS_FP64
               ? solve_refined<double>(f, values_dev, nrhs, B_dev, X_dev, ld, tol, max_iter, rep, st)
               : solve_refined<float>(f, values_dev, nrhs, B_dev, X_dev, ld, tol, max_iter, rep, st);
}

int wcs_spmv(wcs_factor f, const double *values_dev, int32_t nrhs, const double *X_dev, double *Y_dev, int64_t ld,
             wcs_stream stream)
{
    if (f && is_lu(f->prec)) { set_error("wcs_spmv is not defined for an LU factor"); return WCS_EINVAL; }
    if (!f || !values_dev || !X_dev || !Y_dev || nrhs < 1 || ld < f->S->n) {
        set_error("invalid argument to wcs_spmv");
        return WCS_EINVAL;
    }
    if (nrhs > f->max_nrhs) { set_error("wcs_spmv: nrhs exceeds the factor's max_nrhs"); return WCS_EINVAL; }
    hipStream_t st = (hipStream_t)stream;
    int rc = ensure_csr_values(f, values_dev, st);
    if (rc) return rc;
    double *Xp = f->at<double>(f->lay.Xr), *Yp = f->at<double>(f->lay.Rr);
    gather_rows(f, X_dev, ld, nrhs, Xp, st);
    rc = launch_spmv(f, nrhs, Xp, nullptr, Yp, nrhs, 1, st);
    if (rc) return rc;
    scatter_rows(f, Yp, nrhs, Y_dev, ld, st);
    HIP_TRY(hipGetLastError());
    return WCS_OK;
}

int wcs_theta_matrix(wcs_factor f, const double *K_values_dev, double theta, double dt, double *A_values_dev,
                     wcs_stream stream)
{
    if (f && is_lu(f->prec)) { set_error("wcs_theta_matrix is not defined for an LU factor"); return WCS_EINVAL; }
    if (!f || !K_values_dev || !A_values_dev || !(theta > 0 && theta <= 1) || !(dt > 0)) {
        set_error("invalid argument to wcs_theta_matrix");
        return WCS_EINVAL;
    }
    const Symbolic &S = *f->S;
    hipLaunchKernelGGL(k_theta_matrix, dim3(grid_for(S.nnz)), dim3(256), 0, (hipStream_t)stream,
                       f->at<int32_t>(f->lay.rowind), f->at<int32_t>(f->lay.colof), S.nnz, K_values_dev, theta * dt,
                       A_values_dev);
    HIP_TRY(hipGetLastError());
    return WCS_OK;
}

int wcs_theta_steps(wcs_factor f, const double *A_values_dev, double theta, double dt, int32_t nsteps,
                    const double *F_dev, int64_t ldf, double *U_dev, int64_t ldu, double tol, wcs_ir_report *rep,
                    wcs_stream stream)
{
    if (f && is_lu(f->prec)) { set_error("wcs_theta_steps is not defined for an LU factor"); return WCS_EINVAL; }
    if (!f || !A_values_dev || !F_dev || !U_dev || !rep || nsteps < 1 || !(theta > 0 && theta <= 1) || !(dt > 0) ||
        ldf < f->S->n || ldu < f->S->n || !(tol >= 0)) {
        set_error("invalid argument to wcs_theta_steps");
        return WCS_EINVAL;
    }
    if (!f->have_values) { set_error("no numeric factorization yet"); return WCS_ESTATE; }
    hipStream_t st = (hipStream_t)stream;
    return f->prec == WCS_FP64
               ? theta_steps<double>(f, A_values_dev, theta, dt, nsteps, F_dev, ldf, U_dev, ldu, tol, rep, st)
               : theta_steps<float>(f, A_values_dev, theta, dt, nsteps, F_dev, ldf, U_dev, ldu, tol, rep, st);
}

int wcs_field_sample(wcs_factor cov, wcs_factor mass, int32_t nrhs, const double *abar_dev, int64_t lda,
                     const double *X_dev, int64_t ldx, double *out_dev, int64_t ld, wcs_stream stream)
{
    if (!cov || !mass || !X_dev || !out_dev || nrhs < 1 || is_lu(cov->prec) || is_lu(mass->prec) ||
        cov->S->n != mass->S->n || nrhs > cov->max_nrhs || nrhs > mass->max_nrhs || lda < 0 ||
        (lda > 0 && lda < cov->S->n) || ldx < cov->S->n || ld < cov->S->n) {
        set_error("invalid argument to wcs_field_sample");
        return WCS_EINVAL;
    }
    if (!cov->have_values || !mass->have_values) { set_error("no numeric factorization yet"); return WCS_ESTATE; }
    hipStream_t st = (hipStream_t)stream;
    const int n = cov->S->n;
    if (X_dev != out_dev || ldx != ld)
        HIP_TRY(hipMemcpy2DAsync(out_dev, (size_t)ld * 8, X_dev, (size_t)ldx * 8, (size_t)n * 8, (size_t)nrhs,
                                 hipMemcpyDeviceToDevice, st));
    // P_C^T L_C X with the noise in the covariance factor's pivot order
    int rc = cov->prec == WCS_FP32 ? launch_apply<float>(cov, WCS_APPLY_L, nrhs, out_dev, ld, st)
                                   : launch_apply<double>(cov, WCS_APPLY_L, nrhs, out_dev, ld, st);
    if (rc) return rc;
    if (abar_dev)
        hipLaunchKernelGGL(k_add_cols, dim3(grid_for((int64_t)n * nrhs)), dim3(256), 0, st, out_dev, ld, n, nrhs,
                           abar_dev, lda);
    // G^-1 (abar + L X) with the mass matrix's own factor
    rc = mass->prec == WCS_FP32 ? launch_solve<float>(mass, WCS_SOLVE_FULL, nrhs, out_dev, ld, st)
                                : launch_solve<double>(mass, WCS_SOLVE_FULL, nrhs, out_dev, ld, st);
    if (rc) return rc;
    HIP_TRY(hipGetLastError());
    return WCS_OK;
}

int wcs_grad_pattern(wcs_factor f, const double *lam_dev, const double *x_dev, double *gA_dev, wcs_stream stream)
{
    if (f && is_lu(f->prec)) { set_error("wcs_grad_pattern is not defined for an LU factor"); return WCS_EINVAL; }
    if (!f || !lam_dev || !x_dev || !gA_dev) { set_error("invalid argument to wcs_grad_pattern"); return WCS_EINVAL; }
    const Symbolic &S = *f->S;
    hipLaunchKernelGGL(k_grad_pattern, dim3(grid_for(S.nnz)), dim3(256), 0, (hipStream_t)stream,
                       f->at<int32_t>(f->lay.rowind), f->at<int32_t>(f->lay.colof), S.nnz, lam_dev, x_dev, gA_dev);
    HIP_TRY(hipGetLastError());
    return WCS_OK;
}

}  // extern "C"
