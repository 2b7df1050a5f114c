// Host-side ordering and symbolic analysis.
//
// Nested dissection (Section 4): the vertex set of the adjacency graph
// G = (V, E) of the symmetric pattern is split as V = V1 u V2 u S with no edge
// between V1 and V2, ordered V1, V2, S, recursively.  Each split here is
// chosen by a balanced partition of the vertices (by coordinate median when
// positions are supplied, by breadth-first level structure otherwise); S is
// then a minimum vertex cover of the edges that cross that partition
// (Koenig's theorem via Hopcroft-Karp matching), so the block structure holds
// for the graph itself whatever the positions are.  Vertices of very high
// degree (the coarsest wavelet levels touch nearly every other basis
// function) are moved into the root separator before dissecting.
//
// Symbolic factorization of P A P^T (the pattern of Lemma 4.1): elimination
// tree, postorder, column counts by the skeleton-graph / least-common-ancestor
// method, fundamental supernodes, relaxed amalgamation, supernode row
// structures, the assembly tree and its level schedule, extend-add index maps
// and the map of every stored entry of A into the front buffers.
//
// Everything is deterministic: no hashing, no thread-order dependence, every
// sort has a total order.

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <numeric>
#include <queue>
#include <string>
#include <thread>

#include "internal.h"

namespace wcs {

namespace {

struct Graph {
    int32_t n = 0;
    std::vector<int64_t> xadj;
    std::vector<int32_t> adj;
};

int validate(int32_t n, const int64_t *colptr, const int32_t *rowind)
{
    if (n < 0) { set_error("n < 0"); return WCS_EINVAL; }
    if (!colptr || (n > 0 && !rowind)) { set_error("null pattern array"); return WCS_EINVAL; }
    if (colptr[0] != 0) { set_error("colptr[0] != 0"); return WCS_EINVAL; }
    for (int32_t j = 0; j < n; j++) {
        int64_t a = colptr[j], b = colptr[j + 1];
        if (b <= a) { set_error("column " + std::to_string(j) + " is empty (diagonal missing)"); return WCS_EINVAL; }
        if (rowind[a] != j) { set_error("column " + std::to_string(j) + " does not start with its diagonal"); return WCS_EINVAL; }
        for (int64_t p = a + 1; p < b; p++) {
            int32_t r = rowind[p];
            if (r <= rowind[p - 1] || r >= n) {
                set_error("column " + std::to_string(j) + ": rows not strictly ascending or out of range");
                return WCS_EINVAL;
            }
        }
    }
    return WCS_OK;
}

Graph build_graph(int32_t n, const int64_t *colptr, const int32_t *rowind)
{
    Graph g;
    g.n = n;
    g.xadj.assign((size_t)n + 1, 0);
    for (int32_t j = 0; j < n; j++)
        for (int64_t p = colptr[j] + 1; p < colptr[j + 1]; p++) {
            g.xadj[rowind[p] + 1]++;
            g.xadj[j + 1]++;
        }
    for (int32_t v = 0; v < n; v++) g.xadj[v + 1] += g.xadj[v];
    g.adj.resize((size_t)g.xadj[n]);
    std::vector<int64_t> fill(g.xadj.begin(), g.xadj.end() - 1);
    // columns ascending, rows ascending: each list comes out sorted
    for (int32_t j = 0; j < n; j++)
        for (int64_t p = colptr[j] + 1; p < colptr[j + 1]; p++) {
            int32_t i = rowind[p];
            g.adj[fill[i]++] = j;
        }
    for (int32_t j = 0; j < n; j++)
        for (int64_t p = colptr[j] + 1; p < colptr[j + 1]; p++) g.adj[fill[j]++] = rowind[p];
    for (int32_t v = 0; v < n; v++) std::sort(g.adj.begin() + g.xadj[v], g.adj.begin() + g.xadj[v + 1]);
    return g;
}

// ---------------------------------------------------------------------------
// nested dissection

class Dissection {
public:
    Dissection(const Graph &g, const double *coords, int dim, int leaf)
        : g_(g), coords_(coords), dim_(dim), leaf_(leaf < 1 ? 1 : leaf)
    {
        int32_t n = g.n;
        perm_.assign(n, -1);
        stamp_.assign(n, -1);
        side_.assign(n, 0);
        lid_.assign(n, -1);
        rid_.assign(n, -1);
        bfs_level_.assign(n, -1);
    }

    // orders the vertices of V into perm[lo : lo + |V|); returns the node index
    int32_t dissect(std::vector<int32_t> &V, int32_t lo)
    {
        int32_t idx = (int32_t)(tree_.size() / 6);
        tree_.resize(tree_.size() + 6);
        int32_t nv = (int32_t)V.size();
        if (nv <= leaf_) return make_leaf(idx, V, lo);
        int32_t st = next_stamp_++;
        for (int32_t v : V) stamp_[v] = st;
        split(V, st);
        std::vector<int32_t> S = cover(V, st);
        if ((int32_t)S.size() == nv) return make_leaf(idx, V, lo);
        for (int32_t v : S) side_[v] = 2;
        std::vector<int32_t> V1, V2;
        for (int32_t v : V) {
            if (side_[v] == 0) V1.push_back(v);
            else if (side_[v] == 1) V2.push_back(v);
        }
        std::sort(S.begin(), S.end());
        std::vector<int32_t>().swap(V);
        int32_t n1 = (int32_t)V1.size(), n2 = (int32_t)V2.size();
        int32_t c1 = n1 ? dissect(V1, lo) : -1;
        int32_t c2 = n2 ? dissect(V2, lo + n1) : -1;
        int32_t sep = lo + n1 + n2;
        for (size_t t = 0; t < S.size(); t++) perm_[sep + t] = S[t];
        int32_t *nd = &tree_[6 * (size_t)idx];
        nd[0] = lo; nd[1] = lo + n1; nd[2] = sep; nd[3] = sep + (int32_t)S.size(); nd[4] = c1; nd[5] = c2;
        return idx;
    }

    std::vector<int32_t> perm_;
    std::vector<int32_t> tree_;

private:
    int32_t make_leaf(int32_t idx, std::vector<int32_t> &V, int32_t lo)
    {
        std::sort(V.begin(), V.end());
        for (size_t t = 0; t < V.size(); t++) perm_[lo + t] = V[t];
        int32_t *nd = &tree_[6 * (size_t)idx];
        nd[0] = lo; nd[1] = -1; nd[2] = lo; nd[3] = lo + (int32_t)V.size(); nd[4] = -1; nd[5] = -1;
        return idx;
    }

    // side_[v] = 0 for the first half, 1 for the second half of V
    void split(const std::vector<int32_t> &V, int32_t st)
    {
        size_t nv = V.size();
        std::vector<std::pair<double, int32_t>> key(nv);
        if (coords_) {
            int axis = 0;
            double best = -1.0;
            for (int d = 0; d < dim_; d++) {
                double lo = INFINITY, hi = -INFINITY;
                for (int32_t v : V) {
                    double c = coords_[(size_t)v * dim_ + d];
                    lo = std::min(lo, c);
                    hi = std::max(hi, c);
                }
                if (hi - lo > best) { best = hi - lo; axis = d; }
            }
            for (size_t t = 0; t < nv; t++) key[t] = {coords_[(size_t)V[t] * dim_ + axis], V[t]};
        } else {
            bfs_levels(V, st);
            for (size_t t = 0; t < nv; t++) key[t] = {(double)bfs_level_[V[t]], V[t]};
        }
        std::sort(key.begin(), key.end());
        for (size_t t = 0; t < nv; t++) side_[key[t].second] = t < nv / 2 ? 0 : 1;
    }

    // breadth-first levels from a pseudo-peripheral vertex of V's first
    // component; unreached vertices get level INT32_MAX
    void bfs_levels(const std::vector<int32_t> &V, int32_t st)
    {
        int32_t root = *std::min_element(V.begin(), V.end());
        int32_t ecc = -1;
        for (int round = 0; round < 6; round++) {
            int32_t far = bfs(V, st, root);
            int32_t e = bfs_level_[far];
            if (e <= ecc) break;
            ecc = e;
            root = far;
        }
        bfs(V, st, root);
    }

    int32_t bfs(const std::vector<int32_t> &V, int32_t st, int32_t root)
    {
        for (int32_t v : V) bfs_level_[v] = INT32_MAX;
        std::vector<int32_t> q;
        q.reserve(V.size());
        q.push_back(root);
        bfs_level_[root] = 0;
        int32_t far = root;
        for (size_t h = 0; h < q.size(); h++) {
            int32_t u = q[h];
            if (bfs_level_[u] > bfs_level_[far] || (bfs_level_[u] == bfs_level_[far] && u < far)) far = u;
            for (int64_t p = g_.xadj[u]; p < g_.xadj[u + 1]; p++) {
                int32_t w = g_.adj[p];
                if (stamp_[w] != st || bfs_level_[w] != INT32_MAX) continue;
                bfs_level_[w] = bfs_level_[u] + 1;
                q.push_back(w);
            }
        }
        return far;
    }

    // minimum vertex cover of the edges between side 0 and side 1 inside V
    std::vector<int32_t> cover(const std::vector<int32_t> &V, int32_t st)
    {
        std::vector<int32_t> Lb, Rb;
        for (int32_t v : V) {
            bool cut = false;
            for (int64_t p = g_.xadj[v]; p < g_.xadj[v + 1] && !cut; p++) {
                int32_t w = g_.adj[p];
                cut = stamp_[w] == st && side_[w] != side_[v];
            }
            if (!cut) continue;
            if (side_[v] == 0) { lid_[v] = (int32_t)Lb.size(); Lb.push_back(v); }
            else { rid_[v] = (int32_t)Rb.size(); Rb.push_back(v); }
        }
        int32_t nl = (int32_t)Lb.size(), nr = (int32_t)Rb.size();
        std::vector<int64_t> bp((size_t)nl + 1, 0);
        std::vector<int32_t> bi;
        for (int32_t a = 0; a < nl; a++) {
            int32_t v = Lb[a];
            for (int64_t p = g_.xadj[v]; p < g_.xadj[v + 1]; p++) {
                int32_t w = g_.adj[p];
                if (stamp_[w] == st && side_[w] == 1) bi.push_back(rid_[w]);
            }
            bp[a + 1] = (int64_t)bi.size();
        }
        // Hopcroft-Karp
        std::vector<int32_t> ml(nl, -1), mr(nr, -1), dist(nl), it(nl);
        const int32_t INF = INT32_MAX;
        // greedy start
        for (int32_t a = 0; a < nl; a++)
            for (int64_t p = bp[a]; p < bp[a + 1]; p++)
                if (mr[bi[p]] == -1) { ml[a] = bi[p]; mr[bi[p]] = a; break; }
        std::vector<int32_t> q, stk;
        for (;;) {
            q.clear();
            for (int32_t a = 0; a < nl; a++) {
                if (ml[a] == -1) { dist[a] = 0; q.push_back(a); }
                else dist[a] = INF;
            }
            bool found = false;
            for (size_t h = 0; h < q.size(); h++) {
                int32_t a = q[h];
                for (int64_t p = bp[a]; p < bp[a + 1]; p++) {
                    int32_t a2 = mr[bi[p]];
                    if (a2 == -1) found = true;
                    else if (dist[a2] == INF) { dist[a2] = dist[a] + 1; q.push_back(a2); }
                }
            }
            if (!found) break;
            for (int32_t a = 0; a < nl; a++) it[a] = 0;
            for (int32_t a0 = 0; a0 < nl; a0++) {
                if (ml[a0] != -1) continue;
                // iterative layered DFS for an augmenting path from a0
                stk.clear();
                stk.push_back(a0);
                bool aug = false;
                while (!stk.empty() && !aug) {
                    int32_t a = stk.back();
                    int64_t p = bp[a] + it[a];
                    if (p >= bp[a + 1]) { dist[a] = INF; stk.pop_back(); continue; }
                    it[a]++;
                    int32_t b = bi[p];
                    int32_t a2 = mr[b];
                    if (a2 == -1) {
                        // augment along the stack
                        aug = true;
                        int32_t bb = b;
                        for (size_t s = stk.size(); s-- > 0;) {
                            int32_t x = stk[s];
                            int32_t prev = ml[x];
                            ml[x] = bb;
                            mr[bb] = x;
                            bb = prev;
                        }
                    } else if (dist[a2] == dist[a] + 1) {
                        stk.push_back(a2);
                    }
                }
            }
        }
        // Koenig: Z = vertices reachable from free left vertices by alternating paths
        std::vector<char> zl(nl, 0), zr(nr, 0);
        q.clear();
        for (int32_t a = 0; a < nl; a++)
            if (ml[a] == -1) { zl[a] = 1; q.push_back(a); }
        for (size_t h = 0; h < q.size(); h++) {
            int32_t a = q[h];
            for (int64_t p = bp[a]; p < bp[a + 1]; p++) {
                int32_t b = bi[p];
                if (zr[b]) continue;
                zr[b] = 1;
                int32_t a2 = mr[b];
                if (a2 != -1 && !zl[a2]) { zl[a2] = 1; q.push_back(a2); }
            }
        }
        std::vector<int32_t> S;
        for (int32_t a = 0; a < nl; a++) if (!zl[a]) S.push_back(Lb[a]);
        for (int32_t b = 0; b < nr; b++) if (zr[b]) S.push_back(Rb[b]);
        for (int32_t v : Lb) lid_[v] = -1;
        for (int32_t v : Rb) rid_[v] = -1;
        return S;
    }

    const Graph &g_;
    const double *coords_;
    int dim_;
    int32_t leaf_;
    int32_t next_stamp_ = 0;
    std::vector<int32_t> stamp_, lid_, rid_, bfs_level_;
    std::vector<uint8_t> side_;
};

// ---------------------------------------------------------------------------
// symbolic factorization in pivot order

// lower (i > j) and upper (k < i) adjacency of C = P A P^T, per pivot
void permuted_lists(const Graph &g, const std::vector<int32_t> &perm, const std::vector<int32_t> &iperm,
                    std::vector<int64_t> &lp, std::vector<int32_t> &li,
                    std::vector<int64_t> &up, std::vector<int32_t> &ui)
{
    int32_t n = g.n;
    lp.assign((size_t)n + 1, 0);
    up.assign((size_t)n + 1, 0);
    for (int32_t j = 0; j < n; j++) {
        int32_t v = perm[j];
        for (int64_t p = g.xadj[v]; p < g.xadj[v + 1]; p++) {
            int32_t i = iperm[g.adj[p]];
            if (i > j) lp[j + 1]++;
            else up[j + 1]++;
        }
    }
    for (int32_t j = 0; j < n; j++) { lp[j + 1] += lp[j]; up[j + 1] += up[j]; }
    li.resize((size_t)lp[n]);
    ui.resize((size_t)up[n]);
    for (int32_t j = 0; j < n; j++) {
        int32_t v = perm[j];
        int64_t a = lp[j], b = up[j];
        for (int64_t p = g.xadj[v]; p < g.xadj[v + 1]; p++) {
            int32_t i = iperm[g.adj[p]];
            if (i > j) li[a++] = i;
            else ui[b++] = i;
        }
        std::sort(li.begin() + lp[j], li.begin() + lp[j + 1]);
        std::sort(ui.begin() + up[j], ui.begin() + up[j + 1]);
    }
}

// Liu's elimination tree: for each i, climb from every k < i of row i to the
// current root of k's subtree, compressing paths on the way.
void etree(int32_t n, const std::vector<int64_t> &up, const std::vector<int32_t> &ui, std::vector<int32_t> &parent)
{
    parent.assign(n, -1);
    std::vector<int32_t> root(n, -1);
    for (int32_t i = 0; i < n; i++) {
        for (int64_t p = up[i]; p < up[i + 1]; p++) {
            int32_t k = ui[p];
            while (true) {
                int32_t r = root[k];
                if (r == i) break;
                root[k] = i;
                if (r == -1) { parent[k] = i; break; }
                k = r;
            }
        }
    }
}

void postorder(int32_t n, const std::vector<int32_t> &parent, std::vector<int32_t> &post)
{
    std::vector<int32_t> head(n, -1), nxt(n, -1);
    for (int32_t j = n - 1; j >= 0; j--)   // children in ascending order
        if (parent[j] != -1) { nxt[j] = head[parent[j]]; head[parent[j]] = j; }
    post.clear();
    post.reserve(n);
    std::vector<int32_t> stk;
    for (int32_t r = 0; r < n; r++) {
        if (parent[r] != -1) continue;
        stk.push_back(r);
        while (!stk.empty()) {
            int32_t v = stk.back();
            int32_t c = head[v];
            if (c == -1) { post.push_back(v); stk.pop_back(); }
            else { head[v] = nxt[c]; stk.push_back(c); }
        }
    }
}

// Column counts from the skeleton of the row subtrees: every column j gets
// +1 for each row subtree in which it is a leaf, -1 at the least common
// ancestor of consecutive leaves of the same row subtree, and the etree
// itself contributes (leaf ? 1 : 0) - #children; summing over subtrees in
// postorder yields colcount (diagonal included).
void column_counts(int32_t n, const std::vector<int32_t> &parent, const std::vector<int32_t> &post,
                   const std::vector<int64_t> &lp, const std::vector<int32_t> &li, std::vector<int32_t> &cnt)
{
    std::vector<int32_t> first(n, -1), maxfirst(n, -1), prevleaf(n, -1), anc(n);
    std::vector<int64_t> delta(n, 0);
    for (int32_t k = 0; k < n; k++) {
        int32_t j = post[k];
        delta[j] = first[j] == -1 ? 1 : 0;
        for (; j != -1 && first[j] == -1; j = parent[j]) first[j] = k;
    }
    for (int32_t i = 0; i < n; i++) anc[i] = i;
    for (int32_t k = 0; k < n; k++) {
        int32_t j = post[k];
        if (parent[j] != -1) delta[parent[j]]--;
        for (int64_t p = lp[j]; p < lp[j + 1]; p++) {
            int32_t i = li[p];              // i > j, C_ij != 0
            if (first[j] <= maxfirst[i]) continue;   // j is not a leaf of row subtree i
            maxfirst[i] = first[j];
            int32_t jprev = prevleaf[i];
            prevleaf[i] = j;
            delta[j]++;
            if (jprev != -1) {
                int32_t q = jprev;
                while (q != anc[q]) q = anc[q];
                for (int32_t s = jprev; s != q;) { int32_t t = anc[s]; anc[s] = q; s = t; }
                delta[q]--;
            }
        }
        if (parent[j] != -1) anc[j] = parent[j];
    }
    for (int32_t k = 0; k < n; k++) {
        int32_t j = post[k];
        if (parent[j] != -1) delta[parent[j]] += delta[j];
    }
    cnt.resize(n);
    for (int32_t j = 0; j < n; j++) cnt[j] = (int32_t)delta[j];
}

}  // namespace

int analyze(int32_t n, const int64_t *colptr, const int32_t *rowind, const wcs_analyze_opts *opts, Symbolic &S)
{
    int rc = validate(n, colptr, rowind);
    if (rc) return rc;
    wcs_analyze_opts o;
    std::memset(&o, 0, sizeof(o));
    o.leaf_size = 64;
    o.dense_degree_frac = 0.25;
    o.dense_degree_min = 1024;
    o.relax = 1;
    if (opts) o = *opts;
    if (o.coords && (o.coord_dim < 1 || o.coord_dim > 3)) { set_error("coord_dim must be 1..3"); return WCS_EINVAL; }

    S.n = n;
    S.nnz = colptr[n];
    S.colptr.assign(colptr, colptr + n + 1);
    S.rowind.assign(rowind, rowind + S.nnz);
    Graph g = build_graph(n, colptr, rowind);

    // ---- ordering
    if (o.user_perm) {
        S.perm.assign(o.user_perm, o.user_perm + n);
        std::vector<char> seen(n, 0);
        for (int32_t k = 0; k < n; k++) {
            int32_t v = S.perm[k];
            if (v < 0 || v >= n || seen[v]) { set_error("user_perm is not a permutation"); return WCS_EINVAL; }
            seen[v] = 1;
        }
        S.sep_tree = {0, -1, 0, n, -1, -1};
        S.npeeled = 0;
    } else {
        double thr = std::max(o.dense_degree_frac * (double)n, o.dense_degree_min);
        std::vector<int32_t> rest, peeled;
        for (int32_t v = 0; v < n; v++) {
            double deg = (double)(g.xadj[v + 1] - g.xadj[v]);
            (deg >= thr ? peeled : rest).push_back(v);
        }
        Dissection nd(g, o.coords, o.coord_dim, o.leaf_size);
        int32_t nr = (int32_t)rest.size();
        if (nr > 0) nd.dissect(rest, 0);
        else nd.tree_ = {0, -1, 0, 0, -1, -1};
        for (size_t t = 0; t < peeled.size(); t++) nd.perm_[nr + t] = peeled[t];
        nd.tree_[3] = n;   // the root separator also holds the peeled vertices
        S.perm.swap(nd.perm_);
        S.sep_tree.swap(nd.tree_);
        S.npeeled = (int32_t)peeled.size();
    }
    S.iperm.assign(n, 0);
    for (int32_t k = 0; k < n; k++) S.iperm[S.perm[k]] = k;

    // ---- fundamental symbolic structure
    std::vector<int64_t> lp, up;
    std::vector<int32_t> li, ui, post;
    permuted_lists(g, S.perm, S.iperm, lp, li, up, ui);
    etree(n, up, ui, S.parent);
    postorder(n, S.parent, post);
    column_counts(n, S.parent, post, lp, li, S.colcount);
    S.nnz_l = 0;
    S.flops = 0;
    for (int32_t j = 0; j < n; j++) {
        S.nnz_l += S.colcount[j];
        S.flops += (int64_t)S.colcount[j] * S.colcount[j];
    }
    std::vector<int32_t> nchild(n, 0);
    for (int32_t j = 0; j < n; j++) if (S.parent[j] != -1) nchild[S.parent[j]]++;
    S.fund_ptr.clear();
    for (int32_t j = 0; j < n; j++) {
        bool join = j > 0 && S.parent[j - 1] == j && nchild[j] == 1 && S.colcount[j - 1] == S.colcount[j] + 1;
        if (!join) S.fund_ptr.push_back(j);
    }
    S.fund_ptr.push_back(n);
    int32_t nf = (int32_t)S.fund_ptr.size() - 1;

    // ---- relaxed amalgamation: merge a supernode into its parent when it is
    // the parent's immediately preceding child and few explicit zeros result
    // (ncols <= 4 always; <= 16 with <= 80% zeros; <= 48 with <= 10%; else <= 5%)
    std::vector<int32_t> gfirst(nf), gcols(nf), gm(nf);   // per current group (indexed by fundamental id of its top)
    std::vector<int64_t> gzeros(nf, 0);
    std::vector<int32_t> fund_of(n);
    for (int32_t f = 0; f < nf; f++)
        for (int32_t j = S.fund_ptr[f]; j < S.fund_ptr[f + 1]; j++) fund_of[j] = f;
    std::vector<int32_t> group_top_at_end(n + 1, -1);   // last column -> group id (top fundamental)
    std::vector<char> alive(nf, 1);
    for (int32_t f = 0; f < nf; f++) {
        int32_t a = S.fund_ptr[f], b = S.fund_ptr[f + 1];
        gfirst[f] = a;
        gcols[f] = b - a;
        gm[f] = S.colcount[a];
        if (o.relax && a > 0) {
            int32_t c = group_top_at_end[a - 1];        // group ending right before f
            if (c != -1 && S.parent[a - 1] == a && true) {
                // c's last column has parent a (first column of f): c is a child of f
                int64_t cstruct = gm[c] - gcols[c];
                int32_t ncols = gcols[c] + gcols[f];
                int64_t mm = gcols[c] + (int64_t)gm[f];
                int64_t zeros = gzeros[c] + gzeros[f] + (int64_t)gcols[c] * (gm[f] - cstruct);
                int64_t entries = (int64_t)ncols * mm - (int64_t)ncols * (ncols - 1) / 2;
                double z = entries ? (double)zeros / (double)entries : 0.0;
                bool ok = ncols <= 4 || (ncols <= 16 && z <= 0.8) || (ncols <= 48 && z <= 0.1) || z <= 0.05;
                if (ok) {
                    alive[c] = 0;
                    gfirst[f] = gfirst[c];
                    gcols[f] = ncols;
                    gm[f] = (int32_t)mm;
                    gzeros[f] = zeros;
                }
            }
        }
        group_top_at_end[b - 1] = f;
    }
    S.sptr.clear();
    for (int32_t f = 0; f < nf; f++) if (alive[f]) S.sptr.push_back(gfirst[f]);
    S.sptr.push_back(n);
    S.ns = (int32_t)S.sptr.size() - 1;
    int32_t ns = S.ns;
    S.snode_of.assign(n, 0);
    for (int32_t s = 0; s < ns; s++)
        for (int32_t j = S.sptr[s]; j < S.sptr[s + 1]; j++) S.snode_of[j] = s;

    // ---- front row structures: own columns, entries of C below them, and
    // the update rows of every child front (children precede their parent)
    std::vector<int32_t> mark(n, -1);
    std::vector<std::vector<int32_t>> kids(ns);
    S.rptr.assign((size_t)ns + 1, 0);
    S.rows.clear();
    S.sparent.assign(ns, -1);
    std::vector<int32_t> tmp;
    for (int32_t s = 0; s < ns; s++) {
        int32_t f0 = S.sptr[s], f1 = S.sptr[s + 1];
        tmp.clear();
        for (int32_t j = f0; j < f1; j++) { tmp.push_back(j); mark[j] = s; }
        for (int32_t j = f0; j < f1; j++)
            for (int64_t p = lp[j]; p < lp[j + 1]; p++) {
                int32_t i = li[p];
                if (mark[i] != s) { mark[i] = s; tmp.push_back(i); }
            }
        for (int32_t c : kids[s]) {
            int32_t pc = S.p_of(c);
            for (int64_t p = S.rptr[c] + pc; p < S.rptr[c + 1]; p++) {
                int32_t i = S.rows[p];
                if (mark[i] != s) { mark[i] = s; tmp.push_back(i); }
            }
        }
        std::sort(tmp.begin() + (f1 - f0), tmp.end());
        S.rows.insert(S.rows.end(), tmp.begin(), tmp.end());
        S.rptr[s + 1] = (int64_t)S.rows.size();
        if ((int32_t)tmp.size() > f1 - f0) {
            int32_t par = S.snode_of[tmp[f1 - f0]];
            S.sparent[s] = par;
            kids[par].push_back(s);
        }
    }
    // extend-add maps and padded flops
    S.rel.assign(S.rows.size(), -1);
    std::vector<int32_t> pos(n, -1);
    S.flops_padded = 0;
    for (int32_t s = 0; s < ns; s++) {
        int32_t m = S.m_of(s), p = S.p_of(s);
        for (int32_t t = 0; t < p; t++) S.flops_padded += (int64_t)(m - t) * (m - t);
    }
    for (int32_t par = 0; par < ns; par++) {
        for (int64_t q = S.rptr[par]; q < S.rptr[par + 1]; q++) pos[S.rows[q]] = (int32_t)(q - S.rptr[par]);
        for (int32_t c : kids[par]) {
            int32_t pc = S.p_of(c);
            for (int64_t q = S.rptr[c] + pc; q < S.rptr[c + 1]; q++) S.rel[q] = pos[S.rows[q]];
        }
    }
    // levels: height above the leaves
    S.height.assign(ns, 0);
    S.nlevels = ns > 0 ? 1 : 0;
    for (int32_t s = 0; s < ns; s++) {
        if (S.sparent[s] != -1) S.height[S.sparent[s]] = std::max(S.height[S.sparent[s]], S.height[s] + 1);
        S.nlevels = std::max(S.nlevels, S.height[s] + 1);
    }
    // front buffers: m x m column-major with leading dimension front_ld_host(m), one after another
    S.front_off.assign((size_t)ns + 1, 0);
    for (int32_t s = 0; s < ns; s++)
        S.front_off[s + 1] = S.front_off[s] + (int64_t)front_ld_host(S.m_of(s)) * S.m_of(s);
    // stored entries of A -> front offsets: entry (i, j) lands in the front
    // owning column min(pi(i), pi(j)) at row max(pi(i), pi(j))
    S.amap.assign((size_t)S.nnz, 0);
    {
        // group entries by owning front so each front's positions are set once
        std::vector<int64_t> cnt((size_t)ns + 1, 0);
        for (int32_t j = 0; j < n; j++)
            for (int64_t p = colptr[j]; p < colptr[j + 1]; p++) {
                int32_t a = S.iperm[rowind[p]], b = S.iperm[j];
                cnt[S.snode_of[std::min(a, b)] + 1]++;
            }
        for (int32_t s = 0; s < ns; s++) cnt[s + 1] += cnt[s];
        std::vector<int64_t> ent((size_t)S.nnz);
        std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
        for (int32_t j = 0; j < n; j++)
            for (int64_t p = colptr[j]; p < colptr[j + 1]; p++) {
                int32_t a = S.iperm[rowind[p]], b = S.iperm[j];
                ent[fill[S.snode_of[std::min(a, b)]]++] = p;
            }
        std::vector<int32_t> colof(S.nnz);
        for (int32_t j = 0; j < n; j++)
            for (int64_t p = colptr[j]; p < colptr[j + 1]; p++) colof[p] = j;
        for (int32_t s = 0; s < ns; s++) {
            int32_t m = front_ld_host(S.m_of(s));
            for (int64_t q = S.rptr[s]; q < S.rptr[s + 1]; q++) pos[S.rows[q]] = (int32_t)(q - S.rptr[s]);
            for (int64_t t = cnt[s]; t < cnt[s + 1]; t++) {
                int64_t p = ent[t];
                int32_t a = S.iperm[rowind[p]], b = S.iperm[colof[p]];
                int32_t lo = std::min(a, b), hi = std::max(a, b);
                S.amap[p] = S.front_off[s] + (int64_t)(lo - S.sptr[s]) * m + pos[hi];
            }
        }
    }
    // full symmetric CSR of C = P A P^T (pivot order, columns ascending) for
    // the refinement residual; csr_src names the stored entry of each value
    S.csr_ptr.assign((size_t)n + 1, 0);
    for (int32_t j = 0; j < n; j++)
        for (int64_t p = colptr[j]; p < colptr[j + 1]; p++) {
            int32_t i = rowind[p];
            S.csr_ptr[S.iperm[i] + 1]++;
            if (i != j) S.csr_ptr[S.iperm[j] + 1]++;
        }
    for (int32_t i = 0; i < n; i++) S.csr_ptr[i + 1] += S.csr_ptr[i];
    S.csr_col.resize((size_t)S.csr_ptr[n]);
    S.csr_src.resize((size_t)S.csr_ptr[n]);
    {
        std::vector<int64_t> fill(S.csr_ptr.begin(), S.csr_ptr.end() - 1);
        for (int32_t j = 0; j < n; j++)
            for (int64_t p = colptr[j]; p < colptr[j + 1]; p++) {
                int32_t i = rowind[p];
                int32_t a = S.iperm[i], b = S.iperm[j];
                S.csr_col[fill[a]] = b;
                S.csr_src[fill[a]++] = p;
                if (i != j) {
                    S.csr_col[fill[b]] = a;
                    S.csr_src[fill[b]++] = p;
                }
            }
        std::vector<std::pair<int32_t, int64_t>> tmp2;
        for (int32_t r = 0; r < n; r++) {
            int64_t a = S.csr_ptr[r], b = S.csr_ptr[r + 1];
            tmp2.resize((size_t)(b - a));
            for (int64_t q = a; q < b; q++) tmp2[q - a] = {S.csr_col[q], S.csr_src[q]};
            std::sort(tmp2.begin(), tmp2.end());
            for (int64_t q = a; q < b; q++) {
                S.csr_col[q] = tmp2[q - a].first;
                S.csr_src[q] = tmp2[q - a].second;
            }
        }
    }
    S.seg_ptr = {0, n};
    return WCS_OK;
}

// Block-diagonal union: the matrix diag(A_0, ..., A_{count-1}) ordered block by
// block, each block with its own ordering.  Its elimination tree is the forest
// of the parts' trees, so every symbolic quantity is the concatenation of the
// parts' with indices shifted; the level schedule then runs the fronts of equal
// height of all parts together.
int combine(int32_t count, const Symbolic *const *parts, Symbolic &S)
{
    if (count <= 0) { set_error("batch needs at least one part"); return WCS_EINVAL; }
    // totals first, so every array is sized once and filled in place
    int64_t n_tot = 0, nnz_tot = 0, ns_tot = 0, rows_tot = 0, tree_tot = 0, fund_tot = 0, csr_tot = 0;
    for (int32_t b = 0; b < count; b++) {
        const Symbolic *P = parts[b];
        if (!P) { set_error("null part in batch"); return WCS_EINVAL; }
        n_tot += P->n;
        nnz_tot += P->nnz;
        ns_tot += P->ns;
        rows_tot += (int64_t)P->rows.size();
        tree_tot += (int64_t)P->sep_tree.size();
        fund_tot += (int64_t)P->fund_ptr.size() - 1;
        csr_tot += (int64_t)P->csr_col.size();
    }
    if (n_tot > INT32_MAX || ns_tot > INT32_MAX) { set_error("batch too large for 32-bit indices"); return WCS_EINVAL; }
    S = Symbolic();
    S.n = (int32_t)n_tot;
    S.nnz = nnz_tot;
    S.ns = (int32_t)ns_tot;
    S.colptr.resize((size_t)n_tot + 1);
    S.rowind.resize((size_t)nnz_tot);
    S.perm.resize((size_t)n_tot);
    S.iperm.resize((size_t)n_tot);
    S.sep_tree.resize((size_t)tree_tot);
    S.parent.resize((size_t)n_tot);
    S.colcount.resize((size_t)n_tot);
    S.fund_ptr.resize((size_t)fund_tot + 1);
    S.sptr.resize((size_t)ns_tot + 1);
    S.snode_of.resize((size_t)n_tot);
    S.rptr.resize((size_t)ns_tot + 1);
    S.rows.resize((size_t)rows_tot);
    S.rel.resize((size_t)rows_tot);
    S.sparent.resize((size_t)ns_tot);
    S.height.resize((size_t)ns_tot);
    S.front_off.resize((size_t)ns_tot + 1);
    S.amap.resize((size_t)nnz_tot);
    S.csr_ptr.resize((size_t)n_tot + 1);
    S.csr_col.resize((size_t)csr_tot);
    S.csr_src.resize((size_t)csr_tot);
    S.seg_ptr.resize((size_t)count + 1);
    S.colptr[0] = 0;
    S.fund_ptr[0] = 0;
    S.sptr[0] = 0;
    S.rptr[0] = 0;
    S.front_off[0] = 0;
    S.csr_ptr[0] = 0;
    S.seg_ptr[0] = 0;
    // per-part offsets into every concatenated array
    struct Off { int32_t n, s, t; int64_t z, r, f, c, tp, fp; };
    std::vector<Off> off((size_t)count + 1);
    off[0] = Off{0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int32_t b = 0; b < count; b++) {
        const Symbolic &P = *parts[b];
        const Off &o = off[b];
        off[b + 1] = Off{o.n + P.n, o.s + P.ns, o.t + (int32_t)(P.sep_tree.size() / 6), o.z + P.nnz,
                         o.r + (int64_t)P.rows.size(), o.f + P.front_off.back(), o.c + (int64_t)P.csr_col.size(),
                         o.tp + (int64_t)P.sep_tree.size(), o.fp + (int64_t)P.fund_ptr.size() - 1};
        S.seg_ptr[b + 1] = off[b + 1].n;
        S.npeeled += P.npeeled;
        S.nnz_l += P.nnz_l;
        S.flops += P.flops;
        S.flops_padded += P.flops_padded;
        S.nlevels = std::max(S.nlevels, P.nlevels);
    }
    // the parts write disjoint ranges: copy them on a few threads
    auto copy_part = [&](int32_t b) {
        const Symbolic &P = *parts[b];
        const int32_t n = P.n, ns = P.ns;
        const int32_t noff = off[b].n, soff = off[b].s, toff = off[b].t;
        const int64_t zoff = off[b].z, roff = off[b].r, foff = off[b].f, coff = off[b].c, tpos = off[b].tp,
                      fpos = off[b].fp;
        for (int32_t j = 0; j < n; j++) {
            S.colptr[noff + j + 1] = P.colptr[j + 1] + zoff;
            S.perm[noff + j] = P.perm[j] + noff;
            S.iperm[noff + j] = P.iperm[j] + noff;
            S.parent[noff + j] = P.parent[j] < 0 ? -1 : P.parent[j] + noff;
            S.colcount[noff + j] = P.colcount[j];
            S.snode_of[noff + j] = P.snode_of[j] + soff;
            S.csr_ptr[noff + j + 1] = P.csr_ptr[j + 1] + coff;
        }
        for (int64_t q = 0; q < P.nnz; q++) {
            S.rowind[zoff + q] = P.rowind[q] + noff;
            S.amap[zoff + q] = P.amap[q] + foff;
        }
        for (size_t q = 0; q < P.sep_tree.size(); q += 6) {
            const int32_t *nd = &P.sep_tree[q];
            int32_t *od = &S.sep_tree[tpos + q];
            od[0] = nd[0] + noff;
            od[1] = nd[1] < 0 ? -1 : nd[1] + noff;
            od[2] = nd[2] + noff;
            od[3] = nd[3] + noff;
            od[4] = nd[4] < 0 ? -1 : nd[4] + toff;
            od[5] = nd[5] < 0 ? -1 : nd[5] + toff;
        }
        for (size_t q = 1; q < P.fund_ptr.size(); q++) S.fund_ptr[fpos + q] = P.fund_ptr[q] + noff;
        for (int32_t q = 0; q < ns; q++) {
            S.sptr[soff + q + 1] = P.sptr[q + 1] + noff;
            S.rptr[soff + q + 1] = P.rptr[q + 1] + roff;
            S.sparent[soff + q] = P.sparent[q] < 0 ? -1 : P.sparent[q] + soff;
            S.height[soff + q] = P.height[q];
            S.front_off[soff + q + 1] = P.front_off[q + 1] + foff;
        }
        for (size_t q = 0; q < P.rows.size(); q++) {
            S.rows[roff + q] = P.rows[q] + noff;
            S.rel[roff + q] = P.rel[q];
        }
        for (size_t q = 0; q < P.csr_col.size(); q++) {
            S.csr_col[coff + q] = P.csr_col[q] + noff;
            S.csr_src[coff + q] = P.csr_src[q] + zoff;
        }
    };
    unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    nth = std::min<unsigned>(nth, (unsigned)count);
    std::vector<std::thread> pool;
    std::atomic<int32_t> next{0};
    for (unsigned t = 0; t < nth; t++)
        pool.emplace_back([&] {
            for (int32_t b; (b = next.fetch_add(1)) < count;) copy_part(b);
        });
    for (auto &th : pool) th.join();
    return WCS_OK;
}

}  // namespace wcs
