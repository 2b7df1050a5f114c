// Host-only driver of the symbolic analysis for sanitizer builds (test
// infrastructure).  Reads a pattern file, runs wcs_analyze with several
// option sets and wcs_symbolic_batch, checks that malformed patterns are
// rejected, and writes every result to an output file that the test compares
// with the regular library build.
//
// pattern file: int32 n, int64 nnz, int64 colptr[n+1], int32 rowind[nnz], double coords[2n]
// output file:  per analysis: int64 info[14], then int32 arrays perm, parent, colcount (n each),
//               super_ptr (nsuper_fund+1), relaxed_ptr (nsuper+1), front_order (nsuper)
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../include/wcs.h"

static void put_info(FILE *o, const wcs_symbolic_info_t &i)
{
    int64_t v[14] = {i.n, i.nnz_lower, i.nnz_l, i.flops, i.flops_padded, i.nsuper_fund, i.nsuper,
                     i.nlevels, i.max_front, i.nsep_nodes, i.npeeled, i.front_elems, i.nnz_l_padded, i.nseg};
    fwrite(v, sizeof v, 1, o);
}

static int dump(FILE *o, wcs_symbolic s)
{
    wcs_symbolic_info_t in;
    if (wcs_symbolic_info(s, &in) != WCS_OK) return 1;
    put_info(o, in);
    std::vector<int32_t> perm(in.n), parent(in.n), cc(in.n), sp(in.nsuper_fund + 1), rp(in.nsuper + 1),
        fo(in.nsuper);
    if (wcs_symbolic_export(s, perm.data(), parent.data(), cc.data(), sp.data(), nullptr) != WCS_OK) return 1;
    if (wcs_symbolic_fronts(s, rp.data(), fo.data()) != WCS_OK) return 1;
    for (auto *v : {&perm, &parent, &cc, &sp, &rp, &fo}) fwrite(v->data(), 4, v->size(), o);
    return 0;
}

int main(int argc, char **argv)
{
    if (argc != 3) { fprintf(stderr, "usage: %s pattern.bin out.bin\n", argv[0]); return 2; }
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    int32_t n = 0;
    int64_t nnz = 0;
    if (fread(&n, 4, 1, f) != 1 || fread(&nnz, 8, 1, f) != 1) return 2;
    std::vector<int64_t> colptr(n + 1);
    std::vector<int32_t> rowind(nnz);
    std::vector<double> coords(2 * (size_t)n);
    if (fread(colptr.data(), 8, n + 1, f) != (size_t)n + 1 || fread(rowind.data(), 4, nnz, f) != (size_t)nnz ||
        fread(coords.data(), 8, 2 * (size_t)n, f) != 2 * (size_t)n)
        return 2;
    fclose(f);
    FILE *o = fopen(argv[2], "wb");
    if (!o) return 2;
    std::vector<int32_t> rev(n);
    for (int32_t k = 0; k < n; k++) rev[k] = n - 1 - k;
    wcs_analyze_opts opts[4];
    for (auto &op : opts) {
        op.leaf_size = 64;
        op.dense_degree_frac = 0.25;
        op.dense_degree_min = 1024;
        op.coords = nullptr;
        op.coord_dim = 0;
        op.user_perm = nullptr;
        op.relax = 1;
    }
    opts[0].coords = coords.data();
    opts[0].coord_dim = 2;
    opts[1].leaf_size = 16;
    opts[1].dense_degree_min = 64;
    opts[2].user_perm = rev.data();
    opts[3].relax = 0;
    opts[3].coords = coords.data();
    opts[3].coord_dim = 2;
    wcs_symbolic s[4];
    for (int t = 0; t < 4; t++) {
        if (wcs_analyze(n, colptr.data(), rowind.data(), &opts[t], &s[t]) != WCS_OK) {
            fprintf(stderr, "analyze %d: %s\n", t, wcs_last_error());
            return 1;
        }
        if (dump(o, s[t])) return 1;
    }
    wcs_symbolic b;
    if (wcs_symbolic_batch(2, s, &b) != WCS_OK || dump(o, b)) return 1;
    wcs_symbolic_free(b);
    for (auto &x : s) wcs_symbolic_free(x);
    fclose(o);
    // malformed patterns are rejected without touching memory out of bounds
    int bad = 0;
    if (n >= 4 && colptr[2] - colptr[1] >= 3) {
        std::vector<int32_t> r2(rowind);
        std::swap(r2[colptr[1] + 1], r2[colptr[1] + 2]);           // unsorted rows
        wcs_symbolic h = nullptr;
        bad += wcs_analyze(n, colptr.data(), r2.data(), nullptr, &h) != WCS_EINVAL;
        r2 = rowind;
        r2[colptr[1] + 1] = n + 7;                                 // row out of range
        bad += wcs_analyze(n, colptr.data(), r2.data(), nullptr, &h) != WCS_EINVAL;
        r2 = rowind;
        r2[colptr[2]] += 1;                                        // diagonal of column 2 missing
        bad += wcs_analyze(n, colptr.data(), r2.data(), nullptr, &h) != WCS_EINVAL;
        std::vector<int64_t> c2(colptr);
        c2[3] = c2[2];                                             // column 2 empty
        bad += wcs_analyze(n, c2.data(), rowind.data(), nullptr, &h) != WCS_EINVAL;
    }
    printf("ok %d\n", bad);
    return bad ? 1 : 0;
}
