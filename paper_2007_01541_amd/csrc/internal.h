// Internal declarations shared by the host-side parts of the library.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/wcs.h"

namespace wcs {

void set_error(const std::string &msg);

// Leading dimension of an m x m front buffer: m rounded up to 8 elements, so
// every column starts 32-byte (FP32) / 64-byte (FP64) aligned.
inline int32_t front_ld_host(int32_t m) { return (m + 7) & ~7; }

// Result of the ordering + symbolic analysis, plus the static plan derived
// from it (everything here is host memory and independent of the values).
struct Symbolic {
    int32_t n = 0;
    int64_t nnz = 0;
    std::vector<int64_t> colptr;
    std::vector<int32_t> rowind;

    // ordering (perm[k] = original index of pivot k) and separator tree
    std::vector<int32_t> perm, iperm;
    std::vector<int32_t> sep_tree;   // 6 ints per node
    int32_t npeeled = 0;

    // fundamental symbolic structure in pivot order
    std::vector<int32_t> parent, colcount;
    std::vector<int32_t> fund_ptr;   // nsuper_fund + 1
    int64_t nnz_l = 0, flops = 0, flops_padded = 0;

    // amalgamated supernodes = fronts
    int32_t ns = 0;
    std::vector<int32_t> sptr;       // ns + 1 first pivot of each front
    std::vector<int32_t> snode_of;   // pivot -> front
    std::vector<int64_t> rptr;       // ns + 1 offsets into rows / rel
    std::vector<int32_t> rows;       // front row lists (pivot indices, ascending)
    std::vector<int32_t> rel;        // for update rows: position in the parent's row list
    std::vector<int32_t> sparent;    // parent front or -1
    std::vector<int32_t> height;     // 0 for leaves
    int32_t nlevels = 0;
    std::vector<int64_t> front_off;  // ns + 1 element offsets of the front buffers (ld x m, ld = front_ld_host(m))
    std::vector<int64_t> amap;       // per stored entry: element offset inside the fronts

    // full symmetric CSR of P A P^T in pivot order (for the residual), with
    // the stored-entry index each CSR entry takes its value from
    std::vector<int64_t> csr_ptr;
    std::vector<int32_t> csr_col;
    std::vector<int64_t> csr_src;

    // independent diagonal blocks (instances of a batch): block b holds the
    // unknowns [seg_ptr[b], seg_ptr[b+1]) in both the original and the pivot
    // order; a single matrix has one block
    std::vector<int32_t> seg_ptr;

    int32_t m_of(int32_t s) const { return (int32_t)(rptr[s + 1] - rptr[s]); }
    int32_t p_of(int32_t s) const { return sptr[s + 1] - sptr[s]; }
};

int analyze(int32_t n, const int64_t *colptr, const int32_t *rowind, const wcs_analyze_opts *opts,
            Symbolic &out);
// block-diagonal union of independent analyses (one block per part, in order)
int combine(int32_t count, const Symbolic *const *parts, Symbolic &out);

}  // namespace wcs
