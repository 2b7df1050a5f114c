// C ABI: status strings, error detail, and the host-only symbolic calls.
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

struct wcs_symbolic_s {
    wcs::Symbolic s;
};

namespace wcs {
namespace {
thread_local std::string g_last_error;
}
void set_error(const std::string &msg) { g_last_error = msg; }
}  // namespace wcs

extern "C" {

const char *wcs_status_string(int status)
{
    switch (status) {
    case WCS_OK: return "WCS_OK";
    case WCS_EINVAL: return "WCS_EINVAL";
    case WCS_ENOMEM: return "WCS_ENOMEM";
    case WCS_EHIP: return "WCS_EHIP";
    case WCS_ENOTSPD: return "WCS_ENOTSPD";
    case WCS_ENOTCONV: return "WCS_ENOTCONV";
    case WCS_ESTATE: return "WCS_ESTATE";
    case WCS_ESINGULAR: return "WCS_ESINGULAR";
    default: return "WCS_UNKNOWN";
    }
}

const char *wcs_last_error(void) { return wcs::g_last_error.c_str(); }

int wcs_analyze(int32_t n, const int64_t *colptr, const int32_t *rowind, const wcs_analyze_opts *opts,
                wcs_symbolic *out)
{
    if (!out) { wcs::set_error("out is NULL"); return WCS_EINVAL; }
    *out = nullptr;
    wcs_symbolic h = new (std::nothrow) wcs_symbolic_s;
    if (!h) return WCS_ENOMEM;
    int rc;
    try {
        rc = wcs::analyze(n, colptr, rowind, opts, h->s);
    } catch (const std::bad_alloc &) {
        wcs::set_error("host allocation failed in analyze");
        rc = WCS_ENOMEM;
    } catch (...) {
        wcs::set_error("unexpected failure in analyze");
        rc = WCS_EINVAL;
    }
    if (rc != WCS_OK) { delete h; return rc; }
    *out = h;
    return WCS_OK;
}

int wcs_symbolic_info(wcs_symbolic sym, wcs_symbolic_info_t *info)
{
    if (!sym || !info) { wcs::set_error("null argument"); return WCS_EINVAL; }
    const wcs::Symbolic &S = sym->s;
    std::memset(info, 0, sizeof(*info));
    info->n = S.n;
    info->nnz_lower = S.nnz;
    info->nnz_l = S.nnz_l;
    info->flops = S.flops;
    info->flops_padded = S.flops_padded;
    info->nsuper_fund = (int32_t)S.fund_ptr.size() - 1;
    info->nsuper = S.ns;
    info->nlevels = S.nlevels;
    int32_t mx = 0;
    for (int32_t s = 0; s < S.ns; s++) mx = std::max(mx, S.m_of(s));
    info->max_front = mx;
    info->nsep_nodes = (int32_t)(S.sep_tree.size() / 6);
    info->npeeled = S.npeeled;
    info->front_elems = S.front_off.empty() ? 0 : S.front_off.back();
    int64_t pad = 0;
    for (int32_t s = 0; s < S.ns; s++) {
        int64_t m = S.m_of(s), p = S.p_of(s);
        pad += p * m - p * (p - 1) / 2;
    }
    info->nnz_l_padded = pad;
    info->nseg = S.seg_ptr.size() >= 2 ? (int32_t)S.seg_ptr.size() - 1 : 1;
    return WCS_OK;
}

int wcs_symbolic_export(wcs_symbolic sym, int32_t *perm, int32_t *parent, int32_t *colcount, int32_t *super_ptr,
                        int32_t *sep_tree)
{
    if (!sym) { wcs::set_error("null handle"); return WCS_EINVAL; }
    const wcs::Symbolic &S = sym->s;
    size_t n = (size_t)S.n;
    if (perm) std::memcpy(perm, S.perm.data(), n * sizeof(int32_t));
    if (parent) std::memcpy(parent, S.parent.data(), n * sizeof(int32_t));
    if (colcount) std::memcpy(colcount, S.colcount.data(), n * sizeof(int32_t));
    if (super_ptr) std::memcpy(super_ptr, S.fund_ptr.data(), S.fund_ptr.size() * sizeof(int32_t));
    if (sep_tree) std::memcpy(sep_tree, S.sep_tree.data(), S.sep_tree.size() * sizeof(int32_t));
    return WCS_OK;
}

int wcs_symbolic_fronts(wcs_symbolic sym, int32_t *relaxed_ptr, int32_t *front_order)
{
    if (!sym) { wcs::set_error("null handle"); return WCS_EINVAL; }
    const wcs::Symbolic &S = sym->s;
    if (relaxed_ptr) std::memcpy(relaxed_ptr, S.sptr.data(), S.sptr.size() * sizeof(int32_t));
    if (front_order)
        for (int32_t s = 0; s < S.ns; s++) front_order[s] = S.m_of(s);
    return WCS_OK;
}

int wcs_symbolic_batch(int32_t count, const wcs_symbolic *parts, wcs_symbolic *out)
{
    if (!out || !parts || count <= 0) { wcs::set_error("invalid argument to wcs_symbolic_batch"); return WCS_EINVAL; }
    *out = nullptr;
    wcs_symbolic h = new (std::nothrow) wcs_symbolic_s;
    if (!h) return WCS_ENOMEM;
    int rc;
    try {
        std::vector<const wcs::Symbolic *> ps((size_t)count);
        for (int32_t b = 0; b < count; b++) ps[b] = parts[b] ? &parts[b]->s : nullptr;
        rc = wcs::combine(count, ps.data(), h->s);
    } catch (const std::bad_alloc &) {
        wcs::set_error("host allocation failed in wcs_symbolic_batch");
        rc = WCS_ENOMEM;
    }
    if (rc != WCS_OK) { delete h; return rc; }
    *out = h;
    return WCS_OK;
}

int wcs_symbolic_segments(wcs_symbolic sym, int32_t *seg_ptr)
{
    if (!sym || !seg_ptr) { wcs::set_error("null argument"); return WCS_EINVAL; }
    const wcs::Symbolic &S = sym->s;
    if (S.seg_ptr.size() >= 2)
        std::memcpy(seg_ptr, S.seg_ptr.data(), S.seg_ptr.size() * sizeof(int32_t));
    else {
        seg_ptr[0] = 0;
        seg_ptr[1] = S.n;
    }
    return WCS_OK;
}

void wcs_symbolic_free(wcs_symbolic sym) { delete sym; }

}  // extern "C"

namespace wcs {
const Symbolic &symbolic_of(wcs_symbolic h) { return h->s; }
}  // namespace wcs
