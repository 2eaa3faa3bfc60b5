// Host-only part of the C ABI: options, status strings, the thread-local error detail, and
// the calls that expose the library's phi and operators without a GPU.
#include "lfmm.h"
#include "api_common.h"
#include "host_math.h"

#include <cstring>
#include <exception>
#include <new>
#include <string>

namespace lfmm {

thread_local std::string g_last_error;

lfmm_status fail(lfmm_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

lfmm_status validate_options(const lfmm_options* o) {
    if (!(o->eps > 0.0 && o->eps < 1e-2)) return fail(LFMM_E_INVAL, "eps must lie in (0, 1e-2)");
    if (o->max_leaf < 0 || o->max_leaf > 4096) return fail(LFMM_E_INVAL, "max_leaf must lie in [0, 4096]");
    if (o->precision != LFMM_FP64 && o->precision != LFMM_MIXED && o->precision != LFMM_MIXED_BF16)
        return fail(LFMM_E_INVAL, "precision must be LFMM_FP64, LFMM_MIXED or LFMM_MIXED_BF16");
    if (o->proxy_per_edge < 8 || o->proxy_per_edge > 4096)
        return fail(LFMM_E_INVAL, "proxy_per_edge must lie in [8, 4096]");
    if (o->max_rank < 16 || o->max_rank > kMaxRank || o->max_rank % 16 != 0)
        return fail(LFMM_E_INVAL, "max_rank must be 16, 32, 48 or 64");
    if (o->flags & ~(LFMM_FLAG_GRAPH | LFMM_FLAG_CHECK_LOADS | LFMM_FLAG_ADAPTIVE)) return fail(LFMM_E_INVAL, "unknown bits in options.flags");
    if (o->stencil != LFMM_STENCIL_5 && o->stencil != LFMM_STENCIL_9)
        return fail(LFMM_E_INVAL, "stencil must be LFMM_STENCIL_5 or LFMM_STENCIL_9");
    return LFMM_OK;
}

OperatorParams operator_params(const lfmm_options& o) {
    OperatorParams p;
    p.stencil = o.stencil;
    p.eps = o.eps;
    p.proxy_per_edge = o.proxy_per_edge;
    p.max_rank = o.max_rank;
    p.dense_leaf_max = kDenseLeafMax;
    return p;
}

}  // namespace lfmm

using namespace lfmm;

struct lfmm_opset {
    OperatorSet ops;
};

extern "C" {

lfmm_status lfmm_options_init(lfmm_options* opt) {
    if (!opt) return fail(LFMM_E_INVAL, "null options");
    opt->eps = 1e-12;
    opt->max_leaf = 64;
    opt->precision = LFMM_FP64;
    opt->proxy_per_edge = 64;
    opt->max_rank = 48;
    opt->flags = 0;
    opt->stencil = LFMM_STENCIL_5;
    return LFMM_OK;
}

const char* lfmm_status_string(lfmm_status s) {
    switch (s) {
        case LFMM_OK: return "ok";
        case LFMM_W_NONZERO_SUM: return "warning: total load not zero";
        case LFMM_E_INVAL: return "invalid argument";
        case LFMM_E_RANGE: return "out of range";
        case LFMM_E_NOMEM: return "out of memory";
        case LFMM_E_HIP: return "HIP runtime error";
        case LFMM_E_UNSUPPORTED: return "unsupported";
        case LFMM_E_NODEVICE: return "no such device";
        case LFMM_E_BUSY: return "not done yet";
    }
    return "unknown status";
}

const char* lfmm_last_error(void) { return g_last_error.c_str(); }

lfmm_status lfmm_host_phi(int32_t stencil, int64_t n, const int32_t* mxy, double* out) {
    if (n < 0 || (n > 0 && (!mxy || !out))) return fail(LFMM_E_INVAL, "lfmm_host_phi: bad arguments");
    if (stencil != LFMM_STENCIL_5 && stencil != LFMM_STENCIL_9) return fail(LFMM_E_INVAL, "unknown stencil");
    try {
        for (int64_t i = 0; i < n; ++i) out[i] = phi(stencil, mxy[2 * i], mxy[2 * i + 1]);
    } catch (const std::exception& e) {
        return fail(LFMM_E_NOMEM, e.what());
    }
    return LFMM_OK;
}

lfmm_status lfmm_host_opset_create(int64_t leaf_side, int32_t n_levels, const lfmm_options* opt,
                                   lfmm_opset** out) {
    if (!out) return fail(LFMM_E_INVAL, "null output");
    *out = nullptr;
    lfmm_options o;
    lfmm_options_init(&o);
    if (opt) o = *opt;
    lfmm_status st = validate_options(&o);
    if (st != LFMM_OK) return st;
    if (leaf_side < 1 || leaf_side > (int64_t(1) << 20) || (leaf_side & (leaf_side - 1)) != 0)
        return fail(LFMM_E_INVAL, "leaf_side must be a power of two in [1, 2^20]");
    if (leaf_side > kDenseLeafMax) return fail(LFMM_E_UNSUPPORTED, "leaf side above the dense-model limit");
    if (n_levels < 1 || n_levels > 31) return fail(LFMM_E_INVAL, "n_levels must lie in [1, 31]");
    try {
        auto* h = new lfmm_opset;
        h->ops = build_operators(leaf_side, n_levels, operator_params(o));
        *out = h;
    } catch (const std::bad_alloc&) {
        return fail(LFMM_E_NOMEM, "host allocation failed");
    } catch (const std::exception& e) {
        return fail(LFMM_E_INVAL, e.what());
    }
    return LFMM_OK;
}

lfmm_status lfmm_host_opset_level(const lfmm_opset* h, int32_t lev, int64_t* side, int32_t* rank) {
    if (!h || lev < 0 || lev >= h->ops.nlevels) return fail(LFMM_E_INVAL, "bad opset or height");
    if (side) *side = h->ops.level[size_t(lev)].side;
    if (rank) *rank = h->ops.level[size_t(lev)].rank;
    return LFMM_OK;
}

lfmm_status lfmm_host_opset_skeleton(const lfmm_opset* h, int32_t lev, int64_t* out) {
    if (!h || !out || lev < 0 || lev >= h->ops.nlevels) return fail(LFMM_E_INVAL, "bad opset or height");
    const auto& s = h->ops.level[size_t(lev)].skel;
    std::memcpy(out, s.data(), s.size() * sizeof(int64_t));
    return LFMM_OK;
}

lfmm_status lfmm_host_opset_ofo(const lfmm_opset* h, int32_t lev, int32_t c, double* out) {
    if (!h || !out || lev < 1 || lev >= h->ops.nlevels || c < 0 || c > 3)
        return fail(LFMM_E_INVAL, "bad opset, height or child");
    const Mat& T = h->ops.level[size_t(lev)].ofo[c];
    for (int i = 0; i < T.rows; ++i)
        for (int j = 0; j < T.cols; ++j) out[size_t(i) * T.cols + j] = T(i, j);
    return LFMM_OK;
}

lfmm_status lfmm_host_opset_leaf(const lfmm_opset* h, double* out) {
    if (!h || !out) return fail(LFMM_E_INVAL, "bad opset");
    if (!h->ops.leaf.dense) return fail(LFMM_E_UNSUPPORTED, "leaf operator is not dense");
    const Mat& T = h->ops.leaf.T;
    for (int i = 0; i < T.rows; ++i)
        for (int j = 0; j < T.cols; ++j) out[size_t(i) * T.cols + j] = T(i, j);
    return LFMM_OK;
}

lfmm_status lfmm_host_opset_destroy(lfmm_opset* h) {
    delete h;
    return LFMM_OK;
}

}  // extern "C"
