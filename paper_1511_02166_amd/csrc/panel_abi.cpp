// panel_abi.cpp -- host side of the C ABI declared in include/panel.h:
// argument validation (before any HIP call), plan metadata, workspace layout
// and kernel launches.  No device memory is allocated here.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "panel_internal.hpp"

using namespace panel;

// Workspace of panel_solve_noalloc: device memory the library owns, one copy
// per GPU (allocated when the code object is loaded on that device).  In host
// code `scratch` names a host-side stand-in, never the device memory: its
// address on each device comes from hipGetSymbolAddress (scratch_on_device).
static __device__ __align__(256) unsigned char scratch[PANEL_NOALLOC_MAX_BYTES];

struct panel_plan {
    int32_t B = 0;
    int32_t precision = 0;
    int32_t max_n1 = 0;
    int32_t max_k = 0;
    int32_t max_cols = 0;  // max over airfoils of n1 + K
    panel_tiling tiling{PANEL_WAVE_MAX_N1, 0, 0};  // wave_max_n1: largest order given to the one-wavefront LU
    int32_t n_block = 0;       // airfoils factored by the workgroup LU (first in order)
    int32_t max_n1_block = 0;  // their largest order
    // set when the wave limit changed after the last panel_workspace_init:
    // the airfoil order in the workspace no longer matches n_block
    mutable bool order_stale = false;
    std::vector<int32_t> node_off, alpha_off;
    std::vector<double> cost;  // LPT key: (2/3) n1^3 + 2 n1^2 K
    int32_t formulation = PANEL_STREAM_FUNCTION;
    int32_t max_ld = 0;
    int64_t a_total = 0;       // elements of one system section (all airfoils)
    int64_t x_total = 0, piv_total = 0;
    std::vector<char> blob;  // header | meta | order, copied by workspace_init
    WsLayout layout{};
};

namespace {

thread_local std::string g_last_error;

panel_status fail(panel_status s, const std::string &msg) {
    g_last_error = msg;
    return s;
}

panel_status ok() {
    g_last_error.clear();
    return PANEL_OK;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

bool aligned8(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

// Byte offsets of the workspace sections for the plan's batch, precision and
// formulation.
void compute_layout(panel_plan *p) {
    const int32_t B = p->B;
    WsLayout &l = p->layout;
    size_t off = align256(sizeof(WsHeader));
    l.meta = off;
    off = align256(off + sizeof(AirfoilMeta) * B);
    l.order = off;
    off = align256(off + sizeof(int32_t) * B);
    l.queue = off;   // inside the metadata copy: zero after panel_workspace_init
    off = align256(off + sizeof(int32_t) * 4);
    l.flag = off;
    off = align256(off + sizeof(int32_t) * B);
    l.chord = off;
    off = align256(off + sizeof(double) * B);
    l.alpha = off;
    off = align256(off + sizeof(double) * p->alpha_off[B]);
    l.geom = off;
    off = align256(off + sizeof(PanelGeom) * (size_t(p->node_off[B]) - B));
    l.a64 = off;
    off = align256(off + sizeof(double) * size_t(p->a_total));
    if (p->precision == PANEL_FP32_REFINE) {
        l.a32 = off;
        off = align256(off + sizeof(float) * size_t(p->a_total));
    } else {
        l.a32 = 0;
    }
    if (p->formulation == PANEL_HESS_SMITH) {
        l.tg = off;
        off = align256(off + sizeof(double) * size_t(p->a_total));
    } else {
        l.tg = 0;
    }
    l.x = off;
    off = align256(off + sizeof(double) * size_t(p->x_total));
    l.piv = off;
    off = align256(off + sizeof(int32_t) * size_t(p->piv_total));
    l.iters = off;
    off = align256(off + sizeof(int32_t) * B);
    l.total = off;
}

// Airfoils for the workgroup LU first, then those for the one-wavefront LU;
// each group by decreasing cost (longest processing time first), so the
// in-order dispatch of workgroups is an LPT list schedule within each launch.
void build_order(panel_plan *p) {
    const int32_t B = p->B;
    std::vector<int32_t> order(B);
    std::vector<char> big(B);
    p->n_block = 0;
    p->max_n1_block = 0;
    for (int32_t b = 0; b < B; ++b) {
        order[b] = b;
        const int32_t n1 = p->node_off[b + 1] - p->node_off[b];
        big[b] = n1 > p->tiling.wave_max_n1;
        if (big[b]) {
            ++p->n_block;
            p->max_n1_block = std::max(p->max_n1_block, n1);
        }
    }
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t c) {
        if (big[a] != big[c]) return big[a] > big[c];
        return p->cost[a] > p->cost[c];
    });
    std::memcpy(p->blob.data() + p->layout.order, order.data(), sizeof(int32_t) * B);
}

panel_status check_hip(hipError_t e, const char *what) {
    if (e != hipSuccess)
        return fail(PANEL_EHIP, std::string(what) + ": " + hipGetErrorString(e));
    return ok();
}

// Device address of the current device's copy of `scratch`, looked up once
// per device (with that device current) and kept.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

panel_status scratch_on_device(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return check_hip(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(PANEL_EUNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return check_hip(e, "hipGetSymbolAddress(scratch)");
        if (!p || (reinterpret_cast<uintptr_t>(p) & 255u))
            return fail(PANEL_EHIP, "static scratch has no 256-byte aligned device address");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return ok();
}

}  // namespace

extern "C" {

const char *panel_status_str(int32_t s) {
    switch (s) {
        case PANEL_OK: return "PANEL_OK";
        case PANEL_EINVAL: return "PANEL_EINVAL: invalid argument";
        case PANEL_ENOMEM: return "PANEL_ENOMEM: host allocation failed";
        case PANEL_EHIP: return "PANEL_EHIP: HIP runtime error";
        case PANEL_EUNSUPPORTED: return "PANEL_EUNSUPPORTED: unsupported request";
        default: return "unknown panel_status";
    }
}

const char *panel_last_error(void) { return g_last_error.c_str(); }

panel_status panel_plan_create(int32_t B, const int32_t *h_node_offsets,
                               const int32_t *h_alpha_offsets, int32_t precision,
                               panel_plan **out) {
    if (!out) return fail(PANEL_EINVAL, "out is NULL");
    *out = nullptr;
    if (B < 1) return fail(PANEL_EINVAL, "B must be >= 1");
    if (!h_node_offsets || !h_alpha_offsets) return fail(PANEL_EINVAL, "offset array is NULL");
    if (precision != PANEL_FP64 && precision != PANEL_FP32_REFINE)
        return fail(PANEL_EINVAL, "unknown precision");
    if (h_node_offsets[0] != 0 || h_alpha_offsets[0] != 0)
        return fail(PANEL_EINVAL, "offsets must start at 0");
    for (int32_t b = 0; b < B; ++b) {
        int64_t n = int64_t(h_node_offsets[b + 1]) - h_node_offsets[b];
        int64_t k = int64_t(h_alpha_offsets[b + 1]) - h_alpha_offsets[b];
        if (n - 1 < PANEL_NMIN || n - 1 > PANEL_NMAX) {
            char buf[160];
            std::snprintf(buf, sizeof buf, "airfoil %d has %lld panels (allowed %d..%d)", b,
                          (long long)(n - 1), PANEL_NMIN, PANEL_NMAX);
            return fail(PANEL_EINVAL, buf);
        }
        if (k < 1 || k > PANEL_KMAX) {
            char buf[160];
            std::snprintf(buf, sizeof buf, "airfoil %d has %lld angles (allowed 1..%d)", b,
                          (long long)k, PANEL_KMAX);
            return fail(PANEL_EINVAL, buf);
        }
    }
    panel_plan *p = new (std::nothrow) panel_plan;
    if (!p) return fail(PANEL_ENOMEM, "plan allocation");
    try {
        p->B = B;
        p->precision = precision;
        p->node_off.assign(h_node_offsets, h_node_offsets + B + 1);
        p->alpha_off.assign(h_alpha_offsets, h_alpha_offsets + B + 1);
        std::vector<AirfoilMeta> meta(B);
        int64_t a_off = 0, x_off = 0, s_off = 0, piv_off = 0;
        std::vector<double> &cost = p->cost;
        cost.assign(B, 0.0);
        for (int32_t b = 0; b < B; ++b) {
            AirfoilMeta &m = meta[b];
            m.N = h_node_offsets[b + 1] - h_node_offsets[b] - 1;
            m.K = h_alpha_offsets[b + 1] - h_alpha_offsets[b];
            m.n1 = m.N + 1;
            m.ld = (m.n1 + 31) & ~31;
            m.node_off = h_node_offsets[b];
            m.alpha_off = h_alpha_offsets[b];
            m.panel_off = h_node_offsets[b] - b;
            m.a_off = a_off;
            m.x_off = x_off;
            m.s_off = s_off;
            m.piv_off = int32_t(piv_off);
            // keep every system 128-byte aligned in both precisions
            a_off += (int64_t(m.ld) * (m.n1 + m.K) + 31) & ~int64_t(31);
            x_off += int64_t(m.n1) * m.K;
            s_off += int64_t(m.N) * m.K;
            piv_off += m.n1;
            p->max_n1 = std::max(p->max_n1, m.n1);
            p->max_k = std::max(p->max_k, m.K);
            p->max_cols = std::max(p->max_cols, m.n1 + m.K);
            p->max_ld = std::max(p->max_ld, m.ld);
            double n = m.n1;
            cost[b] = n * n * n / 1.5 + 2.0 * n * n * m.K;
        }
        p->a_total = a_off;
        p->x_total = x_off;
        p->piv_total = piv_off;
        compute_layout(p);
        WsHeader hdr{};
        hdr.vinf = 1.0;
        hdr.B = B;
        hdr.precision = precision;
        hdr.max_n1 = p->max_n1;
        const WsLayout &l = p->layout;
        p->blob.assign(l.flag, 0);
        std::memcpy(p->blob.data(), &hdr, sizeof hdr);
        std::memcpy(p->blob.data() + l.meta, meta.data(), sizeof(AirfoilMeta) * B);
        build_order(p);
    } catch (const std::bad_alloc &) {
        delete p;
        return fail(PANEL_ENOMEM, "plan metadata allocation");
    }
    *out = p;
    return ok();
}

void panel_plan_destroy(panel_plan *plan) { delete plan; }

panel_status panel_plan_set_wave_limit(panel_plan *plan, int32_t max_n1) {
    if (!plan) return fail(PANEL_EINVAL, "NULL plan");
    if (max_n1 < 0 || max_n1 > PANEL_WAVE_MAX_N1) {
        char buf[120];
        std::snprintf(buf, sizeof buf, "wave limit must be in 0..%d", PANEL_WAVE_MAX_N1);
        return fail(PANEL_EINVAL, buf);
    }
    if (max_n1 != plan->tiling.wave_max_n1) {
        plan->tiling.wave_max_n1 = max_n1;
        build_order(plan);
        plan->order_stale = true;
    }
    return ok();
}

panel_status panel_plan_set_tiling(panel_plan *plan, const panel_tiling *t) {
    if (!plan || !t) return fail(PANEL_EINVAL, "NULL argument");
    if (t->persistent != 0 && t->persistent != 1) return fail(PANEL_EINVAL, "persistent must be 0 or 1");
    if (t->wg_waves != 0 && t->wg_waves != 4 && t->wg_waves != 8)
        return fail(PANEL_EINVAL, "wg_waves must be 0, 4 or 8");
    panel_status st = panel_plan_set_wave_limit(plan, t->wave_max_n1);
    if (st != PANEL_OK) return st;
    plan->tiling.persistent = t->persistent;
    plan->tiling.wg_waves = t->wg_waves;
    return ok();
}

panel_status panel_plan_set_formulation(panel_plan *plan, int32_t formulation) {
    if (!plan) return fail(PANEL_EINVAL, "NULL plan");
    if (formulation != PANEL_STREAM_FUNCTION && formulation != PANEL_HESS_SMITH)
        return fail(PANEL_EINVAL, "unknown formulation");
    plan->formulation = formulation;
    compute_layout(plan);
    return ok();
}

panel_status panel_plan_get_tiling(const panel_plan *plan, panel_tiling *t) {
    if (!plan || !t) return fail(PANEL_EINVAL, "NULL argument");
    *t = plan->tiling;
    return ok();
}

panel_status panel_workspace_layout(const panel_plan *plan, int32_t b, int64_t *h_desc) {
    if (!plan || !h_desc) return fail(PANEL_EINVAL, "NULL argument");
    if (b < 0 || b >= plan->B) return fail(PANEL_EINVAL, "airfoil index out of range");
    AirfoilMeta m;
    std::memcpy(&m, plan->blob.data() + plan->layout.meta + sizeof(AirfoilMeta) * b, sizeof m);
    const WsLayout &l = plan->layout;
    h_desc[0] = int64_t(l.a64 + sizeof(double) * m.a_off);
    h_desc[1] = l.a32 ? int64_t(l.a32 + sizeof(float) * m.a_off) : -1;
    h_desc[2] = int64_t(l.x + sizeof(double) * m.x_off);
    h_desc[3] = int64_t(l.piv + sizeof(int32_t) * m.piv_off);
    h_desc[4] = m.n1;
    h_desc[5] = m.ld;
    h_desc[6] = m.K;
    h_desc[7] = int64_t(l.iters + sizeof(int32_t) * b);
    h_desc[8] = l.tg ? int64_t(l.tg + sizeof(double) * m.a_off) : -1;
    return ok();
}

panel_status panel_workspace_size(const panel_plan *plan, size_t *bytes) {
    if (!plan || !bytes) return fail(PANEL_EINVAL, "NULL argument");
    *bytes = plan->layout.total;
    return ok();
}

panel_status panel_workspace_init(const panel_plan *plan, void *ws, void *stream) {
    if (!plan || !ws) return fail(PANEL_EINVAL, "NULL argument");
    if (reinterpret_cast<uintptr_t>(ws) & 255u) return fail(PANEL_EINVAL, "workspace must be 256-byte aligned");
    hipError_t e = hipMemcpyAsync(ws, plan->blob.data(), plan->blob.size(), hipMemcpyHostToDevice,
                                  static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return check_hip(e, "workspace metadata copy");
    // The source is pageable host memory owned by the plan; make the copy
    // complete before returning so the plan may be destroyed at any time.
    e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e == hipSuccess) plan->order_stale = false;
    return check_hip(e, "workspace metadata copy");
}

panel_status panel_assemble(const panel_plan *plan, const double *xy, const double *alpha,
                            const double *chord, double vinf, void *ws, void *stream) {
    if (!plan || !xy || !alpha || !ws) return fail(PANEL_EINVAL, "NULL argument");
    if (!aligned8(xy) || !aligned8(alpha) || (chord && !aligned8(chord)))
        return fail(PANEL_EINVAL, "arrays must be 8-byte aligned");
    if (reinterpret_cast<uintptr_t>(ws) & 255u) return fail(PANEL_EINVAL, "workspace must be 256-byte aligned");
    if (!(std::isfinite(vinf) && vinf > 0.0)) return fail(PANEL_EINVAL, "vinf must be finite and > 0");
    WsView v = ws_view(ws, plan->layout);
    const bool mixed = plan->precision == PANEL_FP32_REFINE;
    hipError_t e = plan->formulation == PANEL_HESS_SMITH
                       ? launch_assemble_hs(v, plan->B, plan->max_ld, mixed, xy, alpha, chord, vinf,
                                            static_cast<hipStream_t>(stream))
                       : launch_assemble(v, plan->B, plan->max_cols, mixed, xy, alpha, chord, vinf,
                                         static_cast<hipStream_t>(stream));
    return check_hip(e, "assembly launch");
}

panel_status panel_factor_solve(const panel_plan *plan, void *ws, double refine_tol,
                                int32_t max_iter, int32_t *info, void *stream) {
    if (!plan || !ws || !info) return fail(PANEL_EINVAL, "NULL argument");
    if (reinterpret_cast<uintptr_t>(ws) & 255u) return fail(PANEL_EINVAL, "workspace must be 256-byte aligned");
    const bool mixed = plan->precision == PANEL_FP32_REFINE;
    if (mixed) {
        if (!(std::isfinite(refine_tol) && refine_tol > 0.0))
            return fail(PANEL_EINVAL, "refine_tol must be finite and > 0");
        if (max_iter < 0 || max_iter > 100) return fail(PANEL_EINVAL, "max_iter must be in 0..100");
    }
    if (plan->order_stale)
        return fail(PANEL_EINVAL, "wave limit changed: call panel_workspace_init before factoring");
    WsView v = ws_view(ws, plan->layout);
    hipError_t e = launch_factor_solve(v, plan->B, plan->n_block, plan->max_n1_block, mixed, refine_tol,
                                       max_iter, info, plan->tiling.persistent, plan->tiling.wg_waves,
                                       static_cast<hipStream_t>(stream));
    return check_hip(e, "factor/solve launch");
}

panel_status panel_forces(const panel_plan *plan, const void *ws, double *gamma, double *cp,
                          double *cl, double *cl_p, void *stream) {
    if (!plan || !ws || !cl) return fail(PANEL_EINVAL, "NULL argument");
    if ((gamma && !aligned8(gamma)) || (cp && !aligned8(cp)) || !aligned8(cl) || (cl_p && !aligned8(cl_p)))
        return fail(PANEL_EINVAL, "arrays must be 8-byte aligned");
    WsView v = ws_view(const_cast<void *>(ws), plan->layout);
    hipError_t e = plan->formulation == PANEL_HESS_SMITH
                       ? launch_forces_hs(v, plan->B, plan->max_k, gamma, cp, cl, cl_p, static_cast<hipStream_t>(stream))
                       : launch_forces(v, plan->B, plan->max_k, gamma, cp, cl, cl_p, static_cast<hipStream_t>(stream));
    return check_hip(e, "forces launch");
}

panel_status panel_thwaites(const panel_plan *plan, const void *ws, const double *gamma, const double *cl,
                            double re, double *cd, double *ld, int32_t *sep, void *stream) {
    if (!plan || !ws || !gamma || !cl || !cd || !ld || !sep) return fail(PANEL_EINVAL, "NULL argument");
    if (!aligned8(gamma) || !aligned8(cl) || !aligned8(cd) || !aligned8(ld) || (reinterpret_cast<uintptr_t>(sep) & 3u))
        return fail(PANEL_EINVAL, "arrays must be aligned (8 bytes; sep 4 bytes)");
    if (!(std::isfinite(re) && re > 0.0)) return fail(PANEL_EINVAL, "re must be finite and > 0");
    WsView v = ws_view(const_cast<void *>(ws), plan->layout);
    hipError_t e = launch_thwaites(v, plan->B, plan->max_k, gamma, cl, re, cd, ld, sep,
                                   static_cast<hipStream_t>(stream));
    return check_hip(e, "viscous correction launch");
}

panel_status panel_adjoint(const panel_plan *plan, const void *ws, const double *xy,
                           const double *dcl, const double *dcp, double *dxy, int32_t *info,
                           void *stream) {
    if (!plan || !ws || !xy || !dcl || !dxy) return fail(PANEL_EINVAL, "NULL argument");
    if (!aligned8(xy) || !aligned8(dcl) || !aligned8(dxy) || (dcp && !aligned8(dcp)) ||
        (reinterpret_cast<uintptr_t>(info) & 3u))
        return fail(PANEL_EINVAL, "arrays must be aligned (8 bytes; info 4 bytes)");
    if (reinterpret_cast<uintptr_t>(ws) & 255u) return fail(PANEL_EINVAL, "workspace must be 256-byte aligned");
    if (plan->order_stale)
        return fail(PANEL_EINVAL, "wave limit changed: call panel_workspace_init (and refactor) first");
    WsView v = ws_view(const_cast<void *>(ws), plan->layout);
    const int32_t mixed = plan->precision == PANEL_FP32_REFINE;
    hipError_t e = plan->formulation == PANEL_HESS_SMITH
                       ? launch_adjoint_hs(v, plan->B, mixed, xy, dcl, dcp, dxy, info, static_cast<hipStream_t>(stream))
                       : launch_adjoint(v, plan->B, plan->n_block, plan->max_k, mixed, xy, dcl, dcp, dxy, info,
                                        static_cast<hipStream_t>(stream));
    return check_hip(e, "adjoint launch");
}

panel_status panel_solve_noalloc(const panel_plan *plan, const double *xy, const double *alpha,
                                 const double *chord, double vinf, double refine_tol, int32_t max_iter,
                                 int32_t *info, double *gamma, double *cp, double *cl, double *cl_p,
                                 void *stream) {
    if (!plan || !xy || !alpha || !info || !cl) return fail(PANEL_EINVAL, "NULL argument");
    if (!aligned8(xy) || !aligned8(alpha) || (chord && !aligned8(chord)) || (gamma && !aligned8(gamma)) ||
        (cp && !aligned8(cp)) || !aligned8(cl) || (cl_p && !aligned8(cl_p)) ||
        (reinterpret_cast<uintptr_t>(info) & 3u))
        return fail(PANEL_EINVAL, "arrays must be aligned (8 bytes; info 4 bytes)");
    if (!(std::isfinite(vinf) && vinf > 0.0)) return fail(PANEL_EINVAL, "vinf must be finite and > 0");
    const bool mixed = plan->precision == PANEL_FP32_REFINE;
    if (mixed) {
        if (!(std::isfinite(refine_tol) && refine_tol > 0.0))
            return fail(PANEL_EINVAL, "refine_tol must be finite and > 0");
        if (max_iter < 0 || max_iter > 100) return fail(PANEL_EINVAL, "max_iter must be in 0..100");
    }
    if (plan->layout.total > PANEL_NOALLOC_MAX_BYTES) {
        char buf[200];
        std::snprintf(buf, sizeof buf, "plan needs %zu bytes of workspace; the static scratch holds %zu",
                      plan->layout.total, (size_t)PANEL_NOALLOC_MAX_BYTES);
        return fail(PANEL_EINVAL, buf);
    }
    void *ws = nullptr;
    panel_status st = scratch_on_device(&ws);
    if (st != PANEL_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // the metadata of this plan (its current airfoil order included), then
    // the same launches as the caller-owned workspace path
    hipError_t e = hipMemcpyAsync(ws, plan->blob.data(), plan->blob.size(), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return check_hip(e, "scratch metadata copy");
    WsView v = ws_view(ws, plan->layout);
    e = plan->formulation == PANEL_HESS_SMITH
            ? launch_assemble_hs(v, plan->B, plan->max_ld, mixed, xy, alpha, chord, vinf, s)
            : launch_assemble(v, plan->B, plan->max_cols, mixed, xy, alpha, chord, vinf, s);
    if (e != hipSuccess) return check_hip(e, "assembly launch");
    e = launch_factor_solve(v, plan->B, plan->n_block, plan->max_n1_block, mixed, refine_tol, max_iter, info,
                            plan->tiling.persistent, plan->tiling.wg_waves, s);
    if (e != hipSuccess) return check_hip(e, "factor/solve launch");
    e = plan->formulation == PANEL_HESS_SMITH ? launch_forces_hs(v, plan->B, plan->max_k, gamma, cp, cl, cl_p, s)
                                              : launch_forces(v, plan->B, plan->max_k, gamma, cp, cl, cl_p, s);
    return check_hip(e, "forces launch");
}

panel_status panel_naca4(int32_t B, const int32_t *node_off, int32_t closed_te, const double *mpt,
                         double *xy, void *stream) {
    if (B < 1) return fail(PANEL_EINVAL, "B must be >= 1");
    if (!node_off || !mpt || !xy) return fail(PANEL_EINVAL, "NULL argument");
    if (!aligned8(mpt) || !aligned8(xy)) return fail(PANEL_EINVAL, "arrays must be 8-byte aligned");
    hipError_t e = launch_naca4(B, node_off, closed_te, mpt, xy, static_cast<hipStream_t>(stream));
    return check_hip(e, "naca4 launch");
}

panel_status panel_naca4_vjp(int32_t B, const int32_t *node_off, int32_t closed_te,
                             const double *mpt, const double *dxy, double *dmpt, void *stream) {
    if (B < 1) return fail(PANEL_EINVAL, "B must be >= 1");
    if (!node_off || !mpt || !dxy || !dmpt) return fail(PANEL_EINVAL, "NULL argument");
    if (!aligned8(mpt) || !aligned8(dxy) || !aligned8(dmpt))
        return fail(PANEL_EINVAL, "arrays must be 8-byte aligned");
    hipError_t e = launch_naca4_vjp(B, node_off, closed_te, mpt, dxy, dmpt, static_cast<hipStream_t>(stream));
    return check_hip(e, "naca4 vjp launch");
}

// ---- genetic algorithm ---------------------------------------------------------

static panel_status ga_bounds(int32_t G, const double *lo, const double *hi, GaOps *o) {
    if (!lo || !hi) return fail(PANEL_EINVAL, "NULL bounds");
    for (int g = 0; g < G; ++g) {
        if (!(std::isfinite(lo[g]) && std::isfinite(hi[g]) && lo[g] <= hi[g]))
            return fail(PANEL_EINVAL, "bounds must be finite with lo <= hi");
        o->lo[g] = lo[g];
        o->hi[g] = hi[g];
    }
    return ok();
}

panel_status panel_bspline_nodes(int32_t B, int32_t N, int32_t M, int32_t degree, const double *h_template,
                                 int32_t G, const int32_t *h_gene_map, const double *genome, double *xy,
                                 void *stream) {
    if (B < 1) return fail(PANEL_EINVAL, "B must be >= 1");
    if (N < PANEL_NMIN || N > PANEL_NMAX || (N & 1)) return fail(PANEL_EINVAL, "N must be even, NMIN..NMAX");
    if (degree < 1 || degree > PANEL_GA_MAX_DEGREE) return fail(PANEL_EINVAL, "degree must be 1..PANEL_GA_MAX_DEGREE");
    if (M < degree + 1 || M > PANEL_GA_MAX_CTRL) return fail(PANEL_EINVAL, "need degree + 1 <= M <= PANEL_GA_MAX_CTRL");
    if (G < 0 || G > PANEL_GA_MAX_GENES) return fail(PANEL_EINVAL, "G must be 0..PANEL_GA_MAX_GENES");
    if (!h_template || (G > 0 && (!h_gene_map || !genome)) || !xy) return fail(PANEL_EINVAL, "NULL argument");
    if ((genome && !aligned8(genome)) || !aligned8(xy)) return fail(PANEL_EINVAL, "arrays must be 8-byte aligned");
    GaContour c{};
    c.M = M;
    c.degree = degree;
    c.G = G;
    for (int i = 0; i < 2 * M; ++i) {
        if (!std::isfinite(h_template[i])) return fail(PANEL_EINVAL, "template must be finite");
        c.tmpl[i] = h_template[i];
    }
    if (h_template[0] != h_template[2 * M - 2] || h_template[1] != h_template[2 * M - 1])
        return fail(PANEL_EINVAL, "first and last control points must coincide (the trailing edge)");
    bool used[2 * PANEL_GA_MAX_CTRL] = {};
    for (int g = 0; g < G; ++g) {
        const int32_t t = h_gene_map[g];
        if (t < 2 || t >= 2 * M - 2) return fail(PANEL_EINVAL, "gene_map entries must lie in [2, 2M - 2)");
        if (used[t]) return fail(PANEL_EINVAL, "gene_map entries must be distinct");
        used[t] = true;
        c.gene_map[g] = t;
    }
    hipError_t e = launch_bspline_nodes(c, B, N, genome, xy, static_cast<hipStream_t>(stream));
    return check_hip(e, "B-spline nodes launch");
}

panel_status panel_ga_init(int32_t B, int32_t G, const double *h_lo, const double *h_hi, const double *u,
                           double *genome, void *stream) {
    if (B < 1) return fail(PANEL_EINVAL, "B must be >= 1");
    if (G < 1 || G > PANEL_GA_MAX_GENES) return fail(PANEL_EINVAL, "G must be 1..PANEL_GA_MAX_GENES");
    if (!u || !genome) return fail(PANEL_EINVAL, "NULL argument");
    if (!aligned8(u) || !aligned8(genome)) return fail(PANEL_EINVAL, "arrays must be 8-byte aligned");
    GaOps o{};
    o.G = G;
    panel_status st = ga_bounds(G, h_lo, h_hi, &o);
    if (st != PANEL_OK) return st;
    hipError_t e = launch_ga_init(o, B, u, genome, static_cast<hipStream_t>(stream));
    return check_hip(e, "GA init launch");
}

panel_status panel_ga_fitness(const panel_plan *plan, const void *ws, const double *ld, const int32_t *info,
                              double *fitness, void *stream) {
    if (!plan || !ws || !ld || !info || !fitness) return fail(PANEL_EINVAL, "NULL argument");
    if (!aligned8(ld) || !aligned8(fitness) || (reinterpret_cast<uintptr_t>(info) & 3u))
        return fail(PANEL_EINVAL, "arrays must be aligned (8 bytes; info 4 bytes)");
    if (reinterpret_cast<uintptr_t>(ws) & 255u) return fail(PANEL_EINVAL, "workspace must be 256-byte aligned");
    WsView v = ws_view(const_cast<void *>(ws), plan->layout);
    hipError_t e = launch_ga_fitness(v, plan->B, ld, info, fitness, static_cast<hipStream_t>(stream));
    return check_hip(e, "GA fitness launch");
}

panel_status panel_ga_uniform_count(int32_t B, int32_t k, int64_t *count) {
    if (!count) return fail(PANEL_EINVAL, "NULL argument");
    if (B < 2 || (B & 1)) return fail(PANEL_EINVAL, "B must be even and >= 2");
    if (k < 1 || k > PANEL_GA_MAX_TOURNAMENT) return fail(PANEL_EINVAL, "k must be 1..PANEL_GA_MAX_TOURNAMENT");
    *count = (int64_t)(B / 2) * (4 * k - 1) + 3 * (int64_t)B;
    return ok();
}

panel_status panel_ga_step(int32_t B, int32_t G, int32_t k, double p_sel, double p_mut, double sigma,
                           const double *h_lo, const double *h_hi, const double *fitness,
                           const double *genome_in, const double *u, double *genome_out, int32_t *trace,
                           void *stream) {
    if (B < 2 || (B & 1)) return fail(PANEL_EINVAL, "B must be even and >= 2");
    if (G < 2 || G > PANEL_GA_MAX_GENES) return fail(PANEL_EINVAL, "G must be 2..PANEL_GA_MAX_GENES");
    if (k < 1 || k > PANEL_GA_MAX_TOURNAMENT) return fail(PANEL_EINVAL, "k must be 1..PANEL_GA_MAX_TOURNAMENT");
    if (!(p_sel > 0.0 && p_sel <= 1.0)) return fail(PANEL_EINVAL, "p_sel must be in (0, 1]");
    if (!(p_mut >= 0.0 && p_mut <= 1.0)) return fail(PANEL_EINVAL, "p_mut must be in [0, 1]");
    if (!(std::isfinite(sigma) && sigma >= 0.0)) return fail(PANEL_EINVAL, "sigma must be finite and >= 0");
    if (!fitness || !genome_in || !u || !genome_out) return fail(PANEL_EINVAL, "NULL argument");
    if (genome_in == genome_out) return fail(PANEL_EINVAL, "genome_in and genome_out must differ");
    if (!aligned8(fitness) || !aligned8(genome_in) || !aligned8(u) || !aligned8(genome_out) ||
        (reinterpret_cast<uintptr_t>(trace) & 3u))
        return fail(PANEL_EINVAL, "arrays must be aligned (8 bytes; trace 4 bytes)");
    GaOps o{};
    o.G = G;
    o.k = k;
    o.p_sel = p_sel;
    o.p_mut = p_mut;
    o.sigma = sigma;
    panel_status st = ga_bounds(G, h_lo, h_hi, &o);
    if (st != PANEL_OK) return st;
    hipError_t e = launch_ga_step(o, B, fitness, genome_in, u, genome_out, trace, static_cast<hipStream_t>(stream));
    return check_hip(e, "GA step launch");
}

panel_status panel_ga_record(int32_t B, int32_t G, const double *fitness, const double *genome,
                             int32_t *counter, int32_t max_gen, double *hist_fit, int32_t *hist_idx,
                             double *best_fit, double *best_genome, void *stream) {
    if (B < 1) return fail(PANEL_EINVAL, "B must be >= 1");
    if (G < 1 || G > PANEL_GA_MAX_GENES) return fail(PANEL_EINVAL, "G must be 1..PANEL_GA_MAX_GENES");
    if (max_gen < 0) return fail(PANEL_EINVAL, "max_gen must be >= 0");
    if (!fitness || !genome || !counter || !best_fit || !best_genome || (max_gen > 0 && (!hist_fit || !hist_idx)))
        return fail(PANEL_EINVAL, "NULL argument");
    if (!aligned8(fitness) || !aligned8(genome) || !aligned8(best_fit) || !aligned8(best_genome) ||
        (hist_fit && !aligned8(hist_fit)) || (reinterpret_cast<uintptr_t>(counter) & 3u) ||
        (reinterpret_cast<uintptr_t>(hist_idx) & 3u))
        return fail(PANEL_EINVAL, "arrays must be aligned (8 bytes; int32 4 bytes)");
    hipError_t e = launch_ga_record(B, G, fitness, genome, counter, max_gen, hist_fit, hist_idx, best_fit,
                                    best_genome, static_cast<hipStream_t>(stream));
    return check_hip(e, "GA record launch");
}

panel_status panel_math_eval(int32_t n, const double *x, const double *y, double *log_out,
                             double *atan2_out, void *stream) {
    if (n < 0) return fail(PANEL_EINVAL, "n must be >= 0");
    if (n == 0) return ok();
    if (!x || (atan2_out && !y) || (!log_out && !atan2_out)) return fail(PANEL_EINVAL, "NULL argument");
    if (!aligned8(x) || (y && !aligned8(y)) || (log_out && !aligned8(log_out)) || (atan2_out && !aligned8(atan2_out)))
        return fail(PANEL_EINVAL, "arrays must be 8-byte aligned");
    hipError_t e = launch_math_eval(n, x, y, log_out, atan2_out, static_cast<hipStream_t>(stream));
    return check_hip(e, "math eval launch");
}

}  // extern "C"
