// panel_internal.hpp -- workspace layout and kernel entry declarations shared
// by the host library and the gfx950 kernels of the batched panel method.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/panel.h"

namespace panel {

// Per-airfoil record, written once by panel_workspace_init.
struct AirfoilMeta {
    int64_t a_off;      // element offset of the augmented system [M | rhs]
                        // (ld rows x (n1 + K) columns, column-major) in A64
                        // and, for the mixed path, in A32
    int64_t x_off;      // element offset of the K solutions (n1 each) in X
    int64_t s_off;      // offset of gamma / cp outputs: sum N_b' K_b'
    int32_t N;          // panels
    int32_t K;          // angles of attack
    int32_t n1;         // system order N + 1
    int32_t ld;         // leading dimension (n1 rounded up to 32)
    int32_t node_off;   // first node of the airfoil in xy
    int32_t alpha_off;  // first angle in alpha / cl
    int32_t panel_off;  // first panel in the geometry cache (node_off - b)
    int32_t piv_off;    // first pivot (sum n1_b')
};
static_assert(sizeof(AirfoilMeta) == 56, "meta layout");

// Geometry cached by the assembly for the forces / adjoint steps.
struct PanelGeom {
    double L, tx, ty, pad;
};

// Byte offsets of the workspace sections (all 256-byte aligned).
struct WsLayout {
    size_t meta, order, queue, flag, chord, alpha, geom, a64, a32, tg, x, piv, iters, total;
};

// Scalars copied with the metadata.
struct WsHeader {
    double vinf;
    int32_t B;
    int32_t precision;
    int32_t max_n1;
    int32_t pad;
};

// Device view of a workspace.
struct WsView {
    WsHeader *hdr;
    AirfoilMeta *meta;
    int32_t *order;     // airfoils by decreasing cost (LPT order)
    int32_t *queue;     // work-queue counters of the persistent factorisation
                        // (zero between launches; the last workgroup out resets them)
    int32_t *flag;      // per airfoil: 0 ok, -1 bad geometry (set by assembly)
    double *chord;      // per airfoil
    double *alpha;      // per angle
    PanelGeom *geom;    // per panel
    double *a64;        // FP64 systems (factored in place for PANEL_FP64)
    float *a32;         // FP32 systems (mixed path; factored in place)
    double *tg;         // tangential-velocity influence matrices (Hess-Smith; same offsets as a64)
    double *x;          // solutions
    int32_t *piv;       // pivots (0-based row exchanged at each step)
    int32_t *iters;     // refinement sweeps per airfoil
};

inline __host__ __device__ WsView ws_view(void *ws, const WsLayout &l) {
    char *b = static_cast<char *>(ws);
    WsView v;
    v.hdr = reinterpret_cast<WsHeader *>(b);
    v.meta = reinterpret_cast<AirfoilMeta *>(b + l.meta);
    v.order = reinterpret_cast<int32_t *>(b + l.order);
    v.queue = reinterpret_cast<int32_t *>(b + l.queue);
    v.flag = reinterpret_cast<int32_t *>(b + l.flag);
    v.chord = reinterpret_cast<double *>(b + l.chord);
    v.alpha = reinterpret_cast<double *>(b + l.alpha);
    v.geom = reinterpret_cast<PanelGeom *>(b + l.geom);
    v.a64 = reinterpret_cast<double *>(b + l.a64);
    v.a32 = l.a32 ? reinterpret_cast<float *>(b + l.a32) : nullptr;
    v.tg = l.tg ? reinterpret_cast<double *>(b + l.tg) : nullptr;
    v.x = reinterpret_cast<double *>(b + l.x);
    v.piv = reinterpret_cast<int32_t *>(b + l.piv);
    v.iters = reinterpret_cast<int32_t *>(b + l.iters);
    return v;
}

// Kernel launchers (each enqueues on `stream`, returns hipGetLastError()).
hipError_t launch_naca4(int32_t B, const int32_t *node_off, int32_t closed_te, const double *mpt,
                        double *xy, hipStream_t stream);
hipError_t launch_naca4_vjp(int32_t B, const int32_t *node_off, int32_t closed_te,
                            const double *mpt, const double *dxy, double *dmpt, hipStream_t stream);
hipError_t launch_assemble(const WsView &v, int32_t B, int32_t max_cols, int32_t mixed,
                           const double *xy, const double *alpha, const double *chord, double vinf,
                           hipStream_t stream);
// Systems of order up to PANEL_WAVE_MAX_N1 can be factored by one wavefront
// each (lu_wave.hip); larger ones by a workgroup each (lu.hip).  The plan
// puts the workgroup-kernel airfoils first in `order` (n_block of them, each
// group in LPT order).
constexpr int PANEL_WAVE_RMAX = 5;
constexpr int PANEL_WAVE_MAX_N1 = 64 * PANEL_WAVE_RMAX;
// persistent: one launch that pops both kinds of systems from the order
// (and refines each FP32 solution right after its factorisation); used when
// every workgroup-kernel system fits four wavefronts (n1 <= 768) and
// wg_waves != 8.  wg_waves: 4 or 8 wavefronts per workgroup-kernel system,
// 0 = eight when the batch has at most one airfoil per CU.
hipError_t launch_factor_solve(const WsView &v, int32_t B, int32_t n_block, int32_t max_n1_block,
                               int32_t mixed, double tol, int32_t max_iter, int32_t *info,
                               int32_t persistent, int32_t wg_waves, hipStream_t stream);
hipError_t launch_lu_wave(const WsView &v, int32_t first, int32_t count, int32_t mixed, int32_t *info,
                          hipStream_t stream);
hipError_t launch_refine_wave(const WsView &v, int32_t first, int32_t count, int32_t *info, double tol,
                              int32_t max_iter, hipStream_t stream);
hipError_t launch_forces(const WsView &v, int32_t B, int32_t max_k, double *gamma, double *cp,
                         double *cl, double *cl_p, hipStream_t stream);
// Viscous correction (viscous.hip): one wavefront per (airfoil, angle).
hipError_t launch_thwaites(const WsView &v, int32_t B, int32_t max_k, const double *gamma, const double *cl,
                           double re, double *cd, double *ld, int32_t *sep, hipStream_t stream);
// Hess-Smith formulation (assemble_hs.hip): assembly + Kutta row, and forces.
hipError_t launch_assemble_hs(const WsView &v, int32_t B, int32_t max_ld, int32_t mixed, const double *xy,
                              const double *alpha, const double *chord, double vinf, hipStream_t stream);
hipError_t launch_forces_hs(const WsView &v, int32_t B, int32_t max_k, double *gamma, double *cp, double *cl,
                            double *cl_p, hipStream_t stream);
hipError_t launch_math_eval(int32_t n, const double *x, const double *y, double *lg, double *at,
                            hipStream_t stream);
// ka < 0: one pass with cl cotangents for all angles; ka >= 0: angle ka
// only, with its cl and (dcp non-NULL) cp cotangents, added to dxy for ka > 0.
hipError_t launch_adjoint(const WsView &v, int32_t B, int32_t n_block, int32_t max_k, int32_t mixed,
                          const double *xy, const double *dcl, const double *dcp, double *dxy, int32_t *info,
                          hipStream_t stream);
hipError_t launch_adjoint_wave(const WsView &v, int32_t first, int32_t count, int32_t mixed, const double *xy,
                               const double *dcl, const double *dcp, int32_t ka, double *dxy, int32_t *info,
                               hipStream_t stream);
// Hess-Smith formulation: one workgroup per airfoil, all angles, cl and (dcp
// non-NULL) cp cotangents.
hipError_t launch_adjoint_hs(const WsView &v, int32_t B, int32_t mixed, const double *xy, const double *dcl,
                             const double *dcp, double *dxy, int32_t *info, hipStream_t stream);

// Genetic algorithm (ga.hip).  Small tables travel by value as kernel
// arguments.
struct GaContour {
    int32_t M, degree, G;
    int32_t gene_map[PANEL_GA_MAX_GENES];
    double tmpl[2 * PANEL_GA_MAX_CTRL];
};
struct GaOps {
    int32_t G, k;
    double p_sel, p_mut, sigma;
    double lo[PANEL_GA_MAX_GENES], hi[PANEL_GA_MAX_GENES];
};
hipError_t launch_bspline_nodes(const GaContour &c, int32_t B, int32_t N, const double *genome, double *xy,
                                hipStream_t stream);
hipError_t launch_ga_init(const GaOps &o, int32_t B, const double *u, double *genome, hipStream_t stream);
hipError_t launch_ga_fitness(const WsView &v, int32_t B, const double *ld, const int32_t *info, double *fitness,
                             hipStream_t stream);
hipError_t launch_ga_step(const GaOps &o, int32_t B, const double *fitness, const double *gin, const double *u,
                          double *gout, int32_t *trace, hipStream_t stream);
hipError_t launch_ga_record(int32_t B, int32_t G, const double *fitness, const double *genome, int32_t *counter,
                            int32_t max_gen, double *hist_fit, int32_t *hist_idx, double *best_fit,
                            double *best_genome, hipStream_t stream);

}  // namespace panel
