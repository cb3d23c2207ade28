/*
 * panel.h -- C ABI of the batched 2-D panel-method library for AMD MI355X
 * (gfx950).  Reference method: Einkemmer, arXiv:1511.02166, Sec. 2
 * ("Numerical algorithm") and Sec. 3 (assembly O(n^2) with logarithms and
 * arctangents, LU (2/3)n^3).
 *
 * A batch holds B airfoils.  Airfoil b has N_b panels between N_b + 1 nodes
 * P_0..P_N (trailing edge first, counter-clockwise: upper surface, leading
 * edge, lower surface; P_N = P_0 for a closed section) and K_b angles of
 * attack.  For each airfoil the library assembles the bordered
 * (N_b + 1) x (N_b + 1) system of Sec. 2
 *     sum_i G_ji gamma_i - C = -phi_v(m_j)      (j < N_b, midpoints m_j)
 *     gamma_0 + gamma_{N_b - 1} = 0              (Kutta condition)
 * with G_ji the integral of -(1/2pi) log|m_j - s| over panel i, factors it
 * once by LU with partial pivoting, solves it for the K_b right-hand sides
 * phi_v = vinf (y cos alpha - x sin alpha), and reduces the surface speed
 * gamma_i, Cp_i = 1 - (gamma_i / vinf)^2 and the lift coefficient.
 *
 * Conventions for every entry point:
 *  - Array arguments are DEVICE pointers unless the name starts with h_.
 *    Every floating-point array is IEEE double, 8-byte aligned.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls that take a stream only enqueue work on it: they never
 *    synchronise the device and never allocate device memory, so the
 *    sequence assemble -> factor_solve -> forces (and adjoint) may be
 *    captured into a HIP graph.  The one exception is
 *    panel_workspace_init, a host-to-device copy of the plan's metadata
 *    that returns only once the copy is complete (so the plan may be
 *    destroyed right after it); it is not meant for graph capture.
 *  - The caller owns all device memory, including the workspace, whose size
 *    panel_workspace_size reports.  The library keeps no device pointers
 *    between calls.  A plan owns host memory only.
 *  - Return value: PANEL_OK, or an error code.  Argument checks run on the
 *    host before any HIP call; on failure nothing is enqueued and
 *    panel_last_error() (thread-local) describes the problem.
 *  - Per-airfoil outcomes are reported on the device in info[b]:
 *       0   success
 *       k>0 exact zero pivot in column k (1-based, LAPACK getrf convention);
 *           that airfoil's outputs are NaN
 *      -1   non-finite node coordinate or zero-length panel; outputs NaN
 *      -2   mixed precision: refinement did not reach the tolerance within
 *           max_iter sweeps (the last iterate is returned)
 *      -3   the workspace's airfoil order sends a system to a kernel that
 *           cannot hold it (the plan changed after panel_workspace_init);
 *           outputs NaN
 */
#ifndef PANEL_H
#define PANEL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PANEL_OK = 0,
    PANEL_EINVAL = 1,       /* bad argument (reported before any HIP call)  */
    PANEL_ENOMEM = 2,       /* host allocation failed                        */
    PANEL_EHIP = 3,         /* a HIP runtime call or kernel launch failed    */
    PANEL_EUNSUPPORTED = 4  /* valid request this build does not support     */
} panel_status;

typedef enum {
    PANEL_FP64 = 0,         /* FP64 assembly, FP64 LU and solve              */
    PANEL_FP32_REFINE = 1   /* FP64 assembly; FP32 LU; FP64 residual-based
                               iterative refinement of the solution          */
} panel_precision;

typedef enum {
    PANEL_STREAM_FUNCTION = 0,  /* Sec. 2: constant-density vortex sheet on each
                                   panel, stream function constant on the
                                   contour, Kutta row gamma_0 + gamma_{N-1} = 0 */
    PANEL_HESS_SMITH = 1        /* constant source density per panel plus one
                                   vortex density shared by all panels, flow
                                   tangency at the midpoints, Kutta row: equal
                                   and opposite tangential speeds on the two
                                   trailing-edge panels                         */
} panel_formulation;

/* Largest supported panel count per airfoil. */
#define PANEL_NMAX 1024
/* Smallest supported panel count per airfoil. */
#define PANEL_NMIN 4
/* Largest supported number of angles of attack per airfoil. */
#define PANEL_KMAX 16

typedef struct panel_plan panel_plan;

/* Create a plan for a batch (host metadata only; no HIP call).
 *   B                 number of airfoils, B >= 1
 *   h_node_offsets    host int32[B+1], nondecreasing, [0] = 0; airfoil b owns
 *                     nodes h_node_offsets[b] .. h_node_offsets[b+1]-1, i.e.
 *                     N_b = diff - 1 panels, PANEL_NMIN <= N_b <= PANEL_NMAX
 *   h_alpha_offsets   host int32[B+1], [0] = 0; K_b = diff,
 *                     1 <= K_b <= PANEL_KMAX
 *   precision         a panel_precision value
 *   out               receives the plan (release with panel_plan_destroy)
 * The offsets are copied; the caller may free them afterwards.            */
panel_status panel_plan_create(int32_t B, const int32_t *h_node_offsets,
                               const int32_t *h_alpha_offsets, int32_t precision,
                               panel_plan **out);

/* Release a plan (NULL is ignored). */
void panel_plan_destroy(panel_plan *plan);

/* Choose the LU kernel by system order (Sec. 3: many independent dense
 * factorisations).  Systems with n1 = N_b + 1 <= max_n1 are factored by one
 * wavefront each; larger ones by a workgroup of four wavefronts each.
 *   max_n1   0 .. 320; 0 sends every system to the workgroup kernel.
 *            Default 320.
 * Both kernels produce LAPACK getrf factors and pivots (largest |a|, lowest
 * row on ties).  Takes effect at the next panel_workspace_init (the airfoil
 * order lives in the workspace): after a change, panel_factor_solve and
 * panel_adjoint return PANEL_EINVAL until it has run.  PANEL_EINVAL
 * outside the range.                                                       */
panel_status panel_plan_set_wave_limit(panel_plan *plan, int32_t max_n1);

/* Select the panel formulation (default PANEL_STREAM_FUNCTION).  Both give
 * an (N_b + 1) x (N_b + 1) system per airfoil, factored and solved alike.
 * PANEL_HESS_SMITH unknowns: the N_b source densities, then the vortex
 * density; its workspace also keeps the tangential-velocity influence
 * matrix (one more system-sized section), so call this before
 * panel_workspace_size.  panel_forces reports, for both, the tangential
 * surface speed at the panel midpoints (the `gamma` output), Cp, Cl from the
 * circulation -2 sum_i u_i L_i / (vinf c) and Cl_p; panel_adjoint
 * differentiates either.                                                  */
panel_status panel_plan_set_formulation(panel_plan *plan, int32_t formulation);

/* How the factorisation maps a batch onto the GPU (Sec. 3: many independent
 * dense systems; Sec. 4 splits the population into slices, here the batch
 * is one queue).  This is the entry of the tile table that the Python
 * autotuner (PanelSolver.autotune) fills by timing candidates per batch.
 *   wave_max_n1  systems with n1 <= wave_max_n1 (0..320) are factored by one
 *                wavefront each, larger ones by a workgroup each
 *   persistent   1: one launch of persistent workgroups pops the airfoils in
 *                LPT order, whole workgroups taking the large systems and
 *                single wavefronts the rest, and (PANEL_FP32_REFINE) refines
 *                each solution right after its factorisation; 0: one launch
 *                per kernel family.  Batches with systems above 768 rows, or
 *                wg_waves = 8, always take separate launches.
 *   wg_waves     wavefronts per workgroup-factored system: 4, 8, or 0 (eight
 *                when the batch has at most one airfoil per CU; systems above
 *                768 rows always take eight)
 * Default {320, 0, 0} (the faster choice on the batches measured; the
 * persistent kernel holds both paths and spills more registers).  Changing
 * wave_max_n1 takes effect at the next panel_workspace_init, as for
 * panel_plan_set_wave_limit.                                               */
typedef struct {
    int32_t wave_max_n1;
    int32_t persistent;
    int32_t wg_waves;
} panel_tiling;

panel_status panel_plan_set_tiling(panel_plan *plan, const panel_tiling *tiling);
panel_status panel_plan_get_tiling(const panel_plan *plan, panel_tiling *tiling);

/* Bytes of device workspace the plan needs (256-byte aligned base). */
panel_status panel_workspace_size(const panel_plan *plan, size_t *bytes);

/* Where airfoil b's data sit inside a workspace (for inspection and tests):
 * h_desc receives 9 int64 values: byte offsets of the FP64 augmented system
 * (column-major, ld rows, n1 + K columns), of the FP32 system (-1 unless
 * PANEL_FP32_REFINE), of the K solutions, of the n1 int32 pivots, then n1,
 * ld, K, the byte offset of the int32 refinement-sweep counter, and of the
 * tangential-velocity matrix (column-major, ld rows, n1 columns; -1 unless
 * PANEL_HESS_SMITH).                                                        */
panel_status panel_workspace_layout(const panel_plan *plan, int32_t b, int64_t *h_desc);

/* Write the plan's per-airfoil metadata into the workspace (one host-to-
 * device copy on `stream`).  Must precede the first panel_assemble on a
 * workspace; the metadata stays valid until the workspace is reused for
 * another plan.  Not meant to be captured in a graph.                      */
panel_status panel_workspace_init(const panel_plan *plan, void *ws, void *stream);

/* Assembly (Sec. 2: panel integrals at the midpoints, the constant C, the
 * Kutta row, free-stream right-hand sides).  Everything in FP64; with
 * PANEL_FP32_REFINE an FP32 copy of the system is also written for the
 * factorisation.
 *   xy      2 * node_offsets[B] doubles, node k of the batch at (xy[2k], xy[2k+1])
 *   alpha   alpha_offsets[B] angles of attack in radians
 *   chord   B reference lengths for the lift coefficient, or NULL (all 1)
 *   vinf    free-stream speed, finite and > 0
 *   ws      workspace of panel_workspace_size bytes, initialised          */
panel_status panel_assemble(const panel_plan *plan, const double *xy, const double *alpha,
                            const double *chord, double vinf, void *ws, void *stream);

/* LU factorisation with partial pivoting (largest |a_ik|, lowest row index
 * on ties) of every assembled system, and solution for its K_b right-hand
 * sides (Sec. 3: LU, (2/3)n^3 operations).  With PANEL_FP32_REFINE the
 * factorisation is in FP32 and the solution is refined: r = b - A x in
 * FP64, correction from the FP32 factors, x += correction, until
 * ||correction||_inf <= refine_tol * ||x||_inf, or the correction that the
 * last two predict for the next sweep under linear convergence at a rate
 * below 1/2, ||d_k||^2 / (||d_{k-1}|| - ||d_k||), is, or until the residual
 * sits at the FP64 backward-error floor ||r||_inf <= sqrt(n) eps ||A||_inf
 * ||x||_inf (no sweep can improve x further), or max_iter sweeps (info -2).
 * max_iter = 0 disables refinement and reports -2 (result unverified).
 *   refine_tol  > 0 (ignored for PANEL_FP64)
 *   max_iter    0..100 (ignored for PANEL_FP64)
 *   info        device int32[B], written per airfoil (codes above)        */
panel_status panel_factor_solve(const panel_plan *plan, void *ws, double refine_tol,
                                int32_t max_iter, int32_t *info, void *stream);

/* Surface speed, pressure coefficient and lift (forces step; the paper
 * reports C_L without printing its formula):
 *   gamma[s_b + k N_b + i] = gamma_i   (tangential speed, CCW tangent)
 *   cp   [s_b + k N_b + i] = 1 - (gamma_i / vinf)^2
 *   cl   [alpha_offsets[b] + k] = -2 sum_i gamma_i L_i / (vinf c_b)
 *   cl_p [alpha_offsets[b] + k] = -(1/c_b) sum_i Cp_i L_i (n_i . e_L),
 *          n_i outward normal, e_L = (-sin alpha, cos alpha)
 * with s_b = sum_{b'<b} N_b' K_b'.  gamma, cp, cl_p may be NULL.          */
panel_status panel_forces(const panel_plan *plan, const void *ws, double *gamma, double *cp,
                          double *cl, double *cl_p, void *stream);

/* Viscous correction (Sec. 2: the inviscid solution gives no drag, so a
 * laminar boundary-layer method, Thwaites', corrects it; the genetic
 * algorithm's fitness is the lift-to-drag ratio).  On the surface speed of
 * each airfoil and angle: from the stagnation point (between the first pair
 * of panel midpoints with gamma_j < 0 <= gamma_{j+1}) along both surfaces,
 * theta^2 = 0.45 nu U^-6 int U^5 ds (U = |gamma| piecewise linear in the arc
 * length), lambda = theta^2 U' / nu, laminar separation at the first station
 * with lambda < -0.09, and up to it the wall shear of Thwaites' correlation
 * integrated along the free stream:
 *   cd [alpha_offsets[b] + k]  skin-friction drag / ((1/2) rho vinf^2 c_b),
 *                              nu = vinf c_b / re
 *   ld [.]                     cl / cd
 *   sep[2 (alpha_offsets[b] + k) + {0, 1}]  panel where the upper / lower
 *                              layer separates, -1 if it reaches the
 *                              trailing edge, -2 (cd, ld NaN) if no
 *                              stagnation point is found or info != 0
 *   gamma, cl  the outputs of panel_forces for this workspace (the layer is
 *              run on whatever they hold)
 *   re         chord Reynolds number, finite and > 0                      */
panel_status panel_thwaites(const panel_plan *plan, const void *ws, const double *gamma, const double *cl,
                            double re, double *cd, double *ld, int32_t *sep, void *stream);

/* Reverse-mode sensitivity of the forces outputs to every node (the shape
 * gradient of the Sec. 2 system, M(P) x = r(P, alpha)):
 *   dxy[2k + c] = sum over the airfoil's angles a of
 *                   dcl[a] dCl_a/dP_k,c + sum_i dcp[a, i] dCp_{a,i}/dP_k,c
 * for all N_b + 1 nodes of each airfoil (node 0 and node N are separate
 * variables), with cl and cp as panel_forces defines them
 * (dCp_i/dgamma_i = -2 gamma_i / vinf^2).  Uses the factors left in the
 * workspace by panel_factor_solve (transposed solve; refined in FP64 for
 * PANEL_FP32_REFINE) and re-evaluates the assembly derivatives on the fly.
 * Stream function: without dcp one pass serves every angle; with dcp the
 * work is one pass per angle index.  Hess-Smith (gamma is the surface speed
 * u = T x + vinf e.t): one transposed solve per angle, lambda = M^-T T^T
 * dF/du, with the tangential matrix kept by panel_assemble.
 *   xy     the node array passed to panel_assemble
 *   dcl    alpha_offsets[B] cotangents of cl
 *   dcp    cotangents of cp in panel_forces' layout, or NULL (all zero)
 *   dxy    2 * node_offsets[B] doubles, overwritten
 *   info   device int32[B] or NULL: 0, the factorisation's code for
 *          airfoils that failed there, or -2 when (PANEL_FP32_REFINE) the
 *          FP64 refinement of the transposed solve did not converge within
 *          10 sweeps (the gradient is then less accurate)
 * Airfoils whose factorisation failed get NaN.                            */
panel_status panel_adjoint(const panel_plan *plan, const void *ws, const double *xy,
                           const double *dcl, const double *dcp, double *dxy, int32_t *info,
                           void *stream);

/* NACA 4-digit sections (geometry helper for the GA population): cosine
 * spacing x = (1 + cos(pi s / (N/2)))/2, s = min(k, N - k), nodes 0..N/2 on
 * the upper surface; thickness coefficient a4 = -0.1036 (closed_te != 0,
 * node N = node 0) or -0.1015.
 *   B         number of sections
 *   node_off  DEVICE int32[B+1] node offsets (N_b even, 4..PANEL_NMAX)
 *   mpt       B x 3 doubles (max camber m, its position p in (0,1),
 *             thickness t)
 *   xy        2 * node_off[B] doubles, written                             */
panel_status panel_naca4(int32_t B, const int32_t *node_off, int32_t closed_te,
                         const double *mpt, double *xy, void *stream);

/* Vector-Jacobian product of panel_naca4:
 *   dmpt[3b + q] = sum_k dxy[2k + c] * d xy[2k + c] / d mpt[3b + q]
 * over the nodes of section b (the node-N entry of a closed section is
 * routed to node 0, of which it is a copy).                                */
panel_status panel_naca4_vjp(int32_t B, const int32_t *node_off, int32_t closed_te,
                             const double *mpt, const double *dxy, double *dmpt, void *stream);

/* ---- Genetic algorithm (Sec. 2, the shape optimisation) -------------------
 * The genome is the list of B-spline coefficients of the contour, ordered
 * from the trailing edge over the upper surface to the trailing edge on the
 * lower surface; a generation evaluates every individual with the panel
 * method (fitness: lift-to-drag ratio with the viscous correction), selects
 * parents by tournament, recombines them by one-point crossover and mutates
 * children with some probability.  The paper does not fix the spline, the
 * bounds or the operator parameters; the readings here: clamped B-spline
 * of degree d, uniform interior knots; tournament draws with replacement;
 * crossover position in 1..G-1; a mutation moves one gene by a uniform
 * amount of at most sigma (hi - lo) and clamps it; no elitism.  Random
 * numbers are inputs: DEVICE arrays of uniforms in [0, 1).
 * Genomes are B x G doubles, row-major.                                    */
#define PANEL_GA_MAX_GENES 64
#define PANEL_GA_MAX_CTRL 64
#define PANEL_GA_MAX_DEGREE 7
#define PANEL_GA_MAX_TOURNAMENT 16

/* Contour nodes of B genomes: control points Q (h_template, M points, x y
 * interleaved) with genome[b G + g] written to coordinate h_gene_map[g] of
 * Q; the clamped B-spline of degree d on Q (knots t_j = 0 for j <= d,
 * (j - d)/(M - d) between, 1 for j >= M) is sampled at
 *   u_k = (1 - cos(2 pi k / N)) / 4  (k <= N/2),  u_k = 1 - u_{N-k} above,
 * clustering nodes at both trailing-edge ends and at the middle of the
 * parameter range.  The first and last template points must coincide (the
 * trailing edge) and carry no gene, so node N equals node 0 exactly.
 *   N           even, PANEL_NMIN..PANEL_NMAX; xy gets B (N + 1) nodes, the
 *               layout of a plan with node_offsets b (N + 1)
 *   h_template  HOST, 2M finite doubles, degree + 1 <= M <= PANEL_GA_MAX_CTRL
 *   h_gene_map  HOST, G distinct indices in [2, 2M - 2), G <= PANEL_GA_MAX_GENES
 *   genome      DEVICE B x G;  xy  DEVICE 2 B (N + 1), written           */
panel_status panel_bspline_nodes(int32_t B, int32_t N, int32_t M, int32_t degree, const double *h_template,
                                 int32_t G, const int32_t *h_gene_map, const double *genome, double *xy,
                                 void *stream);

/* Random initial genomes: genome[b G + g] = lo_g + (hi_g - lo_g) u[b G + g].
 *   h_lo, h_hi  HOST, G finite bounds with lo <= hi;  u DEVICE B x G      */
panel_status panel_ga_init(int32_t B, int32_t G, const double *h_lo, const double *h_hi, const double *u,
                           double *genome, void *stream);

/* Fitness of each airfoil of a plan: the mean over its angles of ld (the
 * output of panel_thwaites), or -infinity when info[b] != 0 (the output of
 * panel_factor_solve) or one of its ld values is not finite.
 *   ld DEVICE alpha_offsets[B];  info DEVICE int32 B;  fitness DEVICE B   */
panel_status panel_ga_fitness(const panel_plan *plan, const void *ws, const double *ld, const int32_t *info,
                              double *fitness, void *stream);

/* Number of uniforms one generation of panel_ga_step reads:
 * (B/2)(4k - 1) + 3B.                                                      */
panel_status panel_ga_uniform_count(int32_t B, int32_t k, int64_t *count);

/* One generation: B/2 child pairs, then each child's mutation trial.  For
 * pair q, u[q (4k-1) ...] holds tournament 1 (k draws, index
 * min(B-1, floor(U B)); k-1 rank trials: the rank taken is the first
 * r < k-1 whose trial is < p_sel, else k-1, ranks counting fitness
 * descending, equal fitness in draw order), tournament 2 (the same) and the
 * crossover draw c = 1 + min(G-2, floor(U (G-1))); child 2q takes genes
 * [0, c) from the first parent and [c, G) from the second, child 2q+1 the
 * reverse.  For child i, u[(B/2)(4k-1) + 3i ...] = (X, Y, Z): if X < p_mut,
 * gene j = min(G-1, floor(Y G)) becomes
 * clamp(gene + sigma (hi_j - lo_j)(2Z - 1), lo_j, hi_j).
 *   B even >= 2;  2 <= G <= PANEL_GA_MAX_GENES;  1 <= k <= PANEL_GA_MAX_TOURNAMENT
 *   p_sel in (0, 1];  p_mut in [0, 1];  sigma finite >= 0
 *   fitness     DEVICE B, no NaN (-infinity marks an unusable individual)
 *   genome_in / genome_out  DEVICE B x G, distinct buffers
 *   u           DEVICE, panel_ga_uniform_count values
 *   trace       DEVICE int32 4B or NULL: per child, first parent, second
 *               parent, crossover position, mutated gene (-1 if none)    */
panel_status panel_ga_step(int32_t B, int32_t G, int32_t k, double p_sel, double p_mut, double sigma,
                           const double *h_lo, const double *h_hi, const double *fitness,
                           const double *genome_in, const double *u, double *genome_out, int32_t *trace,
                           void *stream);

/* History of the run, kept on the device: the generation's best individual
 * (highest fitness, lowest index among equals) is written to slot *counter
 * of hist_fit / hist_idx when *counter < max_gen; if it beats *best_fit it
 * replaces *best_fit and its genome is copied to best_genome; *counter then
 * advances.  The caller sets *counter = 0 and *best_fit = -infinity first.
 *   counter DEVICE int32[1];  hist_fit DEVICE max_gen;  hist_idx DEVICE
 *   int32 max_gen;  best_fit DEVICE [1];  best_genome DEVICE G            */
panel_status panel_ga_record(int32_t B, int32_t G, const double *fitness, const double *genome,
                             int32_t *counter, int32_t max_gen, double *hist_fit, int32_t *hist_idx,
                             double *best_fit, double *best_genome, void *stream);

/* Largest workspace panel_solve_noalloc can hold (bytes of the library's
 * static device scratch array, one per GPU, held until the process ends). */
#define PANEL_NOALLOC_MAX_BYTES ((size_t)256 << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * sequence panel_workspace_init -> panel_assemble -> panel_factor_solve ->
 * panel_forces in one call, with the workspace in a static device array of
 * the library instead of caller memory.  Arguments as for those calls; the
 * caller still provides every input and output array.
 *  - The plan's workspace (panel_workspace_size) must not exceed
 *    PANEL_NOALLOC_MAX_BYTES, else PANEL_EINVAL before any HIP call (at
 *    N = 256 that is about 440 airfoils in FP64, 290 in FP32 + refinement).
 *  - Allocates nothing and does not synchronise: the plan's metadata is
 *    copied from host memory owned by the plan on `stream`, so the plan must
 *    stay alive and unchanged until the call has completed on the stream.
 *    The first call on a device looks up that device's copy of the array.
 *  - All calls on one GPU share its array, which keeps the last call's
 *    contents (nothing in it needs to start at zero): calls that overlap in
 *    time on one GPU (different streams or threads) race and corrupt each
 *    other.  Serialise them, or use the caller-owned workspace calls.
 *  - The workspace stays private: panel_adjoint cannot follow this call.  */
panel_status panel_solve_noalloc(const panel_plan *plan, const double *xy, const double *alpha,
                                 const double *chord, double vinf, double refine_tol, int32_t max_iter,
                                 int32_t *info, double *gamma, double *cp, double *cl, double *cl_p,
                                 void *stream);

/* Diagnostic: evaluates the FP64 logarithm and two-argument arctangent the
 * assembly and adjoint kernels use (the library's own, not the device libm),
 * for accuracy tests:
 *   log_out[i] = log(x[i])          (x[i] > 0; NULL log_out skips it)
 *   atan2_out[i] = atan2(y[i], x[i])  (NULL atan2_out skips it)
 * All arrays are device arrays of n doubles.                               */
panel_status panel_math_eval(int32_t n, const double *x, const double *y, double *log_out,
                             double *atan2_out, void *stream);

/* Static description of a status code. */
const char *panel_status_str(int32_t status);

/* Message for the last error on the calling thread ("" if none). */
const char *panel_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PANEL_H */
