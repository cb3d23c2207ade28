/*
 * panel_oracle_hs.c -- plain FP64 CPU oracle for the Hess-Smith panel
 * formulation (TEST INFRASTRUCTURE ONLY; nothing in the product links it).
 *
 * The paper's own scheme (Sec. 2) is a vortex sheet with the stream function
 * held constant on the contour; its opening describes the influence matrix
 * in terms of sources and vortices.  The Hess-Smith discretisation written
 * out here is the classical source+vortex variant of the same problem, kept
 * as a second formulation with the same (N+1) x (N+1) system shape:
 *
 *   unknowns   q_0..q_{N-1} (constant source density on each panel) and
 *              one vortex density g shared by all panels;
 *   rows j < N flow tangency at the panel midpoints m_j:
 *              (V_inf + sum_i q_i S_i(m_j) + g sum_i W_i(m_j)) . n_j = 0
 *   row N      Kutta condition: the tangential speeds at the midpoints of
 *              the two trailing-edge panels (0 and N-1, tangents taken in
 *              node order) are equal and opposite:
 *              V(m_0) . t_0 + V(m_{N-1}) . t_{N-1} = 0
 *
 * S_i(x) is the velocity induced at x by panel i carrying a unit source
 * density, W_i(x) by a unit counter-clockwise vortex density.  In the
 * panel's frame (origin P_i, xi along t_i, eta along the outward normal
 * n_i = (t_y, -t_x)), with r1 = |x - P_i|, r2 = |x - P_{i+1}| and beta the
 * angle the panel subtends at x,
 *     S = (1/2pi) [ log(r1/r2) t_i + beta n_i ],
 *     W = (1/2pi) [ beta t_i - log(r1/r2) n_i ]   (S turned by +90 degrees)
 * written out from the integrals of (1/2pi)(x - s)/|x - s|^2 over the panel.
 * At the panel's own midpoint log(r1/r2) = 0 and beta = pi (the limit from
 * the fluid side).
 *
 * Outputs per angle, in the same form as the stream-function oracle:
 *   u_j   = V(m_j) . t_j      (tangential surface speed at the midpoints)
 *   Cp_j  = 1 - (u_j / vinf)^2
 *   Cl    = -2 sum_j u_j L_j / (vinf c)
 *   Cl_p  = -(1/c) sum_j Cp_j L_j (n_j . e_L),  e_L = (-sin a, cos a)
 * Everything is double precision and written out plainly: two logarithms
 * (one per end point) and two atan2 per influence pair.
 */
#include <math.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define HS_PI 3.14159265358979323846

int oracle_lu(int n, double *A, int *piv);
void oracle_lu_solve(int n, const double *LU, const int *piv, int K, double *B);

static void frame(const double *xy, int i, double *L, double *tx, double *ty)
{
    double hx = xy[2 * i + 2] - xy[2 * i];
    double hy = xy[2 * i + 3] - xy[2 * i + 1];
    *L = sqrt(hx * hx + hy * hy);
    *tx = hx / *L;
    *ty = hy / *L;
}

/* Velocities induced at (x, y) by panel i: unit source (sx, sy) and unit
 * counter-clockwise vortex (wx, wy).  self != 0: (x, y) is the panel's own
 * midpoint.                                                                */
void oracle_hs_influence(const double *xy, int i, double x, double y, int self, double *sx, double *sy,
                         double *wx, double *wy)
{
    double L, tx, ty;
    frame(xy, i, &L, &tx, &ty);
    const double nx = ty, ny = -tx;
    double lg, beta;
    if (self) {
        lg = 0.0;
        beta = HS_PI;
    } else {
        const double dx = x - xy[2 * i], dy = y - xy[2 * i + 1];
        const double xi = dx * tx + dy * ty;
        const double eta = dx * nx + dy * ny;
        const double r1 = sqrt(xi * xi + eta * eta);
        const double r2 = sqrt((xi - L) * (xi - L) + eta * eta);
        lg = log(r1 / r2);
        beta = atan2(eta, xi - L) - atan2(eta, xi);
    }
    const double us = lg / (2.0 * HS_PI), vs = beta / (2.0 * HS_PI);
    *sx = us * tx + vs * nx;
    *sy = us * ty + vs * ny;
    *wx = vs * tx - us * nx;
    *wy = vs * ty - us * ny;
}

/* Normal- and tangential-velocity influence matrices of the N panels at the
 * N midpoints: Mn[j*(N+1) + i] = S_i(m_j) . n_j (i < N), Mn[j*(N+1) + N] =
 * sum_i W_i(m_j) . n_j, and Mt likewise with t_j.  Row-major, N rows.      */
void oracle_hs_influence_matrices(int N, const double *xy, double *Mn, double *Mt)
{
    const int n1 = N + 1;
    for (int j = 0; j < N; ++j) {
        double Lj, tjx, tjy;
        frame(xy, j, &Lj, &tjx, &tjy);
        const double njx = tjy, njy = -tjx;
        const double mx = 0.5 * (xy[2 * j] + xy[2 * j + 2]);
        const double my = 0.5 * (xy[2 * j + 1] + xy[2 * j + 3]);
        double vn = 0.0, vt = 0.0;
        for (int i = 0; i < N; ++i) {
            double sx, sy, wx, wy;
            oracle_hs_influence(xy, i, mx, my, i == j, &sx, &sy, &wx, &wy);
            Mn[j * n1 + i] = sx * njx + sy * njy;
            Mt[j * n1 + i] = sx * tjx + sy * tjy;
            vn += wx * njx + wy * njy;
            vt += wx * tjx + wy * tjy;
        }
        Mn[j * n1 + N] = vn;
        Mt[j * n1 + N] = vt;
    }
}

/* Bordered system M [(N+1) x (N+1), row-major] and right-hand sides R[k*(N+1)
 * + j] for K angles; also the tangential matrix Mt [N x (N+1)].            */
void oracle_hs_assemble(int N, const double *xy, int K, const double *alpha, double vinf, double *M, double *R,
                        double *Mt)
{
    const int n1 = N + 1;
    oracle_hs_influence_matrices(N, xy, M, Mt);
    for (int i = 0; i < n1; ++i)
        M[N * n1 + i] = Mt[0 * n1 + i] + Mt[(N - 1) * n1 + i];
    double L0, t0x, t0y, Le, tex, tey;
    frame(xy, 0, &L0, &t0x, &t0y);
    frame(xy, N - 1, &Le, &tex, &tey);
    for (int k = 0; k < K; ++k) {
        const double ca = cos(alpha[k]), sa = sin(alpha[k]);
        for (int j = 0; j < N; ++j) {
            double Lj, tjx, tjy;
            frame(xy, j, &Lj, &tjx, &tjy);
            R[k * n1 + j] = -vinf * (ca * tjy - sa * tjx);   /* -V_inf . n_j, n_j = (t_y, -t_x) */
        }
        R[k * n1 + N] = -vinf * (ca * (t0x + tex) + sa * (t0y + tey));
    }
}

/* Surface speed, Cp, Cl and Cl_p from the solutions X[k*(N+1) + i].         */
void oracle_hs_forces(int N, const double *xy, int K, const double *alpha, const double *X, const double *Mt,
                      double vinf, double chord, double *u, double *cp, double *cl, double *cl_p)
{
    const int n1 = N + 1;
    for (int k = 0; k < K; ++k) {
        const double ca = cos(alpha[k]), sa = sin(alpha[k]);
        const double ex = -sa, ey = ca;
        double circ = 0.0, fl = 0.0;
        for (int j = 0; j < N; ++j) {
            double Lj, tjx, tjy;
            frame(xy, j, &Lj, &tjx, &tjy);
            double s = vinf * (ca * tjx + sa * tjy);
            for (int i = 0; i < n1; ++i)
                s += Mt[j * n1 + i] * X[k * n1 + i];
            const double c = 1.0 - (s / vinf) * (s / vinf);
            u[k * N + j] = s;
            cp[k * N + j] = c;
            circ += s * Lj;
            fl += c * Lj * (tjy * ex - tjx * ey);
        }
        cl[k] = -2.0 * circ / (vinf * chord);
        if (cl_p)
            cl_p[k] = -fl / chord;
    }
}

/* One airfoil end to end; returns the LU info (0 ok).                       */
int oracle_hs_solve_airfoil(int N, const double *xy, int K, const double *alpha, double vinf, double chord,
                            double *u, double *cp, double *cl, double *cl_p)
{
    const int n1 = N + 1;
    double *M = malloc(sizeof(double) * (size_t)n1 * n1);
    double *Mt = malloc(sizeof(double) * (size_t)n1 * n1);
    double *X = malloc(sizeof(double) * (size_t)n1 * K);
    int *piv = malloc(sizeof(int) * (size_t)n1);
    oracle_hs_assemble(N, xy, K, alpha, vinf, M, X, Mt);
    int info = oracle_lu(n1, M, piv);
    if (info == 0) {
        oracle_lu_solve(n1, M, piv, K, X);
        oracle_hs_forces(N, xy, K, alpha, X, Mt, vinf, chord, u, cp, cl, cl_p);
    } else {
        for (int q = 0; q < N * K; ++q)
            u[q] = cp[q] = NAN;
        for (int k = 0; k < K; ++k) {
            cl[k] = NAN;
            if (cl_p)
                cl_p[k] = NAN;
        }
    }
    free(M);
    free(Mt);
    free(X);
    free(piv);
    return info;
}

/* A whole batch, packed like oracle_solve_batch (OpenMP over airfoils).    */
int oracle_hs_solve_batch(int B, const int *node_off, const double *xy, const int *alpha_off, const double *alpha,
                          const double *chord, double vinf, double *u, double *cp, double *cl, double *cl_p,
                          int *info, int nthreads)
{
    long long *sol_off = malloc(sizeof(long long) * (size_t)(B + 1));
    sol_off[0] = 0;
    for (int b = 0; b < B; ++b)
        sol_off[b + 1] = sol_off[b] + (long long)(node_off[b + 1] - node_off[b] - 1) * (alpha_off[b + 1] - alpha_off[b]);
    int used = 1;
#ifdef _OPENMP
    if (nthreads <= 0)
        nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
    for (int b = 0; b < B; ++b) {
        const int N = node_off[b + 1] - node_off[b] - 1;
        const int K = alpha_off[b + 1] - alpha_off[b];
        info[b] = oracle_hs_solve_airfoil(N, xy + 2 * (size_t)node_off[b], K, alpha + alpha_off[b], vinf,
                                          chord ? chord[b] : 1.0, u + sol_off[b], cp + sol_off[b],
                                          cl + alpha_off[b], cl_p ? cl_p + alpha_off[b] : NULL);
    }
#ifdef _OPENMP
    used = nthreads;
#endif
    free(sol_off);
    return used;
}

/* ------------------------------------------------------------------------- */
/* Gradient of the weighted forces of one angle in the Hess-Smith scheme,
 *     F = dcl * Cl + sum_j dcp[j] * Cp_j,
 * with respect to every node coordinate (grad[2k + c], k = 0..N): for each
 * coordinate the whole complex-valued assembly is re-evaluated with that
 * coordinate moved by i*h (complex step, Squire & Trapp 1998), giving dM,
 * dR and the derivative of the tangential matrix and of the free-stream
 * tangential speeds; then dx = M^{-1}(dR - dM x) with the real factors, and
 * du = dMt x + Mt dx + d(V_inf . t), dF from u and the panel lengths.
 * O(N^3) per coordinate: for small N only.                                 */
#include <complex.h>

#define HS_H 1e-30

typedef double complex cplx;

static cplx c_atan2(cplx y, cplx x)
{
    double yr = creal(y), xr = creal(x);
    return atan2(yr, xr) + I * ((xr * cimag(y) - yr * cimag(x)) / (xr * xr + yr * yr));
}

static void c_frame(const cplx *z, int i, cplx *L, cplx *tx, cplx *ty)
{
    cplx hx = z[2 * i + 2] - z[2 * i], hy = z[2 * i + 3] - z[2 * i + 1];
    *L = csqrt(hx * hx + hy * hy);
    *tx = hx / *L;
    *ty = hy / *L;
}

static void c_influence(const cplx *z, int i, cplx x, cplx y, int self, cplx *sx, cplx *sy, cplx *wx, cplx *wy)
{
    cplx L, tx, ty;
    c_frame(z, i, &L, &tx, &ty);
    cplx nx = ty, ny = -tx, lg, beta;
    if (self) {
        lg = 0.0;
        beta = HS_PI;
    } else {
        cplx dx = x - z[2 * i], dy = y - z[2 * i + 1];
        cplx xi = dx * tx + dy * ty, eta = dx * nx + dy * ny;
        lg = 0.5 * (clog(xi * xi + eta * eta) - clog((xi - L) * (xi - L) + eta * eta));
        beta = c_atan2(eta, xi - L) - c_atan2(eta, xi);
    }
    cplx us = lg / (2.0 * HS_PI), vs = beta / (2.0 * HS_PI);
    *sx = us * tx + vs * nx;
    *sy = us * ty + vs * ny;
    *wx = vs * tx - us * nx;
    *wy = vs * ty - us * ny;
}

/* complex system: M [(N+1)^2], R [N+1], Mt [N*(N+1)], tangential free-stream
 * speeds ft [N] = V_inf . t_j, panel lengths Ls [N]                         */
static void c_assemble(int N, const cplx *z, double alpha, double vinf, cplx *M, cplx *R, cplx *Mt, cplx *ft,
                       cplx *Ls)
{
    const int n1 = N + 1;
    const double ca = cos(alpha), sa = sin(alpha);
    for (int j = 0; j < N; ++j) {
        cplx Lj, tjx, tjy;
        c_frame(z, j, &Lj, &tjx, &tjy);
        Ls[j] = Lj;
        cplx njx = tjy, njy = -tjx;
        cplx mx = 0.5 * (z[2 * j] + z[2 * j + 2]), my = 0.5 * (z[2 * j + 1] + z[2 * j + 3]);
        cplx vn = 0.0, vt = 0.0;
        for (int i = 0; i < N; ++i) {
            cplx sx, sy, wx, wy;
            c_influence(z, i, mx, my, i == j, &sx, &sy, &wx, &wy);
            M[j * n1 + i] = sx * njx + sy * njy;
            Mt[j * n1 + i] = sx * tjx + sy * tjy;
            vn += wx * njx + wy * njy;
            vt += wx * tjx + wy * tjy;
        }
        M[j * n1 + N] = vn;
        Mt[j * n1 + N] = vt;
        R[j] = -vinf * (ca * tjy - sa * tjx);
        ft[j] = vinf * (ca * tjx + sa * tjy);
    }
    for (int i = 0; i < n1; ++i)
        M[N * n1 + i] = Mt[i] + Mt[(N - 1) * n1 + i];
    cplx L0, t0x, t0y, Le, tex, tey;
    c_frame(z, 0, &L0, &t0x, &t0y);
    c_frame(z, N - 1, &Le, &tex, &tey);
    R[N] = -vinf * (ca * (t0x + tex) + sa * (t0y + tey));
}

int oracle_hs_force_gradient(int N, const double *xy, double alpha, double vinf, double chord, double dcl,
                             const double *dcp, double *grad)
{
    const int n1 = N + 1, nc = 2 * (N + 1);
    cplx *z = malloc(sizeof(cplx) * (size_t)nc);
    cplx *M = malloc(sizeof(cplx) * (size_t)n1 * n1);
    cplx *Mt = malloc(sizeof(cplx) * (size_t)n1 * n1);
    cplx *R = malloc(sizeof(cplx) * (size_t)n1);
    cplx *ft = malloc(sizeof(cplx) * (size_t)N);
    cplx *Ls = malloc(sizeof(cplx) * (size_t)N);
    double *A = malloc(sizeof(double) * (size_t)n1 * n1);
    double *x = malloc(sizeof(double) * (size_t)n1);
    double *v = malloc(sizeof(double) * (size_t)n1);
    double *Mtr = malloc(sizeof(double) * (size_t)n1 * n1);
    double *u = malloc(sizeof(double) * (size_t)N);
    int *piv = malloc(sizeof(int) * (size_t)n1);
    for (int q = 0; q < nc; ++q)
        z[q] = xy[q];
    c_assemble(N, z, alpha, vinf, M, R, Mt, ft, Ls);
    for (int q = 0; q < n1 * n1; ++q) {
        A[q] = creal(M[q]);
        Mtr[q] = creal(Mt[q]);
    }
    for (int j = 0; j < n1; ++j)
        x[j] = creal(R[j]);
    int info = oracle_lu(n1, A, piv);
    if (info == 0) {
        oracle_lu_solve(n1, A, piv, 1, x);
        for (int j = 0; j < N; ++j) {
            double s = creal(ft[j]);
            for (int i = 0; i < n1; ++i)
                s += Mtr[j * n1 + i] * x[i];
            u[j] = s;
        }
        const double scale = -2.0 / (vinf * chord);
        for (int q = 0; q < nc; ++q) {
            z[q] = xy[q] + I * HS_H;
            c_assemble(N, z, alpha, vinf, M, R, Mt, ft, Ls);
            for (int j = 0; j < n1; ++j) {
                double s = cimag(R[j]) / HS_H;
                for (int i = 0; i < n1; ++i)
                    s -= cimag(M[j * n1 + i]) / HS_H * x[i];
                v[j] = s;
            }
            oracle_lu_solve(n1, A, piv, 1, v);   /* dx */
            double dF = 0.0;
            for (int j = 0; j < N; ++j) {
                double du = cimag(ft[j]) / HS_H;
                for (int i = 0; i < n1; ++i)
                    du += cimag(Mt[j * n1 + i]) / HS_H * x[i] + Mtr[j * n1 + i] * v[i];
                dF += dcl * scale * (du * creal(Ls[j]) + u[j] * cimag(Ls[j]) / HS_H);
                if (dcp)
                    dF += dcp[j] * (-2.0 * u[j] * du / (vinf * vinf));
            }
            grad[q] = dF;
            z[q] = xy[q];
        }
    }
    free(z);
    free(M);
    free(Mt);
    free(R);
    free(ft);
    free(Ls);
    free(A);
    free(x);
    free(v);
    free(Mtr);
    free(u);
    free(piv);
    return info;
}
