/*
 * panel_oracle.c -- plain, slow, FP64 CPU oracle for the batched 2-D panel
 * method (Einkemmer, arXiv:1511.02166, Sec. 2 "Numerical algorithm").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links or calls
 * this file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header or table with the GPU path.
 *
 * What it computes, per airfoil with nodes P_0..P_N (P_N = P_0 for a closed
 * section, trailing edge first, counter-clockwise: upper surface, leading
 * edge, lower surface) and per angle of attack alpha:
 *
 *   G_ji  = integral over panel i of -(1/2pi) log|m_j - s| ds      (Sec. 2,
 *           fundamental solution, constant density on each panel, boundary
 *           condition collocated at the panel midpoints m_j)
 *   rows j < N :  sum_i G_ji gamma_i - C = -phi_v(m_j),
 *                 phi_v(x, y) = vinf (y cos alpha - x sin alpha)
 *                 (Sec. 2, stream function of the free stream and the
 *                 boundary condition phi = C on the contour)
 *   row N      :  gamma_0 + gamma_{N-1} = 0      (Sec. 2, Kutta condition)
 *
 * solved by Gaussian elimination with partial pivoting (Sec. 3: LU, (2/3)n^3).
 * Surface quantities (the paper reports C_L but prints no formula for it):
 *   u_i = gamma_i (tangential speed, counter-clockwise tangent; the interior
 *         stream function is constant so the outer slip speed equals the
 *         sheet strength), Cp_i = 1 - (u_i / vinf)^2,
 *   Cl   = -2 sum_i gamma_i L_i / (vinf c)          (Kutta-Joukowski lift of
 *          the counter-clockwise circulation sum_i gamma_i L_i),
 *   Cl_p = -(1/c) sum_i Cp_i L_i (n_i . e_L),  e_L = (-sin alpha, cos alpha).
 *
 * Sign reading: the closed form printed for the panel integral in Sec. 2 is
 * the negative of the integral it is said to equal; this file uses the
 * integral as defined (the printed sign would only flip the sign of gamma).
 * The self-influence (j = i) is the limit of the integral at the panel
 * midpoint, (L/2pi)(1 - log(L/2)).
 *
 * Everything is double precision, written out plainly: two logs and two
 * atan2 per off-diagonal entry exactly as the closed form reads.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846

/* ------------------------------------------------------------------------- */
/* NACA 4-digit section (standard definition: thickness polynomial with
 * a4 = -0.1036 for a closed trailing edge or -0.1015 for the classic open
 * one; two-branch camber line; thickness laid off along the camber normal).
 * Cosine spacing x = (1 + cos(pi s / (N/2))) / 2 with s = min(k, N - k), so
 * node k and node N - k sit at the same x (uniform spacing: x = 1 - s/(N/2)).  Nodes 0..N/2 are on the upper
 * surface, N/2..N on the lower; the leading-edge node is k = N/2.
 * For a closed section node N is set equal to node 0. N must be even.       */
void oracle_naca4_spaced(double m, double p, double t, int N, int closed_te, int uniform, double *xy)
{
    const double a4 = closed_te ? -0.1036 : -0.1015;
    const int half = N / 2;
    for (int k = 0; k <= N; ++k) {
        int s = (k <= half) ? k : N - k;
        double x = uniform ? 1.0 - (double)s / (double)half
                           : 0.5 * (1.0 + cos(OR_PI * (double)s / (double)half));
        double yt = 5.0 * t * (0.2969 * sqrt(x) - 0.1260 * x - 0.3516 * x * x
                               + 0.2843 * x * x * x + a4 * x * x * x * x);
        double yc, dyc;
        if (m == 0.0) {
            yc = 0.0;
            dyc = 0.0;
        } else if (x < p) {
            yc = m / (p * p) * (2.0 * p * x - x * x);
            dyc = 2.0 * m / (p * p) * (p - x);
        } else {
            yc = m / ((1.0 - p) * (1.0 - p)) * ((1.0 - 2.0 * p) + 2.0 * p * x - x * x);
            dyc = 2.0 * m / ((1.0 - p) * (1.0 - p)) * (p - x);
        }
        double th = atan(dyc);
        if (k <= half) {
            xy[2 * k] = x - yt * sin(th);
            xy[2 * k + 1] = yc + yt * cos(th);
        } else {
            xy[2 * k] = x + yt * sin(th);
            xy[2 * k + 1] = yc - yt * cos(th);
        }
    }
    if (closed_te) {
        xy[2 * N] = xy[0];
        xy[2 * N + 1] = xy[1];
    }
}

void oracle_naca4(double m, double p, double t, int N, int closed_te, double *xy)
{
    oracle_naca4_spaced(m, p, t, N, closed_te, 0, xy);
}

/* ------------------------------------------------------------------------- */
/* Panel i runs from P_i to P_{i+1}; returns its length and unit tangent.   */
static double panel_frame(const double *xy, int i, double *tx, double *ty)
{
    double hx = xy[2 * i + 2] - xy[2 * i];
    double hy = xy[2 * i + 3] - xy[2 * i + 1];
    double L = sqrt(hx * hx + hy * hy);
    *tx = hx / L;
    *ty = hy / L;
    return L;
}

/* G_ji: integral over panel i of -(1/2pi) log|m_j - s| ds (Sec. 2, panel
 * integral).  With local coordinates of the midpoint m_j relative to P_i,
 * xi along the panel and eta along n_i = (ty, -tx):
 *   int_0^L log((xi - s)^2 + eta^2) ds
 *     = xi log r1^2 - (xi - L) log r2^2 - 2L - 2 eta [atan2(eta, xi) - atan2(eta, xi - L)]
 * and G_ji = -(1/4pi) times that.  j == i is the midpoint limit.           */
double oracle_g_entry(const double *xy, int j, int i)
{
    double tx, ty;
    double L = panel_frame(xy, i, &tx, &ty);
    if (i == j)
        return L / (2.0 * OR_PI) * (1.0 - log(0.5 * L));
    double mx = 0.5 * (xy[2 * j] + xy[2 * j + 2]);
    double my = 0.5 * (xy[2 * j + 1] + xy[2 * j + 3]);
    double dx = mx - xy[2 * i];
    double dy = my - xy[2 * i + 1];
    double xi = dx * tx + dy * ty;
    double eta = dx * ty - dy * tx;
    double r1s = xi * xi + eta * eta;
    double r2s = (xi - L) * (xi - L) + eta * eta;
    double delta = atan2(eta, xi) - atan2(eta, xi - L);
    return -1.0 / (4.0 * OR_PI) * (xi * log(r1s) - (xi - L) * log(r2s) - 2.0 * L - 2.0 * eta * delta);
}

/* Free-stream stream function phi_v = vinf (y cos a - x sin a) (Sec. 2).    */
static double phi_v(double x, double y, double vinf, double a)
{
    return vinf * (y * cos(a) - x * sin(a));
}

/* Bordered (N+1)x(N+1) system, row-major M[j*(N+1) + i]; right-hand sides
 * R[k*(N+1) + j] for the K angles.  Unknowns (gamma_0..gamma_{N-1}, C).    */
void oracle_assemble(int N, const double *xy, int K, const double *alpha, double vinf,
                     double *M, double *R)
{
    const int n1 = N + 1;
    for (int j = 0; j < N; ++j) {
        for (int i = 0; i < N; ++i)
            M[j * n1 + i] = oracle_g_entry(xy, j, i);
        M[j * n1 + N] = -1.0;
    }
    for (int i = 0; i < n1; ++i)
        M[N * n1 + i] = 0.0;
    M[N * n1 + 0] += 1.0;
    M[N * n1 + N - 1] += 1.0;
    for (int k = 0; k < K; ++k) {
        for (int j = 0; j < N; ++j) {
            double mx = 0.5 * (xy[2 * j] + xy[2 * j + 2]);
            double my = 0.5 * (xy[2 * j + 1] + xy[2 * j + 3]);
            R[k * n1 + j] = -phi_v(mx, my, vinf, alpha[k]);
        }
        R[k * n1 + N] = 0.0;
    }
}

/* Gaussian elimination with partial pivoting, row-major, in place.
 * Pivot = largest |a_ik| over i >= k, lowest index on ties; piv[k] is the
 * (0-based) row exchanged with row k.  Returns 0, or k+1 for the first exact
 * zero pivot (elimination continues past it, as LAPACK getrf does).        */
int oracle_lu(int n, double *A, int *piv)
{
    int info = 0;
    for (int k = 0; k < n; ++k) {
        int p = k;
        double amax = fabs(A[k * n + k]);
        for (int i = k + 1; i < n; ++i) {
            if (fabs(A[i * n + k]) > amax) {
                amax = fabs(A[i * n + k]);
                p = i;
            }
        }
        piv[k] = p;
        if (A[p * n + k] == 0.0) {
            if (info == 0)
                info = k + 1;
            continue;
        }
        if (p != k) {
            for (int j = 0; j < n; ++j) {
                double tmp = A[k * n + j];
                A[k * n + j] = A[p * n + j];
                A[p * n + j] = tmp;
            }
        }
        for (int i = k + 1; i < n; ++i) {
            double l = A[i * n + k] / A[k * n + k];
            A[i * n + k] = l;
            for (int j = k + 1; j < n; ++j)
                A[i * n + j] -= l * A[k * n + j];
        }
    }
    return info;
}

/* Solve A X = B from the factors of oracle_lu; B holds K right-hand sides
 * stored one after another (B[k*n + i]) and is overwritten by X.          */
void oracle_lu_solve(int n, const double *LU, const int *piv, int K, double *B)
{
    for (int k = 0; k < K; ++k) {
        double *b = B + (size_t)k * n;
        for (int i = 0; i < n; ++i) {
            int p = piv[i];
            if (p != i) {
                double tmp = b[i];
                b[i] = b[p];
                b[p] = tmp;
            }
        }
        for (int i = 0; i < n; ++i) {
            double s = b[i];
            for (int j = 0; j < i; ++j)
                s -= LU[i * n + j] * b[j];
            b[i] = s;
        }
        for (int i = n - 1; i >= 0; --i) {
            double s = b[i];
            for (int j = i + 1; j < n; ++j)
                s -= LU[i * n + j] * b[j];
            b[i] = s / LU[i * n + i];
        }
    }
}

/* Transposed solve A^T Y = W from the same factors (P A = L U, so
 * A^T = U^T L^T P): solve U^T z = w, then L^T y' = z, then y = P^T y'.     */
void oracle_lu_solve_t(int n, const double *LU, const int *piv, double *w)
{
    for (int i = 0; i < n; ++i) {
        double s = w[i];
        for (int j = 0; j < i; ++j)
            s -= LU[j * n + i] * w[j];
        w[i] = s / LU[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = w[i];
        for (int j = i + 1; j < n; ++j)
            s -= LU[j * n + i] * w[j];
        w[i] = s;
    }
    for (int i = n - 1; i >= 0; --i) {
        int p = piv[i];
        if (p != i) {
            double tmp = w[i];
            w[i] = w[p];
            w[p] = tmp;
        }
    }
}

/* Surface speed, Cp, Cl (circulation) and Cl (pressure) for K angles.
 * X holds the K solutions (gamma_0..gamma_{N-1}, C) one after another.     */
void oracle_forces(int N, const double *xy, int K, const double *alpha, const double *X,
                   double vinf, double chord, double *gamma, double *cp, double *cl, double *cl_p)
{
    const int n1 = N + 1;
    for (int k = 0; k < K; ++k) {
        double circ = 0.0, fl = 0.0;
        double ex = -sin(alpha[k]), ey = cos(alpha[k]);
        for (int i = 0; i < N; ++i) {
            double tx, ty;
            double L = panel_frame(xy, i, &tx, &ty);
            double g = X[k * n1 + i];
            double c = 1.0 - (g / vinf) * (g / vinf);
            gamma[k * N + i] = g;
            cp[k * N + i] = c;
            circ += g * L;
            fl += c * L * (ty * ex - tx * ey);
        }
        cl[k] = -2.0 * circ / (vinf * chord);
        if (cl_p)
            cl_p[k] = -fl / chord;
    }
}

/* Input screening: 0 if all nodes are finite and no panel has zero length. */
static int screen_nodes(int N, const double *xy)
{
    for (int k = 0; k < 2 * (N + 1); ++k)
        if (!isfinite(xy[k]))
            return -1;
    for (int i = 0; i < N; ++i) {
        double hx = xy[2 * i + 2] - xy[2 * i];
        double hy = xy[2 * i + 3] - xy[2 * i + 1];
        if (hx == 0.0 && hy == 0.0)
            return -1;
    }
    return 0;
}

/* One airfoil end to end: assemble, factor, solve, forces.  Scratch is
 * allocated here; returns info (0, k>0 zero pivot, -1 bad input).          */
int oracle_solve_airfoil(int N, const double *xy, int K, const double *alpha, double vinf,
                         double chord, double *gamma, double *cp, double *cl, double *cl_p)
{
    const int n1 = N + 1;
    int info = screen_nodes(N, xy);
    if (info == 0) {
        double *M = malloc(sizeof(double) * (size_t)n1 * n1);
        double *X = malloc(sizeof(double) * (size_t)n1 * K);
        int *piv = malloc(sizeof(int) * (size_t)n1);
        oracle_assemble(N, xy, K, alpha, vinf, M, X);
        info = oracle_lu(n1, M, piv);
        if (info == 0) {
            oracle_lu_solve(n1, M, piv, K, X);
            oracle_forces(N, xy, K, alpha, X, vinf, chord, gamma, cp, cl, cl_p);
        }
        free(M);
        free(X);
        free(piv);
    }
    if (info != 0) {
        for (int q = 0; q < N * K; ++q)
            gamma[q] = cp[q] = NAN;
        for (int k = 0; k < K; ++k) {
            cl[k] = NAN;
            if (cl_p)
                cl_p[k] = NAN;
        }
    }
    return info;
}

/* A whole batch (packed like the GPU library's arrays):
 *   xy       2 * node_off[B] doubles, airfoil b owns nodes node_off[b]..node_off[b+1]-1
 *   alpha    alpha_off[B] angles
 *   gamma,cp sum_b N_b K_b values, airfoil b at sum_{b'<b} N_b' K_b', angle-major
 *   cl,cl_p  alpha_off[B] values
 * Airfoils are distributed over `nthreads` OpenMP threads (<= 0: default).
 * Returns the thread count used.                                           */
int oracle_solve_batch(int B, const int *node_off, const double *xy, const int *alpha_off,
                       const double *alpha, const double *chord, double vinf, double *gamma,
                       double *cp, double *cl, double *cl_p, int *info, int nthreads)
{
    long long *sol_off = malloc(sizeof(long long) * (size_t)(B + 1));
    sol_off[0] = 0;
    for (int b = 0; b < B; ++b) {
        long long N = node_off[b + 1] - node_off[b] - 1;
        long long K = alpha_off[b + 1] - alpha_off[b];
        sol_off[b + 1] = sol_off[b] + N * K;
    }
    int used = 1;
#ifdef _OPENMP
    if (nthreads <= 0)
        nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
    for (int b = 0; b < B; ++b) {
        int N = node_off[b + 1] - node_off[b] - 1;
        int K = alpha_off[b + 1] - alpha_off[b];
        double c = chord ? chord[b] : 1.0;
        info[b] = oracle_solve_airfoil(N, xy + 2 * (size_t)node_off[b], K, alpha + alpha_off[b], vinf, c,
                                       gamma + sol_off[b], cp + sol_off[b], cl + alpha_off[b],
                                       cl_p ? cl_p + alpha_off[b] : NULL);
    }
#ifdef _OPENMP
    used = nthreads;
#endif
    free(sol_off);
    return used;
}
