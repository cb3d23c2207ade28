/*
 * panel_oracle_grad.c -- FP64 CPU oracle for the geometric sensitivity of the
 * lift coefficient (TEST INFRASTRUCTURE ONLY; not linked into the product).
 *
 * Forward (tangent-linear) sensitivity of the system of Sec. 2
 *     M(P) x = r(P, alpha),   Cl = -2 sum_i x_i L_i(P) / (vinf c)
 * with respect to every node coordinate P_k (all N+1 nodes are independent
 * variables; for a closed section the physical trailing-edge derivative is
 * the sum of the entries of node 0 and node N):
 *     dx = M^{-1} (dr - dM x),
 *     dCl = -2/(vinf c) * sum_i (dx_i L_i + x_i dL_i).
 * The entry derivatives dM_ji and dL_i are obtained by the complex-step method
 * (Squire & Trapp, SIAM Review 40, 1998): evaluate the defining closed form
 * with one coordinate perturbed by i*h and read Im(.)/h, which carries no
 * subtractive cancellation.  The factorisation of M is reused for every
 * direction.  The NACA Jacobian d P / d(m, p, t) is obtained the same way.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OG_PI 3.14159265358979323846
#define OG_H 1e-30

int oracle_lu(int n, double *A, int *piv);
void oracle_lu_solve(int n, const double *LU, const int *piv, int K, double *B);
void oracle_assemble(int N, const double *xy, int K, const double *alpha, double vinf,
                     double *M, double *R);
void oracle_naca4(double m, double p, double t, int N, int closed_te, double *xy);

/* atan2 continued to complex arguments with small imaginary parts: the real
 * part is the usual atan2 of the real parts, the imaginary part carries the
 * first-order change (x dy - y dx) / (x^2 + y^2).                          */
static double complex c_atan2(double complex y, double complex x)
{
    double yr = creal(y), xr = creal(x);
    double d = (xr * cimag(y) - yr * cimag(x)) / (xr * xr + yr * yr);
    return atan2(yr, xr) + I * d;
}

/* Complex evaluation of the panel influence G_ji (same closed form as the
 * real oracle: integral over panel i of -(1/2pi) log|m_j - s| ds).         */
static double complex g_entry_c(const double complex *z, int j, int i)
{
    double complex hx = z[2 * i + 2] - z[2 * i];
    double complex hy = z[2 * i + 3] - z[2 * i + 1];
    double complex L = csqrt(hx * hx + hy * hy);
    if (i == j)
        return L / (2.0 * OG_PI) * (1.0 - clog(0.5 * L));
    double complex tx = hx / L, ty = hy / L;
    double complex mx = 0.5 * (z[2 * j] + z[2 * j + 2]);
    double complex my = 0.5 * (z[2 * j + 1] + z[2 * j + 3]);
    double complex dx = mx - z[2 * i], dy = my - z[2 * i + 1];
    double complex xi = dx * tx + dy * ty;
    double complex eta = dx * ty - dy * tx;
    double complex r1s = xi * xi + eta * eta;
    double complex r2s = (xi - L) * (xi - L) + eta * eta;
    double complex delta = c_atan2(eta, xi) - c_atan2(eta, xi - L);
    return -1.0 / (4.0 * OG_PI) * (xi * clog(r1s) - (xi - L) * clog(r2s) - 2.0 * L - 2.0 * eta * delta);
}

static double panel_len(const double *xy, int i)
{
    double hx = xy[2 * i + 2] - xy[2 * i], hy = xy[2 * i + 3] - xy[2 * i + 1];
    return sqrt(hx * hx + hy * hy);
}

/* dCl/dP for every node coordinate: grad[2k + c], k = 0..N, c = x, y.
 * Also returns dCl/dalpha in dcl_dalpha[0].  Returns the LU info.          */
int oracle_cl_gradient(int N, const double *xy, double alpha, double vinf, double chord,
                       double *grad, double *dcl_dalpha)
{
    const int n1 = N + 1;
    const int nc = 2 * (N + 1);
    double *M = malloc(sizeof(double) * (size_t)n1 * n1);
    double *x = malloc(sizeof(double) * (size_t)n1);
    double *v = malloc(sizeof(double) * (size_t)n1);
    int *piv = malloc(sizeof(int) * (size_t)n1);
    double complex *z = malloc(sizeof(double complex) * (size_t)nc);
    oracle_assemble(N, xy, 1, &alpha, vinf, M, x);
    int info = oracle_lu(n1, M, piv);
    if (info != 0)
        goto done;
    oracle_lu_solve(n1, M, piv, 1, x);
    for (int q = 0; q < nc; ++q)
        z[q] = xy[q];
    const double ca = cos(alpha), sa = sin(alpha);
    const double scale = -2.0 / (vinf * chord);

    for (int q = 0; q < nc; ++q) {
        const int k = q / 2;          /* node index          */
        const int c = q % 2;          /* 0: x, 1: y          */
        z[q] = xy[q] + I * OG_H;
        /* panels touching node k: k-1 (ends at P_k) and k (starts at P_k);
         * control points touching node k: the same indices.               */
        int lo = k - 1 < 0 ? 0 : k - 1;
        int hi = k > N - 1 ? N - 1 : k;
        for (int j = 0; j < n1; ++j)
            v[j] = 0.0;
        /* dr_j for the moving control points m_j = (P_j + P_{j+1}) / 2,
         * r_j = -vinf (m_y cos a - m_x sin a)                              */
        for (int j = lo; j <= hi; ++j) {
            double dm = 0.5;
            v[j] = c == 0 ? vinf * sa * dm : -vinf * ca * dm;
        }
        /* -(dM x)_j: entries whose panel or control point moves with P_k  */
        for (int j = 0; j < N; ++j) {
            int row_moves = (j >= lo && j <= hi);
            for (int i = 0; i < N; ++i) {
                int col_moves = (i >= lo && i <= hi);
                if (!row_moves && !col_moves)
                    continue;
                double dG = cimag(g_entry_c(z, j, i)) / OG_H;
                v[j] -= dG * x[i];
            }
        }
        oracle_lu_solve(n1, M, piv, 1, v);
        double d = 0.0;
        for (int i = 0; i < N; ++i) {
            double dL = 0.0;
            if (i >= lo && i <= hi) {
                double complex hx = z[2 * i + 2] - z[2 * i], hy = z[2 * i + 3] - z[2 * i + 1];
                dL = cimag(csqrt(hx * hx + hy * hy)) / OG_H;
            }
            d += v[i] * panel_len(xy, i) + x[i] * dL;
        }
        grad[q] = scale * d;
        z[q] = xy[q];
    }
    if (dcl_dalpha) {
        /* dr/dalpha_j = -vinf (-m_y sin a - m_x cos a); M does not depend on alpha */
        for (int j = 0; j < N; ++j) {
            double mx = 0.5 * (xy[2 * j] + xy[2 * j + 2]);
            double my = 0.5 * (xy[2 * j + 1] + xy[2 * j + 3]);
            v[j] = vinf * (my * sa + mx * ca);
        }
        v[N] = 0.0;
        oracle_lu_solve(n1, M, piv, 1, v);
        double d = 0.0;
        for (int i = 0; i < N; ++i)
            d += v[i] * panel_len(xy, i);
        dcl_dalpha[0] = scale * d;
    }
done:
    free(M);
    free(x);
    free(v);
    free(piv);
    free(z);
    return info;
}

/* Complex-step NACA 4-digit node (same definition as oracle_naca4).        */
static void naca_node_c(double complex m, double complex p, double complex t, int k, int N, int closed_te,
                        double complex *X, double complex *Y)
{
    const double a4 = closed_te ? -0.1036 : -0.1015;
    const int half = N / 2;
    int s = (k <= half) ? k : N - k;
    double x = 0.5 * (1.0 + cos(OG_PI * (double)s / (double)half));
    double complex yt = 5.0 * t * (0.2969 * sqrt(x) - 0.1260 * x - 0.3516 * x * x + 0.2843 * x * x * x
                                   + a4 * x * x * x * x);
    double complex yc, dyc;
    if (creal(m) == 0.0 && cimag(m) == 0.0) {
        yc = 0.0;
        dyc = 0.0;
    } else if (x < creal(p)) {
        yc = m / (p * p) * (2.0 * p * x - x * x);
        dyc = 2.0 * m / (p * p) * (p - x);
    } else {
        yc = m / ((1.0 - p) * (1.0 - p)) * ((1.0 - 2.0 * p) + 2.0 * p * x - x * x);
        dyc = 2.0 * m / ((1.0 - p) * (1.0 - p)) * (p - x);
    }
    double complex th = catan(dyc);
    if (k <= half) {
        *X = x - yt * csin(th);
        *Y = yc + yt * ccos(th);
    } else {
        *X = x + yt * csin(th);
        *Y = yc - yt * ccos(th);
    }
}

/* J[(2k + c)*3 + q] = d P_k,c / d theta_q, theta = (m, p, t), k = 0..N.     */
void oracle_naca4_jacobian(double m, double p, double t, int N, int closed_te, double *J)
{
    for (int q = 0; q < 3; ++q) {
        double complex mm = m, pp = p, tt = t;
        if (q == 0)
            mm += I * OG_H;
        if (q == 1)
            pp += I * OG_H;
        if (q == 2)
            tt += I * OG_H;
        for (int k = 0; k <= N; ++k) {
            int kk = (closed_te && k == N) ? 0 : k;
            double complex X, Y;
            naca_node_c(mm, pp, tt, kk, N, closed_te, &X, &Y);
            J[(2 * k) * 3 + q] = cimag(X) / OG_H;
            J[(2 * k + 1) * 3 + q] = cimag(Y) / OG_H;
        }
    }
}

/* Gradient of the weighted forces of one angle of attack,
 *     F = dcl * Cl + sum_i dcp[i] * Cp_i,   Cp_i = 1 - (x_i / vinf)^2,
 * with respect to every node coordinate (grad[2k + c], k = 0..N), by the
 * same tangent-linear sweep as oracle_cl_gradient: per coordinate,
 * dx = M^{-1}(dr - dM x), then dCl as above and dCp_i = -2 x_i dx_i / vinf^2.
 * dcp may be NULL (then F is dcl * Cl).  Returns the LU info.              */
int oracle_force_gradient(int N, const double *xy, double alpha, double vinf, double chord, double dcl,
                          const double *dcp, double *grad)
{
    const int n1 = N + 1;
    const int nc = 2 * (N + 1);
    double *M = malloc(sizeof(double) * (size_t)n1 * n1);
    double *x = malloc(sizeof(double) * (size_t)n1);
    double *v = malloc(sizeof(double) * (size_t)n1);
    int *piv = malloc(sizeof(int) * (size_t)n1);
    double complex *z = malloc(sizeof(double complex) * (size_t)nc);
    oracle_assemble(N, xy, 1, &alpha, vinf, M, x);
    int info = oracle_lu(n1, M, piv);
    if (info != 0)
        goto done;
    oracle_lu_solve(n1, M, piv, 1, x);
    for (int q = 0; q < nc; ++q)
        z[q] = xy[q];
    const double ca = cos(alpha), sa = sin(alpha);
    const double scale = -2.0 / (vinf * chord);

    for (int q = 0; q < nc; ++q) {
        const int k = q / 2;
        const int c = q % 2;
        z[q] = xy[q] + I * OG_H;
        int lo = k - 1 < 0 ? 0 : k - 1;
        int hi = k > N - 1 ? N - 1 : k;
        for (int j = 0; j < n1; ++j)
            v[j] = 0.0;
        for (int j = lo; j <= hi; ++j)
            v[j] = c == 0 ? vinf * sa * 0.5 : -vinf * ca * 0.5;
        for (int j = 0; j < N; ++j) {
            int row_moves = (j >= lo && j <= hi);
            for (int i = 0; i < N; ++i) {
                int col_moves = (i >= lo && i <= hi);
                if (!row_moves && !col_moves)
                    continue;
                v[j] -= cimag(g_entry_c(z, j, i)) / OG_H * x[i];
            }
        }
        oracle_lu_solve(n1, M, piv, 1, v);
        double dcl_q = 0.0, dcp_q = 0.0;
        for (int i = 0; i < N; ++i) {
            double dL = 0.0;
            if (i >= lo && i <= hi) {
                double complex hx = z[2 * i + 2] - z[2 * i], hy = z[2 * i + 3] - z[2 * i + 1];
                dL = cimag(csqrt(hx * hx + hy * hy)) / OG_H;
            }
            dcl_q += v[i] * panel_len(xy, i) + x[i] * dL;
            if (dcp)
                dcp_q += dcp[i] * (-2.0 * x[i] * v[i] / (vinf * vinf));
        }
        grad[q] = dcl * scale * dcl_q + dcp_q;
        z[q] = xy[q];
    }
done:
    free(M);
    free(x);
    free(v);
    free(piv);
    free(z);
    return info;
}
