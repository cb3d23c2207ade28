/*
 * panel_oracle_bl.c -- plain FP64 CPU oracle of the viscous correction
 * (TEST INFRASTRUCTURE ONLY; nothing in the product links it).
 *
 * Sec. 2 of the paper: the inviscid panel solution gives the lift but no
 * drag, so a laminar boundary-layer correction (Thwaites' method) is run on
 * the surface speed of the panel solution; the genetic algorithm's fitness is
 * the lift-to-drag ratio.  The paper names the method without printing its
 * formulas; the textbook form written out here is:
 *
 *   momentum thickness  theta^2(s) = 0.45 nu U(s)^-6 int_0^s U^5 ds'
 *                       (s: arc length from the stagnation point, U the
 *                       edge speed |u|)
 *   pressure gradient   lambda = theta^2 / nu  dU/ds
 *   wall shear          tau_w = mu U l(lambda) / theta, with the usual
 *                       piecewise fits of Thwaites' correlation,
 *                       l = 0.22 + 1.57 lambda - 1.8 lambda^2     (lambda >= 0)
 *                       l = 0.22 + 1.402 lambda + 0.018 lambda / (lambda + 0.107)
 *                                                                  (lambda < 0)
 *   laminar separation  at the first station with lambda < -0.09; the
 *                       boundary layer is integrated up to it (or to the
 *                       trailing edge)
 *   drag                the friction force of the attached layer on both
 *                       surfaces along the free stream, normalised by
 *                       (1/2) rho vinf^2 c (potential flow carries no
 *                       pressure drag); nu = vinf c / Re.
 *
 * Discretisation (the GPU kernel takes the same steps): stations are the
 * panel midpoints, carrying u_j (tangential speed along the counter-
 * clockwise tangent).  The stagnation point lies between the first pair of
 * midpoints with u_j < 0 <= u_{j+1}, placed by linear interpolation of u
 * along the arc; the upper surface runs from it through j, j-1, ..., 0, the
 * lower surface through j+1, ..., N-1.  U is taken piecewise linear in s
 * between stations (U = 0 at the stagnation point), so the integral of U^5
 * over a segment of length ds is exact for it:
 *     ds (Ua^5 + Ua^4 Ub + Ua^3 Ub^2 + Ua^2 Ub^3 + Ua Ub^4 + Ub^5) / 6;
 * dU/ds by central differences between neighbouring stations (the
 * stagnation point is the first one's left neighbour, the last station
 * uses its left one).  Each station stands for its panel: its shear acts
 * over the panel length, in the flow direction sign(u_j) t_j.
 */
#include <math.h>
#include <stdlib.h>

static double shear_corr(double lam)
{
    if (lam >= 0.0)
        return 0.22 + 1.57 * lam - 1.8 * lam * lam;
    return 0.22 + 1.402 * lam + 0.018 * lam / (lam + 0.107);
}

static double seg_u5(double ds, double a, double b)
{
    return ds * (a * a * a * a * a + a * a * a * a * b + a * a * a * b * b + a * a * b * b * b + a * b * b * b * b +
                 b * b * b * b * b) / 6.0;
}

/* One surface: n stations with edge speeds U[i] > 0; ds[i] is the arc
 * length from station i-1 to station i (ds[0] from the stagnation point).
 * Writes theta[i], lam[i] (n each) and returns the index of the first
 * separated station, or n if the layer stays attached.                    */
int oracle_thwaites_surface(int n, const double *ds, const double *U, double nu, double *theta, double *lam)
{
    double F = 0.0, Uprev = 0.0;
    int sep = n;
    for (int i = 0; i < n; ++i) {
        F += seg_u5(ds[i], Uprev, U[i]);
        Uprev = U[i];
        const double u6 = U[i] * U[i] * U[i] * U[i] * U[i] * U[i];
        theta[i] = sqrt(0.45 * nu * F / u6);
    }
    for (int i = 0; i < n; ++i) {
        double dUds;
        if (n == 1) {
            dUds = U[0] / ds[0];
        } else if (i == 0) {
            dUds = (U[1] - 0.0) / (ds[0] + ds[1]);
        } else if (i == n - 1) {
            dUds = (U[i] - U[i - 1]) / ds[i];
        } else {
            dUds = (U[i + 1] - U[i - 1]) / (ds[i] + ds[i + 1]);
        }
        lam[i] = theta[i] * theta[i] / nu * dUds;
        if (sep == n && lam[i] < -0.09)
            sep = i;
    }
    return sep;
}

static void frame(const double *xy, int i, double *L, double *tx, double *ty)
{
    double hx = xy[2 * i + 2] - xy[2 * i], hy = xy[2 * i + 3] - xy[2 * i + 1];
    *L = sqrt(hx * hx + hy * hy);
    *tx = hx / *L;
    *ty = hy / *L;
}

/* Viscous correction for K angles of one airfoil.  u[k*N + j]: surface
 * speeds of the panel solution (panel_forces' gamma output), cl[k] its lift.
 * Writes cd[k], ld[k] = cl / cd, and sep[2k], sep[2k+1]: the panel at which
 * the upper / lower layer separates (-1 if it reaches the trailing edge;
 * -2 for both if no stagnation point is found, with cd = ld = NaN).        */
void oracle_thwaites(int N, const double *xy, int K, const double *alpha, const double *u, const double *cl,
                     double vinf, double chord, double re, double *cd, double *ld, int *sep)
{
    const double nu = vinf * chord / re;
    double *ds = malloc(sizeof(double) * (size_t)N);
    double *U = malloc(sizeof(double) * (size_t)N);
    double *th = malloc(sizeof(double) * (size_t)N);
    double *lm = malloc(sizeof(double) * (size_t)N);
    int *pan = malloc(sizeof(int) * (size_t)N);
    for (int k = 0; k < K; ++k) {
        const double *uk = u + (size_t)k * N;
        const double ex = cos(alpha[k]), ey = sin(alpha[k]);
        int js = -1;
        for (int j = 0; j + 1 < N; ++j)
            if (uk[j] < 0.0 && uk[j + 1] >= 0.0) {
                js = j;
                break;
            }
        if (js < 0) {
            cd[k] = ld[k] = NAN;
            sep[2 * k] = sep[2 * k + 1] = -2;
            continue;
        }
        double La, Lb, tx, ty;
        frame(xy, js, &La, &tx, &ty);
        frame(xy, js + 1, &Lb, &tx, &ty);
        const double dseg = 0.5 * (La + Lb);
        const double f = -uk[js] / (uk[js + 1] - uk[js]);   /* stagnation point: fraction from m_js */
        double drag = 0.0;
        for (int side = 0; side < 2; ++side) {
            /* upper: js, js-1, ..., 0; lower: js+1, ..., N-1 */
            const int n = side == 0 ? js + 1 : N - 1 - js;
            for (int q = 0; q < n; ++q) {
                const int j = side == 0 ? js - q : js + 1 + q;
                pan[q] = j;
                U[q] = fabs(uk[j]);
                if (q == 0) {
                    ds[q] = side == 0 ? f * dseg : (1.0 - f) * dseg;
                } else {
                    double L1, L2, a, b;
                    frame(xy, pan[q - 1], &L1, &a, &b);
                    frame(xy, j, &L2, &a, &b);
                    ds[q] = 0.5 * (L1 + L2);
                }
            }
            const int s = oracle_thwaites_surface(n, ds, U, nu, th, lm);
            sep[2 * k + side] = s < n ? pan[s] : -1;
            for (int q = 0; q < s; ++q) {
                const int j = pan[q];
                double L, jtx, jty;
                frame(xy, j, &L, &jtx, &jty);
                const double dir = uk[j] >= 0.0 ? 1.0 : -1.0;
                const double cf = 2.0 * nu * U[q] * shear_corr(lm[q]) / (th[q] * vinf * vinf);
                drag += cf * L * dir * (jtx * ex + jty * ey);
            }
        }
        cd[k] = drag / chord;
        ld[k] = cl[k] / cd[k];
    }
    free(ds);
    free(U);
    free(th);
    free(lm);
    free(pan);
}
