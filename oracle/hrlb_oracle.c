/*
 * hrlb_oracle.c -- plain FP64 CPU oracle for the half-range lattice Boltzmann solver of the
 * reduced Shakhov equations in planar Couette flow (Ambrus, Sharipov, Sofonea,
 * arXiv:1810.07803).
 *
 * TEST INFRASTRUCTURE.  This file is the slow, obviously-correct reference that the GPU path is
 * checked against.  Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * may build, load or call it.  It shares no code, header or table generator with the GPU
 * library; it receives its quadrature tables from oracle/quadrature.py (mpmath).
 *
 * Units: m = K_B = 1, L = 1, n_ref = 1, reference momentum p0 = 1.
 *
 * What each function follows (sections and equations of the paper):
 *   orc_gx          equation (gx), Sec. III: half-range polynomial truncation of g(p_x,u_x,T),
 *                   evaluated in binary128 (__float128) because the monomial-moment form of
 *                   (gx) is ill-conditioned in FP64 for expansion orders near 10.
 *   orc_gy          equation (gy), Sec. III: full-range truncation of g(p_y,u_y,T), FP64.
 *   orc_moments     moment definitions of Sec. II (n, u_i, T_ij, T_zz, q_x, q_y, T), two-pass.
 *   orc_tau         equation (tau) with the power-law viscosity of equation (mu), or with the
 *                   tabulated law of equations (mun) and (interp) when a table is given.
 *   orc_prandtl     Pr: the constant, or the piecewise-constant Pr_n of equation (interp).
 *   collision       reduced Shakhov equations (boltz_red) with S_phi, S_chi of Sec. II.
 *   walls           diffuse reflection, equations (diffuse) and (diffuse_nw).
 *   advection       WENO-5 of Jiang & Shu (J. Comput. Phys. 126, 1996) in finite-difference
 *                   form on the stretched grid of equation (stretch); Sec. III names the scheme.
 *   orc_step        third-order TVD Runge-Kutta of Shu & Osher (1988); Sec. III names it.
 *                   Optional local time steps for steady states (not in the paper, see below).
 *   half channel    Sec. II: phi and chi are invariant under (x, p_x, p_y) -> (-x, -p_x, -p_y),
 *                   so the right half [0, 1/2] with one diffuse wall at x = 1/2 is enough; the
 *                   grid of equation (stretch) is then the paper's own (eta in [0, artanh A]).
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *   - full channel [-1/2, 1/2]; left wall moves with -u_w, right wall with +u_w; both diffuse.
 *   - grid: eta uniform on [-artanh A, artanh A], cell centred; x = tanh(eta)/(2A);
 *     A == 0 means a uniform grid.
 *   - wall closure: two ghost layers per wall.  Directions leaving the domain through a wall
 *     use quadratic extrapolation (in cell index) of the three cells next to the wall;
 *     directions entering from a wall use the wall populations n_w g_x g_y.  The face flux
 *     on a wall face is p_x times the wall population for entering directions and p_x times
 *     the WENO face value (with extrapolated ghosts) for leaving directions.
 *   - n_w uses the discrete sums over the velocity set of the leaving face values, which
 *     makes the discrete wall mass flux exactly zero.
 *   - a second closure, selected by wall_closure = 1 and used only to check the first, drops the
 *     WENO candidate stencils that reach beyond a wall (linear weights renormalised over the rest),
 *     so that no ghost value is read; entering wall faces keep the wall population.  Both closures
 *     are consistent, so their results must agree as the grid is refined.
 *   - WENO-5 is applied to phi and chi independently, eps = 1e-6, upwinded by sign(p_x).
 *   - initial state: rest equilibrium n = 1, u = 0, T = T_w.
 *   - local time steps (lts_cap > 1, a steady-state accelerator that is not in the paper): cell s
 *     advances with dt_s = dt * max(1, min(J_s / min J, lts_cap, tau_w / (2 dt))), tau_w the
 *     relaxation time at n = 1, T = T_w (no last term when collisionless), so every cell runs at
 *     the Courant number of the smallest one.  Fluxes then leave and enter neighbouring cells with
 *     different weights, so the transient does not conserve mass: at every residual check the
 *     populations are rescaled to the rest-state mass sum_s J_s deta (n_ref = 1).  The residual is
 *     || (f_new - f_old) / dt_s || / || f_old ||.  The fixed point R(f) = 0 is the same.
 *   - half channel: the ghost cells -1, -2, -3 of velocity (p_x, p_y) hold the values of the
 *     mirrored velocity (-p_x, -p_y) in cells 0, 1, 2 (the symmetry above at x_{-1-s} = -x_s);
 *     the face at x = 0 is an ordinary WENO face for both signs of p_x.
 *
 * Velocity ordering (shared convention with the GPU library, no shared code):
 *   v = (h*Qx + i)*Qy + j,  p_x = +z_i for h = 0 and -z_i for h = 1,  p_y = z_j (ascending).
 * Population arrays are [v][cell], cells contiguous.
 */
#include <math.h>
#include <quadmath.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_EPS_WENO 1e-6

typedef struct {
    int Qx, Nx, Qy, Ny;            /* half-range order, x expansion order, full-range order, y order */
    const double *zx, *wx;         /* [Qx] positive half-range nodes and weights (sum w = 1/2)      */
    const double *phi_hi, *phi_lo; /* [(Nx+1)*Qx] Phi_{s,i} as hi + lo double pairs                */
    const double *zy, *wy;         /* [Qy] full-range nodes (ascending) and weights (sum w = 1)     */
    int ncell;                     /* number of cells across the full channel                       */
    double stretch_A;              /* 0 <= A < 1; 0 means uniform                                   */
    double delta, uw, Tw, Pr, omega;
    double dt;
    int collisionless;             /* 1: no collision term (delta -> 0 limit)                       */
    int half;                      /* 1: right half [0, 1/2] with the point symmetry at x = 0        */
    int ntab;                      /* 0: mu ~ T^omega and constant Pr; >= 2: the tabulated law      */
    const double *tabT, *tabMu, *tabPr; /* [ntab] T_n ascending, mu_n, Pr_n (= c_p mu_n / kappa_n)   */
    double lts_cap;                /* > 1: local time steps up to lts_cap * dt (steady states only)  */
    int wall_closure;              /* 0: extrapolated ghosts (the solver's reading); 1: truncated      */
                                   /* WENO stencils at the walls (a second consistent closure)         */
} orc_problem;

/* ----------------------------------------------------------------------------------------- */
/* small helpers                                                                               */
/* ----------------------------------------------------------------------------------------- */
static int nvel(const orc_problem *P) { return 2 * P->Qx * P->Qy; }

static double vel_px(const orc_problem *P, int v)
{
    int hi = v / P->Qy; /* h*Qx + i */
    int h = hi / P->Qx, i = hi % P->Qx;
    return h == 0 ? P->zx[i] : -P->zx[i];
}

static double vel_py(const orc_problem *P, int v) { return P->zy[v % P->Qy]; }

/* the velocity (-p_x, -p_y) of velocity v: the other sign of the same half-range node, and the
 * full-range node of opposite sign (the nodes are symmetric about 0, ascending) */
static int vel_mirror(const orc_problem *P, int v)
{
    int hi = v / P->Qy, j = v % P->Qy;
    int h = hi / P->Qx, i = hi % P->Qx;
    return ((1 - h) * P->Qx + i) * P->Qy + (P->Qy - 1 - j);
}

/* grid of equation (stretch): eta uniform on [0, artanh A] for the half channel (the paper's
 * cells), on [-artanh A, artanh A] for the full channel */
int orc_grid(const orc_problem *P, double *x, double *J, double *deta)
{
    int N = P->ncell;
    if (N < 1) return -1;
    if (P->half) {
        if (P->stretch_A == 0.0) {
            *deta = 0.5 / N;
            for (int s = 0; s < N; ++s) {
                x[s] = (s + 0.5) * (*deta);
                J[s] = 1.0;
            }
        } else {
            double A = P->stretch_A;
            *deta = atanh(A) / N;
            for (int s = 0; s < N; ++s) {
                double eta = (s + 0.5) * (*deta);
                double c = cosh(eta);
                x[s] = tanh(eta) / (2.0 * A);
                J[s] = 1.0 / (2.0 * A * c * c);
            }
        }
        return 0;
    }
    if (P->stretch_A == 0.0) {
        *deta = 1.0 / N;
        for (int s = 0; s < N; ++s) {
            x[s] = -0.5 + (s + 0.5) / N;
            J[s] = 1.0;
        }
    } else {
        double A = P->stretch_A;
        double emax = atanh(A);
        *deta = 2.0 * emax / N;
        for (int s = 0; s < N; ++s) {
            double eta = -emax + (s + 0.5) * (*deta);
            double c = cosh(eta);
            x[s] = tanh(eta) / (2.0 * A);
            J[s] = 1.0 / (2.0 * A * c * c);
        }
    }
    return 0;
}

/* ----------------------------------------------------------------------------------------- */
/* equilibrium truncations                                                                     */
/* ----------------------------------------------------------------------------------------- */

/* equation (gx): g_{x,i} = (w_i/2) sum_s (T/2)^{s/2} [ (1+erf z) P+_s(z) + 2 e^{-z^2}/sqrt(pi) P*_s(z) ] Phi_{s,i}
 * with z = sigma_i u sqrt(1/(2T)).  P+_s = e^{-z^2} d^s/dz^s e^{z^2} and P-_s = e^{z^2} d^s/dz^s e^{-z^2}
 * obey P+_{s+1} = 2z P+_s + 2s P+_{s-1} and P-_{s+1} = -2z P-_s - 2s P-_{s-1} (differentiate the
 * definitions once); P*_s = sum_{j<s} C(s,j) P+_j P-_{s-1-j}. */
int orc_gx(const orc_problem *P, double u, double T, double *out)
{
    int Q = P->Qx, N = P->Nx;
    if (N < 0 || N > 63 || T <= 0) return -1;
    __float128 Pp[64], Pm[64], Ps[64], binom[64][64];
    for (int s = 0; s <= N; ++s) {
        binom[s][0] = 1;
        for (int j = 1; j <= s; ++j) binom[s][j] = binom[s][j - 1] * (s - j + 1) / j;
    }
    for (int h = 0; h < 2; ++h) {
        __float128 sigma = h == 0 ? 1 : -1;
        __float128 Tq = T;
        __float128 z = sigma * (__float128)u * sqrtq(1 / (2 * Tq));
        Pp[0] = 1;
        Pm[0] = 1;
        if (N >= 1) {
            Pp[1] = 2 * z;
            Pm[1] = -2 * z;
        }
        for (int s = 1; s < N; ++s) {
            Pp[s + 1] = 2 * z * Pp[s] + 2 * s * Pp[s - 1];
            Pm[s + 1] = -2 * z * Pm[s] - 2 * s * Pm[s - 1];
        }
        for (int s = 0; s <= N; ++s) {
            __float128 acc = 0;
            for (int j = 0; j < s; ++j) acc += binom[s][j] * Pp[j] * Pm[s - 1 - j];
            Ps[s] = acc;
        }
        __float128 E = 1 + erfq(z);
        __float128 G = 2 * expq(-z * z) / sqrtq(M_PIq);
        for (int i = 0; i < Q; ++i) {
            __float128 sum = 0;
            __float128 scale = 1; /* (T/2)^{s/2} */
            __float128 half_T_root = sqrtq(Tq / 2);
            for (int s = 0; s <= N; ++s) {
                __float128 phi = (__float128)P->phi_hi[s * Q + i] + (__float128)P->phi_lo[s * Q + i];
                sum += scale * (E * Pp[s] + G * Ps[s]) * phi;
                scale *= half_T_root;
            }
            out[h * Q + i] = (double)((__float128)P->wx[i] / 2 * sum);
        }
    }
    return 0;
}

/* equation (gy): g_{y,j} = w_j sum_{l=0}^{Ny} He_l(z_j) sum_{s=0}^{l/2} (T-1)^s u^{l-2s} / (2^s s! (l-2s)!) */
int orc_gy(const orc_problem *P, double u, double T, double *out)
{
    int Q = P->Qy, N = P->Ny;
    if (N < 0 || N > 170) return -1;
    for (int j = 0; j < Q; ++j) {
        double z = P->zy[j];
        double he_prev = 0.0, he = 1.0; /* He_{-1}, He_0 */
        double sum = 0.0;
        for (int l = 0; l <= N; ++l) {
            double c = 0.0;
            for (int s = 0; 2 * s <= l; ++s) {
                double term = pow(T - 1.0, s) * pow(u, l - 2 * s) /
                              (pow(2.0, s) * tgamma(s + 1.0) * tgamma(l - 2 * s + 1.0));
                c += term;
            }
            sum += he * c;
            double he_next = z * he - l * he_prev;
            he_prev = he;
            he = he_next;
        }
        out[j] = P->wy[j] * sum;
    }
    return 0;
}

/* ----------------------------------------------------------------------------------------- */
/* moments (Sec. II), two-pass: raw sums for n and u, then central moments                     */
/* fields[k*N + s], k = n, u_x, u_y, T, P_xx, P_xy, P_yy, T_zz, q_x, q_y                      */
/* ----------------------------------------------------------------------------------------- */
int orc_moments(const orc_problem *P, const double *phi, const double *chi, double *fields)
{
    int N = P->ncell, V = nvel(P);
#pragma omp parallel for schedule(static)
    for (int s = 0; s < N; ++s) {
        double n = 0, jx = 0, jy = 0;
        for (int v = 0; v < V; ++v) {
            double f = phi[(size_t)v * N + s];
            n += f;
            jx += vel_px(P, v) * f;
            jy += vel_py(P, v) * f;
        }
        double ux = jx / n, uy = jy / n;
        double pxx = 0, pxy = 0, pyy = 0, tzz = 0, qx = 0, qy = 0;
        for (int v = 0; v < V; ++v) {
            double f = phi[(size_t)v * N + s], g = chi[(size_t)v * N + s];
            double xx = vel_px(P, v) - ux, xy = vel_py(P, v) - uy;
            double x2 = xx * xx + xy * xy;
            pxx += xx * xx * f;
            pxy += xx * xy * f;
            pyy += xy * xy * f;
            tzz += g;
            qx += 0.5 * (x2 * xx * f + xx * g);
            qy += 0.5 * (x2 * xy * f + xy * g);
        }
        double T = (pxx + pyy + tzz) / (3.0 * n);
        double *o = fields;
        o[0 * N + s] = n;
        o[1 * N + s] = ux;
        o[2 * N + s] = uy;
        o[3 * N + s] = T;
        o[4 * N + s] = pxx;
        o[5 * N + s] = pxy;
        o[6 * N + s] = pyy;
        o[7 * N + s] = tzz;
        o[8 * N + s] = qx;
        o[9 * N + s] = qy;
    }
    return 0;
}

/* index of the table interval that holds T: the largest k with T_k <= T, -1 below T_0
 * (0-based: the paper's T_n is tabT[n-1]) */
static int table_index(const orc_problem *P, double T)
{
    int k = -1;
    for (int m = 0; m < P->ntab; ++m)
        if (P->tabT[m] <= T) k = m;
    return k;
}

/* equations (mun) and (interp): on the paper's interval [T_n, T_{n+1}] the power law through the two
 * tabulated values, mu_n (T/T_n)^omega_n with omega_n = ln(mu_{n+1}/mu_n)/ln(T_{n+1}/T_n); below T_2
 * the first interval's law, above T_N the last one's */
static double mu_table(const orc_problem *P, double T)
{
    int k = table_index(P, T);
    int s = k < 0 ? 0 : (k > P->ntab - 2 ? P->ntab - 2 : k);
    double om = log(P->tabMu[s + 1] / P->tabMu[s]) / log(P->tabT[s + 1] / P->tabT[s]);
    return P->tabMu[s] * pow(T / P->tabT[s], om);
}

/* equation (interp) for Pr: Pr_1 below T_2, Pr_n on T_n <= T < T_{n+1}, Pr_N from T_N on */
double orc_prandtl(const orc_problem *P, double T)
{
    if (P->ntab < 2) return P->Pr;
    int N = P->ntab;
    if (T < P->tabT[1]) return P->tabPr[0];
    if (T >= P->tabT[N - 1]) return P->tabPr[N - 1];
    return P->tabPr[table_index(P, T)];
}

/* equation (tau) with mu(T)/mu(T_w) from equation (mu) or the table, t_ref = L/v_ref = 1/sqrt(T_w) */
double orc_tau(const orc_problem *P, double n, double T)
{
    double mu_ratio = P->ntab >= 2 ? mu_table(P, T) / mu_table(P, P->Tw) : pow(T / P->Tw, P->omega);
    return mu_ratio / (n * (T / P->Tw)) / (P->delta * sqrt(2.0)) / sqrt(P->Tw);
}

/* Collision targets phi_eq (1 + S_phi) and chi_eq (1 + S_chi) of the reduced Shakhov model at one
 * cell, for all velocities; used by the right-hand side and by the tests. */
int orc_collision_target(const orc_problem *P, const double *cell /* n,ux,uy,T,qx,qy */,
                         double *tphi, double *tchi)
{
    int Qx = P->Qx, Qy = P->Qy, V = nvel(P);
    double n = cell[0], ux = cell[1], uy = cell[2], T = cell[3], qx = cell[4], qy = cell[5];
    double *gx = malloc(sizeof(double) * 2 * Qx);
    double *gy = malloc(sizeof(double) * Qy);
    if (!gx || !gy) { free(gx); free(gy); return -1; }
    orc_gx(P, ux, T, gx);
    orc_gy(P, uy, T, gy);
    double pref = (1.0 - orc_prandtl(P, T)) / (n * T * T);
    for (int v = 0; v < V; ++v) {
        int hi = v / Qy, j = v % Qy;
        double feq = n * gx[hi] * gy[j];
        double xx = vel_px(P, v) - ux, xy = vel_py(P, v) - uy;
        double x2 = xx * xx + xy * xy;
        double qxi = qx * xx + qy * xy;
        double Sphi = pref * (x2 / (5.0 * T) - 4.0 / 5.0) * qxi;
        double Schi = pref * (x2 / (5.0 * T) - 2.0 / 5.0) * qxi;
        tphi[v] = feq * (1.0 + Sphi);
        tchi[v] = T * feq * (1.0 + Schi);
    }
    free(gx);
    free(gy);
    return 0;
}

/* ----------------------------------------------------------------------------------------- */
/* WENO-5 (Jiang & Shu): face value from five values ordered along the upwind direction,       */
/* a = f_{c-2}, b = f_{c-1}, c = f_c (upwind cell), d = f_{c+1}, e = f_{c+2}.                  */
/* orc_weno5_sub keeps only the candidate stencils whose bit is set in mask (bit k: stencil k, */
/* 0 = {a,b,c}, 1 = {b,c,d}, 2 = {c,d,e}), with their linear weights renormalised by dropping  */
/* the others; the values of the dropped stencils are never read.  mask = 7 is plain WENO-5.   */
/* ----------------------------------------------------------------------------------------- */
double orc_weno5_sub(double a, double b, double c, double d, double e, int mask)
{
    double num = 0.0, den = 0.0;
    if (mask & 1) {
        double q0 = (2.0 * a - 7.0 * b + 11.0 * c) / 6.0;
        double b0 = 13.0 / 12.0 * (a - 2.0 * b + c) * (a - 2.0 * b + c) + 0.25 * (a - 4.0 * b + 3.0 * c) * (a - 4.0 * b + 3.0 * c);
        double a0 = 0.1 / ((ORC_EPS_WENO + b0) * (ORC_EPS_WENO + b0));
        num += a0 * q0;
        den += a0;
    }
    if (mask & 2) {
        double q1 = (-b + 5.0 * c + 2.0 * d) / 6.0;
        double b1 = 13.0 / 12.0 * (b - 2.0 * c + d) * (b - 2.0 * c + d) + 0.25 * (b - d) * (b - d);
        double a1 = 0.6 / ((ORC_EPS_WENO + b1) * (ORC_EPS_WENO + b1));
        num += a1 * q1;
        den += a1;
    }
    if (mask & 4) {
        double q2 = (2.0 * c + 5.0 * d - e) / 6.0;
        double b2 = 13.0 / 12.0 * (c - 2.0 * d + e) * (c - 2.0 * d + e) + 0.25 * (3.0 * c - 4.0 * d + e) * (3.0 * c - 4.0 * d + e);
        double a2 = 0.3 / ((ORC_EPS_WENO + b2) * (ORC_EPS_WENO + b2));
        num += a2 * q2;
        den += a2;
    }
    return num / den;
}

double orc_weno5(double a, double b, double c, double d, double e) { return orc_weno5_sub(a, b, c, d, e, 7); }

/* Lagrange quadratic through (0,y0), (1,y1), (2,y2), evaluated at t */
static double extrap_quadratic(double y0, double y1, double y2, double t)
{
    double l0 = (t - 1.0) * (t - 2.0) / 2.0;
    double l1 = -t * (t - 2.0);
    double l2 = t * (t - 1.0) / 2.0;
    return l0 * y0 + l1 * y1 + l2 * y2;
}

#define NG 3 /* ghost layers per side in the extended arrays */

/* extended array e[NG + s] for s in [-NG, N+NG) */
static void fill_interior(const double *f, int N, double *e)
{
    for (int s = 0; s < N; ++s) e[NG + s] = f[s];
}

static void fill_left_extrap(double *e)
{
    for (int k = 1; k <= NG; ++k) e[NG - k] = extrap_quadratic(e[NG], e[NG + 1], e[NG + 2], -k);
}

/* half channel: cell -k holds the mirrored velocity's value in cell k-1 */
static void fill_left_mirror(double *e, const double *fm)
{
    for (int k = 1; k <= NG; ++k) e[NG - k] = fm[k - 1];
}

static void fill_right_extrap(double *e, int N)
{
    for (int k = 0; k < NG; ++k)
        e[NG + N + k] = extrap_quadratic(e[NG + N - 3], e[NG + N - 2], e[NG + N - 1], 3 + k);
}

/* face value at face f (between cells f-1 and f) for the sign of px.  Extrapolated-ghost closure:
 * plain WENO-5 over the extended row.  Truncated closure: the candidate stencils that reach a cell
 * beyond a wall (below lo or above N-1) are dropped; lo = 0 at a wall, lo = -NG where the half
 * channel's mirrored ghosts continue the row. */
static double face_value_c(const orc_problem *P, const double *e, int N, int f, double px)
{
    const double *c = e + NG;
    int mask = 7;
    if (P->wall_closure == 1) {
        int lo = P->half ? -NG : 0, hi = N - 1;
        /* first cell of stencil k in upwind order: p_x > 0 reads cells f-3+k .. f-1+k; p_x < 0 reads
         * cells f-k .. f+2-k */
        mask = 0;
        for (int k = 0; k < 3; ++k) {
            int first = px > 0 ? f - 3 + k : f - k, last = first + 2;
            if (first >= lo && last <= hi) mask |= 1 << k;
        }
        if (mask == 0) return 0.0; /* only wall faces of entering directions, whose value is overridden */
    }
    if (px > 0) return orc_weno5_sub(c[f - 3], c[f - 2], c[f - 1], c[f], c[f + 1], mask);
    return orc_weno5_sub(c[f + 2], c[f + 1], c[f], c[f - 1], c[f - 2], mask);
}

typedef struct {
    double *gxw;         /* [2Qx] g_x(0, T_w) */
    double *gyl, *gyr;   /* [Qy] g_y(-u_w, T_w), g_y(+u_w, T_w) */
} wall_tables;

static int make_wall_tables(const orc_problem *P, wall_tables *W)
{
    W->gxw = malloc(sizeof(double) * 2 * P->Qx);
    W->gyl = malloc(sizeof(double) * P->Qy);
    W->gyr = malloc(sizeof(double) * P->Qy);
    if (!W->gxw || !W->gyl || !W->gyr) return -1;
    orc_gx(P, 0.0, P->Tw, W->gxw);
    orc_gy(P, -P->uw, P->Tw, W->gyl);
    orc_gy(P, +P->uw, P->Tw, W->gyr);
    return 0;
}

static void free_wall_tables(wall_tables *W)
{
    free(W->gxw);
    free(W->gyl);
    free(W->gyr);
}

/* The extended row of one velocity (cells -NG .. N+NG-1) as the right-hand side builds it: ghosts
 * of directions leaving through a wall by quadratic extrapolation, of directions entering from a wall
 * the wall population (wall_l at the left wall, wall_r at the right one); in the half channel the
 * left ghosts hold the mirrored velocity's row fm.  Then the N+1 face values, the wall faces of
 * entering directions being the wall population (diffuse reflection, equation (diffuse)). */
int orc_row_faces(const orc_problem *P, double px, const double *f, double wall_l, double wall_r, const double *fm,
                  double *e, double *F)
{
    int N = P->ncell;
    fill_interior(f, N, e);
    if (px > 0) {
        for (int k = 1; k <= NG; ++k) e[NG - k] = wall_l;
        fill_right_extrap(e, N);
    } else {
        fill_left_extrap(e);
        for (int k = 0; k < NG; ++k) e[NG + N + k] = wall_r;
    }
    if (P->half) {
        if (!fm) return -1;
        fill_left_mirror(e, fm);
    }
    for (int fc = 0; fc <= N; ++fc) {
        if (px > 0 && fc == 0 && !P->half)
            F[fc] = wall_l;
        else if (px < 0 && fc == N)
            F[fc] = wall_r;
        else
            F[fc] = face_value_c(P, e, N, fc, px);
    }
    return 0;
}

/* ----------------------------------------------------------------------------------------- */
/* right-hand side L(f) of the reduced equations (boltz_red) for both distributions           */
/* wall_info (optional, 4 doubles): n_wL, n_wR, and the y-momentum fluxes sum_v p_x p_y F at  */
/* the left and right wall faces (half channel: n_wL = 0 and the flux through the face x = 0).  */
/* ----------------------------------------------------------------------------------------- */
int orc_rhs(const orc_problem *P, const double *phi, const double *chi, double *dphi, double *dchi,
            double *wall_info)
{
    int N = P->ncell, V = nvel(P), Qy = P->Qy;
    if (N < 8) return -1;
    double *x = malloc(sizeof(double) * N), *J = malloc(sizeof(double) * N), deta;
    double *fields = malloc(sizeof(double) * 10 * N);
    double *tphi = malloc(sizeof(double) * (size_t)V * N), *tchi = malloc(sizeof(double) * (size_t)V * N);
    double *inv_tau = malloc(sizeof(double) * N);
    double *out_face_l = malloc(sizeof(double) * V), *out_face_r = malloc(sizeof(double) * V);
    wall_tables W;
    if (!x || !J || !fields || !tphi || !tchi || !inv_tau || !out_face_l || !out_face_r ||
        make_wall_tables(P, &W))
        return -2;
    orc_grid(P, x, J, &deta);
    orc_moments(P, phi, chi, fields);

    /* collision targets per cell */
#pragma omp parallel for schedule(dynamic)
    for (int s = 0; s < N; ++s) {
        double cell[6] = {fields[0 * N + s], fields[1 * N + s], fields[2 * N + s],
                          fields[3 * N + s], fields[8 * N + s], fields[9 * N + s]};
        double *tp = malloc(sizeof(double) * V), *tc = malloc(sizeof(double) * V);
        orc_collision_target(P, cell, tp, tc);
        for (int v = 0; v < V; ++v) {
            tphi[(size_t)v * N + s] = tp[v];
            tchi[(size_t)v * N + s] = tc[v];
        }
        free(tp);
        free(tc);
        inv_tau[s] = P->collisionless ? 0.0 : 1.0 / orc_tau(P, cell[0], cell[3]);
    }

    /* leaving face values at both walls (the closure's face values), equation (diffuse_nw) */
#pragma omp parallel for schedule(static)
    for (int v = 0; v < V; ++v) {
        double *e = malloc(sizeof(double) * (N + 2 * NG));
        double px = vel_px(P, v);
        fill_interior(phi + (size_t)v * N, N, e);
        fill_left_extrap(e);
        fill_right_extrap(e, N);
        out_face_l[v] = px < 0 ? face_value_c(P, e, N, 0, px) : 0.0;
        out_face_r[v] = px > 0 ? face_value_c(P, e, N, N, px) : 0.0;
        free(e);
    }
    double numl = 0, denl = 0, numr = 0, denr = 0;
    for (int v = 0; v < V; ++v) {
        double px = vel_px(P, v);
        int hi = v / Qy, j = v % Qy;
        if (px < 0) {
            numl += px * out_face_l[v];
            denr += px * W.gxw[hi] * W.gyr[j];
        } else {
            numr += px * out_face_r[v];
            denl += px * W.gxw[hi] * W.gyl[j];
        }
    }
    double nwl = P->half ? 0.0 : -numl / denl, nwr = -numr / denr;

    double mflux_l = 0, mflux_r = 0;
    double *face_l = malloc(sizeof(double) * V), *face_r = malloc(sizeof(double) * V);
#pragma omp parallel for schedule(static)
    for (int v = 0; v < V; ++v) {
        double px = vel_px(P, v);
        int hi = v / Qy, j = v % Qy;
        double wl = nwl * W.gxw[hi] * W.gyl[j]; /* left wall population (phi) */
        double wr = nwr * W.gxw[hi] * W.gyr[j]; /* right wall population (phi) */
        double *e = malloc(sizeof(double) * (N + 2 * NG));
        double *F = malloc(sizeof(double) * (N + 1));
        for (int dist = 0; dist < 2; ++dist) {
            const double *f = (dist == 0 ? phi : chi) + (size_t)v * N;
            double *df = (dist == 0 ? dphi : dchi) + (size_t)v * N;
            const double *tg = (dist == 0 ? tphi : tchi) + (size_t)v * N;
            double wscale = dist == 0 ? 1.0 : P->Tw; /* chi_wall = K_B T_w phi_wall */
            const double *fm = P->half ? (dist == 0 ? phi : chi) + (size_t)vel_mirror(P, v) * N : NULL;
            orc_row_faces(P, px, f, wscale * wl, wscale * wr, fm, e, F);
            for (int s = 0; s < N; ++s) {
                double adv = -px * (F[s + 1] - F[s]) / (J[s] * deta);
                double col = (tg[s] - f[s]) * inv_tau[s];
                df[s] = adv + col;
            }
            if (dist == 0) {
                face_l[v] = F[0];
                face_r[v] = F[N];
            }
        }
        free(e);
        free(F);
    }
    for (int v = 0; v < V; ++v) {
        double px = vel_px(P, v), py = vel_py(P, v);
        mflux_l += px * py * face_l[v];
        mflux_r += px * py * face_r[v];
    }
    if (wall_info) {
        wall_info[0] = nwl;
        wall_info[1] = nwr;
        wall_info[2] = mflux_l;
        wall_info[3] = mflux_r;
    }
    free(face_l);
    free(face_r);
    free(x);
    free(J);
    free(fields);
    free(tphi);
    free(tchi);
    free(inv_tau);
    free(out_face_l);
    free(out_face_r);
    free_wall_tables(&W);
    return 0;
}

/* rest equilibrium n = 1, u = 0, T = T_w:  phi = g_x(0,T_w) g_y(0,T_w),  chi = T_w phi */
int orc_init_state(const orc_problem *P, double *phi, double *chi)
{
    int N = P->ncell, V = nvel(P), Qy = P->Qy;
    double *gx = malloc(sizeof(double) * 2 * P->Qx), *gy = malloc(sizeof(double) * Qy);
    if (!gx || !gy) return -1;
    orc_gx(P, 0.0, P->Tw, gx);
    orc_gy(P, 0.0, P->Tw, gy);
    for (int v = 0; v < V; ++v)
        for (int s = 0; s < N; ++s) {
            phi[(size_t)v * N + s] = gx[v / Qy] * gy[v % Qy];
            chi[(size_t)v * N + s] = P->Tw * phi[(size_t)v * N + s];
        }
    free(gx);
    free(gy);
    return 0;
}

/* relative residual || (f_new - f_old)/dt_s || / || f_old ||, J-weighted L2 over cells,
 * velocities and both distributions (dt_s = dt without local time steps) */
static double residual(const orc_problem *P, const double *J, const double *dts, const double *p0,
                       const double *c0, const double *p1, const double *c1)
{
    int N = P->ncell, V = nvel(P);
    double num = 0, den = 0;
    for (int v = 0; v < V; ++v)
        for (int s = 0; s < N; ++s) {
            size_t k = (size_t)v * N + s;
            double d2 = (p1[k] - p0[k]) * (p1[k] - p0[k]) + (c1[k] - c0[k]) * (c1[k] - c0[k]);
            num += J[s] * d2 / (dts[s] * dts[s]);
            den += J[s] * (p0[k] * p0[k] + c0[k] * c0[k]);
        }
    return sqrt(num) / sqrt(den);
}

/* per-cell time steps: dt everywhere, or the local steps of lts_cap (see the header) */
static void cell_time_steps(const orc_problem *P, const double *J, double *dts)
{
    int N = P->ncell;
    double jmin = J[0];
    for (int s = 1; s < N; ++s) jmin = J[s] < jmin ? J[s] : jmin;
    double rcoll = HUGE_VAL;
    if (!P->collisionless) rcoll = 0.5 * orc_tau(P, 1.0, P->Tw) / P->dt;
    for (int s = 0; s < N; ++s) {
        double f = 1.0;
        if (P->lts_cap > 1.0) {
            f = J[s] / jmin;
            if (f > P->lts_cap) f = P->lts_cap;
            if (f > rcoll) f = rcoll;
            if (f < 1.0) f = 1.0;
        }
        dts[s] = P->dt * f;
    }
}

/* Advance n_steps SSP-RK3 steps in place:
 *   f1 = f + dt L(f);  f2 = 3/4 f + 1/4 (f1 + dt L(f1));  f_new = 1/3 f + 2/3 (f2 + dt L(f2)).
 * If tol > 0, stop after the first step whose residual (checked every check_every steps) is
 * below tol.  Returns the number of steps taken; *res_out receives the last residual computed
 * (or -1 if none was). */
long orc_step(const orc_problem *P, double *phi, double *chi, long n_steps, int check_every, double tol,
              double *res_out)
{
    int N = P->ncell, V = nvel(P);
    size_t M = (size_t)V * N;
    double *buf = malloc(sizeof(double) * M * 8);
    double *x = malloc(sizeof(double) * N), *J = malloc(sizeof(double) * N), deta;
    double *dts = malloc(sizeof(double) * N);
    if (!buf || !x || !J || !dts) return -1;
    orc_grid(P, x, J, &deta);
    cell_time_steps(P, J, dts);
    double *p1 = buf, *c1 = buf + M, *p2 = buf + 2 * M, *c2 = buf + 3 * M;
    double *dp = buf + 4 * M, *dc = buf + 5 * M, *p0 = buf + 6 * M, *c0 = buf + 7 * M;
    double res = -1.0;
    long step;
    for (step = 0; step < n_steps; ++step) {
        memcpy(p0, phi, sizeof(double) * M);
        memcpy(c0, chi, sizeof(double) * M);
        orc_rhs(P, phi, chi, dp, dc, NULL);
        for (size_t k = 0; k < M; ++k) {
            double dt = dts[k % N];
            p1[k] = phi[k] + dt * dp[k];
            c1[k] = chi[k] + dt * dc[k];
        }
        orc_rhs(P, p1, c1, dp, dc, NULL);
        for (size_t k = 0; k < M; ++k) {
            double dt = dts[k % N];
            p2[k] = 0.75 * phi[k] + 0.25 * (p1[k] + dt * dp[k]);
            c2[k] = 0.75 * chi[k] + 0.25 * (c1[k] + dt * dc[k]);
        }
        orc_rhs(P, p2, c2, dp, dc, NULL);
        for (size_t k = 0; k < M; ++k) {
            double dt = dts[k % N];
            phi[k] = phi[k] / 3.0 + 2.0 / 3.0 * (p2[k] + dt * dp[k]);
            chi[k] = chi[k] / 3.0 + 2.0 / 3.0 * (c2[k] + dt * dc[k]);
        }
        if (check_every > 0 && (step + 1) % check_every == 0) {
            res = residual(P, J, dts, p0, c0, phi, chi);
            if (P->lts_cap > 1.0) {
                /* local steps: back to the rest-state mass sum_s J_s deta (n = 1) */
                double m = 0.0, m0 = 0.0;
                for (int s = 0; s < N; ++s) {
                    double n = 0.0;
                    for (int v = 0; v < V; ++v) n += phi[(size_t)v * N + s];
                    m += J[s] * deta * n;
                    m0 += J[s] * deta;
                }
                double scale = m0 / m;
                for (size_t k = 0; k < M; ++k) {
                    phi[k] *= scale;
                    chi[k] *= scale;
                }
            }
            if (tol > 0 && res < tol) {
                ++step;
                break;
            }
            if (!(res == res)) { /* NaN: diverged */
                ++step;
                break;
            }
        }
    }
    if (res_out) *res_out = res;
    free(buf);
    free(x);
    free(J);
    free(dts);
    return step;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
