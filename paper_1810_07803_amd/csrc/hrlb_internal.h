// hrlb_internal.h -- data layout shared by the host runtime and the gfx950 kernels of the
// half-range lattice Boltzmann Couette solver.  Not part of the public ABI (see include/hrlb.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hrlb_plan.h"

namespace hrlb {

// ---- stage kernel tiling ------------------------------------------------------------------
// A block of kThreads threads covers kTileCells consecutive cells (kStrip per thread, kTPR
// threads per velocity row) and kRows velocity rows.  A row walks `vpt` velocities sharing the
// same p_x (consecutive j), so the x-advection upwind direction is uniform along a row.  The
// walls need 3 cells per side and 16-byte loads need n_cells to be a multiple of kStrip = 4.
constexpr int kThreads = 256;
constexpr int kStrip = 4;
constexpr int kTPR = 16;
constexpr int kRows = kThreads / kTPR;        // 16
constexpr int kTileCells = kStrip * kTPR;     // 64
static_assert(kTileCells == kPlanTileCells, "tile width of the work lists");
constexpr int kMaxVpt = kTPR;                 // velocities per row are bounded by the lanes of a row
constexpr int kMomPerPass = 4;                // moments reduced per LDS pass
constexpr int kCellThreads = 256;             // threads per block of the per-cell kernel
static_assert(kCellThreads == kPlanCellThreads, "block size of the per-cell kernel's work list");
constexpr int kMaxCellLanes = 16;             // lanes per cell of the per-cell kernel (4, 8 or 16)

// auxiliary half-range Gauss rule used to project the Maxwellian on the half-range Hermite
// basis (well-conditioned replacement of the monomial-moment form of eq. gx).  The rule of a case is
// the standard one scaled to the wall temperature: nodes sqrt(T_w) Z_k, weights sqrt(T_w) W_k, i.e.
// the Gauss rule of the weight exp(-p^2/(2 T_w)), so that its accuracy depends on T/T_w and
// u/sqrt(T_w) only.  Measured against the binary128 form of eq. gx (N_x = 10, Q_x = 16 and 80,
// T_w = 1 and 3), relative to max_i |g_x,i|: at most 4e-15 for 0.3 <= T/T_w <= 2 and
// |u_x| <= 2 sqrt(T_w); 2e-13 at T/T_w = 2.4 with |u_x| <= sqrt(T_w); 4e-11 at T/T_w = 3.
constexpr int kAux = 48;
// the band in which the 48-node projection is verified to 2e-13: a cell outside it raises DY_RANGE
constexpr double kAuxTlo = 0.3, kAuxThi = 2.4, kAuxUmax = 1.0;
// A second, 24-node rule (scaled the same way) serves the cells near the wall equilibrium, where it
// is as accurate: measured the same way, at most 3e-15 for 0.7 <= T/T_w <= 1.15 and
// |u_x| <= 0.75 sqrt(T_w) (T_w = 1 and 3), but 3e-13 at T/T_w = 1.5, u = 0 and 1e-9 at T/T_w = 1.5,
// u = sqrt(T_w); so it is used for 0.7 <= T/T_w <= 1.15, |u_x| <= 0.75 sqrt(T_w).
constexpr int kAux2 = 24;
constexpr double kAux2Tlo = 0.7, kAux2Thi = 1.15, kAux2Umax = 0.75;

constexpr int kMaxQx = 128, kMaxNx = 16, kMaxQy = 64;
constexpr int kMaxViscTable = 256;  // rows of a tabulated transport law
constexpr int kNMom = 11;  // raw moment accumulators per cell

// per-cell scalars of the collision, FP64 for both storage precisions (the Shakhov factor's
// temperature and heat-flux terms are evaluated in FP64), slot-major [slot][nx]: u_x, u_y, T, 1/tau,
// 0.8 A, 0.4 A and A/(5T) with A = (1 - Pr)/(n T^2), q_x, q_y
enum : int { SC_UX = 0, SC_UY, SC_T, SC_INVTAU, SC_S8, SC_S4, SC_AS5T, SC_QX, SC_QY, kNSc };
// per-cell table in the storage precision, slot-major [slot][nx]: 1/(J_s deta), then g_x at the
// 2 Q_x nodes, then g_y at the Q_y nodes
constexpr int kGIjd = 0, kGx0 = 1;
__host__ __device__ constexpr int g_slots(int qx, int qy) { return 1 + 2 * qx + qy; }
// FP64 output fields [field][nx]
enum : int { F_N = 0, F_UX, F_UY, F_T, F_PXX, F_PXY, F_PYY, F_TZZ, F_QX, F_QY, kNFields };
// mutable per-instance FP64 scalars
enum : int {
    DY_NWL = 0,   // wall density of the left wall for the current state
    DY_NWR,       // right wall
    DY_SHEAR_L,   // y-momentum flux through the left wall face
    DY_SHEAR_R,
    DY_STEP,      // completed steps (double, exact below 2^53)
    DY_RES_NUM,   // last residual numerator  sum J (f_new - f_old)^2
    DY_RES_DEN,   // last residual denominator sum J f_old^2
    DY_PXY_MEAN,  // J-weighted channel mean of P_xy at the last check
    DY_MASS,      // sum_s J_s deta n_s at the last check
    DY_FLAGS,     // nonzero if a non-finite value was met
    DY_AVG_ON,    // nonzero: every completed step adds the fields to the running sums
    DY_AVG_STEPS, // steps summed since the last start
    DY_RANGE,     // nonzero once a cell's T/T_w or u_x/sqrt(T_w) left the verified band of eq. gx
    kNDyn = 16
};

struct InstDesc {
    int nx;        // cells
    int qx, qy;    // quadrature orders
    int nv;        // 2 qx qy
    int nxo, nyo;  // expansion orders N_x, N_y
    int vpt;       // velocities per row (divides qy)
    int segs_per_line;  // qy / vpt
    int nseg;      // 2 qx qy / vpt
    int ngroups;   // ceil(nseg / kRows)
    int nctiles;   // ceil(nx / kTileCells)
    int precision; // 0 fp64, 1 fp32 storage
    int rounding;  // 0 nearest, 1 stochastic (fp32 only)
    int collisionless;
    uint32_t seed;
    int ktab_n;    // doubles of the per-cell kernel's LDS copy of the quadrature tables (padded rows)
    int cell_lanes;  // lanes per cell in the per-cell kernel (1, 2, 4, 8 or 16)
    int nxb;       // rows of the padded h tables: gx_rows(nxo)
    int nyb;       // rows of the padded He table: gy_rows(nyo), 0 = evaluated without the table padding
    int half;      // 1: right half of the channel, mirrored ghosts at x = 0 (no left wall)
    int ntab;      // 0: mu ~ T^omega, constant Pr; >= 2: rows of the tabulated transport law
    int lts;       // 1: local time steps (mass rescaled at checked steps)
    double dt, Tw, Pr, omega;
    double mu_w;         // tabulated law: mu(T_w)
    double tau_pref;     // delta sqrt(2) sqrt(T_w): 1/tau = tau_pref n (T/T_w)^(1-omega)
    double den_l, den_r; // sum over entering directions of p_x g_x(0,T_w) g_y(-/+u_w,T_w)
    double mom_l, mom_r; // same sums weighted by p_y (incoming momentum flux per unit n_w)
    double jsum;         // sum_s J_s deta (channel width in x)
    double inv_Tw;       // 1/T_w
    double visc_y;       // 1 - omega: (T/T_w)^(1-omega) = exp(visc_y log(T inv_Tw))
    double band_tlo, band_thi, band_u;  // kAuxTlo T_w, kAuxThi T_w, kAuxUmax sqrt(T_w)
    double aux2_tlo, aux2_thi, aux2_u;  // kAux2Tlo T_w, kAux2Thi T_w, kAux2Umax sqrt(T_w)
    // device pointers (all inside the case workspace)
    void* f[3];          // state buffers, each [2][nv][nx] in the storage precision
    double* sc;          // [kNSc][nx] FP64 per-cell scalars of the collision
    void* cell;          // [g_slots(qx, qy)][nx] storage precision: 1/(J deta), g_x, g_y
    double* fields;      // [kNFields][nx]
    double* avg;         // [kNFields][nx] running sums of the fields over completed steps
    double* mom_part;    // [ngroups][kNMom][nx]
    double* res_part;    // [nctiles * ngroups][2]
    double* dyn;         // [kNDyn]
    const double* px;    // [2 qx]
    const double* py;    // [qy]
    const double* wx;    // [qx]
    const double* wy;    // [qy]
    const double* hz;    // [(nxo+1)][qx]   orthonormal half-range polynomials at the nodes
    const double* auxZ;  // [kAux]  nodes of the auxiliary rule, scaled by sqrt(T_w)
    const double* auxW;  // [kAux]  its weights, scaled by sqrt(T_w)
    const double* hZ;    // [(nxo+1)][kAux] the same polynomials at the auxiliary nodes
    const double* auxZ2; // [kAux2] the smaller auxiliary rule
    const double* auxW2; // [kAux2]
    const double* hZ2;   // [(nxo+1)][kAux2]
    const double* ktab;  // [cell_lds(qx, qy, nxb, nyb, nyo, true).total] the per-cell kernels' LDS table image
    const double* he;    // [(nyo+1)][qy]   probabilists' Hermite polynomials at the y nodes
    const double* inv_jdeta; // [nx]
    const double* jdeta;     // [nx]
    const double* gw_l;  // [nv] g_x(0,T_w) g_y(-u_w,T_w)
    const double* gw_r;  // [nv] g_x(0,T_w) g_y(+u_w,T_w)
    const double* g0;    // [nv] initial populations (rest equilibrium, n = 1)
    const double* vT;    // [ntab] tabulated law: T_k ascending
    const double* vMu;   // [ntab] mu_k
    const double* vOm;   // [ntab - 1] omega_k = ln(mu_{k+1}/mu_k) / ln(T_{k+1}/T_k)
    const double* vPr;   // [ntab] Pr_k
    const double* dts;   // [nx] time step of each cell (dt everywhere without local time steps)
    const double* jres;  // [nx] residual weight J_s deta (dt/dt_s)^2
};

// ---- padded table shapes of the per-cell kernel ---------------------------------------------
// The per-cell kernel evaluates eqs. (gx) and (gy) with loops over the expansion order unrolled at
// compile time for a few row counts; the tables are copied to LDS with zero rows up to that count.
__host__ __device__ constexpr int gx_rows(int nxo)
{
    return nxo + 1 <= 4 ? 4 : nxo + 1 <= 8 ? 8 : nxo + 1 <= 11 ? 11 : 17;
}
__host__ __device__ constexpr int gy_rows(int nyo)
{
    return nyo + 1 <= 4 ? 4 : nyo + 1 <= 8 ? 8 : nyo + 1 <= 12 ? 12 : nyo + 1 <= 16 ? 16 : nyo + 1 <= 20 ? 20
         : nyo + 1 <= 32 ? 32 : 0;
}
// LDS layout (doubles): wx[qx] wy[qy] auxZ[kAux] auxW[kAux] hZ[nxb][kAux] hz[nxb][qx] he[rows][qy]
// auxZ2[kAux2] auxW2[kAux2] hZ2[nxb][kAux2], the last three only for plans that use the 24-node rule
// (at most 8 lanes per cell; uses_aux2)
struct CellLds {
    int wx, wy, az, aw, hZ, hz, he, az2, aw2, hZ2, total;
};
__host__ __device__ constexpr bool uses_aux2(int cell_lanes) { return cell_lanes <= 8; }
__host__ __device__ inline CellLds cell_lds(int qx, int qy, int nxb, int nyb, int nyo, bool aux2)
{
    CellLds o;
    o.wx = 0;
    o.wy = o.wx + qx;
    o.az = o.wy + qy;
    o.aw = o.az + kAux;
    o.hZ = o.aw + kAux;
    o.hz = o.hZ + nxb * kAux;
    o.he = o.hz + nxb * qx;
    o.az2 = o.he + (nyb > 0 ? nyb : nyo + 1) * qy;
    o.aw2 = o.az2 + (aux2 ? kAux2 : 0);
    o.hZ2 = o.aw2 + (aux2 ? kAux2 : 0);
    o.total = o.hZ2 + (aux2 ? nxb * kAux2 : 0);
    return o;
}

// ---- tabulated transport law (host and device) -------------------------------------------
// eqs. (mun), (interp): k = the last row with T_k <= t (binary search, rows strictly increasing);
// mu from the power law of interval clamp(k, 0, n-2), i.e. the first interval's law below T_1 and the
// last one's above T_{n-1}; Pr = Pr_0 below T_1, Pr_k on [T_k, T_{k+1}), Pr_{n-1} from T_{n-1} on.
__host__ __device__ inline void visc_lookup(const double* T, const double* mu, const double* om, const double* pr,
                                            int n, double t, double* mu_out, double* pr_out)
{
    int lo = -1, hi = n;  // T[lo] <= t < T[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (T[mid] <= t)
            lo = mid;
        else
            hi = mid;
    }
    const int s = lo < 0 ? 0 : (lo > n - 2 ? n - 2 : lo);
    *mu_out = mu[s] * pow(t / T[s], om[s]);
    *pr_out = lo < 1 ? pr[0] : pr[lo];
}

// ---- equilibrium truncations (host and device) ------------------------------------------
// g_{x,i}(u,T), i < 2 qx, following eq. gx as a projection: g_{x,i} = w_i sum_l h_l(z_i) I_l with
// I_l = int_0^inf g(p; sigma_i u, T) h_l(p) dp evaluated with the auxiliary half-range rule scaled to
// T_w (nodes Z, weights W of the weight exp(-p^2/(2 T_w))/sqrt(2 pi)), on which
// g/omega_w = exp(p^2/(2 T_w) - (p-u)^2/(2T))/sqrt(T).
__host__ __device__ inline void eval_gx(int qx, int nxo, const double* wx, const double* hz,
                                        const double* auxZ, const double* auxW, const double* hZ,
                                        double Tw, double u, double T, double* out)
{
    const double inv2T = 0.5 / T;
    const double rsT = 1.0 / sqrt(T);
    for (int h = 0; h < 2; ++h) {
        const double us = h == 0 ? u : -u;
        double I[kMaxNx + 1];
        for (int l = 0; l <= nxo; ++l) I[l] = 0.0;
        for (int k = 0; k < kAux; ++k) {
            const double Z = auxZ[k];
            const double e = (Z * Z * ((T - Tw) / Tw) + 2.0 * Z * us - us * us) * inv2T;
            const double wk = auxW[k] * exp(e) * rsT;
            for (int l = 0; l <= nxo; ++l) I[l] += wk * hZ[l * kAux + k];
        }
        for (int i = 0; i < qx; ++i) {
            double s = 0.0;
            for (int l = 0; l <= nxo; ++l) s += I[l] * hz[l * qx + i];
            out[h * qx + i] = wx[i] * s;
        }
    }
}

// g_{y,j}(u,T), eq. gy: w_j sum_l He_l(y_j) c_l with c_l the coefficient of t^l in
// exp(u t + (T-1) t^2/2), i.e. l c_l = u c_{l-1} + (T-1) c_{l-2}.
__host__ __device__ inline void eval_gy(int qy, int nyo, const double* wy, const double* he, double u,
                                        double T, double* out, int stride = 1)
{
    double c[kMaxQy];
    c[0] = 1.0;
    if (nyo >= 1) c[1] = u;
    for (int l = 2; l <= nyo; ++l) c[l] = (u * c[l - 1] + (T - 1.0) * c[l - 2]) / l;
    for (int j = 0; j < qy; ++j) {
        double s = 0.0;
        for (int l = 0; l <= nyo; ++l) s += c[l] * he[l * qy + j];
        out[j * stride] = wy[j] * s;
    }
}

}  // namespace hrlb
