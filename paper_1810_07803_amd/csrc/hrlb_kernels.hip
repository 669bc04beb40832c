// hrlb_kernels.hip -- gfx950 kernels of the half-range lattice Boltzmann Couette solver.
//
// Per Runge-Kutta stage two launches cover every instance of a batch:
//   stage_kernel  one pass over (cell, velocity) units: WENO-5 face values of the stage input
//                 (diffuse-wall ghosts at the channel ends), reduced Shakhov collision, the SSP-RK3
//                 stage combine, the store of the stage output, and FP64 partial sums of that
//                 output's moments, wall out-fluxes and (optionally) residual, reduced per tile in
//                 LDS in a fixed order.
//   cell_kernel   per cell: sums the partials over velocity groups, forms the moments of Sec. II,
//                 the relaxation time of eq. (tau), the Shakhov prefactor and the truncated
//                 equilibria of eqs. (gx), (gy) that the next stage's collision uses; per instance:
//                 the wall densities of eq. (diffuse_nw).
// Layout: populations [dist][v][cell] with cells contiguous; a thread owns 4 consecutive cells
// of one velocity, a block 64 cells x 16 velocity rows.
#include "hrlb_internal.h"

namespace hrlb {

enum : int { FLAG_RESID = 1, FLAG_STEP_DONE = 2 };

// ---- vector loads / stores of 4 consecutive cells ------------------------------------------
__device__ __forceinline__ void ld4(const float* p, float (&o)[4])
{
    const float4 v = *reinterpret_cast<const float4*>(p);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}
__device__ __forceinline__ void ld4(const double* p, double (&o)[4])
{
    const double2 a = *reinterpret_cast<const double2*>(p);
    const double2 b = *reinterpret_cast<const double2*>(p + 2);
    o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
}
__device__ __forceinline__ void st4(float* p, const float (&o)[4])
{
    *reinterpret_cast<float4*>(p) = make_float4(o[0], o[1], o[2], o[3]);
}
__device__ __forceinline__ void st4(double* p, const double (&o)[4])
{
    *reinterpret_cast<double2*>(p) = make_double2(o[0], o[1]);
    *reinterpret_cast<double2*>(p + 2) = make_double2(o[2], o[3]);
}

__device__ __forceinline__ float fast_div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double fast_div(double a, double b) { return a / b; }

// WENO-5 (Jiang & Shu) face value; a..e ordered along the upwind direction, c the upwind cell.
// The three nonlinear weights share one denominator: alpha_k (eps+b0)^2 (eps+b1)^2 (eps+b2)^2.
template <typename T>
__device__ __forceinline__ T weno5(T a, T b, T c, T d, T e)
{
    const T eps = T(1e-6);
    const T q0 = (T(2) * a - T(7) * b + T(11) * c) * T(1.0 / 6.0);
    const T q1 = (-b + T(5) * c + T(2) * d) * T(1.0 / 6.0);
    const T q2 = (T(2) * c + T(5) * d - e) * T(1.0 / 6.0);
    const T s0 = a - T(2) * b + c, r0 = a - T(4) * b + T(3) * c;
    const T s1 = b - T(2) * c + d, r1 = b - d;
    const T s2 = c - T(2) * d + e, r2 = T(3) * c - T(4) * d + e;
    const T t0 = eps + (T(13.0 / 12.0) * s0 * s0 + T(0.25) * r0 * r0);
    const T t1 = eps + (T(13.0 / 12.0) * s1 * s1 + T(0.25) * r1 * r1);
    const T t2 = eps + (T(13.0 / 12.0) * s2 * s2 + T(0.25) * r2 * r2);
    const T u0 = t0 * t0, u1 = t1 * t1, u2 = t2 * t2;
    const T a0 = T(0.1) * (u1 * u2), a1 = T(0.6) * (u0 * u2), a2 = T(0.3) * (u0 * u1);
    return fast_div(a0 * q0 + a1 * q1 + a2 * q2, a0 + a1 + a2);
}

// counter-based 32-bit hash (integer avalanche "lowbias32", C. Wellons, 2018)
__device__ __forceinline__ uint32_t hash32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// Stochastic rounding of an FP64 value to FP32 with 16 random bits: the 29 bits a conversion
// drops are incremented by r << 13 before truncation, so the value rounds away from zero with
// probability equal to its dropped fraction (resolution 2^-16 ulp).
__device__ __forceinline__ float round_stochastic(double x, uint32_t r16)
{
    unsigned long long b = (unsigned long long)__double_as_longlong(x);
    b += (unsigned long long)(r16 & 0xffffu) << 13;
    b &= ~0x1fffffffull;
    return (float)__longlong_as_double((long long)b);
}

template <typename T>
__device__ __forceinline__ T store_round(double x, int stochastic, uint32_t r16);
template <>
__device__ __forceinline__ double store_round<double>(double x, int, uint32_t) { return x; }
template <>
__device__ __forceinline__ float store_round<float>(double x, int stochastic, uint32_t r16)
{
    return stochastic ? round_stochastic(x, r16) : (float)x;
}

// Quadratic extrapolation (in cell index) of the three cells next to a wall, used for the
// ghosts of directions leaving the domain: nodes y0, y1, y2 at 0, 1, 2.
template <typename T>
__device__ __forceinline__ T ext_p3(T y0, T y1, T y2) { return y0 - T(3) * y1 + T(3) * y2; }   // t = 3
template <typename T>
__device__ __forceinline__ T ext_p4(T y0, T y1, T y2) { return T(3) * y0 - T(8) * y1 + T(6) * y2; }  // t = 4
template <typename T>
__device__ __forceinline__ T ext_m1(T y0, T y1, T y2) { return T(3) * y0 - T(3) * y1 + y2; }   // t = -1
template <typename T>
__device__ __forceinline__ T ext_m2(T y0, T y1, T y2) { return T(6) * y0 - T(8) * y1 + T(3) * y2; }  // t = -2

// ANALYZE: no update; partials of the current state f[0] (used after set-up or a state upload)
template <typename T, bool ANALYZE>
__global__ __launch_bounds__(kThreads) void stage_kernel(const InstDesc* __restrict__ descs,
                                                         const TileRef* __restrict__ tiles, int ntiles,
                                                         int stage, int flags)
{
    __shared__ double lds_mom[kMomPerPass][kRows][kTileCells];
    __shared__ double lds_red[kThreads / 64][6];

    const int tid = threadIdx.x;
    const int row = tid / kTPR, strip = tid % kTPR;
    constexpr bool analyze = ANALYZE;
    const int in_idx = analyze ? 0 : (stage == 0 ? 0 : stage == 1 ? 1 : 2);
    const int out_idx = analyze ? 0 : (stage == 0 ? 1 : stage == 1 ? 2 : 0);
    const double ca = stage == 1 ? 0.75 : stage == 2 ? (1.0 / 3.0) : 0.0;
    const double cb = stage == 1 ? 0.25 : stage == 2 ? (2.0 / 3.0) : 1.0;
    const bool want_res = (flags & FLAG_RESID) && stage == 2;

    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const TileRef tr = tiles[t];
        const InstDesc& D = descs[tr.inst];
        const int nx = D.nx, nv = D.nv, qx = D.qx, qy = D.qy;
        const int cell0 = tr.ctile * kTileCells + strip * kStrip;
        const int seg = tr.group * kRows + row;
        const bool active = cell0 < nx && seg < D.nseg;
        const bool first = cell0 == 0, last = cell0 + kStrip == nx;

        double acc[6][kStrip];
#pragma unroll
        for (int a = 0; a < 6; ++a)
#pragma unroll
            for (int c = 0; c < kStrip; ++c) acc[a][c] = 0.0;
        double wflux_l = 0, wflux_r = 0, wmom_l = 0, wmom_r = 0, rnum = 0, rden = 0;
        double pxd = 0.0;

        if (active) {
            const int hi = seg / D.segs_per_line;
            const int jc = seg - hi * D.segs_per_line;
            pxd = D.px[hi];
            const T px = (T)pxd;
            const T* __restrict__ cell = (const T*)D.cell;
            const T* __restrict__ fin = (const T*)D.f[in_idx];
            const T* __restrict__ fnn = (const T*)D.f[0];
            T* __restrict__ fout = (T*)D.f[out_idx];
            T ux[4], uy[4], Tt[4], itau[4], AS[4], A5[4], qxv[4], qyv[4], ijd[4], Gx[4];
            if (!analyze) {
                ld4(cell + SC_UX * nx + cell0, ux);
                ld4(cell + SC_UY * nx + cell0, uy);
                ld4(cell + SC_T * nx + cell0, Tt);
                ld4(cell + SC_INVTAU * nx + cell0, itau);
                ld4(cell + SC_AS * nx + cell0, AS);
                ld4(cell + SC_AS5T * nx + cell0, A5);
                ld4(cell + SC_QX * nx + cell0, qxv);
                ld4(cell + SC_QY * nx + cell0, qyv);
                ld4(cell + SC_IJD * nx + cell0, ijd);
                ld4(cell + (kNSc + hi) * nx + cell0, Gx);
            }
            double jw[4] = {0, 0, 0, 0};
            if (want_res) {
                for (int c = 0; c < 4; ++c) jw[c] = D.jdeta[cell0 + c];
            }
            const double nwl = D.dyn[DY_NWL], nwr = D.dyn[DY_NWR];
            const double Tw = D.Tw;
            const double dt = D.dt;
            uint32_t rkey = 0;
            if (D.rounding) {
                const uint32_t stepc = (uint32_t)D.dyn[DY_STEP];
                rkey = hash32(D.seed ^ hash32(stepc * 3u + (uint32_t)stage + 0x9e3779b9u));
            }
            const int vbase = hi * qy + jc * D.vpt;
            for (int k = 0; k < D.vpt; ++k) {
                const int v = vbase + k;
                const int j = v - hi * qy;
                const double pyd = D.py[j];
                const T py = (T)pyd;
                T wp[12], wc[12];
                {
                    const T* rp = fin + (size_t)v * nx;
                    const T* rc = fin + ((size_t)nv + v) * nx;
                    T tmp[4];
                    ld4(rp + (first ? cell0 : cell0 - 4), tmp);
                    for (int c = 0; c < 4; ++c) wp[c] = tmp[c];
                    ld4(rp + cell0, tmp);
                    for (int c = 0; c < 4; ++c) wp[4 + c] = tmp[c];
                    ld4(rp + (last ? cell0 : cell0 + 4), tmp);
                    for (int c = 0; c < 4; ++c) wp[8 + c] = tmp[c];
                    ld4(rc + (first ? cell0 : cell0 - 4), tmp);
                    for (int c = 0; c < 4; ++c) wc[c] = tmp[c];
                    ld4(rc + cell0, tmp);
                    for (int c = 0; c < 4; ++c) wc[4 + c] = tmp[c];
                    ld4(rc + (last ? cell0 : cell0 + 4), tmp);
                    for (int c = 0; c < 4; ++c) wc[8 + c] = tmp[c];
                }
                T op[4], oc[4];
                double ope[4], oce[4];  // FP64 value before rounding to the storage type
                if (analyze) {
                    for (int c = 0; c < 4; ++c) {
                        op[c] = wp[4 + c];
                        oc[c] = wc[4 + c];
                    }
                } else {
                    T fnp[4], fnc[4];
                    if (stage > 0) {
                        ld4(fnn + (size_t)v * nx + cell0, fnp);
                        ld4(fnn + ((size_t)nv + v) * nx + cell0, fnc);
                    }
                    const T phiwl = (T)(nwl * D.gw_l[v]), phiwr = (T)(nwr * D.gw_r[v]);
                    const T chiwl = (T)(Tw * nwl * D.gw_l[v]), chiwr = (T)(Tw * nwr * D.gw_r[v]);
                    T Fp[5], Fc[5];
                    if (px > T(0)) {
                        if (first) {
                            wp[1] = wp[2] = wp[3] = phiwl;
                            wc[1] = wc[2] = wc[3] = chiwl;
                        }
                        if (last) {
                            wp[8] = ext_p3(wp[5], wp[6], wp[7]);
                            wp[9] = ext_p4(wp[5], wp[6], wp[7]);
                            wc[8] = ext_p3(wc[5], wc[6], wc[7]);
                            wc[9] = ext_p4(wc[5], wc[6], wc[7]);
                        }
#pragma unroll
                        for (int f = 0; f < 5; ++f) {
                            Fp[f] = weno5(wp[f + 1], wp[f + 2], wp[f + 3], wp[f + 4], wp[f + 5]);
                            Fc[f] = weno5(wc[f + 1], wc[f + 2], wc[f + 3], wc[f + 4], wc[f + 5]);
                        }
                        if (first) {
                            Fp[0] = phiwl;
                            Fc[0] = chiwl;
                        }
                    } else {
                        if (first) {
                            wp[3] = ext_m1(wp[4], wp[5], wp[6]);
                            wp[2] = ext_m2(wp[4], wp[5], wp[6]);
                            wc[3] = ext_m1(wc[4], wc[5], wc[6]);
                            wc[2] = ext_m2(wc[4], wc[5], wc[6]);
                        }
                        if (last) {
                            wp[8] = wp[9] = wp[10] = phiwr;
                            wc[8] = wc[9] = wc[10] = chiwr;
                        }
#pragma unroll
                        for (int f = 0; f < 5; ++f) {
                            Fp[f] = weno5(wp[f + 6], wp[f + 5], wp[f + 4], wp[f + 3], wp[f + 2]);
                            Fc[f] = weno5(wc[f + 6], wc[f + 5], wc[f + 4], wc[f + 3], wc[f + 2]);
                        }
                        if (last) {
                            Fp[4] = phiwr;
                            Fc[4] = chiwr;
                        }
                    }
                    T Gy[4];
                    ld4(cell + (kNSc + 2 * qx + j) * nx + cell0, Gy);
                    uint32_t rbits[4] = {0, 0, 0, 0};
                    if (D.rounding) {
                        const uint32_t base = rkey ^ ((uint32_t)v * 0x85ebca6bu) ^ ((uint32_t)cell0 * 0xc2b2ae35u);
                        for (int q = 0; q < 4; ++q) rbits[q] = hash32(base + (uint32_t)q);
                    }
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const T p = wp[4 + c], x = wc[4 + c];
                        // reduced Shakhov collision, Sec. II
                        const T xx = px - ux[c], xy = py - uy[c];
                        const T x2 = xx * xx + xy * xy;
                        const T qxi = qxv[c] * xx + qyv[c] * xy;
                        const T sp = qxi * (A5[c] * x2 - T(0.8) * AS[c]);
                        const T sc = qxi * (A5[c] * x2 - T(0.4) * AS[c]);
                        const T feq = Gx[c] * Gy[c];
                        const T tp = feq + feq * sp;
                        const T tc = Tt[c] * (feq + feq * sc);
                        const T Lp = -px * (Fp[c + 1] - Fp[c]) * ijd[c] + (tp - p) * itau[c];
                        const T Lc = -px * (Fc[c + 1] - Fc[c]) * ijd[c] + (tc - x) * itau[c];
                        const double fnpd = stage > 0 ? (double)fnp[c] : 0.0;
                        const double fncd = stage > 0 ? (double)fnc[c] : 0.0;
                        // SSP-RK3 stage: out = a f^n + b (f_in + dt L(f_in)), combined in FP64
                        ope[c] = ca * fnpd + cb * ((double)p + dt * (double)Lp);
                        oce[c] = ca * fncd + cb * ((double)x + dt * (double)Lc);
                        op[c] = store_round<T>(ope[c], D.rounding, rbits[c]);
                        oc[c] = store_round<T>(oce[c], D.rounding, rbits[c] >> 16);
                        if (want_res) {
                            const double dp = ope[c] - fnpd, dc = oce[c] - fncd;
                            rnum += jw[c] * (dp * dp + dc * dc);
                            rden += jw[c] * (fnpd * fnpd + fncd * fncd);
                        }
                    }
                    st4(fout + (size_t)v * nx + cell0, op);
                    st4(fout + ((size_t)nv + v) * nx + cell0, oc);
                }
                // moments of the output (FP64): sums over this row's j of phi p_y^a and chi p_y^b
                const double py2 = pyd * pyd, py3 = py2 * pyd;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const double o = (double)op[c], x = (double)oc[c];
                    acc[0][c] += o;
                    acc[1][c] += pyd * o;
                    acc[2][c] += py2 * o;
                    acc[3][c] += py3 * o;
                    acc[4][c] += x;
                    acc[5][c] += pyd * x;
                }
                // leaving face value of the output at a wall (eq. diffuse_nw for the next stage)
                if (last && pxd > 0) {
                    const T o1 = op[1], o2 = op[2], o3 = op[3];
                    const T F = weno5(o1, o2, o3, ext_p3(o1, o2, o3), ext_p4(o1, o2, o3));
                    wflux_r += pxd * (double)F;
                    wmom_r += pxd * pyd * (double)F;
                }
                if (first && pxd < 0) {
                    const T o0 = op[0], o1 = op[1], o2 = op[2];
                    const T F = weno5(o2, o1, o0, ext_m1(o0, o1, o2), ext_m2(o0, o1, o2));
                    wflux_l += pxd * (double)F;
                    wmom_l += pxd * pyd * (double)F;
                }
            }
        }

        // ---- moments: combine the row sums with the powers of p_x, reduce rows in LDS ----------
        double m11[kNMom][kStrip];
        {
            const double px1 = pxd, px2 = pxd * pxd, px3 = px2 * pxd;
#pragma unroll
            for (int c = 0; c < kStrip; ++c) {
                const double A0 = acc[0][c], A1 = acc[1][c], A2 = acc[2][c], A3 = acc[3][c];
                const double B0 = acc[4][c], B1 = acc[5][c];
                m11[0][c] = A0;
                m11[1][c] = px1 * A0;
                m11[2][c] = A1;
                m11[3][c] = px2 * A0;
                m11[4][c] = px1 * A1;
                m11[5][c] = A2;
                m11[6][c] = px3 * A0 + px1 * A2;
                m11[7][c] = px2 * A1 + A3;
                m11[8][c] = B0;
                m11[9][c] = px1 * B0;
                m11[10][c] = B1;
            }
        }
#pragma unroll
        for (int pass = 0; pass < (kNMom + kMomPerPass - 1) / kMomPerPass; ++pass) {
#pragma unroll
            for (int mm = 0; mm < kMomPerPass; ++mm) {
                const int m = pass * kMomPerPass + mm;
                if (m < kNMom) {
#pragma unroll
                    for (int c = 0; c < kStrip; ++c) lds_mom[mm][row][strip * kStrip + c] = m11[m][c];
                }
            }
            __syncthreads();
            {
                const int mm = tid / kTileCells, cc = tid % kTileCells;
                const int m = pass * kMomPerPass + mm;
                const int cellx = tr.ctile * kTileCells + cc;
                if (m < kNMom && cellx < nx) {
                    double s = 0.0;
#pragma unroll
                    for (int r = 0; r < kRows; ++r) s += lds_mom[mm][r][cc];
                    D.mom_part[((size_t)tr.group * kNMom + m) * nx + cellx] = s;
                }
            }
            __syncthreads();
        }

        // ---- wall out-fluxes and residual: block sums in a fixed order -------------------------
        const bool has_l = tr.ctile == 0, has_r = tr.ctile == D.nctiles - 1;
        if (has_l || has_r || want_res) {
            double vals[6] = {wflux_l, wflux_r, wmom_l, wmom_r, rnum, rden};
            const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                double s = vals[q];
                for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
                if (lane == 0) lds_red[wave][q] = s;
            }
            __syncthreads();
            if (tid == 0) {
                double tot[6];
                for (int q = 0; q < 6; ++q) {
                    double s = 0.0;
                    for (int w = 0; w < kThreads / 64; ++w) s += lds_red[w][q];
                    tot[q] = s;
                }
                if (has_l) {
                    D.wall_part[tr.group * 4 + 0] = tot[0];
                    D.wall_part[tr.group * 4 + 2] = tot[2];
                }
                if (has_r) {
                    D.wall_part[tr.group * 4 + 1] = tot[1];
                    D.wall_part[tr.group * 4 + 3] = tot[3];
                }
                if (want_res) {
                    D.res_part[tr.tile_id * 2 + 0] = tot[4];
                    D.res_part[tr.tile_id * 2 + 1] = tot[5];
                }
            }
            __syncthreads();
        }
    }
}

// ---- per-cell kernel --------------------------------------------------------------------------
constexpr int kCyReg = 32;  // expansion orders N_y below this keep their coefficients in registers

template <typename T>
__global__ __launch_bounds__(kCellBlock) void cell_kernel(const InstDesc* __restrict__ descs,
                                                          const CellRef* __restrict__ cells, int flags)
{
    extern __shared__ double ktab[];
    const CellRef cr = cells[blockIdx.x];
    const InstDesc& D = descs[cr.inst];
    const int nx = D.nx;
    const int s = cr.cell0 + threadIdx.x;

    // the instance's quadrature tables are contiguous from wx to the end of he: stage them in LDS
    const double* gbase = D.wx;
    for (int k = threadIdx.x; k < D.ktab_n; k += blockDim.x) ktab[k] = gbase[k];
    __syncthreads();
    const double* s_wx = ktab;
    const double* s_wy = ktab + (D.wy - gbase);
    const double* s_hz = ktab + (D.hz - gbase);
    const double* s_az = ktab + (D.auxZ - gbase);
    const double* s_aw = ktab + (D.auxW - gbase);
    const double* s_hZ = ktab + (D.hZ - gbase);
    const double* s_he = ktab + (D.he - gbase);

    if (cr.cell0 == 0 && threadIdx.x == 0) {
        // eq. (diffuse_nw) with the discrete leaving fluxes of the current state
        double fl = 0, fr = 0, ml = 0, mr = 0;
        for (int g = 0; g < D.ngroups; ++g) {
            fl += D.wall_part[g * 4 + 0];
            fr += D.wall_part[g * 4 + 1];
            ml += D.wall_part[g * 4 + 2];
            mr += D.wall_part[g * 4 + 3];
        }
        const double nwl = -fl / D.den_l, nwr = -fr / D.den_r;
        D.dyn[DY_NWL] = nwl;
        D.dyn[DY_NWR] = nwr;
        D.dyn[DY_SHEAR_L] = ml + nwl * D.mom_l;
        D.dyn[DY_SHEAR_R] = mr + nwr * D.mom_r;
        if (flags & FLAG_STEP_DONE) D.dyn[DY_STEP] += 1.0;
    }
    if (s >= nx) return;

    double R[kNMom];
#pragma unroll
    for (int m = 0; m < kNMom; ++m) R[m] = 0.0;
    for (int g = 0; g < D.ngroups; ++g)
#pragma unroll
        for (int m = 0; m < kNMom; ++m) R[m] += D.mom_part[((size_t)g * kNMom + m) * nx + s];

    // moments of Sec. II from the raw sums (shift to the peculiar velocity xi = p - u)
    const double n = R[0];
    const double ux = R[1] / n, uy = R[2] / n;
    const double pxx = R[3] - n * ux * ux;
    const double pxy = R[4] - n * ux * uy;
    const double pyy = R[5] - n * uy * uy;
    const double tzz = R[8];
    const double Tm = (pxx + pyy + tzz) / (3.0 * n);
    const double u2 = ux * ux + uy * uy;
    const double b = R[3] + R[5];
    const double c0 = ux * R[1] + uy * R[2];
    const double cx = ux * R[3] + uy * R[4];
    const double cy = ux * R[4] + uy * R[5];
    const double qx = 0.5 * (R[6] - ux * b - 2.0 * cx + 2.0 * ux * c0 + u2 * (R[1] - ux * R[0]) + R[9] - ux * R[8]);
    const double qy = 0.5 * (R[7] - uy * b - 2.0 * cy + 2.0 * uy * c0 + u2 * (R[2] - uy * R[0]) + R[10] - uy * R[8]);

    double* F = D.fields;
    F[F_N * nx + s] = n;
    F[F_UX * nx + s] = ux;
    F[F_UY * nx + s] = uy;
    F[F_T * nx + s] = Tm;
    F[F_PXX * nx + s] = pxx;
    F[F_PXY * nx + s] = pxy;
    F[F_PYY * nx + s] = pyy;
    F[F_TZZ * nx + s] = tzz;
    F[F_QX * nx + s] = qx;
    F[F_QY * nx + s] = qy;

    // eq. (tau) with mu ~ T^omega; Shakhov prefactor (1 - Pr)/(n K_B^2 T^2)
    const double invtau = D.collisionless ? 0.0 : D.tau_pref * n * pow(Tm / D.Tw, 1.0 - D.omega);
    const double As = (1.0 - D.Pr) / (n * Tm * Tm);
    T* cell = (T*)D.cell;
    cell[SC_UX * nx + s] = (T)ux;
    cell[SC_UY * nx + s] = (T)uy;
    cell[SC_T * nx + s] = (T)Tm;
    cell[SC_INVTAU * nx + s] = (T)invtau;
    cell[SC_AS * nx + s] = (T)As;
    cell[SC_AS5T * nx + s] = (T)(As / (5.0 * Tm));
    cell[SC_QX * nx + s] = (T)qx;
    cell[SC_QY * nx + s] = (T)qy;
    cell[SC_IJD * nx + s] = (T)D.inv_jdeta[s];

    // g_x (eq. gx) as the projection of g/omega on h_0..h_N computed with the auxiliary rule;
    // the exponent for the two half-lines differs only in the sign of the term linear in u
    const int qxn = D.qx, nxo = D.nxo;
    const double inv2T = 0.5 / Tm;
    const double rsT = 1.0 / sqrt(Tm);
    double Ip[kMaxNx + 1], Im[kMaxNx + 1];
#pragma unroll
    for (int l = 0; l <= kMaxNx; ++l) Ip[l] = Im[l] = 0.0;
    for (int k = 0; k < kAux; ++k) {
        const double Z = s_az[k];
        const double a = (Z * Z * (Tm - 1.0) - ux * ux) * inv2T;
        const double bb = Z * ux * (2.0 * inv2T);
        const double wk = s_aw[k] * rsT;
        const double ep = wk * exp(a + bb), em = wk * exp(a - bb);
#pragma unroll
        for (int l = 0; l <= kMaxNx; ++l)
            if (l <= nxo) {
                const double hz = s_hZ[l * kAux + k];
                Ip[l] += ep * hz;
                Im[l] += em * hz;
            }
    }
    for (int i = 0; i < qxn; ++i) {
        double ap = 0.0, am = 0.0;
#pragma unroll
        for (int l = 0; l <= kMaxNx; ++l)
            if (l <= nxo) {
                const double hz = s_hz[l * qxn + i];
                ap += Ip[l] * hz;
                am += Im[l] * hz;
            }
        const double nw = n * s_wx[i];
        cell[(kNSc + i) * nx + s] = (T)(nw * ap);
        cell[(kNSc + qxn + i) * nx + s] = (T)(nw * am);
    }

    // g_y (eq. gy): c_l = coefficient of t^l in exp(u t + (T-1) t^2/2), l c_l = u c_{l-1} + (T-1) c_{l-2}
    const int nqy = D.qy, nyo = D.nyo;
    const double tm1 = Tm - 1.0;
    if (nyo < kCyReg) {
        double cl[kCyReg];
        cl[0] = 1.0;
        cl[1] = uy;
#pragma unroll
        for (int l = 2; l < kCyReg; ++l) cl[l] = (uy * cl[l - 1] + tm1 * cl[l - 2]) * (1.0 / l);
        for (int j = 0; j < nqy; ++j) {
            double acc = 0.0;
#pragma unroll
            for (int l = 0; l < kCyReg; ++l)
                if (l <= nyo) acc += cl[l] * s_he[l * nqy + j];
            cell[(kNSc + 2 * qxn + j) * nx + s] = (T)(s_wy[j] * acc);
        }
    } else {
        for (int j = 0; j < nqy; ++j) {
            double c2 = 1.0, c1 = uy;
            double acc = s_he[j] + uy * s_he[nqy + j];
            for (int l = 2; l <= nyo; ++l) {
                const double c = (uy * c1 + tm1 * c2) / l;
                acc += c * s_he[l * nqy + j];
                c2 = c1;
                c1 = c;
            }
            cell[(kNSc + 2 * qxn + j) * nx + s] = (T)(s_wy[j] * acc);
        }
    }
}

// ---- per-instance reductions at a check point: residual, mean P_xy, mass ----------------------
__global__ __launch_bounds__(256) void finalize_kernel(const InstDesc* __restrict__ descs, int with_res)
{
    __shared__ double red[256][4];
    const InstDesc& D = descs[blockIdx.x];
    const int nx = D.nx;
    double a = 0, b = 0, c = 0, d = 0;
    if (with_res) {
        const int nt = D.nctiles * D.ngroups;
        for (int t = threadIdx.x; t < nt; t += 256) {
            a += D.res_part[t * 2 + 0];
            b += D.res_part[t * 2 + 1];
        }
    }
    for (int s = threadIdx.x; s < nx; s += 256) {
        c += D.jdeta[s] * D.fields[F_PXY * nx + s];
        d += D.jdeta[s] * D.fields[F_N * nx + s];
    }
    red[threadIdx.x][0] = a;
    red[threadIdx.x][1] = b;
    red[threadIdx.x][2] = c;
    red[threadIdx.x][3] = d;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int q = 0; q < 4; ++q) red[threadIdx.x][q] += red[threadIdx.x + w][q];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double jsum = D.jsum;
        if (with_res) {
            D.dyn[DY_RES_NUM] = red[0][0];
            D.dyn[DY_RES_DEN] = red[0][1];
        }
        D.dyn[DY_PXY_MEAN] = red[0][2] / jsum;
        D.dyn[DY_MASS] = red[0][3];
        const double chk = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        if (!(chk == chk) || chk - chk != 0.0) D.dyn[DY_FLAGS] = 1.0;
    }
}

// ---- state initialisation: rest equilibrium phi = g0[v], chi = T_w g0[v] -----------------------
template <typename T>
__global__ __launch_bounds__(256) void init_kernel(const InstDesc* __restrict__ descs, int inst)
{
    const InstDesc& D = descs[inst];
    const size_t total = (size_t)D.nv * D.nx;
    T* f0 = (T*)D.f[0];
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (size_t)gridDim.x * blockDim.x) {
        const int v = (int)(k / D.nx);
        const double g = D.g0[v];
        f0[k] = (T)g;
        f0[total + k] = (T)(D.Tw * g);
    }
}

}  // namespace hrlb

// ---- host-callable launchers (C linkage inside the library) --------------------------------------
using namespace hrlb;

extern "C" __attribute__((visibility("hidden"))) hipError_t hrlbk_stage(int fp32, const InstDesc* descs, const TileRef* tiles, int ntiles, int grid,
                                  int stage, int flags, hipStream_t st)
{
    if (ntiles <= 0) return hipSuccess;
    if (stage < 0) {
        if (fp32)
            hipLaunchKernelGGL((stage_kernel<float, true>), dim3(grid), dim3(kThreads), 0, st, descs, tiles, ntiles, 0, 0);
        else
            hipLaunchKernelGGL((stage_kernel<double, true>), dim3(grid), dim3(kThreads), 0, st, descs, tiles, ntiles, 0, 0);
    } else if (fp32) {
        hipLaunchKernelGGL((stage_kernel<float, false>), dim3(grid), dim3(kThreads), 0, st, descs, tiles, ntiles, stage,
                           flags);
    } else {
        hipLaunchKernelGGL((stage_kernel<double, false>), dim3(grid), dim3(kThreads), 0, st, descs, tiles, ntiles, stage,
                           flags);
    }
    return hipGetLastError();
}

extern "C" __attribute__((visibility("hidden"))) hipError_t hrlbk_cell(int fp32, const InstDesc* descs, const CellRef* cells, int ncells, int flags,
                                 size_t shmem, hipStream_t st)
{
    if (ncells <= 0) return hipSuccess;
    if (fp32)
        hipLaunchKernelGGL(cell_kernel<float>, dim3(ncells), dim3(kCellBlock), shmem, st, descs, cells, flags);
    else
        hipLaunchKernelGGL(cell_kernel<double>, dim3(ncells), dim3(kCellBlock), shmem, st, descs, cells, flags);
    return hipGetLastError();
}

extern "C" __attribute__((visibility("hidden"))) hipError_t hrlbk_finalize(const InstDesc* descs, int ninst, int with_res, hipStream_t st)
{
    if (ninst <= 0) return hipSuccess;
    hipLaunchKernelGGL(finalize_kernel, dim3(ninst), dim3(256), 0, st, descs, with_res);
    return hipGetLastError();
}

extern "C" __attribute__((visibility("hidden"))) hipError_t hrlbk_init(int fp32, const InstDesc* descs, int inst, size_t units, hipStream_t st)
{
    int grid = (int)((units + 255) / 256);
    if (grid > 65535) grid = 65535;
    if (grid < 1) grid = 1;
    if (fp32)
        hipLaunchKernelGGL(init_kernel<float>, dim3(grid), dim3(256), 0, st, descs, inst);
    else
        hipLaunchKernelGGL(init_kernel<double>, dim3(grid), dim3(256), 0, st, descs, inst);
    return hipGetLastError();
}
