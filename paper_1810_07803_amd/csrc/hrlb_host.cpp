// hrlb_host.cpp -- host runtime behind include/hrlb.h: velocity sets, case set-up inside a
// caller-owned device workspace, launch sequences of the SSP-RK3 step, steady-state loop,
// read-back, and batches of cases advanced by shared launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hrlb.h"
#include "hrlb_internal.h"
#include "hrlb_plan.h"
#include "hrlb_quadrature.h"
#include "hrlb_runtime.h"

using namespace hrlb;

namespace hrlb {

namespace {
thread_local std::string g_err;
}

hrlb_status fail(hrlb_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

}  // namespace hrlb

// ------------------------------------------------------------------------------------------------
// velocity set
extern "C" hrlb_status hrlb_init_quadrature(int Qx, int Nx_order, int Qy, int Ny_order, double p0, hrlb_quad** out)
{
    if (!out) return fail(HRLB_E_INVALID, "out is NULL");
    *out = nullptr;
    if (Qx < 3 || Qx > kMaxQx) return fail(HRLB_E_INVALID, "Qx=%d outside [3,%d]", Qx, kMaxQx);
    if (Qy < 3 || Qy > kMaxQy) return fail(HRLB_E_INVALID, "Qy=%d outside [3,%d]", Qy, kMaxQy);
    if (Nx_order < 2 || Nx_order > Qx - 1 || Nx_order > kMaxNx)
        return fail(HRLB_E_INVALID, "Nx_order=%d outside [2, min(Qx-1,%d)]", Nx_order, kMaxNx);
    if (Ny_order < 2 || Ny_order > Qy - 1) return fail(HRLB_E_INVALID, "Ny_order=%d outside [2, Qy-1]", Ny_order);
    if (p0 != 1.0) return fail(HRLB_E_INVALID, "p0 must be 1 (nondimensional units)");
    hrlb_quad* q = new (std::nothrow) hrlb_quad;
    if (!q) return fail(HRLB_E_NOMEM, "host allocation failed");
    q->qx = Qx;
    q->nxo = Nx_order;
    q->qy = Qy;
    q->nyo = Ny_order;
    const int nrec = std::max(Qx, kAux) + 1;
    Recurrence hr = half_range_recurrence(nrec);
    std::vector<long double> nodes, weights;
    gauss_from_recurrence(hr, Qx, nodes, weights);
    q->zx.resize(Qx);
    q->wx.resize(Qx);
    for (int i = 0; i < Qx; ++i) {
        q->zx[i] = (double)nodes[i];
        q->wx[i] = (double)weights[i];
    }
    q->px.resize(2 * Qx);
    q->wx2.resize(2 * Qx);
    for (int i = 0; i < Qx; ++i) {
        q->px[i] = q->zx[i];
        q->px[Qx + i] = -q->zx[i];
        q->wx2[i] = q->wx2[Qx + i] = q->wx[i];
    }
    std::vector<long double> hv(nrec + 1);
    q->hz.assign((size_t)(Nx_order + 1) * Qx, 0.0);
    for (int i = 0; i < Qx; ++i) {
        orthonormal_values(hr, Nx_order, nodes[i], hv.data());
        for (int l = 0; l <= Nx_order; ++l) q->hz[(size_t)l * Qx + i] = (double)hv[l];
    }
    std::vector<long double> an, aw;
    gauss_from_recurrence(hr, kAux, an, aw);
    q->hr = hr;
    q->auxZl = an;
    q->auxWl = aw;
    q->auxZ.resize(kAux);
    q->auxW.resize(kAux);
    q->hZ.assign((size_t)(Nx_order + 1) * kAux, 0.0);
    for (int k = 0; k < kAux; ++k) {
        q->auxZ[k] = (double)an[k];
        q->auxW[k] = (double)aw[k];
        orthonormal_values(hr, Nx_order, an[k], hv.data());
        for (int l = 0; l <= Nx_order; ++l) q->hZ[(size_t)l * kAux + k] = (double)hv[l];
    }
    gauss_from_recurrence(hr, kAux2, an, aw);
    q->auxZ2l = an;
    q->auxW2l = aw;
    q->auxZ2.resize(kAux2);
    q->auxW2.resize(kAux2);
    q->hZ2.assign((size_t)(Nx_order + 1) * kAux2, 0.0);
    for (int k = 0; k < kAux2; ++k) {
        q->auxZ2[k] = (double)an[k];
        q->auxW2[k] = (double)aw[k];
        orthonormal_values(hr, Nx_order, an[k], hv.data());
        for (int l = 0; l <= Nx_order; ++l) q->hZ2[(size_t)l * kAux2 + k] = (double)hv[l];
    }
    Recurrence fr = hermite_recurrence(Qy + 1);
    std::vector<long double> yn, yw;
    gauss_from_recurrence(fr, Qy, yn, yw);
    q->zy.resize(Qy);
    q->wy.resize(Qy);
    q->he.assign((size_t)(Ny_order + 1) * Qy, 0.0);
    for (int j = 0; j < Qy; ++j) {
        q->zy[j] = (double)yn[j];
        q->wy[j] = (double)yw[j];
        long double prev = 0.0L, cur = 1.0L;
        for (int l = 0; l <= Ny_order; ++l) {
            q->he[(size_t)l * Qy + j] = (double)cur;
            const long double nx = yn[j] * cur - l * prev;
            prev = cur;
            cur = nx;
        }
    }
    *out = q;
    return HRLB_OK;
}

extern "C" hrlb_status hrlb_quadrature_nodes(const hrlb_quad* q, double* px, double* wx, double* py, double* wy)
{
    if (!q) return fail(HRLB_E_INVALID, "quadrature is NULL");
    if (px) std::copy(q->px.begin(), q->px.end(), px);
    if (wx) std::copy(q->wx2.begin(), q->wx2.end(), wx);
    if (py) std::copy(q->zy.begin(), q->zy.end(), py);
    if (wy) std::copy(q->wy.begin(), q->wy.end(), wy);
    return HRLB_OK;
}

extern "C" void hrlb_free_quadrature(hrlb_quad* q) { delete q; }

extern "C" const char* hrlb_last_error(void) { return g_err.c_str(); }

// ------------------------------------------------------------------------------------------------
// case set-up
namespace {

hrlb_status validate(const hrlb_quad* q, const hrlb_case_params* p)
{
    if (!q || !p) return fail(HRLB_E_INVALID, "NULL quadrature or parameters");
    if (!(p->delta >= 0.0) || !std::isfinite(p->delta)) return fail(HRLB_E_INVALID, "delta must be >= 0");
    if (!(p->T_w > 0.0) || !std::isfinite(p->T_w)) return fail(HRLB_E_INVALID, "T_w must be > 0");
    if (!(p->Pr > 0.0) || !std::isfinite(p->Pr)) return fail(HRLB_E_INVALID, "Pr must be > 0");
    // |u_w| <= 2 sqrt(T_w): the viscous heating of Couette flow stays below the collisionless value
    // T/T_w = 1 + u_w^2/(3 T_w) <= 2.33, inside the band where eq. (gx) is evaluated to 2e-13
    if (!std::isfinite(p->u_w) || std::fabs(p->u_w) > 2.0 * std::sqrt(p->T_w))
        return fail(HRLB_E_INVALID, "|u_w| must be <= 2 sqrt(T_w)");
    if (!std::isfinite(p->omega) || p->omega < 0.0 || p->omega > 2.0) return fail(HRLB_E_INVALID, "omega outside [0,2]");
    if (p->n_cells < 8 || p->n_cells > 65536 || p->n_cells % kStrip != 0)
        return fail(HRLB_E_INVALID, "n_cells=%d must be a multiple of %d in [8, 65536]", p->n_cells, kStrip);
    if (!(p->stretch_A >= 0.0 && p->stretch_A < 1.0)) return fail(HRLB_E_INVALID, "stretch_A outside [0,1)");
    {
        const double es = p->precision == HRLB_FP64 ? 8.0 : 4.0;
        const double state = 2.0 * 2.0 * q->qx * q->qy * (double)p->n_cells * es;
        if (state >= 2147483648.0)
            return fail(HRLB_E_INVALID, "one state buffer (%.3g bytes) must stay below 2 GiB", state);
    }
    if (p->precision != HRLB_FP64 && p->precision != HRLB_FP32_STORE_FP64_MOM)
        return fail(HRLB_E_INVALID, "unknown precision %d", p->precision);
    if (p->rounding != HRLB_ROUND_NEAREST && p->rounding != HRLB_ROUND_STOCHASTIC)
        return fail(HRLB_E_INVALID, "unknown rounding %d", p->rounding);
    if (p->dt <= 0.0 && !(p->cfl > 0.0 && p->cfl <= 2.0)) return fail(HRLB_E_INVALID, "cfl must be in (0,2] when dt <= 0");
    if (!std::isfinite(p->dt)) return fail(HRLB_E_INVALID, "dt not finite");
    if (p->tile_vpt < 0 || p->tile_vpt > kMaxVpt || (p->tile_vpt > 0 && q->qy % p->tile_vpt != 0))
        return fail(HRLB_E_INVALID, "tile_vpt=%d must be 0 or a divisor of Qy=%d up to %d", p->tile_vpt, q->qy, kMaxVpt);
    if (p->cell_lanes < 0 || p->cell_lanes > kMaxCellLanes || (p->cell_lanes & (p->cell_lanes - 1)))
        return fail(HRLB_E_INVALID, "cell_lanes=%d must be 0 or a power of two up to %d", p->cell_lanes, kMaxCellLanes);
    if (p->half_channel != 0 && p->half_channel != 1) return fail(HRLB_E_INVALID, "half_channel must be 0 or 1");
    if (!(p->local_dt_cap >= 0.0 && p->local_dt_cap <= 1e6)) return fail(HRLB_E_INVALID, "local_dt_cap outside [0, 1e6]");
    if (p->kernel_path != HRLB_PATH_AUTO && p->kernel_path != HRLB_PATH_TILED && p->kernel_path != HRLB_PATH_SMALL)
        return fail(HRLB_E_INVALID, "unknown kernel_path %d", p->kernel_path);
    if (p->visc_table_n != 0) {
        const int nt = p->visc_table_n;
        if (nt < 2 || nt > kMaxViscTable) return fail(HRLB_E_INVALID, "visc_table_n=%d outside [2, %d]", nt, kMaxViscTable);
        if (!p->visc_T || !p->visc_mu || !p->visc_Pr) return fail(HRLB_E_INVALID, "NULL transport table");
        for (int k = 0; k < nt; ++k) {
            if (!(p->visc_T[k] > 0.0) || !std::isfinite(p->visc_T[k]) || (k > 0 && !(p->visc_T[k] > p->visc_T[k - 1])))
                return fail(HRLB_E_INVALID, "visc_T must be positive, finite and strictly increasing (row %d)", k);
            if (!(p->visc_mu[k] > 0.0) || !std::isfinite(p->visc_mu[k]))
                return fail(HRLB_E_INVALID, "visc_mu[%d] must be positive and finite", k);
            if (!(p->visc_Pr[k] > 0.0) || !std::isfinite(p->visc_Pr[k]))
                return fail(HRLB_E_INVALID, "visc_Pr[%d] must be positive and finite", k);
        }
    }
    return HRLB_OK;
}


// velocities per row: the requested divisor, or the largest divisor of qy not above 8 that still
// fills the 16 rows of a group
int choose_vpt(int qx, int qy, int requested)
{
    if (requested > 0) return requested;
    const int nv = 2 * qx * qy;
    int best = 1;
    for (int d = 1; d <= std::min(std::min(qy, 8), kMaxVpt); ++d)
        if (qy % d == 0 && nv / d >= kRows) best = d;
    return best;
}

// persistent grid: at most 4096 blocks, a multiple of 8 so that block b stays on XCD b % 8

// lanes per cell of the per-cell kernel: about a quarter of the x nodes of one half-line
int auto_cell_lanes(int qx)
{
    // two lanes per cell measured best for large ragged batches on MI355X (fewer redundant per-cell
    // operations than wider splits, more parallelism than one lane); the autotuner picks wider
    // splits for a lone case with few cells
    (void)qx;
    return 2;
}

Layout make_layout(const hrlb_quad* q, const hrlb_case_params* p)
{
    Layout L{};
    const int nx = p->n_cells, qx = q->qx, qy = q->qy, nv = 2 * qx * qy;
    const size_t es = p->precision == HRLB_FP64 ? 8 : 4;
    L.vpt = choose_vpt(qx, qy, p->tile_vpt);
    const int nseg = nv / L.vpt;
    L.ngroups = (nseg + kRows - 1) / kRows;
    L.nctiles = (nx + kTileCells - 1) / kTileCells;
    L.cell_lanes = p->cell_lanes > 0 ? p->cell_lanes : auto_cell_lanes(qx);
    const int cpb = kCellThreads / L.cell_lanes;
    L.ncellblocks = cell_block_count(nx, cpb, wall_blocks_of_their_own(qx, qy));
    size_t off = 0;
    L.desc = off;
    off = align256(off + sizeof(InstDesc));
    L.dyn = off;
    off = align256(off + sizeof(double) * kNDyn);
    L.tables = off;
    size_t t = 0;
    L.t_px = t; t += 2 * qx;
    L.t_py = t; t += qy;
    L.t_wx = t; t += qx;
    L.t_wy = t; t += qy;
    L.t_hz = t; t += (size_t)(q->nxo + 1) * qx;
    L.t_az = t; t += kAux;
    L.t_aw = t; t += kAux;
    L.t_hZ = t; t += (size_t)(q->nxo + 1) * kAux;
    L.t_he = t; t += (size_t)(q->nyo + 1) * qy;
    L.t_ijd = t; t += nx;
    L.t_jd = t; t += nx;
    L.t_gwl = t; t += nv;
    L.t_gwr = t; t += nv;
    L.t_g0 = t; t += nv;
    const int nt = p->visc_table_n;
    L.t_vT = t; t += nt;
    L.t_vMu = t; t += nt;
    L.t_vOm = t; t += nt > 0 ? nt - 1 : 0;
    L.t_vPr = t; t += nt;
    L.t_dts = t; t += nx;
    L.t_jres = t; t += nx;
    L.t_az2 = t; t += kAux2;
    L.t_aw2 = t; t += kAux2;
    L.t_hZ2 = t; t += (size_t)(q->nxo + 1) * kAux2;
    // the per-cell kernels' LDS image of the quadrature tables (layout of cell_lds with the 24-node rule;
    // the layout without it is a prefix)
    L.t_img = t; t += cell_lds(qx, qy, gx_rows(q->nxo), gy_rows(q->nyo), q->nyo, true).total;
    L.t_n = t;
    off = align256(off + sizeof(double) * t);
    L.cell = off;  // FP64 scalars [kNSc][nx], then the storage-precision table [g_slots][nx]
    L.cell_g = align256(sizeof(double) * kNSc * nx);
    off = align256(off + L.cell_g + es * (size_t)g_slots(qx, qy) * nx);
    L.fields = off;
    off = align256(off + sizeof(double) * kNFields * nx);
    L.avg = off;
    off = align256(off + sizeof(double) * kNFields * nx);
    L.mom = off;
    off = align256(off + sizeof(double) * (size_t)L.ngroups * kNMom * nx);
    L.res = off;
    off = align256(off + sizeof(double) * (size_t)L.nctiles * L.ngroups * 2);
    L.tiles = off;
    L.ntile_list = (int)case_tiles(L.nctiles, L.ngroups).size();
    off = align256(off + sizeof(TileRef) * (size_t)L.ntile_list);
    L.cells = off;
    off = align256(off + sizeof(CellRef) * L.ncellblocks);
    L.ctr = off;
    off = align256(off + sizeof(unsigned) * (kXcds + 1));
    L.aux_total = off;
    // the populations: three state buffers, offsets relative to the state region
    size_t so = 0;
    for (int k = 0; k < 3; ++k) {
        L.f[k] = so;
        so = align256(so + es * 2 * (size_t)nv * nx);
    }
    L.state_total = so;
    L.total = L.aux_total + L.state_total;  // a workspace holds the auxiliary region, then the state
    return L;
}

// cell centres and J_s deta of eq. (stretch): eta uniform on [0, artanh A] for the half channel
// (Sec. III), on [-artanh A, artanh A] for the full one; A = 0 is the uniform grid
void grid_of(const hrlb_case_params* p, std::vector<double>& x, std::vector<double>& jdeta)
{
    const int N = p->n_cells;
    x.resize(N);
    jdeta.resize(N);
    if (p->half_channel) {
        if (p->stretch_A == 0.0) {
            for (int s = 0; s < N; ++s) {
                x[s] = (s + 0.5) * (0.5 / N);
                jdeta[s] = 0.5 / N;
            }
        } else {
            const double A = p->stretch_A, de = std::atanh(A) / N;
            for (int s = 0; s < N; ++s) {
                const double eta = (s + 0.5) * de;
                const double c = std::cosh(eta);
                x[s] = std::tanh(eta) / (2.0 * A);
                jdeta[s] = de / (2.0 * A * c * c);
            }
        }
        return;
    }
    if (p->stretch_A == 0.0) {
        for (int s = 0; s < N; ++s) {
            x[s] = -0.5 + (s + 0.5) / N;
            jdeta[s] = 1.0 / N;
        }
    } else {
        const double A = p->stretch_A, emax = std::atanh(A), de = 2.0 * emax / N;
        for (int s = 0; s < N; ++s) {
            const double eta = -emax + (s + 0.5) * de;
            const double c = std::cosh(eta);
            x[s] = std::tanh(eta) / (2.0 * A);
            jdeta[s] = de / (2.0 * A * c * c);
        }
    }
}



hrlb_status enqueue_eager(const Launcher& L, long n_steps, bool check_last, hipStream_t st)
{
    // the small cases: all n_steps in one launch (their check, rescaling and re-analysis inside)
    if (L.nsmall > 0 && n_steps > 0)
        HIP_TRY(hrlbk_small(L.fp32, L.small_descs, L.nsmall, (int)n_steps, check_last ? 1 : 0, L.small_lds, st));
    for (long s = 0; s < n_steps; ++s) {
        const bool chk = check_last && s + 1 == n_steps;
        for (int stage = 0; stage < 3; ++stage) {
            const int fl = (stage == 2 && chk) ? FLAG_RESID : 0;
            HIP_TRY(hrlbk_stage(L.fp32, L.descs, L.tiles, L.ntiles, L.ctr, stage, fl, L.qy_max, st));
            HIP_TRY(hrlbk_cell(L.fp32, L.descs, L.cells, L.ncellblocks, stage == 0 ? 1 : stage == 1 ? 2 : 0,
                               stage == 2 ? FLAG_STEP_DONE : 0, L.shmem, st));
        }
        if (chk) HIP_TRY(hrlbk_finalize(L.descs, L.ninst, 1, st));
        if (chk && L.any_lts) {
            // local time steps: rescale to the rest-state mass, then recompute the moments, walls and
            // equilibrium tables of the rescaled state (reproduces bit for bit what the other
            // instances of the launch already hold)
            HIP_TRY(hrlbk_renorm(L.fp32, L.descs, L.ninst, st));
            HIP_TRY(hrlbk_stage(L.fp32, L.descs, L.tiles, L.ntiles, L.ctr, -1, 0, L.qy_max, st));
            HIP_TRY(hrlbk_cell(L.fp32, L.descs, L.cells, L.ncellblocks, 0, FLAG_FIELDS, L.shmem, st));
        }
    }
    return HRLB_OK;
}

// A block of graph_steps steps (with or without the residual check on its last step) is captured
// once on a private stream and replayed on the caller's stream.
hrlb_status graph_for(Launcher& L, bool check, hipGraphExec_t* out)
{
    hipGraphExec_t& slot = check ? L.graph_check : L.graph_plain;
    if (slot && L.graph_len == L.graph_steps) {
        *out = slot;
        return HRLB_OK;
    }
    if (L.graph_len != L.graph_steps) L.drop_graphs();
    hipStream_t cap = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    hrlb_status st = HRLB_OK;
    if (e == hipSuccess) st = enqueue_eager(L, L.graph_steps, check, cap);
    hipError_t e2 = hipStreamEndCapture(cap, &g);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess && st == HRLB_OK) e = hipGraphInstantiate(&slot, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cap);
    if (st != HRLB_OK) return st;
    if (e != hipSuccess) {
        slot = nullptr;
        return fail(HRLB_E_DEVICE, "graph capture: %s", hipGetErrorString(e));
    }
    L.graph_len = L.graph_steps;
    *out = slot;
    return HRLB_OK;
}


hrlb_status analyze_case(hrlb_case* c)
{
    const int fp32 = c->p.precision == HRLB_FP32_STORE_FP64_MOM;
    HIP_TRY(hrlbk_stage(fp32, c->d_desc, c->d_tiles, c->ntiles, c->d_ctr, -1, 0, c->q->qy, c->stream));
    HIP_TRY(hrlbk_cell(fp32, c->d_desc, c->d_cells, c->L.ncellblocks, 0, FLAG_FIELDS, c->shmem, c->stream));
    HIP_TRY(hrlbk_finalize(c->d_desc, 1, 0, c->stream));
    c->needs_analyze = false;
    return HRLB_OK;
}

hrlb_status ensure_analyzed(hrlb_case* c) { return c->needs_analyze ? analyze_case(c) : HRLB_OK; }

}  // namespace

hrlb_status hrlb::enqueue_steps(Launcher& L, long n_steps, bool check_last)
{
    const int G = L.graph_steps;
    if (G < 2 || n_steps < G) return enqueue_eager(L, n_steps, check_last, L.stream);
    const long blocks = n_steps / G, rest = n_steps % G;
    for (long b = 0; b < blocks; ++b) {
        const bool chk = check_last && rest == 0 && b + 1 == blocks;
        hipGraphExec_t ex = nullptr;
        hrlb_status st = graph_for(L, chk, &ex);
        if (st != HRLB_OK) return st;
        HIP_TRY(hipGraphLaunch(ex, L.stream));
    }
    return rest ? enqueue_eager(L, rest, check_last, L.stream) : HRLB_OK;
}

extern "C" hrlb_status hrlb_case_workspace_bytes(const hrlb_quad* q, const hrlb_case_params* p, size_t* bytes)
{
    hrlb_status st = validate(q, p);
    if (st != HRLB_OK) return st;
    if (!bytes) return fail(HRLB_E_INVALID, "bytes is NULL");
    const Layout L = make_layout(q, p);
    if (!tiles_valid(case_tiles(L.nctiles, L.ngroups), (size_t)L.ntile_list, 1, &L.nctiles, &L.ngroups))
        return fail(HRLB_E_INVALID, "internal: inconsistent tile list");
    *bytes = L.total;
    return HRLB_OK;
}

namespace {
// A case whose auxiliary region (descriptor, tables, cell tables, moment and residual partials, work
// lists, counters) starts at aux and whose three state buffers start at state; both device memory of
// the caller (hrlb_init_case) or the state alone with aux in the library's static scratch
// (hrlb_init_case_static).  Validated parameters and layout.
hrlb_status init_case_in(const hrlb_quad* q, const hrlb_case_params* p, const Layout& L, char* aux, char* state,
                         hipStream_t stream, int static_dev, hrlb_case** out)
{
    hrlb_case* c = new (std::nothrow) hrlb_case;
    if (!c) return fail(HRLB_E_NOMEM, "host allocation failed");
    c->p = *p;
    c->q = q;
    c->ws = aux;
    c->ws_bytes = L.total;
    c->stream = stream;
    c->L = L;
    c->steps_done = 0;
    c->static_dev = static_dev;
    c->static_gen = 0;
    const int nx = p->n_cells, qx = q->qx, qy = q->qy, nv = 2 * qx * qy;
    c->nv = nv;
    grid_of(p, c->x, c->jdeta);

    // host tables
    std::vector<double> tab(L.t_n, 0.0);
    std::copy(q->px.begin(), q->px.end(), tab.begin() + L.t_px);
    std::copy(q->zy.begin(), q->zy.end(), tab.begin() + L.t_py);
    std::copy(q->wx.begin(), q->wx.end(), tab.begin() + L.t_wx);
    std::copy(q->wy.begin(), q->wy.end(), tab.begin() + L.t_wy);
    std::copy(q->hz.begin(), q->hz.end(), tab.begin() + L.t_hz);
    // auxiliary rules of eq. (gx) scaled to the wall temperature: nodes and weights times sqrt(T_w), the
    // orthonormal h_l at the scaled nodes (extended precision, rounded once)
    {
        const long double sw = std::sqrt((long double)p->T_w);
        std::vector<long double> hv(q->nxo + 1);
        auto scaled = [&](const std::vector<long double>& Z, const std::vector<long double>& W, size_t tz, size_t tw,
                          size_t th) {
            const int K = (int)Z.size();
            for (int k = 0; k < K; ++k) {
                const long double z = sw * Z[k];
                tab[tz + k] = (double)z;
                tab[tw + k] = (double)(sw * W[k]);
                orthonormal_values(q->hr, q->nxo, z, hv.data());
                for (int l = 0; l <= q->nxo; ++l) tab[th + (size_t)l * K + k] = (double)hv[l];
            }
        };
        scaled(q->auxZl, q->auxWl, L.t_az, L.t_aw, L.t_hZ);
        scaled(q->auxZ2l, q->auxW2l, L.t_az2, L.t_aw2, L.t_hZ2);
    }
    std::copy(q->he.begin(), q->he.end(), tab.begin() + L.t_he);
    {
        // the LDS image: every table at its offset of cell_lds, its rows beyond N_x (N_y) zero up to the
        // padded row counts (the vector starts zeroed)
        const int nxr = q->nxo + 1, nyr = q->nyo + 1;
        const CellLds lay = cell_lds(qx, qy, gx_rows(q->nxo), gy_rows(q->nyo), q->nyo, true);
        double* im = tab.data() + L.t_img;
        auto put = [&](int at, size_t from, int n) { std::copy(tab.begin() + from, tab.begin() + from + n, im + at); };
        put(lay.wx, L.t_wx, qx);
        put(lay.wy, L.t_wy, qy);
        put(lay.az, L.t_az, kAux);
        put(lay.aw, L.t_aw, kAux);
        put(lay.hZ, L.t_hZ, nxr * kAux);
        put(lay.hz, L.t_hz, nxr * qx);
        put(lay.he, L.t_he, nyr * qy);
        put(lay.az2, L.t_az2, kAux2);
        put(lay.aw2, L.t_aw2, kAux2);
        put(lay.hZ2, L.t_hZ2, nxr * kAux2);
    }
    for (int s = 0; s < nx; ++s) {
        tab[L.t_ijd + s] = 1.0 / c->jdeta[s];
        tab[L.t_jd + s] = c->jdeta[s];
    }
    // tabulated transport law: rows and the exponent of each interval, eq. (mun)
    const int nt = p->visc_table_n;
    for (int k = 0; k < nt; ++k) {
        tab[L.t_vT + k] = p->visc_T[k];
        tab[L.t_vMu + k] = p->visc_mu[k];
        tab[L.t_vPr + k] = p->visc_Pr[k];
        if (k + 1 < nt)
            tab[L.t_vOm + k] = std::log(p->visc_mu[k + 1] / p->visc_mu[k]) / std::log(p->visc_T[k + 1] / p->visc_T[k]);
    }
    std::vector<double> gxw(2 * qx), gyl(qy), gyr(qy), gy0(qy);
    eval_gx(qx, q->nxo, q->wx.data(), q->hz.data(), tab.data() + L.t_az, tab.data() + L.t_aw, tab.data() + L.t_hZ,
            p->T_w, 0.0, p->T_w, gxw.data());
    eval_gy(qy, q->nyo, q->wy.data(), q->he.data(), -p->u_w, p->T_w, gyl.data());
    eval_gy(qy, q->nyo, q->wy.data(), q->he.data(), +p->u_w, p->T_w, gyr.data());
    eval_gy(qy, q->nyo, q->wy.data(), q->he.data(), 0.0, p->T_w, gy0.data());
    double den_l = 0, den_r = 0, mom_l = 0, mom_r = 0;
    for (int v = 0; v < nv; ++v) {
        const int hi = v / qy, j = v % qy;
        tab[L.t_gwl + v] = gxw[hi] * gyl[j];
        tab[L.t_gwr + v] = gxw[hi] * gyr[j];
        tab[L.t_g0 + v] = gxw[hi] * gy0[j];
        const double pxv = q->px[hi], pyv = q->zy[j];
        if (pxv > 0) {  // enters through the left wall
            den_l += pxv * tab[L.t_gwl + v];
            mom_l += pxv * pyv * tab[L.t_gwl + v];
        } else {        // enters through the right wall
            den_r += pxv * tab[L.t_gwr + v];
            mom_r += pxv * pyv * tab[L.t_gwr + v];
        }
    }

    // time step
    double dt = p->dt;
    if (dt <= 0.0) {
        double mind = 1e300;
        for (int s = 0; s < nx; ++s) mind = std::min(mind, c->jdeta[s]);
        double maxp = 0.0;
        for (double z : q->zx) maxp = std::max(maxp, z);
        dt = p->cfl * mind / maxp;
        if (p->delta > 0.0) {
            const double tau_w = 1.0 / (p->delta * std::sqrt(2.0)) / std::sqrt(p->T_w);
            dt = std::min(dt, 0.5 * tau_w);
        }
    }
    c->dt = dt;
    // time step of each cell: dt, or the local steps of local_dt_cap (every cell at the Courant
    // number of the smallest, capped, and within half the rest-state relaxation time)
    {
        double jmin = c->jdeta[0];
        for (int s = 1; s < nx; ++s) jmin = std::min(jmin, c->jdeta[s]);
        const double rcoll = p->delta > 0.0 ? 0.5 * (1.0 / (p->delta * std::sqrt(2.0)) / std::sqrt(p->T_w)) / dt : HUGE_VAL;
        for (int s = 0; s < nx; ++s) {
            double f = 1.0;
            if (p->local_dt_cap > 1.0) {
                f = c->jdeta[s] / jmin;
                if (f > p->local_dt_cap) f = p->local_dt_cap;
                if (f > rcoll) f = rcoll;
                if (f < 1.0) f = 1.0;
            }
            const double dts = dt * f;
            tab[L.t_dts + s] = dts;
            tab[L.t_jres + s] = c->jdeta[s] * ((dt / dts) * (dt / dts));
        }
    }

    // descriptor
    InstDesc& D = c->desc;
    std::memset(&D, 0, sizeof D);
    D.nx = nx;
    D.qx = qx;
    D.qy = qy;
    D.nv = nv;
    D.nxo = q->nxo;
    D.nyo = q->nyo;
    D.vpt = L.vpt;
    D.segs_per_line = qy / L.vpt;
    D.nseg = nv / L.vpt;
    D.ngroups = L.ngroups;
    D.nctiles = L.nctiles;
    D.precision = p->precision;
    D.rounding = p->precision == HRLB_FP32_STORE_FP64_MOM ? p->rounding : 0;
    D.collisionless = p->delta == 0.0;
    D.seed = p->seed;
    D.nxb = gx_rows(q->nxo);
    D.nyb = gy_rows(q->nyo);
    D.ktab_n = cell_lds(qx, qy, D.nxb, D.nyb, q->nyo, uses_aux2(L.cell_lanes)).total;
    D.cell_lanes = L.cell_lanes;
    D.half = p->half_channel;
    D.lts = p->local_dt_cap > 1.0;
    D.ntab = nt;
    if (nt > 0) {
        double prw = 0.0;
        visc_lookup(tab.data() + L.t_vT, tab.data() + L.t_vMu, tab.data() + L.t_vOm, tab.data() + L.t_vPr, nt, p->T_w,
                    &D.mu_w, &prw);
    }
    c->shmem = sizeof(double) * (size_t)D.ktab_n;
    c->run.shmem = c->shmem;
    D.dt = dt;
    D.Tw = p->T_w;
    D.Pr = p->Pr;
    D.omega = p->omega;
    D.tau_pref = p->delta * std::sqrt(2.0) * std::sqrt(p->T_w);
    D.den_l = den_l;
    D.den_r = den_r;
    D.mom_l = mom_l;
    D.mom_r = mom_r;
    D.jsum = 0.0;
    for (int s = 0; s < nx; ++s) D.jsum += c->jdeta[s];
    D.inv_Tw = 1.0 / p->T_w;
    D.visc_y = 1.0 - p->omega;
    D.band_tlo = kAuxTlo * p->T_w;
    D.band_thi = kAuxThi * p->T_w;
    D.band_u = kAuxUmax * std::sqrt(p->T_w);
    D.aux2_tlo = kAux2Tlo * p->T_w;
    D.aux2_thi = kAux2Thi * p->T_w;
    D.aux2_u = kAux2Umax * std::sqrt(p->T_w);
    char* ws = aux;
    for (int k = 0; k < 3; ++k) D.f[k] = state + L.f[k];
    D.sc = (double*)(ws + L.cell);
    D.cell = ws + L.cell + L.cell_g;
    D.fields = (double*)(ws + L.fields);
    D.avg = (double*)(ws + L.avg);
    D.mom_part = (double*)(ws + L.mom);
    D.res_part = (double*)(ws + L.res);
    D.dyn = (double*)(ws + L.dyn);
    const double* tb = (const double*)(ws + L.tables);
    D.px = tb + L.t_px;
    D.py = tb + L.t_py;
    D.wx = tb + L.t_wx;
    D.wy = tb + L.t_wy;
    D.hz = tb + L.t_hz;
    D.auxZ = tb + L.t_az;
    D.auxW = tb + L.t_aw;
    D.hZ = tb + L.t_hZ;
    D.auxZ2 = tb + L.t_az2;
    D.auxW2 = tb + L.t_aw2;
    D.hZ2 = tb + L.t_hZ2;
    D.ktab = tb + L.t_img;
    D.he = tb + L.t_he;
    D.inv_jdeta = tb + L.t_ijd;
    D.jdeta = tb + L.t_jd;
    D.gw_l = tb + L.t_gwl;
    D.gw_r = tb + L.t_gwr;
    D.g0 = tb + L.t_g0;
    D.vT = tb + L.t_vT;
    D.vMu = tb + L.t_vMu;
    D.vOm = tb + L.t_vOm;
    D.vPr = tb + L.t_vPr;
    D.dts = tb + L.t_dts;
    D.jres = tb + L.t_jres;
    c->d_desc = (InstDesc*)(ws + L.desc);
    c->d_tiles = (TileRef*)(ws + L.tiles);
    c->d_ctr = (unsigned*)(ws + L.ctr);
    c->d_cells = (CellRef*)(ws + L.cells);

    std::vector<TileRef> tiles = case_tiles(L.nctiles, L.ngroups);
    if (!tiles_valid(tiles, (size_t)L.ntile_list, 1, &L.nctiles, &L.ngroups)) {
        delete c;
        return fail(HRLB_E_INVALID, "internal: inconsistent tile list");
    }
    c->ntiles = (int)tiles.size();
    // the small-case kernel when the case fits its LDS (kernel_path)
    // the small path holds a case in one workgroup's LDS: up to what the device gives a workgroup (160 KB
    // on MI355X; the kernel's registers keep it at one block per compute unit whatever its LDS)
    c->small_lds = hrlbk_small_lds(&D);
    const size_t small_max = hrlbk_small_lds_max();
    const bool fits = c->small_lds <= small_max && D.nxb <= 11 && D.nyb != 0 && D.nyb <= 12;
    if (p->kernel_path == HRLB_PATH_SMALL && !fits) {
        const size_t need = c->small_lds;
        delete c;
        return fail(HRLB_E_INVALID,
                    "the small path takes cases of at most %zu bytes of LDS (this one: %zu) and expansion orders "
                    "N_x <= 10, N_y <= 11", small_max, need);
    }
    c->small = p->kernel_path == HRLB_PATH_SMALL || (p->kernel_path == HRLB_PATH_AUTO && fits);
    c->run.fp32 = p->precision == HRLB_FP32_STORE_FP64_MOM;
    c->run.stream = c->stream;
    c->run.qy_max = qy;
    if (c->small) {
        c->run.small_descs = c->d_desc;
        c->run.nsmall = 1;
        c->run.small_lds = c->small_lds;
    } else {
        c->run.descs = c->d_desc;
        c->run.ninst = 1;
        c->run.tiles = c->d_tiles;
        c->run.ctr = c->d_ctr;
        c->run.ntiles = c->ntiles;
        c->run.cells = c->d_cells;
        c->run.ncellblocks = L.ncellblocks;
        c->run.any_lts = p->local_dt_cap > 1.0;
    }
    std::vector<CellRef> cells;
    cells = plan_cell_blocks(std::vector<int>{nx}, std::vector<int>{kCellThreads / L.cell_lanes},
                             std::vector<char>{(char)wall_blocks_of_their_own(qx, qy)});
    if ((int)cells.size() != L.ncellblocks) {
        delete c;
        return fail(HRLB_E_INVALID, "internal: inconsistent cell-block list");
    }
    std::vector<double> dyn(kNDyn, 0.0);
    dyn[DY_NWL] = dyn[DY_NWR] = 1.0;

    hipError_t e = hipSuccess;
    auto cp = [&](size_t off, const void* src, size_t n) {
        if (e == hipSuccess) e = hipMemcpyAsync(ws + off, src, n, hipMemcpyHostToDevice, c->stream);
    };
    cp(L.desc, &D, sizeof D);
    cp(L.dyn, dyn.data(), sizeof(double) * kNDyn);
    cp(L.tables, tab.data(), sizeof(double) * tab.size());
    cp(L.tiles, tiles.data(), sizeof(TileRef) * tiles.size());
    cp(L.cells, cells.data(), sizeof(CellRef) * cells.size());
    const std::vector<unsigned> zeros(kXcds + 1, 0u);
    cp(L.ctr, zeros.data(), sizeof(unsigned) * zeros.size());
    if (e == hipSuccess) e = hrlbk_init(p->precision == HRLB_FP32_STORE_FP64_MOM, c->d_desc, 0, (size_t)nv * nx, c->stream);
    // the host staging vectors above must outlive the enqueued copies: wait on every path
    const hipError_t es = hipStreamSynchronize(c->stream);
    if (e != hipSuccess || es != hipSuccess) {
        delete c;
        return fail(HRLB_E_DEVICE, "case upload: %s", hipGetErrorString(e != hipSuccess ? e : es));
    }
    // moments and equilibrium tables of the initial state are computed lazily (one analysis pass per
    // case, or one for a whole batch); the initial mass follows from the uniform rest state
    c->needs_analyze = true;
    double n0 = 0.0;
    for (int v = 0; v < nv; ++v) n0 += tab[L.t_g0 + v];
    c->mass0 = n0 * D.jsum;
    *out = c;
    return HRLB_OK;
}

// generation of the static case last created on each device (0: none yet)
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
unsigned long g_static_gen[kMaxDevices] = {};
}  // namespace

// a case created by hrlb_init_case_static is live until the next one on its device replaces it
hrlb_status hrlb::case_live(const hrlb_case* c)
{
    if (!c) return fail(HRLB_E_INVALID, "case is NULL");
    if (c->static_dev < 0) return HRLB_OK;
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (g_static_gen[c->static_dev] != c->static_gen)
        return fail(HRLB_E_INVALID, "static case superseded by a later hrlb_init_case_static on device %d",
                    c->static_dev);
    return HRLB_OK;
}

extern "C" hrlb_status hrlb_init_case(const hrlb_quad* q, const hrlb_case_params* p, void* dev_workspace,
                                      size_t ws_bytes, void* hip_stream, hrlb_case** out)
{
    if (!out) return fail(HRLB_E_INVALID, "out is NULL");
    *out = nullptr;
    hrlb_status st = validate(q, p);
    if (st != HRLB_OK) return st;
    if (!dev_workspace) return fail(HRLB_E_INVALID, "device workspace is NULL");
    if (((uintptr_t)dev_workspace) & 255) return fail(HRLB_E_INVALID, "device workspace must be 256-byte aligned");
    const Layout L = make_layout(q, p);
    if (ws_bytes < L.total)
        return fail(HRLB_E_NOMEM, "workspace of %zu bytes < %zu required", ws_bytes, L.total);
    char* ws = (char*)dev_workspace;
    return init_case_in(q, p, L, ws, ws + L.aux_total, (hipStream_t)hip_stream, -1, out);
}

extern "C" hrlb_status hrlb_case_state_bytes(const hrlb_quad* q, const hrlb_case_params* p, size_t* bytes)
{
    hrlb_status st = validate(q, p);
    if (st != HRLB_OK) return st;
    if (!bytes) return fail(HRLB_E_INVALID, "bytes is NULL");
    *bytes = make_layout(q, p).state_total;
    return HRLB_OK;
}

extern "C" hrlb_status hrlb_init_case_static(const hrlb_quad* q, const hrlb_case_params* p, void* dev_state,
                                             size_t state_bytes, void* hip_stream, hrlb_case** out)
{
    if (!out) return fail(HRLB_E_INVALID, "out is NULL");
    *out = nullptr;
    hrlb_status st = validate(q, p);
    if (st != HRLB_OK) return st;
    if (!dev_state) return fail(HRLB_E_INVALID, "device state buffer is NULL");
    if (((uintptr_t)dev_state) & 255) return fail(HRLB_E_INVALID, "device state buffer must be 256-byte aligned");
    const Layout L = make_layout(q, p);
    if (state_bytes < L.state_total)
        return fail(HRLB_E_NOMEM, "state buffer of %zu bytes < %zu required", state_bytes, L.state_total);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(HRLB_E_DEVICE, "device %d beyond the supported %d", dev, kMaxDevices);
    void* scratch = nullptr;
    size_t scratch_bytes = 0;
    HIP_TRY(hrlbk_scratch(&scratch, &scratch_bytes));
    if (L.aux_total > scratch_bytes)
        return fail(HRLB_E_INVALID,
                    "the case needs %zu bytes of tables and partial sums, beyond the %zu bytes of the static scratch",
                    L.aux_total, scratch_bytes);
    hrlb_case* c = nullptr;
    st = init_case_in(q, p, L, (char*)scratch, (char*)dev_state, (hipStream_t)hip_stream, dev, &c);
    if (st != HRLB_OK) return st;
    {
        std::lock_guard<std::mutex> lock(g_static_mu);
        c->static_gen = ++g_static_gen[dev];
    }
    *out = c;
    return HRLB_OK;
}

extern "C" void hrlb_free_case(hrlb_case* c) { delete c; }

void hrlb::range_message(long steps)
{
    fail(HRLB_E_RANGE,
         "a cell left %.1f <= T/T_w <= %.1f, |u_x| <= %.1f sqrt(T_w), where eq. (gx) is evaluated to 2e-13 "
         "(after %ld steps)", kAuxTlo, kAuxThi, kAuxUmax, steps);
}

extern "C" hrlb_status hrlb_case_flags(hrlb_case* c, unsigned* flags)
{
    if (!c || !flags) return fail(HRLB_E_INVALID, "NULL argument");
    {
        const hrlb_status sl = case_live(c);
        if (sl != HRLB_OK) return sl;
    }
    double dy[kNDyn];
    HIP_TRY(hipMemcpyAsync(dy, c->desc.dyn, sizeof dy, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    *flags = (dy[DY_FLAGS] != 0.0 ? HRLB_FLAG_NONFINITE : 0u) | (dy[DY_RANGE] != 0.0 ? HRLB_FLAG_RANGE : 0u);
    return HRLB_OK;
}

extern "C" hrlb_status hrlb_case_kernel_path(const hrlb_case* c, int* path)
{
    if (!c || !path) return fail(HRLB_E_INVALID, "NULL argument");
    *path = c->small ? HRLB_PATH_SMALL : HRLB_PATH_TILED;
    return HRLB_OK;
}

extern "C" hrlb_status hrlb_case_info(const hrlb_case* c, double* dt, int* n_vel, int* n_cells, long* steps_done)
{
    if (!c) return fail(HRLB_E_INVALID, "case is NULL");
    {
        const hrlb_status sl = case_live(c);
        if (sl != HRLB_OK) return sl;
    }
    if (dt) *dt = c->dt;
    if (n_vel) *n_vel = c->nv;
    if (n_cells) *n_cells = c->p.n_cells;
    if (steps_done) *steps_done = c->steps_done;
    return HRLB_OK;
}

extern "C" hrlb_status hrlb_step(hrlb_case* c, long n_steps)
{
    if (!c) return fail(HRLB_E_INVALID, "case is NULL");
    {
        const hrlb_status sl = case_live(c);
        if (sl != HRLB_OK) return sl;
    }
    if (n_steps < 0) return fail(HRLB_E_INVALID, "n_steps < 0");
    hrlb_status st0 = ensure_analyzed(c);
    if (st0 != HRLB_OK) return st0;
    hrlb_status st = enqueue_steps(c->run, n_steps, false);
    if (st == HRLB_OK) c->steps_done += n_steps;
    return st;
}

extern "C" hrlb_status hrlb_tune_workspace_bytes(const hrlb_quad* q, const hrlb_case_params* p, size_t* bytes)
{
    hrlb_status st = validate(q, p);
    if (st != HRLB_OK) return st;
    if (!bytes) return fail(HRLB_E_INVALID, "bytes is NULL");
    size_t mx = 0;
    for (int d = 1; d <= std::min(q->qy, kMaxVpt); ++d) {
        if (q->qy % d) continue;
        for (int l = 1; l <= kMaxCellLanes; l *= 2) {
            hrlb_case_params pp = *p;
            pp.tile_vpt = d;
            pp.cell_lanes = l;
            mx = std::max(mx, make_layout(q, &pp).total);
        }
    }
    *bytes = mx;
    return HRLB_OK;
}

namespace {
// ms per step of one plan, timed with events after a warm-up step (the case is freed again)
hrlb_status time_plan(const hrlb_quad* q, const hrlb_case_params* pp, void* ws, size_t ws_bytes, hipStream_t s,
                      int n_steps, hipEvent_t e0, hipEvent_t e1, double* ms_out)
{
    hrlb_case* c = nullptr;
    hrlb_status st = hrlb_init_case(q, pp, ws, ws_bytes, s, &c);
    if (st != HRLB_OK) return st;
    st = hrlb_step(c, 1);
    float ms = 0.0f;
    hipError_t e = hipSuccess;
    if (st == HRLB_OK) e = hipEventRecord(e0, s);
    if (st == HRLB_OK && e == hipSuccess) st = hrlb_step(c, n_steps);
    if (st == HRLB_OK && e == hipSuccess) e = hipEventRecord(e1, s);
    if (st == HRLB_OK && e == hipSuccess) e = hipEventSynchronize(e1);
    if (st == HRLB_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (st == HRLB_OK && e != hipSuccess) st = fail(HRLB_E_DEVICE, "tuning events: %s", hipGetErrorString(e));
    (void)hipStreamSynchronize(s);
    hrlb_free_case(c);
    *ms_out = ms / n_steps;
    return st;
}
}  // namespace

extern "C" hrlb_status hrlb_tune_plan(const hrlb_quad* q, const hrlb_case_params* p, void* dev_workspace,
                                      size_t ws_bytes, void* hip_stream, int n_steps, int* best_vpt,
                                      int* best_lanes, double* best_ms_per_step)
{
    size_t need = 0;
    hrlb_status st = hrlb_tune_workspace_bytes(q, p, &need);
    if (st != HRLB_OK) return st;
    if (ws_bytes < need) return fail(HRLB_E_NOMEM, "tuning workspace of %zu bytes < %zu", ws_bytes, need);
    if (n_steps < 1 || !best_vpt || !best_lanes) return fail(HRLB_E_INVALID, "n_steps < 1 or NULL output");
    hipStream_t s = (hipStream_t)hip_stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    hrlb_case_params pp = *p;
    if (pp.cell_lanes == 0) pp.cell_lanes = auto_cell_lanes(q->qx);
    double best_ms = 1e300;
    int bv = 0, bl = pp.cell_lanes;
    for (int d = 1; d <= std::min(q->qy, kMaxVpt) && st == HRLB_OK; ++d) {
        if (q->qy % d) continue;
        pp.tile_vpt = d;
        double ms = 0;
        st = time_plan(q, &pp, dev_workspace, ws_bytes, s, n_steps, e0, e1, &ms);
        if (st == HRLB_OK && ms < best_ms) {
            best_ms = ms;
            bv = d;
        }
    }
    pp.tile_vpt = bv;
    for (int l = 1; l <= kMaxCellLanes && st == HRLB_OK; l *= 2) {
        if (l == bl) continue;
        pp.cell_lanes = l;
        double ms = 0;
        st = time_plan(q, &pp, dev_workspace, ws_bytes, s, n_steps, e0, e1, &ms);
        if (st == HRLB_OK && ms < best_ms) {
            best_ms = ms;
            bl = l;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != HRLB_OK) return st;
    *best_vpt = bv;
    *best_lanes = bl;
    if (best_ms_per_step) *best_ms_per_step = best_ms;
    return HRLB_OK;
}

// Remaining absolute error of the last of m checked means of P_xy (m >= 3): the m - 1 differences d are
// taken as decaying geometrically, their rate r per check fitted by least squares to log|d| (a fit over
// several checks is not thrown off by two modes overlapping, which makes a three-point extrapolation
// under-estimate), and the error bounded by max(|d_last|, |d_prev|) r / (1 - r).  0 when the last two
// differences are exactly zero; HUGE_VAL while the fitted rate is >= 1 or another difference is zero.
double hrlb::pxy_error_bound(const double* m, int count)
{
    const int W = count - 1;
    double est = HUGE_VAL;
    bool zero = false;
    for (int k = 0; k < W; ++k) zero = zero || m[k + 1] == m[k];
    if (m[W] == m[W - 1] && m[W - 1] == m[W - 2]) return 0.0;
    if (zero) return est;
    double sy = 0.0, sxy = 0.0, sxx = 0.0;
    for (int k = 0; k < W; ++k) sy += std::log(std::fabs(m[k + 1] - m[k]));
    const double xm = 0.5 * (W - 1), ym = sy / W;
    for (int k = 0; k < W; ++k) {
        sxy += (k - xm) * (std::log(std::fabs(m[k + 1] - m[k])) - ym);
        sxx += (k - xm) * (k - xm);
    }
    const double r = std::exp(sxy / sxx);
    if (r < 1.0) est = std::max(std::fabs(m[W] - m[W - 1]), std::fabs(m[W - 1] - m[W - 2])) * r / (1.0 - r);
    return est;
}

extern "C" hrlb_status hrlb_pxy_error_estimate(const double* means, int count, double* estimate)
{
    if (!means || !estimate || count < 3) return fail(HRLB_E_INVALID, "need at least 3 means and an output pointer");
    const double last = std::fabs(means[count - 1]);
    *estimate = pxy_error_bound(means, count) / std::max(last, 1e-300);
    return HRLB_OK;
}

hrlb_status hrlb::steady_update(SteadyTrack& t, const double* dy, long n, double dt, double tol, int stop_rule)
{
    t.res = std::sqrt(dy[DY_RES_NUM]) / (dt * std::sqrt(dy[DY_RES_DEN]));
    const double pxy = dy[DY_PXY_MEAN];
    if (!std::isfinite(t.res) || !std::isfinite(pxy) || dy[DY_FLAGS] != 0.0) return HRLB_E_DIVERGED;
    if (dy[DY_RANGE] != 0.0) return HRLB_E_RANGE;
    if (t.have_prev) t.drift = std::fabs(pxy - t.pxy_prev) / (n * dt * std::max(std::fabs(pxy), 1e-300));
    t.have_prev = true;
    t.pxy_prev = pxy;
    constexpr int W = SteadyTrack::kPxyWin;
    for (int k = 0; k < W; ++k) t.pxy[k] = t.pxy[k + 1];
    t.pxy[W] = pxy;
    if (++t.nchk > W) {
        const double est = pxy_error_bound(t.pxy, W + 1);
        t.err = est / std::max(std::fabs(pxy), 1e-300);
        t.below = t.err < tol ? t.below + 1 : 0;
    }
    if (stop_rule == HRLB_STOP_PXY_ERR) return t.below >= 2 ? HRLB_OK : HRLB_NOT_CONVERGED;
    const double crit = stop_rule == HRLB_STOP_RESIDUAL ? t.res : t.drift;
    return (crit >= 0.0 && crit < tol) ? HRLB_OK : HRLB_NOT_CONVERGED;
}

extern "C" hrlb_status hrlb_run_to_steady(hrlb_case* c, double tol, long max_steps, int check_every, int stop_rule,
                                          hrlb_steady_info* info)
{
    if (!c) return fail(HRLB_E_INVALID, "case is NULL");
    {
        const hrlb_status sl = case_live(c);
        if (sl != HRLB_OK) return sl;
    }
    if (check_every < 1 || max_steps < 0 || !(tol > 0.0)) return fail(HRLB_E_INVALID, "bad tol/max_steps/check_every");
    if (stop_rule != HRLB_STOP_RESIDUAL && stop_rule != HRLB_STOP_PXY && stop_rule != HRLB_STOP_PXY_ERR)
        return fail(HRLB_E_INVALID, "bad stop rule");
    const auto t0 = std::chrono::steady_clock::now();
    {
        hrlb_status sa = ensure_analyzed(c);
        if (sa != HRLB_OK) return sa;
    }
    long taken = 0;
    hrlb_status decision = HRLB_NOT_CONVERGED;
    double dy[kNDyn];
    SteadyTrack track;
    while (taken < max_steps) {
        const long n = std::min<long>(check_every, max_steps - taken);
        hrlb_status st = enqueue_steps(c->run, n, true);
        if (st != HRLB_OK) return st;
        HIP_TRY(hipMemcpyAsync(dy, c->desc.dyn, sizeof dy, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        taken += n;
        c->steps_done += n;
        const hrlb_status v = steady_update(track, dy, n, c->dt, tol, stop_rule);
        if (v != HRLB_NOT_CONVERGED) {
            decision = v;
            if (v == HRLB_E_DIVERGED) fail(HRLB_E_DIVERGED, "non-finite residual after %ld steps", c->steps_done);
            if (v == HRLB_E_RANGE) range_message(c->steps_done);
            break;
        }
    }
    const double res = track.res, drift = track.drift;
    if (info) {
        info->steps = taken;
        info->residual = res;
        info->pxy_drift = drift;
        info->pxy_err = track.err;
        info->sim_time = c->steps_done * c->dt;
        info->wall_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        info->mass_drift = taken > 0 ? (dy[DY_MASS] - c->mass0) / c->mass0 : 0.0;
    }
    return decision;
}

extern "C" hrlb_status hrlb_moments(hrlb_case* c, double* fields, double* x, double* Pi, double* wall_shear)
{
    if (!c) return fail(HRLB_E_INVALID, "case is NULL");
    {
        const hrlb_status sl = case_live(c);
        if (sl != HRLB_OK) return sl;
    }
    {
        hrlb_status sa = ensure_analyzed(c);
        if (sa != HRLB_OK) return sa;
    }
    const int nx = c->p.n_cells;
    std::vector<double> f((size_t)kNFields * nx);
    double dy[kNDyn];
    {
        Copies cp(c->stream);
        cp.add(f.data(), c->desc.fields, sizeof(double) * f.size(), hipMemcpyDeviceToHost);
        cp.add(dy, c->desc.dyn, sizeof dy, hipMemcpyDeviceToHost);
        const hrlb_status sc = cp.finish("moments");
        if (sc != HRLB_OK) return sc;
    }
    if (fields) std::copy(f.begin(), f.end(), fields);
    if (x) std::copy(c->x.begin(), c->x.end(), x);
    if (Pi) {
        double num = 0, den = 0;
        for (int s = 0; s < nx; ++s) {
            num += c->jdeta[s] * f[(size_t)F_PXY * nx + s];
            den += c->jdeta[s];
        }
        const double pxy = num / den;
        const double vref = std::sqrt(c->p.T_w), pref = c->p.T_w;
        *Pi = c->p.u_w != 0.0 ? -pxy * vref / (pref * c->p.u_w * std::sqrt(2.0)) : 0.0;
    }
    if (wall_shear) {
        wall_shear[0] = c->p.half_channel ? dy[DY_SHEAR_R] : dy[DY_SHEAR_L];
        wall_shear[1] = dy[DY_SHEAR_R];
    }
    return HRLB_OK;
}

extern "C" hrlb_status hrlb_average_start(hrlb_case* c)
{
    if (!c) return fail(HRLB_E_INVALID, "case is NULL");
    {
        const hrlb_status sl = case_live(c);
        if (sl != HRLB_OK) return sl;
    }
    HIP_TRY(hrlbk_average(c->d_desc, 1, c->p.n_cells, c->stream));
    return HRLB_OK;
}

extern "C" hrlb_status hrlb_average_stop(hrlb_case* c)
{
    if (!c) return fail(HRLB_E_INVALID, "case is NULL");
    {
        const hrlb_status sl = case_live(c);
        if (sl != HRLB_OK) return sl;
    }
    HIP_TRY(hrlbk_average(c->d_desc, 0, c->p.n_cells, c->stream));
    return HRLB_OK;
}

extern "C" hrlb_status hrlb_average_read(hrlb_case* c, double* fields, double* Pi, long* steps)
{
    if (!c) return fail(HRLB_E_INVALID, "case is NULL");
    {
        const hrlb_status sl = case_live(c);
        if (sl != HRLB_OK) return sl;
    }
    const int nx = c->p.n_cells;
    std::vector<double> a((size_t)kNFields * nx);
    double dy[kNDyn];
    {
        Copies cp(c->stream);
        cp.add(a.data(), c->desc.avg, sizeof(double) * a.size(), hipMemcpyDeviceToHost);
        cp.add(dy, c->desc.dyn, sizeof dy, hipMemcpyDeviceToHost);
        const hrlb_status sc = cp.finish("average read");
        if (sc != HRLB_OK) return sc;
    }
    const double m = dy[DY_AVG_STEPS];
    if (steps) *steps = (long)m;
    if (!(m > 0.0)) return fail(HRLB_E_INVALID, "no step has been averaged");
    for (double& v : a) v /= m;
    if (fields) std::copy(a.begin(), a.end(), fields);
    if (Pi) {
        double num = 0, den = 0;
        for (int s = 0; s < nx; ++s) {
            num += c->jdeta[s] * a[(size_t)F_PXY * nx + s];
            den += c->jdeta[s];
        }
        const double vref = std::sqrt(c->p.T_w), pref = c->p.T_w;
        *Pi = c->p.u_w != 0.0 ? -(num / den) * vref / (pref * c->p.u_w * std::sqrt(2.0)) : 0.0;
    }
    return HRLB_OK;
}

extern "C" hrlb_status hrlb_get_state(hrlb_case* c, double* host_state)
{
    if (!c || !host_state) return fail(HRLB_E_INVALID, "NULL argument");
    {
        const hrlb_status sl = case_live(c);
        if (sl != HRLB_OK) return sl;
    }
    const size_t n = 2 * (size_t)c->nv * c->p.n_cells;
    if (c->p.precision == HRLB_FP64) {
        HIP_TRY(hipMemcpyAsync(host_state, c->desc.f[0], sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
    } else {
        std::vector<float> tmp(n);
        HIP_TRY(hipMemcpyAsync(tmp.data(), c->desc.f[0], sizeof(float) * n, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        for (size_t k = 0; k < n; ++k) host_state[k] = tmp[k];
    }
    return HRLB_OK;
}

extern "C" hrlb_status hrlb_set_state(hrlb_case* c, const double* host_state)
{
    if (!c || !host_state) return fail(HRLB_E_INVALID, "NULL argument");
    {
        const hrlb_status sl = case_live(c);
        if (sl != HRLB_OK) return sl;
    }
    const size_t n = 2 * (size_t)c->nv * c->p.n_cells;
    for (size_t k = 0; k < n; ++k)
        if (!std::isfinite(host_state[k])) return fail(HRLB_E_INVALID, "state holds a non-finite value at %zu", k);
    if (c->p.precision == HRLB_FP64) {
        HIP_TRY(hipMemcpyAsync(c->desc.f[0], host_state, sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
    } else {
        std::vector<float> tmp(n);
        for (size_t k = 0; k < n; ++k) tmp[k] = (float)host_state[k];
        HIP_TRY(hipMemcpyAsync(c->desc.f[0], tmp.data(), sizeof(float) * n, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
    }
    hrlb_status st = analyze_case(c);
    if (st != HRLB_OK) return st;
    double dy[kNDyn];
    HIP_TRY(hipMemcpyAsync(dy, c->desc.dyn, sizeof dy, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->mass0 = dy[DY_MASS];  // mass drift is reported relative to the uploaded state
    return HRLB_OK;
}

// ------------------------------------------------------------------------------------------------
// batches
namespace {
constexpr int kMaxBatchParts = 4;
constexpr double kSplitUnits = 2e7;  // cell-velocity units from which a batch is split over kSplitParts streams
constexpr int kSplitParts = 3;

// cases of a batch split into n parts of about equal work (units = velocities x cells): largest first
// onto the least loaded part; each part keeps its cases in ascending order
// The cases of the tiled path split into `parts` parts of about equal work, and the cases of the small
// path (if any) in one part of their own after them, whose one launch per block of steps then overlaps
// the tiled parts' launches on its own stream.  all_tiled: every case counts as tiled (analysis passes).
std::vector<std::vector<int>> split_batch(hrlb_case* const* cases, int n, int parts, bool all_tiled = false)
{
    std::vector<int> order, smalls;
    for (int i = 0; i < n; ++i) (all_tiled || !cases[i]->small ? order : smalls).push_back(i);
    const int nt = (int)order.size();
    parts = std::max(1, std::min(parts, nt));
    if (nt == 0) return {smalls};
    auto units = [&](int i) { return (double)cases[i]->nv * cases[i]->p.n_cells; };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return units(a) > units(b); });
    std::vector<std::vector<int>> out(parts);
    std::vector<double> load(parts, 0.0);
    for (int i : order) {
        const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        out[k].push_back(i);
        load[k] += units(i);
    }
    for (auto& v : out) std::sort(v.begin(), v.end());
    if (!smalls.empty()) out.push_back(smalls);
    return out;
}

// tile list of a set of cases: natural sequence over the cases, then the XCD-aware order
std::vector<TileRef> part_tiles(hrlb_case* const* cases, const std::vector<int>& idx)
{
    std::vector<PlanShape> shapes;
    for (int i : idx)
        shapes.push_back(PlanShape{cases[i]->L.nctiles, cases[i]->L.ngroups, cases[i]->L.vpt, cases[i]->p.n_cells});
    return plan_batch_tiles(shapes);
}

struct PartLayout {
    size_t descs, tiles, cells, ctr;
    int ntiles, ncellblocks;
};

// workspace layout of a batch split into `parts` parts (descriptors, tile list and cell list per part)
// the cases of a part in launch order: those on the tiled kernels, then those on the small-case kernel
// (every case on the tiled kernels for an analysis pass, which runs them on any case)
std::vector<int> launch_order(hrlb_case* const* cases, const std::vector<int>& idx, bool all_tiled, int* ntiled)
{
    std::vector<int> out;
    for (int i : idx)
        if (all_tiled || !cases[i]->small) out.push_back(i);
    *ntiled = (int)out.size();
    for (int i : idx)
        if (!all_tiled && cases[i]->small) out.push_back(i);
    return out;
}

size_t parts_layout(hrlb_case* const* cases, const std::vector<std::vector<int>>& split, std::vector<PartLayout>* L,
                    bool all_tiled = false)
{
    size_t off = 0;
    if (L) L->clear();
    for (const auto& part : split) {
        PartLayout P{};
        int ntiled = 0;
        const std::vector<int> idx = launch_order(cases, part, all_tiled, &ntiled);
        const std::vector<int> tiled(idx.begin(), idx.begin() + ntiled);
        P.ntiles = (int)part_tiles(cases, tiled).size();
        P.ncellblocks = 0;
        for (int i : tiled) P.ncellblocks += cases[i]->L.ncellblocks;
        P.descs = off;
        off = align256(off + sizeof(InstDesc) * idx.size());
        P.tiles = off;
        off = align256(off + sizeof(TileRef) * P.ntiles);
        P.cells = off;
        off = align256(off + sizeof(CellRef) * P.ncellblocks);
        P.ctr = off;
        off = align256(off + sizeof(unsigned) * (kXcds + 1));
        if (L) L->push_back(P);
    }
    return off;
}

hrlb_status batch_check(hrlb_case* const* cases, int n)
{
    if (!cases || n < 1) return fail(HRLB_E_INVALID, "empty batch");
    for (int i = 0; i < n; ++i) {
        if (!cases[i]) return fail(HRLB_E_INVALID, "case %d is NULL", i);
        {
            const hrlb_status sl = case_live(cases[i]);
            if (sl != HRLB_OK) return sl;
        }
        if (cases[i]->p.precision != cases[0]->p.precision) return fail(HRLB_E_INVALID, "mixed precisions in a batch");
        if (cases[i]->stream != cases[0]->stream) return fail(HRLB_E_INVALID, "cases of a batch must share a stream");
    }
    return HRLB_OK;
}

// workspace that holds the launch tables of any split into 1..kMaxBatchParts parts
size_t batch_bytes(hrlb_case* const* cases, int n)
{
    size_t m = parts_layout(cases, split_batch(cases, n, 1, true), nullptr, true);
    for (int p = 1; p <= kMaxBatchParts; ++p) m = std::max(m, parts_layout(cases, split_batch(cases, n, p), nullptr));
    return m;
}

// (re)builds the parts of a batch inside its workspace and uploads their tables (synchronous);
// all_tiled: every case on the tiled kernels (the batch's analysis pass)
hrlb_status batch_build_parts(hrlb_batch* b, int nparts, bool all_tiled = false)
{
    const int n = (int)b->cases.size();
    hrlb_case* const* cases = b->cases.data();
    const auto split = split_batch(cases, n, nparts, all_tiled);
    std::vector<PartLayout> L;
    const size_t need = parts_layout(cases, split, &L, all_tiled);
    if (need > b->ws_bytes) return fail(HRLB_E_INVALID, "internal: batch workspace too small for %d parts", nparts);
    HIP_TRY(hipStreamSynchronize(b->stream));
    b->parts.clear();
    for (size_t k = 0; k < split.size(); ++k) {
        auto part = std::make_unique<hrlb_batch_part>();
        hrlb_batch_part& P = *part;
        P.idx = launch_order(cases, split[k], all_tiled, &P.ntiled);
        P.d_descs = (InstDesc*)(b->ws + L[k].descs);
        P.d_tiles = (TileRef*)(b->ws + L[k].tiles);
        P.d_cells = (CellRef*)(b->ws + L[k].cells);
        P.d_ctr = (unsigned*)(b->ws + L[k].ctr);
        P.ntiles = L[k].ntiles;
        P.ncellblocks = L[k].ncellblocks;
        if (k == 0) {
            P.stream = b->stream;
        } else {
            HIP_TRY(hipStreamCreateWithFlags(&P.stream, hipStreamNonBlocking));
            P.own_stream = true;
            HIP_TRY(hipEventCreateWithFlags(&P.done, hipEventDisableTiming));
        }
        const int ni = (int)P.idx.size(), nt = P.ntiled;
        std::vector<InstDesc> descs(ni);
        std::vector<int> nct(nt), ngr(nt), ncell(nt), cpb(nt);
        std::vector<char> own(nt);
        size_t small_lds = 0;
        for (int q = 0; q < ni; ++q) {
            const hrlb_case* c = cases[P.idx[q]];
            descs[q] = c->desc;
            if (q >= nt) {
                small_lds = std::max(small_lds, c->small_lds);
                continue;
            }
            nct[q] = c->L.nctiles;
            ngr[q] = c->L.ngroups;
            ncell[q] = c->p.n_cells;
            cpb[q] = kCellThreads / c->L.cell_lanes;
            own[q] = wall_blocks_of_their_own(c->q->qx, c->q->qy);
        }
        std::vector<CellRef> cells = plan_cell_blocks(ncell, cpb, own);
        {
            // per-cell work of an instance: the projection of eq. (gx) and its 2 Q_x output nodes
            // scale with (N_x + 1) (Q_x + 8), plus the moment shift and tau
            std::vector<double> w(nt);
            for (int q = 0; q < nt; ++q) {
                const hrlb_case* c = cases[P.idx[q]];
                w[q] = (double)(c->q->nxo + 1) * (c->q->qx + 8) + 40.0;
            }
            size_t first = 0;
            while (first < cells.size() && cells[first].cell0 < 0) ++first;
            int ncu = 0, dev = 0;
            if (hipGetDevice(&dev) != hipSuccess ||
                hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
                ncu = 0;  // keep the plain order
            balance_cell_blocks(cells, first, w, ncu);
        }
        const std::vector<TileRef> tiles = part_tiles(cases, std::vector<int>(P.idx.begin(), P.idx.begin() + nt));
        if ((int)tiles.size() != P.ntiles || (int)cells.size() != P.ncellblocks ||
            !tiles_valid(tiles, (size_t)P.ntiles, nt, nct.data(), ngr.data()))
            return fail(HRLB_E_INVALID, "internal: inconsistent batch tile list");
        static const unsigned zeros[kXcds + 1] = {};
        Copies cp(b->stream);  // the staging vectors end with this iteration
        cp.add(P.d_descs, descs.data(), sizeof(InstDesc) * ni, hipMemcpyHostToDevice);
        cp.add(P.d_tiles, tiles.data(), sizeof(TileRef) * tiles.size(), hipMemcpyHostToDevice);
        cp.add(P.d_cells, cells.data(), sizeof(CellRef) * cells.size(), hipMemcpyHostToDevice);
        cp.add(P.d_ctr, zeros, sizeof zeros, hipMemcpyHostToDevice);
        const hrlb_status sc = cp.finish("batch upload");
        if (sc != HRLB_OK) return sc;
        P.run.fp32 = b->fp32;
        P.run.descs = P.d_descs;
        P.run.ninst = nt;
        P.run.small_descs = P.d_descs + nt;
        P.run.nsmall = ni - nt;
        P.run.small_lds = small_lds;
        P.run.tiles = P.d_tiles;
        P.run.ctr = P.d_ctr;
        P.run.ntiles = P.ntiles;
        P.run.cells = P.d_cells;
        P.run.ncellblocks = P.ncellblocks;
        P.run.shmem = b->shmem;
        P.run.qy_max = b->qy_max;
        P.run.any_lts = false;
        for (int q = 0; q < nt; ++q) P.run.any_lts = P.run.any_lts || cases[P.idx[q]]->p.local_dt_cap > 1.0;
        P.run.stream = P.stream;
        P.run.graph_steps = b->graph_steps;
        b->parts.push_back(std::move(part));
    }
    HIP_TRY(hipStreamSynchronize(b->stream));
    return HRLB_OK;
}

// parts 1.. start after everything already on the batch's stream and the batch's stream waits for them
hrlb_status batch_fork(hrlb_batch* b)
{
    if (b->parts.size() < 2) return HRLB_OK;
    HIP_TRY(hipEventRecord(b->fork, b->stream));
    for (size_t k = 1; k < b->parts.size(); ++k) HIP_TRY(hipStreamWaitEvent(b->parts[k]->stream, b->fork, 0));
    return HRLB_OK;
}
hrlb_status batch_join(hrlb_batch* b)
{
    for (size_t k = 1; k < b->parts.size(); ++k) {
        HIP_TRY(hipEventRecord(b->parts[k]->done, b->parts[k]->stream));
        HIP_TRY(hipStreamWaitEvent(b->stream, b->parts[k]->done, 0));
    }
    return HRLB_OK;
}
}  // namespace

extern "C" hrlb_status hrlb_batch_workspace_bytes(hrlb_case* const* cases, int n_cases, size_t* bytes)
{
    hrlb_status st = batch_check(cases, n_cases);
    if (st != HRLB_OK) return st;
    if (!bytes) return fail(HRLB_E_INVALID, "bytes is NULL");
    *bytes = batch_bytes(cases, n_cases);
    return HRLB_OK;
}

extern "C" hrlb_status hrlb_batch_create(hrlb_case* const* cases, int n_cases, void* dev_workspace, size_t ws_bytes,
                                         hrlb_batch** out)
{
    if (!out) return fail(HRLB_E_INVALID, "out is NULL");
    *out = nullptr;
    hrlb_status st = batch_check(cases, n_cases);
    if (st != HRLB_OK) return st;
    if (!dev_workspace || ((uintptr_t)dev_workspace & 255)) return fail(HRLB_E_INVALID, "workspace NULL or misaligned");
    const size_t need = batch_bytes(cases, n_cases);
    if (ws_bytes < need) return fail(HRLB_E_NOMEM, "batch workspace of %zu bytes < %zu", ws_bytes, need);
    std::unique_ptr<hrlb_batch> b(new (std::nothrow) hrlb_batch);
    if (!b) return fail(HRLB_E_NOMEM, "host allocation failed");
    b->cases.assign(cases, cases + n_cases);
    b->ws = (char*)dev_workspace;
    b->ws_bytes = ws_bytes;
    b->fp32 = cases[0]->p.precision == HRLB_FP32_STORE_FP64_MOM;
    b->stream = cases[0]->stream;
    for (int i = 0; i < n_cases; ++i) {
        b->shmem = std::max(b->shmem, cases[i]->shmem);
        b->qy_max = std::max(b->qy_max, cases[i]->q->qy);
    }
    HIP_TRY(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
    // one analysis pass brings every case's moments up to date (it reproduces bit for bit what a
    // case already analysed holds); it runs on one part holding all cases
    bool any = false;
    for (int i = 0; i < n_cases; ++i) any = any || cases[i]->needs_analyze;
    if (any) {
        st = batch_build_parts(b.get(), 1, true);
        if (st != HRLB_OK) return st;
        const hrlb_batch_part& P = *b->parts[0];
        HIP_TRY(hrlbk_stage(b->fp32, P.d_descs, P.d_tiles, P.ntiles, P.d_ctr, -1, 0, b->qy_max, b->stream));
        HIP_TRY(hrlbk_cell(b->fp32, P.d_descs, P.d_cells, P.ncellblocks, 0, FLAG_FIELDS, b->shmem, b->stream));
        HIP_TRY(hrlbk_finalize(P.d_descs, (int)P.idx.size(), 0, b->stream));
    }
    // three parts on three streams for large batches: one part's per-cell kernel overlaps another's
    // stage kernel.  Measured on MI355X (512-instance FP32 batches, one box): 1 / 2 / 3 / 4 parts
    // give 4.91 / 5.18 / 5.30 / 5.15e10 updates/s at 5.2e7 units and 4.23 / 4.33 / 4.75 / 4.72e10
    // at 2.6e7 units (half channel); at 1e7 units two parts were 16% slower than one (the parts'
    // launches then compete for the chip), hence one part below kSplitUnits
    double units = 0.0;
    for (int i = 0; i < n_cases; ++i) units += (double)cases[i]->nv * cases[i]->p.n_cells;
    st = batch_build_parts(b.get(), units >= kSplitUnits ? std::min(kSplitParts, n_cases) : 1);
    if (st != HRLB_OK) return st;
    for (int i = 0; i < n_cases; ++i) cases[i]->needs_analyze = false;
    *out = b.release();
    return HRLB_OK;
}

extern "C" hrlb_status hrlb_batch_set_streams(hrlb_batch* b, int n_streams)
{
    if (!b || n_streams < 1 || n_streams > kMaxBatchParts)
        return fail(HRLB_E_INVALID, "NULL batch or n_streams outside [1, %d]", kMaxBatchParts);
    return batch_build_parts(b, n_streams);
}

extern "C" hrlb_status hrlb_batch_step(hrlb_batch* b, long n_steps, int check)
{
    if (!b) return fail(HRLB_E_INVALID, "batch is NULL");
    if (n_steps < 0) return fail(HRLB_E_INVALID, "n_steps < 0");
    hrlb_status st = batch_fork(b);
    for (auto& P : b->parts)
        if (st == HRLB_OK) st = enqueue_steps(P->run, n_steps, check != 0);
    if (st == HRLB_OK) st = batch_join(b);
    if (st == HRLB_OK)
        for (hrlb_case* c : b->cases) c->steps_done += n_steps;
    return st;
}

extern "C" hrlb_status hrlb_batch_poll(hrlb_batch* b, double* residual, double* pxy_mean)
{
    if (!b) return fail(HRLB_E_INVALID, "batch is NULL");
    const int n = (int)b->cases.size();
    std::vector<double> dy((size_t)kNDyn * n);
    {
        Copies cp(b->stream);
        for (int i = 0; i < n; ++i)
            cp.add(dy.data() + (size_t)i * kNDyn, b->cases[i]->desc.dyn, sizeof(double) * kNDyn, hipMemcpyDeviceToHost);
        const hrlb_status sc = cp.finish("batch poll");
        if (sc != HRLB_OK) return sc;
    }
    for (int i = 0; i < n; ++i) {
        const double* d = dy.data() + (size_t)i * kNDyn;
        if (residual) residual[i] = std::sqrt(d[DY_RES_NUM]) / (b->cases[i]->dt * std::sqrt(d[DY_RES_DEN]));
        if (pxy_mean) pxy_mean[i] = d[DY_PXY_MEAN];
    }
    return HRLB_OK;
}

extern "C" void hrlb_batch_free(hrlb_batch* b) { delete b; }

extern "C" hrlb_status hrlb_case_set_graph_steps(hrlb_case* c, int steps_per_graph)
{
    if (!c || steps_per_graph < 0) return fail(HRLB_E_INVALID, "NULL case or negative steps");
    {
        const hrlb_status sl = case_live(c);
        if (sl != HRLB_OK) return sl;
    }
    c->run.drop_graphs();
    c->run.graph_steps = steps_per_graph;
    return HRLB_OK;
}

extern "C" hrlb_status hrlb_batch_set_graph_steps(hrlb_batch* b, int steps_per_graph)
{
    if (!b || steps_per_graph < 0) return fail(HRLB_E_INVALID, "NULL batch or negative steps");
    b->graph_steps = steps_per_graph;
    for (auto& P : b->parts) {
        P->run.drop_graphs();
        P->run.graph_steps = steps_per_graph;
    }
    return HRLB_OK;
}

extern "C" hrlb_status hrlb_batch_profile(hrlb_batch* b, long n_steps, double* stage_kernel_ms, double* cell_kernel_ms)
{
    if (!b || n_steps < 1) return fail(HRLB_E_INVALID, "NULL batch or n_steps < 1");
    const long nl = n_steps * 3;
    const size_t np = b->parts.size();
    std::vector<hipEvent_t> ev(4 * nl * np, nullptr);
    hrlb_status st = HRLB_OK;
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            st = fail(HRLB_E_DEVICE, "hipEventCreate failed");
            break;
        }
    if (st == HRLB_OK) st = batch_fork(b);
    // the launch sequence of hrlb_batch_step, with an event pair around every launch on its stream
    for (size_t q = 0; q < np && st == HRLB_OK; ++q) {
        const hrlb_batch_part& P = *b->parts[q];
        for (long k = 0; k < nl && st == HRLB_OK; ++k) {
            hipEvent_t* e4 = &ev[4 * (q * nl + k)];
            const int stage = (int)(k % 3);
            hipError_t e = hipEventRecord(e4[0], P.stream);
            if (e == hipSuccess) e = hrlbk_stage(b->fp32, P.d_descs, P.d_tiles, P.ntiles, P.d_ctr, stage, 0, b->qy_max, P.stream);
            if (e == hipSuccess) e = hipEventRecord(e4[1], P.stream);
            if (e == hipSuccess) e = hipEventRecord(e4[2], P.stream);
            if (e == hipSuccess)
                e = hrlbk_cell(b->fp32, P.d_descs, P.d_cells, P.ncellblocks, stage == 0 ? 1 : stage == 1 ? 2 : 0,
                               stage == 2 ? FLAG_STEP_DONE : 0, b->shmem, P.stream);
            if (e == hipSuccess) e = hipEventRecord(e4[3], P.stream);
            if (e != hipSuccess) st = fail(HRLB_E_DEVICE, "profiled launch: %s", hipGetErrorString(e));
        }
        // the part's small cases take the same steps (not timed)
        if (st == HRLB_OK && P.run.nsmall > 0) {
            const hipError_t e = hrlbk_small(b->fp32, P.run.small_descs, P.run.nsmall, (int)n_steps, 0,
                                             P.run.small_lds, P.stream);
            if (e != hipSuccess) st = fail(HRLB_E_DEVICE, "small-case launch: %s", hipGetErrorString(e));
        }
    }
    if (st == HRLB_OK) st = batch_join(b);
    // the mean over the launches of the parts that hold tiled cases (the small-case part has none)
    double ts = 0, tc = 0;
    size_t timed = 0;
    if (st == HRLB_OK) {
        hipError_t e = hipStreamSynchronize(b->stream);
        for (size_t i = 0; i < nl * np && e == hipSuccess; ++i) {
            if (b->parts[i / nl]->ntiles == 0) continue;
            float a = 0, c = 0;
            e = hipEventElapsedTime(&a, ev[4 * i], ev[4 * i + 1]);
            if (e == hipSuccess) e = hipEventElapsedTime(&c, ev[4 * i + 2], ev[4 * i + 3]);
            ts += a;
            tc += c;
            ++timed;
        }
        if (e != hipSuccess) st = fail(HRLB_E_DEVICE, "profile events: %s", hipGetErrorString(e));
    }
    for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
    if (st != HRLB_OK) return st;
    for (hrlb_case* c : b->cases) c->steps_done += n_steps;
    if (stage_kernel_ms) *stage_kernel_ms = timed ? ts / (double)timed : 0.0;
    if (cell_kernel_ms) *cell_kernel_ms = timed ? tc / (double)timed : 0.0;
    return HRLB_OK;
}
