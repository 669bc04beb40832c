// hrlb_runtime.h -- host-side objects behind the opaque handles of include/hrlb.h, shared by the
// host runtime (hrlb_host.cpp) and the request server (hrlb_serve.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <memory>
#include <string>
#include <vector>

#include "../../include/hrlb.h"
#include "hrlb_internal.h"
#include "hrlb_plan.h"
#include "hrlb_quadrature.h"

extern "C" hipError_t hrlbk_stage(int fp32, const hrlb::InstDesc* descs, const hrlb::TileRef* tiles, int ntiles, unsigned* ctr,
                                  int stage, int flags, int qy_max, hipStream_t st);
extern "C" hipError_t hrlbk_cell(int fp32, const hrlb::InstDesc* descs, const hrlb::CellRef* cells, int ncells, int buf,
                                 int flags, size_t shmem, hipStream_t st);
extern "C" hipError_t hrlbk_renorm(int fp32, const hrlb::InstDesc* descs, int ninst, hipStream_t st);
extern "C" hipError_t hrlbk_finalize(const hrlb::InstDesc* descs, int ninst, int with_res, hipStream_t st);
extern "C" hipError_t hrlbk_init(int fp32, const hrlb::InstDesc* descs, int inst, size_t units, hipStream_t st);
extern "C" hipError_t hrlbk_average(const hrlb::InstDesc* desc, int start, int nx, hipStream_t st);
extern "C" hipError_t hrlbk_scratch(void** ptr, size_t* bytes);
extern "C" size_t hrlbk_small_lds(const hrlb::InstDesc* D);
extern "C" size_t hrlbk_small_lds_max();
extern "C" hipError_t hrlbk_small(int fp32, const hrlb::InstDesc* descs, int ninst, int n_steps, int check, size_t lds,
                                  hipStream_t st);

namespace hrlb {

// FLAG_FIELDS: the per-cell kernel also stores the FP64 fields (always at the end of a step, with
// FLAG_STEP_DONE; analysis passes ask for them; the stages inside a step do not need them)
enum : int { FLAG_RESID = 1, FLAG_STEP_DONE = 2, FLAG_FIELDS = 4 };

hrlb_status fail(hrlb_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return fail(HRLB_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_));  \
    } while (0)

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Copies between device memory and host buffers that end with the caller's scope: every copy is
// enqueued on one stream, and finish() always waits for that stream (also after a failed copy), so
// that no copy outlives its host buffer.
struct Copies {
    explicit Copies(hipStream_t s) : st(s) {}
    void add(void* dst, const void* src, size_t bytes, hipMemcpyKind kind)
    {
        if (e == hipSuccess) e = hipMemcpyAsync(dst, src, bytes, kind, st);
    }
    hrlb_status finish(const char* what)
    {
        const hipError_t es = hipStreamSynchronize(st);
        if (e == hipSuccess) e = es;
        return e == hipSuccess ? HRLB_OK : fail(HRLB_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
    }
    hipStream_t st;
    hipError_t e = hipSuccess;
};

// launch parameters of a case or a batch, with its cached step-block graphs
struct Launcher {
    int fp32 = 0;
    const InstDesc* descs = nullptr;
    int ninst = 0;
    const TileRef* tiles = nullptr;
    int ntiles = 0;
    unsigned* ctr = nullptr;  // work-queue counters of the stage kernel (kXcds + 1, zeroed)
    const CellRef* cells = nullptr;
    int ncellblocks = 0;
    size_t shmem = 0;
    int qy_max = 0;
    bool any_lts = false;  // some instance takes local time steps: rescale + re-analyse after checks
    const InstDesc* small_descs = nullptr;  // instances on the small-case kernel (one block each)
    int nsmall = 0;
    size_t small_lds = 0;                   // dynamic LDS of that launch (its largest instance)
    hipStream_t stream = nullptr;
    int graph_steps = 0;  // steps per captured graph; < 2 launches directly (faster on this stack)
    int graph_len = 0;
    hipGraphExec_t graph_plain = nullptr, graph_check = nullptr;
    void drop_graphs()
    {
        if (graph_plain) (void)hipGraphExecDestroy(graph_plain);
        if (graph_check) (void)hipGraphExecDestroy(graph_check);
        graph_plain = graph_check = nullptr;
        graph_len = 0;
    }
    ~Launcher() { drop_graphs(); }
};

// residual and P_xy-drift bookkeeping of a steady-state run; the same rule serves
// hrlb_run_to_steady and the request server, so both stop a case after the same step
struct SteadyTrack {
    bool have_prev = false;
    double pxy_prev = 0.0;
    double res = -1.0, drift = -1.0;
    // P_xy error rule: the last kPxyWin + 1 checked means, how many were seen, the last estimate, and how
    // many consecutive estimates were below the tolerance
    static constexpr int kPxyWin = 8;
    double pxy[kPxyWin + 1] = {};
    int nchk = 0;
    double err = -1.0;
    int below = 0;
};
// dy: the case's dynamic scalars read after a block of n steps whose last step was checked.
// Returns HRLB_OK when the stop criterion is below tol, HRLB_NOT_CONVERGED to go on, and
// HRLB_E_DIVERGED (with the message set) on a non-finite value.
hrlb_status steady_update(SteadyTrack& t, const double* dy, long n, double dt, double tol, int stop_rule);
// remaining absolute error of the last of count checked means of P_xy (the P_xy error rule)
double pxy_error_bound(const double* means, int count);
// sets the thread's error message of HRLB_E_RANGE
void range_message(long steps);
// HRLB_OK unless the case lives in the static scratch and a later static case on its device replaced it
hrlb_status case_live(const hrlb_case* c);

// byte offsets of the regions of a case workspace
struct Layout {
    // auxiliary region (offsets from its base): descriptor, dynamic scalars, tables, cell tables,
    // fields, averages, moment and residual partials, work lists, counters; state region (offsets
    // from its own base): the three population buffers f[0..2]
    size_t desc, dyn, tables, cell, cell_g, fields, avg, mom, res, tiles, cells, ctr, aux_total;
    size_t f[3], state_total;
    size_t total;  // aux_total + state_total: one workspace holding both regions
    // table offsets in doubles relative to `tables`
    size_t t_px, t_py, t_wx, t_wy, t_hz, t_az, t_aw, t_hZ, t_he, t_ijd, t_jd, t_gwl, t_gwr, t_g0, t_vT, t_vMu, t_vOm,
        t_vPr, t_dts, t_jres, t_az2, t_aw2, t_hZ2, t_img, t_n;
    int ngroups, nctiles, vpt, ncellblocks, cell_lanes;
    int ntile_list;  // records in the case's tile list (XCD-aware order, padded)
};

}  // namespace hrlb

struct hrlb_quad {
    int qx, nxo, qy, nyo;
    hrlb::Recurrence hr;               // half-range recurrence (orthonormal h_l at any point)
    std::vector<long double> auxZl, auxWl, auxZ2l, auxW2l;  // unscaled auxiliary rules, extended precision
    std::vector<double> zx, wx;        // [qx] positive nodes, weights
    std::vector<double> px, wx2;       // [2qx] h-major
    std::vector<double> zy, wy;        // [qy]
    std::vector<double> hz;            // [(nxo+1)][qx]
    std::vector<double> auxZ, auxW;    // [kAux]
    std::vector<double> hZ;            // [(nxo+1)][kAux]
    std::vector<double> auxZ2, auxW2;  // [kAux2]
    std::vector<double> hZ2;           // [(nxo+1)][kAux2]
    std::vector<double> he;            // [(nyo+1)][qy]
};

struct hrlb_case {
    hrlb_case_params p;
    const hrlb_quad* q;
    char* ws;
    size_t ws_bytes;
    hipStream_t stream;
    hrlb::Layout L;
    hrlb::InstDesc desc;  // host copy of the device descriptor
    hrlb::InstDesc* d_desc;
    hrlb::TileRef* d_tiles;
    hrlb::CellRef* d_cells;
    unsigned* d_ctr;
    int ntiles;
    int nv;
    size_t shmem;  // dynamic LDS of the per-cell kernel
    double dt;
    long steps_done;
    double mass0;
    std::vector<double> x, jdeta;
    bool needs_analyze;  // moments/tables of the stored state not computed yet
    bool small;          // advanced by the small-case kernel (kernel_path)
    size_t small_lds;    // its dynamic LDS
    int static_dev;      // device whose static scratch holds the auxiliary region, -1 for a workspace case
    unsigned long static_gen;  // generation of that static case (hrlb::case_live)
    hrlb::Launcher run;
};

// cases of a batch advanced on one stream by shared launches
struct hrlb_batch_part {
    std::vector<int> idx;  // indices into hrlb_batch::cases, ascending: the tiled cases, then the small ones
    int ntiled = 0;        // the first ntiled of idx run the tiled kernels, the rest the small-case kernel
    hrlb::InstDesc* d_descs = nullptr;  // descriptors of idx in that order
    hrlb::TileRef* d_tiles = nullptr;
    hrlb::CellRef* d_cells = nullptr;
    unsigned* d_ctr = nullptr;
    int ntiles = 0, ncellblocks = 0;
    hipStream_t stream = nullptr;  // part 0: the batch's stream; others: owned by the library
    bool own_stream = false;
    hipEvent_t done = nullptr;     // join event of parts 1..
    hrlb::Launcher run;
    ~hrlb_batch_part()
    {
        run.drop_graphs();
        if (done) (void)hipEventDestroy(done);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
};

struct hrlb_batch {
    std::vector<hrlb_case*> cases;
    int fp32 = 0;
    size_t shmem = 0;
    int qy_max = 0;
    hipStream_t stream = nullptr;  // the cases' stream: every call is ordered on it
    char* ws = nullptr;
    size_t ws_bytes = 0;
    int graph_steps = 0;
    std::vector<std::unique_ptr<hrlb_batch_part>> parts;
    hipEvent_t fork = nullptr;
    ~hrlb_batch()
    {
        parts.clear();
        if (fork) (void)hipEventDestroy(fork);
    }
};

namespace hrlb {
// enqueue n steps of a case or a batch on its stream (residual check on the last step if asked)
hrlb_status enqueue_steps(Launcher& L, long n_steps, bool check_last);
}  // namespace hrlb
