// hrlb_serve.cpp -- request server of include/hrlb.h: continuous batching of Couette solves whose
// populations stay resident in a caller-owned device arena from admission to their stop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <map>
#include <memory>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "../../include/hrlb.h"
#include "hrlb_runtime.h"
#include "hrlb_sched.h"

using namespace hrlb;

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    long id = 0;
    hrlb_solve_request r{};
    const hrlb_quad* q = nullptr;
    size_t bytes = 0;
    int state = HRLB_REQ_WAITING;
    hrlb_status status = HRLB_OK;
    int bypassed = 0;
    long long off = -1;  // arena block of the case workspace
    hrlb_case* c = nullptr;
    SteadyTrack track;
    long taken = 0;
    double t_arrival = -1.0, t_admit = -1.0, t_done = -1.0;
    double pi = 0.0, mass_drift = 0.0, sim_time = 0.0;
    std::vector<double> fields, x;
    std::vector<double> vT, vMu, vPr;  // the request's transport table (its params point here)
};

using QuadKey = std::tuple<int, int, int, int>;

}  // namespace

struct hrlb_server {
    hrlb_server_config cfg{};
    char* base = nullptr;
    Arena arena;
    hipStream_t stream = nullptr;
    Clock::time_point t0;
    std::map<QuadKey, hrlb_quad*> quads;
    std::unordered_map<long, std::unique_ptr<Request>> all;
    std::vector<Request*> waiting;  // arrival order
    std::vector<Request*> active;
    hrlb_batch* batch = nullptr;
    long long batch_off = -1;
    long next_id = 1;
    int n_done = 0, n_failed = 0;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }

    void drop_batch()
    {
        if (batch) hrlb_batch_free(batch);
        batch = nullptr;
        if (batch_off >= 0) arena.release((size_t)batch_off);
        batch_off = -1;
    }

    // launch tables of the resident set, placed in the arena; HRLB_E_NOMEM if they do not fit
    hrlb_status build_batch()
    {
        drop_batch();
        if (active.empty()) return HRLB_OK;
        std::vector<hrlb_case*> cs;
        for (Request* rq : active) cs.push_back(rq->c);
        size_t bb = 0;
        hrlb_status st = hrlb_batch_workspace_bytes(cs.data(), (int)cs.size(), &bb);
        if (st != HRLB_OK) return st;
        batch_off = arena.alloc(bb);
        if (batch_off < 0) return fail(HRLB_E_NOMEM, "no arena room for the batch tables (%zu bytes)", bb);
        st = hrlb_batch_create(cs.data(), (int)cs.size(), base + batch_off, bb, &batch);
        if (st != HRLB_OK) {
            arena.release((size_t)batch_off);
            batch_off = -1;
        }
        return st;
    }

    // ends a resident solve: results to the host (DONE) or the error (FAILED); frees its memory
    void retire(Request* rq, hrlb_status decision, const double* dy)
    {
        rq->t_done = now();
        rq->status = decision;
        if (decision == HRLB_OK || decision == HRLB_NOT_CONVERGED) {
            const int nx = rq->r.params.n_cells;
            rq->fields.assign((size_t)kNFields * nx, 0.0);
            rq->x.assign(nx, 0.0);
            const hrlb_status st = hrlb_moments(rq->c, rq->fields.data(), rq->x.data(), &rq->pi, nullptr);
            if (st != HRLB_OK) rq->status = st;
        }
        if (dy) rq->mass_drift = (dy[DY_MASS] - rq->c->mass0) / rq->c->mass0;
        rq->sim_time = rq->c->steps_done * rq->c->dt;
        rq->state = (rq->status == HRLB_OK || rq->status == HRLB_NOT_CONVERGED) ? HRLB_REQ_DONE : HRLB_REQ_FAILED;
        if (rq->state == HRLB_REQ_DONE)
            ++n_done;
        else
            ++n_failed;
        hrlb_free_case(rq->c);
        rq->c = nullptr;
        arena.release((size_t)rq->off);
        rq->off = -1;
    }

    ~hrlb_server()
    {
        drop_batch();
        for (Request* rq : active)
            if (rq->c) hrlb_free_case(rq->c);
        for (auto& kv : quads) hrlb_free_quadrature(kv.second);
    }
};

extern "C" hrlb_status hrlb_server_create(const hrlb_server_config* cfg, void* dev_arena, size_t arena_bytes,
                                          void* hip_stream, hrlb_server** out)
{
    if (!out) return fail(HRLB_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!cfg) return fail(HRLB_E_INVALID, "config is NULL");
    if (cfg->max_active < 1 || cfg->check_every < 1 || cfg->max_bypass < 0)
        return fail(HRLB_E_INVALID, "max_active and check_every must be >= 1, max_bypass >= 0");
    if (cfg->precision != HRLB_FP64 && cfg->precision != HRLB_FP32_STORE_FP64_MOM)
        return fail(HRLB_E_INVALID, "unknown precision %d", cfg->precision);
    if (!dev_arena || ((uintptr_t)dev_arena & 255)) return fail(HRLB_E_INVALID, "arena NULL or not 256-byte aligned");
    hrlb_server* s = new (std::nothrow) hrlb_server;
    if (!s) return fail(HRLB_E_NOMEM, "host allocation failed");
    s->cfg = *cfg;
    s->base = (char*)dev_arena;
    s->arena.reset(arena_bytes);
    s->stream = (hipStream_t)hip_stream;
    s->t0 = Clock::now();
    *out = s;
    return HRLB_OK;
}

extern "C" double hrlb_server_clock(const hrlb_server* s) { return s ? s->now() : -1.0; }

extern "C" hrlb_status hrlb_server_submit(hrlb_server* s, const hrlb_solve_request* r, long* id)
{
    if (!s || !r || !id) return fail(HRLB_E_INVALID, "NULL argument");
    if (r->params.precision != s->cfg.precision)
        return fail(HRLB_E_INVALID, "request precision %d differs from the server's %d", r->params.precision,
                    s->cfg.precision);
    if (r->max_steps < 1 || r->max_steps % s->cfg.check_every != 0)
        return fail(HRLB_E_INVALID, "max_steps=%ld must be a positive multiple of check_every=%d", r->max_steps,
                    s->cfg.check_every);
    if (!(r->tol > 0.0)) return fail(HRLB_E_INVALID, "tol must be > 0");
    if (r->stop_rule != HRLB_STOP_RESIDUAL && r->stop_rule != HRLB_STOP_PXY && r->stop_rule != HRLB_STOP_PXY_ERR)
        return fail(HRLB_E_INVALID, "bad stop rule");
    const QuadKey key{r->Qx, r->Nx_order, r->Qy, r->Ny_order};
    auto it = s->quads.find(key);
    if (it == s->quads.end()) {
        hrlb_quad* q = nullptr;
        const hrlb_status st = hrlb_init_quadrature(r->Qx, r->Nx_order, r->Qy, r->Ny_order, 1.0, &q);
        if (st != HRLB_OK) return st;
        it = s->quads.emplace(key, q).first;
    }
    size_t bytes = 0;
    const hrlb_status st = hrlb_case_workspace_bytes(it->second, &r->params, &bytes);
    if (st != HRLB_OK) return st;
    // room for the solve and, generously, its share of the batch tables (a few KB per solve)
    const size_t need = Arena::round_up(bytes) + Arena::round_up(bytes / 16) + (size_t(64) << 10);
    if (need > s->arena.capacity())
        return fail(HRLB_E_NOMEM, "solve needs %zu bytes with its launch tables, the arena holds %zu", need,
                    s->arena.capacity());
    auto rq = std::make_unique<Request>();
    rq->id = s->next_id++;
    rq->r = *r;
    if (r->params.visc_table_n > 0) {  // validated above; the caller's arrays may go away after this call
        const int nt = r->params.visc_table_n;
        rq->vT.assign(r->params.visc_T, r->params.visc_T + nt);
        rq->vMu.assign(r->params.visc_mu, r->params.visc_mu + nt);
        rq->vPr.assign(r->params.visc_Pr, r->params.visc_Pr + nt);
        rq->r.params.visc_T = rq->vT.data();
        rq->r.params.visc_mu = rq->vMu.data();
        rq->r.params.visc_Pr = rq->vPr.data();
    }
    rq->q = it->second;
    rq->bytes = bytes;
    rq->t_arrival = r->arrival_s >= 0.0 ? r->arrival_s : s->now();
    s->waiting.push_back(rq.get());
    *id = rq->id;
    s->all.emplace(rq->id, std::move(rq));
    return HRLB_OK;
}

extern "C" hrlb_status hrlb_server_pump(hrlb_server* s, hrlb_server_stats* stats)
{
    if (!s) return fail(HRLB_E_INVALID, "server is NULL");
    const double t_round = s->now();
    int admitted_n = 0, retired_n = 0;
    long steps = 0;
    double units = 0.0;

    // ---- admission.  The batch tables are rebuilt whenever the resident set changes, so their block
    // is returned first; new members are placed in arrival order (with bounded backfill), created,
    // and the newest of them are sent back to wait if the tables of the grown set do not fit.
    if (!s->waiting.empty() && (int)s->active.size() < s->cfg.max_active) {
        s->drop_batch();
        std::vector<Waiting> q(s->waiting.size());
        for (size_t i = 0; i < q.size(); ++i) q[i].bypassed = s->waiting[i]->bypassed;
        const int free_slots = s->cfg.max_active - (int)s->active.size();
        const std::vector<int> idx = admit_in_order(q, free_slots, s->cfg.max_bypass, [&](int i) {
            const long long off = s->arena.alloc(s->waiting[i]->bytes);
            if (off < 0) return false;
            s->waiting[i]->off = off;
            return true;
        });
        for (size_t i = 0; i < q.size(); ++i) s->waiting[i]->bypassed = q[i].bypassed;
        std::vector<Request*> fresh;
        for (int i : idx) {
            Request* rq = s->waiting[i];
            hrlb_case* c = nullptr;
            const hrlb_status st = hrlb_init_case(rq->q, &rq->r.params, s->base + rq->off, rq->bytes, s->stream, &c);
            rq->t_admit = s->now();
            if (st != HRLB_OK) {
                rq->status = st;
                rq->state = HRLB_REQ_FAILED;
                rq->t_done = rq->t_admit;
                s->arena.release((size_t)rq->off);
                rq->off = -1;
                ++s->n_failed;
                continue;
            }
            rq->c = c;
            rq->state = HRLB_REQ_ACTIVE;
            s->active.push_back(rq);
            fresh.push_back(rq);
        }
        for (;;) {
            const hrlb_status st = s->build_batch();
            if (st == HRLB_OK) break;
            if (st != HRLB_E_NOMEM || fresh.empty()) return st;
            Request* last = fresh.back();
            fresh.pop_back();
            hrlb_free_case(last->c);
            last->c = nullptr;
            s->arena.release((size_t)last->off);
            last->off = -1;
            last->state = HRLB_REQ_WAITING;
            last->t_admit = -1.0;
            s->active.pop_back();
        }
        admitted_n = (int)fresh.size();
        std::vector<Request*> still;
        for (Request* rq : s->waiting)
            if (rq->state == HRLB_REQ_WAITING) still.push_back(rq);
        s->waiting.swap(still);
    }

    if (!s->active.empty()) {
        if (!s->batch) {
            const hrlb_status st = s->build_batch();
            if (st != HRLB_OK) return st;
        }
        const long n = s->cfg.check_every;
        hrlb_status st = hrlb_batch_step(s->batch, n, 1);
        if (st != HRLB_OK) return st;
        std::vector<double> dy((size_t)kNDyn * s->active.size());
        {
            Copies cp(s->stream);
            for (size_t i = 0; i < s->active.size(); ++i)
                cp.add(dy.data() + i * kNDyn, s->active[i]->c->desc.dyn, sizeof(double) * kNDyn, hipMemcpyDeviceToHost);
            st = cp.finish("server check");
            if (st != HRLB_OK) return st;
        }
        steps = n;
        std::vector<Request*> keep;
        for (size_t i = 0; i < s->active.size(); ++i) {
            Request* rq = s->active[i];
            units += (double)rq->c->nv * rq->c->p.n_cells * n;
            rq->taken += n;
            const double* d = dy.data() + i * kNDyn;
            hrlb_status v = steady_update(rq->track, d, n, rq->c->dt, rq->r.tol, rq->r.stop_rule);
            if (v == HRLB_NOT_CONVERGED && rq->taken < rq->r.max_steps) {
                keep.push_back(rq);
                continue;
            }
            if (v == HRLB_E_DIVERGED) fail(HRLB_E_DIVERGED, "request %ld: non-finite residual", rq->id);
            if (v == HRLB_E_RANGE) range_message(rq->c->steps_done);
            s->retire(rq, v, d);
            ++retired_n;
        }
        s->active.swap(keep);
        if (retired_n) s->drop_batch();
    }

    if (stats) {
        stats->waiting = (int)s->waiting.size();
        stats->active = (int)s->active.size();
        stats->done = s->n_done;
        stats->failed = s->n_failed;
        stats->admitted = admitted_n;
        stats->retired = retired_n;
        stats->steps = steps;
        stats->units = units;
        stats->round_s = s->now() - t_round;
        stats->arena_used = s->arena.used_bytes();
        stats->arena_largest_free = s->arena.largest_free();
    }
    return HRLB_OK;
}

extern "C" hrlb_status hrlb_server_request(hrlb_server* s, long id, hrlb_request_info* info, double* fields, double* x,
                                           int release)
{
    if (!s) return fail(HRLB_E_INVALID, "server is NULL");
    auto it = s->all.find(id);
    if (it == s->all.end()) return fail(HRLB_E_INVALID, "unknown request id %ld", id);
    Request* rq = it->second.get();
    if (info) {
        info->state = rq->state;
        info->status = rq->status;
        info->steps = rq->taken;
        info->residual = rq->track.res;
        info->pxy_drift = rq->track.drift;
        info->pxy_err = rq->track.err;
        info->Pi = rq->pi;
        info->sim_time = rq->sim_time;
        info->mass_drift = rq->mass_drift;
        info->t_arrival = rq->t_arrival;
        info->t_admit = rq->t_admit;
        info->t_done = rq->t_done;
        info->n_cells = rq->r.params.n_cells;
        info->n_vel = 2 * rq->r.Qx * rq->r.Qy;
        info->bytes = rq->bytes;
    }
    if (rq->state == HRLB_REQ_DONE) {
        if (fields) std::copy(rq->fields.begin(), rq->fields.end(), fields);
        if (x) std::copy(rq->x.begin(), rq->x.end(), x);
    }
    if (release && (rq->state == HRLB_REQ_DONE || rq->state == HRLB_REQ_FAILED)) s->all.erase(it);
    return HRLB_OK;
}

extern "C" void hrlb_server_free(hrlb_server* s) { delete s; }
