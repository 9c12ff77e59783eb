// server.cpp -- serving form of the step: continuous batching of many solves
// on one device.  Requests of different grids, velocity grids and physics
// queue up, are admitted in arrival order whenever a block of the server's
// workspace large enough for their footprint and an active slot are free,
// and keep their state resident.  Solves smaller than a fusion limit (cell
// x node updates per step) form the fused group: they advance together on
// the server's stream, where one captured HIP graph of K fused steps over
// the group (each step one launch per fill phase and per update tile group,
// spanning the workgroups of all members) is replayed and captured again
// when a member joins or leaves.  Larger solves fill the device on their own
// and run standalone: each has its own stream and captured graph of K
// steps, concurrent with the group.  A new solve is prepared on its own
// stream while replays run and joins the group at the group's next replay.
// After each replay the drag coefficient of every solve in it is checked; a
// solve ends when |C_D(n) - C_D(n - K)| < tol |C_D(n)| or a step cap is
// reached, and releases its memory and slot to the queue.
//
// Built on the public C ABI only (ibdvm_create, ibdvm_batch_graph_create, ...).
#include <hip/hip_runtime_api.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "ibdvm.h"

namespace {

constexpr size_t kAlign = 256;

// first-fit allocator over the server workspace with coalescing frees
class Arena {
public:
    void reset(size_t bytes)
    {
        free_.clear();
        free_[0] = bytes;
        total_ = bytes;
        used_ = 0;
    }
    bool take(size_t bytes, size_t &off)
    {
        bytes = (bytes + kAlign - 1) / kAlign * kAlign;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            off = it->first;
            const size_t rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[off + bytes] = rest;
            used_ += bytes;
            return true;
        }
        return false;
    }
    void give(size_t off, size_t bytes)
    {
        bytes = (bytes + kAlign - 1) / kAlign * kAlign;
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t total() const { return total_; }

private:
    std::map<size_t, size_t> free_;  // offset -> length
    size_t total_ = 0, used_ = 0;
};

struct Request {
    int64_t id = 0;
    ibdvm_grid grid{};
    ibdvm_vgrid vgrid{};
    ibdvm_geometry geom{};
    double Kn = 0, Ma = 0, Pr = 0, gamma = 0, alpha = 1, Tw = 1;
    ibdvm_opts opts{};
    uint64_t seed = 0;
    double amp = 0, tol = 0;
    int64_t max_steps = 0;
    double *moments_out = nullptr;
    size_t bytes = 0;
    double t_submit = 0;
};

struct Active {
    Request rq;
    size_t off = 0;
    ibdvm_ctx *ctx = nullptr;
    bool fused = false;           // member of the fused group
    bool joined = false;          // fused: on the server stream, in the group graph
    hipStream_t stream = nullptr; // standalone solves; fused ones until they join
    hipEvent_t done = nullptr;    // standalone: end of its replay in flight
    ibdvm_graph *graph = nullptr; // standalone: K captured steps
    bool inflight = false;        // standalone
    int64_t steps = 0, updates_per_step = 0;
    double cd_prev = NAN, cd = NAN, cl = NAN;
    double t_admit = 0;
    int32_t tile[3] = {0, 0, 0};
};

}  // namespace

struct ibdvm_server {
    char *ws = nullptr;
    Arena arena;
    int32_t max_active = 1, K = 100;
    int device = 0;
    int64_t fuse_below = 1 << 24;   // solves with fewer updates per step join the fused group
    hipStream_t stream = nullptr;   // the fused group's stream
    hipEvent_t done = nullptr;      // end of the group replay in flight
    ibdvm_graph *graph = nullptr;   // K fused steps of the group; null when the group changed
    bool inflight = false;
    int64_t next_id = 1, finished = 0;
    std::deque<Request> queue;
    std::vector<Active> active;
    std::vector<ibdvm_result> ready;  // finished, not yet returned by poll
    std::map<std::tuple<int, int, int, int, int, int>, std::vector<int32_t>> tiles;  // autotune cache
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    std::string err;
    double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
};

namespace {

ibdvm_status hip_fail(ibdvm_server *s, hipError_t e, const char *what)
{
    s->err = std::string(what) + ": " + hipGetErrorString(e);
    return IBDVM_E_DEVICE;
}

// the active set changes: the captured graph addresses its contexts
void drop_graph(ibdvm_server *s)
{
    if (s->graph) ibdvm_graph_destroy(s->graph);
    s->graph = nullptr;
}

void release(ibdvm_server *s, Active &a)
{
    if (a.joined) drop_graph(s);
    if (a.graph) ibdvm_graph_destroy(a.graph);
    if (a.ctx) ibdvm_destroy(a.ctx);
    if (a.done) (void)hipEventDestroy(a.done);
    if (a.stream) (void)hipStreamDestroy(a.stream);
    a.graph = nullptr;
    a.ctx = nullptr;
    a.done = nullptr;
    a.stream = nullptr;
    s->arena.give(a.off, a.rq.bytes);
}

void retire(ibdvm_server *s, Active &a, ibdvm_status status, int converged)
{
    ibdvm_result r{};
    r.id = a.rq.id;
    r.status = status;
    r.converged = converged;
    r.steps = a.steps;
    r.C_D = a.cd;
    r.C_L = a.cl;
    r.t_submit = a.rq.t_submit;
    r.t_admit = a.t_admit;
    r.updates = a.updates_per_step * a.steps;
    std::memcpy(r.tile, a.tile, sizeof(r.tile));
    if (status == IBDVM_OK && a.rq.moments_out) r.status = ibdvm_moments(a.ctx, a.rq.moments_out, 0);
    release(s, a);
    r.t_done = s->now();
    s->ready.push_back(r);
    s->finished += 1;
}

// creates the context of a request in its workspace block on a stream of its
// own (overlapping the replays in flight); standalone solves also capture
// their graph
ibdvm_status admit(ibdvm_server *s, Active &a)
{
    hipError_t e = hipStreamCreateWithFlags(&a.stream, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(s, e, "stream");
    ibdvm_opts o = a.rq.opts;
    o.workspace = s->ws + a.off;
    o.workspace_bytes = a.rq.bytes;
    o.stream = a.stream;
    ibdvm_status st = ibdvm_create(&a.rq.grid, &a.rq.vgrid, &a.rq.geom, a.rq.Kn, a.rq.Ma, a.rq.Pr, a.rq.gamma,
                                   a.rq.alpha, a.rq.Tw, &o, &a.ctx);
    if (st) return st;
    if ((st = ibdvm_init_freestream_hashed(a.ctx, a.rq.seed, a.rq.amp))) return st;
    int64_t info[7];
    if ((st = ibdvm_info(a.ctx, info))) return st;
    a.updates_per_step = info[5] * info[2];  // fluid cells x velocity nodes
    if (a.rq.grid.dim == 2) {
        const auto key = std::make_tuple(a.rq.grid.n[0], a.rq.grid.n[1], a.rq.vgrid.n[0], a.rq.vgrid.n[1],
                                         (int)a.rq.opts.precision, 0);
        auto it = s->tiles.find(key);
        if (it == s->tiles.end()) {
            int32_t t[3];
            if ((st = ibdvm_autotune(a.ctx, 2, t))) return st;
            it = s->tiles.emplace(key, std::vector<int32_t>{t[0], t[1], t[2]}).first;
        }
        if ((st = ibdvm_set_tile(a.ctx, it->second[0], it->second[1], it->second[2]))) return st;
        if ((st = ibdvm_get_tile(a.ctx, a.tile))) return st;
    }
    a.fused = a.updates_per_step < s->fuse_below;
    if (a.fused) return IBDVM_OK;
    if ((e = hipEventCreateWithFlags(&a.done, hipEventDisableTiming)) != hipSuccess) return hip_fail(s, e, "event");
    return ibdvm_graph_create(a.ctx, s->K, &a.graph);
}

// after a replay: C_D, convergence, retirement; false if the solve ended
bool harvest(ibdvm_server *s, Active &a)
{
    a.steps += s->K;
    double F[3];
    int32_t np = 0;
    ibdvm_status st = ibdvm_surface_forces(a.ctx, F, &a.cd, &a.cl, nullptr, 0, &np);
    if (st) {
        retire(s, a, st, 0);
        return false;
    }
    const bool conv =
        a.rq.tol > 0.0 && std::isfinite(a.cd_prev) && std::fabs(a.cd - a.cd_prev) < a.rq.tol * std::fabs(a.cd);
    a.cd_prev = a.cd;
    if (conv || a.steps >= a.rq.max_steps) {
        retire(s, a, IBDVM_OK, conv ? 1 : 0);
        return false;
    }
    return true;
}

// one pass: harvest finished replays, check convergence, admit, relaunch.
// wait: block on one replay in flight (the group's first) before harvesting
ibdvm_status pass(ibdvm_server *s, bool wait)
{
    bool waited = false;
    auto ready = [&](hipEvent_t ev, hipError_t &q) {
        q = (wait && !waited) ? hipEventSynchronize(ev) : hipEventQuery(ev);
        waited = waited || wait;
        if (q == hipErrorNotReady) {
            (void)hipGetLastError();  // not an error: keep it out of the next launch check
            return false;
        }
        return true;
    };
    hipError_t q;
    if (s->inflight && ready(s->done, q)) {
        if (q != hipSuccess) return hip_fail(s, q, "group replay");
        s->inflight = false;
        for (size_t i = 0; i < s->active.size();) {
            Active &a = s->active[i];
            if (a.joined && !harvest(s, a)) {
                s->active.erase(s->active.begin() + (long)i);
                continue;
            }
            ++i;
        }
    }
    for (size_t i = 0; i < s->active.size();) {
        Active &a = s->active[i];
        if (a.inflight && ready(a.done, q)) {
            if (q != hipSuccess) return hip_fail(s, q, "replay");
            a.inflight = false;
            if (!harvest(s, a)) {
                s->active.erase(s->active.begin() + (long)i);
                continue;
            }
        }
        ++i;
    }
    // the group's stream and event are made at the first admission, so
    // creating a server and queueing requests touch no device
    if (!s->stream && !s->queue.empty()) {
        hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s->done, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(s, e, "server stream");
    }
    // admission in arrival order: the head waits until its block fits
    while (!s->queue.empty() && (int32_t)s->active.size() < s->max_active) {
        Request &rq = s->queue.front();
        size_t off = 0;
        if (!s->arena.take(rq.bytes, off)) break;
        Active a;
        a.rq = rq;
        a.off = off;
        a.t_admit = s->now();
        s->queue.pop_front();
        ibdvm_status st = admit(s, a);
        if (st) {
            if (a.ctx == nullptr) s->err = ibdvm_last_error();
            retire(s, a, st, 0);
            continue;
        }
        s->active.push_back(a);
    }
    // relaunch: standalone solves, then the group (new members join now)
    for (Active &a : s->active)
        if (!a.fused && !a.inflight) {
            ibdvm_status st = ibdvm_graph_launch(a.graph);
            if (st) {
                s->err = ibdvm_last_error();
                return st;
            }
            hipError_t e = hipEventRecord(a.done, a.stream);
            if (e != hipSuccess) return hip_fail(s, e, "event record");
            a.inflight = true;
        }
    if (s->inflight) return IBDVM_OK;
    std::vector<ibdvm_ctx *> group;
    for (Active &a : s->active) {
        if (!a.fused) continue;
        if (!a.joined) {
            ibdvm_status st = ibdvm_set_stream(a.ctx, s->stream);
            if (st) {
                s->err = ibdvm_last_error();
                return st;
            }
            (void)hipStreamDestroy(a.stream);
            a.stream = nullptr;
            a.joined = true;
            drop_graph(s);
        }
        group.push_back(a.ctx);
    }
    if (group.empty()) return IBDVM_OK;
    if (!s->graph) {
        ibdvm_status st = ibdvm_batch_graph_create(group.data(), (int32_t)group.size(), s->K, &s->graph);
        if (st) {
            s->err = ibdvm_last_error();
            return st;
        }
    }
    ibdvm_status st = ibdvm_graph_launch(s->graph);
    if (st) {
        s->err = ibdvm_last_error();
        return st;
    }
    hipError_t e = hipEventRecord(s->done, s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "event record");
    s->inflight = true;
    return IBDVM_OK;
}

}  // namespace

extern "C" {

ibdvm_status ibdvm_server_create(void *workspace, size_t bytes, int32_t max_active, int32_t steps_per_replay,
                                 ibdvm_server **out)
{
    if (!out) return IBDVM_E_INVALID_ARG;
    *out = nullptr;
    if (!workspace || bytes < kAlign || ((uintptr_t)workspace % kAlign) != 0) return IBDVM_E_INVALID_ARG;
    if (max_active < 1 || steps_per_replay < 2 || (steps_per_replay & 1)) return IBDVM_E_INVALID_ARG;
    auto *s = new ibdvm_server;
    s->ws = (char *)workspace;
    s->arena.reset(bytes / kAlign * kAlign);
    s->max_active = max_active;
    s->K = steps_per_replay;
    *out = s;
    return IBDVM_OK;
}

ibdvm_status ibdvm_server_submit(ibdvm_server *s, const ibdvm_grid *grid, const ibdvm_vgrid *vgrid,
                                 const ibdvm_geometry *geom, double Kn, double Ma, double Pr, double gamma,
                                 double alpha, double T_w, const ibdvm_opts *opts, uint64_t seed, double amp,
                                 double tol, int64_t max_steps, double *moments_out, int64_t *id)
{
    if (!s || !grid || !vgrid || !geom || !opts || !id) return IBDVM_E_INVALID_ARG;
    if (grid->dim != 2) {
        s->err = "the serving form takes 2D problems";
        return IBDVM_E_UNSUPPORTED;
    }
    if (max_steps < s->K) return IBDVM_E_INVALID_ARG;
    Request rq;
    rq.grid = *grid;
    rq.vgrid = *vgrid;
    rq.geom = *geom;
    rq.Kn = Kn;
    rq.Ma = Ma;
    rq.Pr = Pr;
    rq.gamma = gamma;
    rq.alpha = alpha;
    rq.Tw = T_w;
    rq.opts = *opts;
    rq.opts.workspace = nullptr;
    rq.opts.stream = nullptr;
    rq.seed = seed;
    rq.amp = amp;
    rq.tol = tol;
    rq.max_steps = max_steps;
    rq.moments_out = moments_out;
    ibdvm_status st = ibdvm_footprint(grid, vgrid, geom, &rq.opts, &rq.bytes);
    if (st) {
        s->err = ibdvm_last_error();
        return st;
    }
    if ((rq.bytes + kAlign - 1) / kAlign * kAlign > s->arena.total()) {
        s->err = "request footprint exceeds the server workspace";
        return IBDVM_E_NO_MEMORY;
    }
    rq.id = s->next_id++;
    rq.t_submit = s->now();
    s->queue.push_back(rq);
    *id = rq.id;
    return IBDVM_OK;
}

ibdvm_status ibdvm_server_poll(ibdvm_server *s, int32_t block, ibdvm_result *done, int32_t cap, int32_t *n_done)
{
    if (!s || !n_done || (cap > 0 && !done)) return IBDVM_E_INVALID_ARG;
    *n_done = 0;
    ibdvm_status st = pass(s, false);
    while (!st && block && s->ready.empty() && !s->active.empty()) st = pass(s, true);
    int32_t n = 0;
    while (n < cap && !s->ready.empty()) {
        done[n++] = s->ready.front();
        s->ready.erase(s->ready.begin());
    }
    *n_done = n;
    return st;
}

ibdvm_status ibdvm_server_cancel(ibdvm_server *s, int64_t id)
{
    if (!s) return IBDVM_E_INVALID_ARG;
    for (auto it = s->queue.begin(); it != s->queue.end(); ++it)
        if (it->id == id) {
            ibdvm_result r{};
            r.id = id;
            r.status = IBDVM_E_CANCELLED;
            r.t_submit = it->t_submit;
            r.t_admit = r.t_done = s->now();
            s->queue.erase(it);
            s->ready.push_back(r);
            s->finished += 1;
            return IBDVM_OK;
        }
    for (size_t i = 0; i < s->active.size(); ++i) {
        Active &a = s->active[i];
        if (a.rq.id != id) continue;
        // the replay in flight that runs this solve ends before its memory is
        // released: its own (standalone, or fused but not yet joined), or the
        // group's (joined); a finished group replay is harvested by the next
        // pass for the other members
        hipError_t e = hipSuccess;
        bool ran = false;  // a replay of this solve was in flight and has now ended
        if (a.joined) {
            ran = s->inflight;
            if (ran) e = hipEventSynchronize(s->done);
        } else if (a.inflight) {
            ran = true;
            e = hipEventSynchronize(a.done);
        } else if (a.stream) {
            e = hipStreamSynchronize(a.stream);
        }
        if (e != hipSuccess) return hip_fail(s, e, "cancel");
        if (ran) a.steps += s->K;
        retire(s, a, IBDVM_E_CANCELLED, 0);
        s->active.erase(s->active.begin() + (long)i);
        return IBDVM_OK;
    }
    s->err = "no queued or active request with this id";
    return IBDVM_E_INVALID_ARG;
}

ibdvm_status ibdvm_server_info(const ibdvm_server *s, int64_t out[5])
{
    if (!s || !out) return IBDVM_E_INVALID_ARG;
    out[0] = (int64_t)s->queue.size();
    out[1] = (int64_t)s->active.size();
    out[2] = s->finished;
    out[3] = (int64_t)s->arena.used();
    out[4] = (int64_t)s->arena.total();
    return IBDVM_OK;
}

double ibdvm_server_clock(const ibdvm_server *s) { return s ? s->now() : 0.0; }

ibdvm_status ibdvm_server_set_fusion(ibdvm_server *s, int64_t updates_per_step)
{
    if (!s || updates_per_step < 0) return IBDVM_E_INVALID_ARG;
    s->fuse_below = updates_per_step;
    return IBDVM_OK;
}

const char *ibdvm_server_error(const ibdvm_server *s) { return s ? s->err.c_str() : ""; }

void ibdvm_server_destroy(ibdvm_server *s)
{
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    for (Active &a : s->active) {
        if (a.stream) (void)hipStreamSynchronize(a.stream);
        release(s, a);
    }
    drop_graph(s);
    if (s->done) (void)hipEventDestroy(s->done);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

}  // extern "C"
