// Serving engine: independent solve requests on resident geometries.
//
// Requests of one geometry share a multi-rhs state; each request owns one
// lane (one rhs) of it from admission to completion.  A worker thread drives
// every geometry's state on a stream of its own: whenever a state's cycle
// has finished it reads the per-lane residual norms, retires converged lanes
// (copies their solution out), admits waiting requests into free lanes, and
// launches the next cycle (a replayed HIP graph) for all running lanes.  New
// requests thus join a batch between two cycles instead of waiting for it to
// drain (continuous batching).  Lane fields are held within a device-memory
// budget; idle states of other geometries are released when a waiting
// geometry needs room, and while a geometry waits for memory the others
// admit nothing new, so their states drain (no geometry starves).
//
// Every lane goes through exactly the operations a one-rhs solve of the same
// request performs (zero start, V-cycles, the same convergence and stall
// tests), and kernels never mix lanes, so a result does not depend on what
// else was in flight.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cmath>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "octmg_internal.hpp"

using namespace octmg;

namespace {

#define SHIP(call)                                                                           \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return api_fail(e_ == hipErrorOutOfMemory ? OCTMG_ERR_OOM : OCTMG_ERR_HIP,       \
                            std::string(#call) + ": " + hipGetErrorString(e_));              \
    } while (0)

#define SSTCK(call)                    \
    do {                               \
        octmg_status s_ = (call);      \
        if (s_ != OCTMG_OK) return s_; \
    } while (0)

struct Request {
    uint64_t id = 0;
    int slot = 0;
    const double *rhs = nullptr;
    int rhs_dev = 0;
    double *out = nullptr;
    int out_dev = 0;
    double rtol = 0.0;
    double t_submit = 0.0, t_admit = 0.0;
};

struct Lane {
    bool busy = false;
    bool running = false;  // admitted and not yet retired
    bool fresh = false;    // admitted in the pass in flight: its first norms are pending
    bool storing = false;  // finished: its solution is being copied out, published next pass
    bool ran = false;      // cycled in the pass in flight
    int status = OCTMG_OK;
    Request req;
    int cycles = 0, stall = 0;
    double r0 = 0.0, cur = 0.0, prev = 0.0;
};

struct Slot {
    octmg_geom geom = nullptr;
    std::vector<double> iface, dom;
    octmg_state state = nullptr;
    size_t bytes = 0;
    std::vector<Lane> lanes;
    std::deque<Request> pending;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool inflight = false;
    double last_used = 0.0;
};

}  // namespace

struct octmg_server_s {
    int device = 0;
    octmg_server_opts opts{};
    std::chrono::steady_clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv;
    bool stop = false;
    std::deque<Request> incoming;
    std::vector<octmg_result> finished;
    std::vector<std::unique_ptr<Slot>> slots;  // grown under mu, read by the worker
    uint64_t next_id = 1;
    size_t used = 0;
    // a geometry waiting for memory: other geometries admit no new requests
    // until it has a state, so their states drain and can be released
    int starving = -1;
    octmg_server_stats stats{};
    std::string worker_error;
    std::thread worker;

    double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }

    void finish(const Request &r, int status, int cycles, double r0, double rf) {
        octmg_result o{};
        o.id = r.id;
        o.status = status;
        o.cycles = cycles;
        o.r0 = r0;
        o.r_final = rf;
        o.t_submit = r.t_submit;
        o.t_admit = r.t_admit;
        o.t_done = now();
        std::lock_guard<std::mutex> g(mu);
        finished.push_back(o);
        stats.completed++;
        if (status != OCTMG_OK) stats.failed++;
    }

    octmg_status release(Slot &S) {
        if (!S.state) return OCTMG_OK;
        octmg_state_destroy(S.state);
        S.state = nullptr;
        S.lanes.clear();
        used -= S.bytes;
        S.bytes = 0;
        stats.states_released++;
        return OCTMG_OK;
    }

    // A state for S with as many lanes as the budget allows (up to
    // max_lanes), releasing idle states of other geometries first if that is
    // what it takes to fit one lane.  A state costs its fixed part plus
    // lane_bytes per lane.
    octmg_status acquire(Slot &S, int idx, bool *rejected) {
        *rejected = false;
        const size_t lane = lane_bytes(S.geom, opts.precision), fixed = state_fixed_bytes(S.geom);
        const size_t per = lane + fixed;  // the smallest state: one lane
        if (per > opts.hbm_budget_bytes) {
            *rejected = true;
            return OCTMG_OK;
        }
        if (used + per > opts.hbm_budget_bytes) {
            std::vector<Slot *> idle;
            for (auto &p : slots)
                if (p.get() != &S && p->state && !p->inflight) {
                    bool any = false;
                    for (auto &l : p->lanes) any |= l.busy;
                    if (!any) idle.push_back(p.get());
                }
            // states nobody waits for first, then the least recently used
            std::sort(idle.begin(), idle.end(), [](Slot *a, Slot *b) {
                if (a->pending.empty() != b->pending.empty()) return a->pending.empty();
                return a->last_used < b->last_used;
            });
            for (Slot *p : idle) {
                if (used + per <= opts.hbm_budget_bytes) break;
                SSTCK(release(*p));
            }
            if (used + per > opts.hbm_budget_bytes) {  // wait for lanes elsewhere to finish
                if (starving < 0) starving = idx;
                return OCTMG_OK;
            }
        }
        const size_t fit = (opts.hbm_budget_bytes - used - fixed) / lane;
        const int n = (int)std::min<size_t>(fit, (size_t)opts.max_lanes);
        octmg_state st = nullptr;
        SSTCK(octmg_state_create(S.geom, n, opts.precision, &st));
        octmg_status r = octmg_set_boundary(st, S.iface.empty() ? nullptr : S.iface.data(), S.dom.data(), 0,
                                            S.stream);
        if (r == OCTMG_OK) r = lanes_prepare(st);
        if (r != OCTMG_OK) {
            octmg_state_destroy(st);
            return r;
        }
        S.state = st;
        S.bytes = fixed + lane * (size_t)n;
        used += S.bytes;
        S.lanes.assign(n, Lane{});
        if (starving == idx) starving = -1;
        stats.states_created++;
        stats.peak_bytes = std::max<uint64_t>(stats.peak_bytes, used);
        return OCTMG_OK;
    }

    // convergence test of one lane after its norm `v`, in the order of a
    // one-rhs solve: non-finite, converged, cycle limit, stall.  Returns
    // false while the lane keeps cycling, else true with its final status.
    bool settle(Lane &l, double v, int *status) {
        l.cur = v;
        if (!std::isfinite(v)) return *status = OCTMG_ERR_NONFINITE, true;
        if (v <= l.req.rtol * l.r0) return *status = OCTMG_OK, true;
        if (l.cycles == opts.max_cycles) return *status = OCTMG_ERR_NOT_CONVERGED, true;
        if (l.cycles > 0) {
            l.stall = v > 0.95 * l.prev ? l.stall + 1 : 0;
            if (l.stall >= 3) return *status = OCTMG_ERR_NOT_CONVERGED, true;
        }
        l.prev = v;
        return false;
    }

    // One pass over a slot; returns whether anything happened.  A pass only
    // enqueues work on the slot's stream and records one event; the next
    // pass, once the event has passed, reads what the work produced:
    //   1. publish the lanes whose solutions were being copied out;
    //   2. settle lanes admitted last pass on their first norms (cycle 0);
    //   3. settle lanes that cycled on the cycle's norms;
    //   4. copy out the lanes that finished, admit waiting requests into
    //      free lanes (load rhs, first norms), launch the next cycle of the
    //      running lanes, record the event.
    // A lane admitted in a pass also cycles in it; a lane that had in fact
    // converged before its first cycle (r0 = 0: phi = 0 is exact) is settled
    // at cycle 0, and its cycle left phi = 0 unchanged.  Host buffers are
    // staged synchronously (lane_load / lane_store wait for them).
    octmg_status service(Slot &S, int idx, bool *progress) {
        if (S.inflight) {
            const hipError_t q = hipEventQuery(S.done);
            if (q == hipErrorNotReady) return OCTMG_OK;
            SHIP(q);
            S.inflight = false;
            *progress = true;
            std::vector<double> nv, r0, rk;
            lanes_norms(S.state, nv);
            lanes_begin_norms(S.state, r0, rk);
            for (int i = 0; i < (int)S.lanes.size(); i++) {
                Lane &l = S.lanes[i];
                if (l.storing) {
                    finish(l.req, l.status, l.cycles, l.r0, l.cur);
                    l = Lane{};
                    continue;
                }
                bool done = false;
                if (l.fresh) {
                    l.fresh = false;
                    l.r0 = r0[i];
                    done = settle(l, rk[i], &l.status);
                }
                if (!done && l.ran) {
                    l.cycles++;
                    done = settle(l, nv[i], &l.status);
                }
                l.ran = false;
                if (done) SSTCK(retire(S, i));
            }
        }
        if (!S.pending.empty() && !S.state) {
            bool rejected = false;
            SSTCK(acquire(S, idx, &rejected));
            if (rejected) {
                while (!S.pending.empty()) {
                    finish(S.pending.front(), OCTMG_ERR_BUDGET, 0, 0.0, 0.0);
                    S.pending.pop_front();
                }
                return OCTMG_OK;
            }
        }
        if (!S.state) return OCTMG_OK;
        std::vector<int> fresh(S.lanes.size(), 0);
        bool any_fresh = false;
        const bool admit = starving < 0 || starving == idx;
        for (int i = 0; i < (int)S.lanes.size() && admit && !S.pending.empty(); i++) {
            Lane &l = S.lanes[i];
            if (l.busy) continue;
            Request r = S.pending.front();
            S.pending.pop_front();
            r.t_admit = now();
            const octmg_status st = lane_load(S.state, i, r.rhs, r.rhs_dev, S.stream);
            if (st != OCTMG_OK) {
                finish(r, st, 0, 0.0, 0.0);
                continue;
            }
            l = Lane{};
            l.busy = l.running = l.fresh = true;
            l.req = r;
            fresh[i] = 1;
            any_fresh = true;
            stats.admitted++;
        }
        if (any_fresh) {
            *progress = true;
            SSTCK(lanes_begin(S.state, fresh, S.stream));
        }
        std::vector<int> run(S.lanes.size(), 0);
        bool any = false, storing = false;
        for (int i = 0; i < (int)S.lanes.size(); i++) {
            if (S.lanes[i].running) run[i] = 1, any = true, S.lanes[i].ran = true;
            storing |= S.lanes[i].storing;
        }
        if (any) {
            SSTCK(lanes_cycle(S.state, run, OCTMG_CYCLE_V, S.stream));
            stats.cycles_launched++;
            int k = 0;
            for (int v : run) k += v;
            stats.lane_cycles += k;
        }
        if (any || storing) {
            SHIP(hipEventRecord(S.done, S.stream));
            S.inflight = true;
            S.last_used = now();
        }
        return OCTMG_OK;
    }

    // lane i has its final status: copy its iterate out (unless it is not
    // finite) and publish it once that copy has passed; a lane that is not
    // copied is published now
    octmg_status retire(Slot &S, int i) {
        Lane &l = S.lanes[i];
        l.running = false;
        if (l.status == OCTMG_ERR_NONFINITE) {
            finish(l.req, l.status, l.cycles, l.r0, l.cur);
            l = Lane{};
            return OCTMG_OK;
        }
        SSTCK(lane_store(S.state, i, l.req.out, l.req.out_dev, S.stream));
        if (l.req.out_dev) {
            l.storing = true;
        } else {  // copied and waited for already
            finish(l.req, l.status, l.cycles, l.r0, l.cur);
            l = Lane{};
        }
        return OCTMG_OK;
    }

    void run() {
        if (hipSetDevice(device) != hipSuccess) {
            worker_error = "hipSetDevice failed in the server thread";
            return;
        }
        for (;;) {
            std::vector<Slot *> view;
            {
                std::unique_lock<std::mutex> g(mu);
                bool busy = !incoming.empty();
                for (auto &p : slots) busy |= p->inflight || !p->pending.empty();
                if (!busy) {
                    if (stop) return;
                    cv.wait_for(g, std::chrono::microseconds(200));
                    if (incoming.empty()) continue;
                }
                for (auto &p : slots) view.push_back(p.get());
                while (!incoming.empty()) {
                    Request r = incoming.front();
                    incoming.pop_front();
                    view[r.slot]->pending.push_back(r);
                }
            }
            bool progress = false;
            for (int i = 0; i < (int)view.size(); i++) {
                const octmg_status st = service(*view[i], i, &progress);
                if (st != OCTMG_OK) {
                    // a device error ends the worker; waiting and running requests fail
                    std::lock_guard<std::mutex> g(mu);
                    worker_error = octmg_last_error();
                    stop = true;
                }
            }
            if (!worker_error.empty()) {
                for (Slot *s : view) {
                    for (auto &l : s->lanes)
                        if (l.busy) finish(l.req, OCTMG_ERR_HIP, l.cycles, l.r0, l.cur);
                    for (auto &r : s->pending) finish(r, OCTMG_ERR_HIP, 0, 0.0, 0.0);
                    s->lanes.clear();
                    s->pending.clear();
                    s->inflight = false;
                }
                std::lock_guard<std::mutex> g(mu);
                for (auto &r : incoming) {
                    octmg_result o{};
                    o.id = r.id;
                    o.status = OCTMG_ERR_HIP;
                    o.t_submit = r.t_submit;
                    o.t_done = now();
                    finished.push_back(o);
                }
                incoming.clear();
                return;
            }
            if (!progress) std::this_thread::yield();
        }
    }
};

extern "C" {

octmg_status octmg_server_create(int device, const octmg_server_opts *o, octmg_server *out) {
    if (!o || !out) return api_fail(OCTMG_ERR_INVALID, "null argument");
    if (o->max_lanes < 1 || o->max_lanes > 4096 || o->max_cycles < 1 || o->max_cycles > 64 ||
        (o->precision != OCTMG_FP64 && o->precision != OCTMG_MIXED) || o->hbm_budget_bytes == 0)
        return api_fail(OCTMG_ERR_INVALID, "bad server options");
    int n = 0;
    SHIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return api_fail(OCTMG_ERR_INVALID, "bad device");
    std::unique_ptr<octmg_server_s> s(new octmg_server_s());
    s->device = device;
    s->opts = *o;
    s->t0 = std::chrono::steady_clock::now();
    s->worker = std::thread([p = s.get()] { p->run(); });
    *out = s.release();
    return OCTMG_OK;
}

octmg_status octmg_server_add_geometry(octmg_server s, octmg_geom g, const double *iface_vals,
                                       const double *domain_vals, int *slot) {
    if (!s || !g || !slot) return api_fail(OCTMG_ERR_INVALID, "null argument");
    int64_t info[8];
    SSTCK(octmg_geom_info(g, info));
    if (geom_device(g) != s->device) return api_fail(OCTMG_ERR_INVALID, "geometry lives on another device");
    const int64_t n_iface = info[2], n_domain = info[3];
    std::unique_ptr<Slot> S(new Slot());
    S->geom = g;
    if (iface_vals && n_iface) S->iface.assign(iface_vals, iface_vals + n_iface);
    S->dom.assign((size_t)n_domain, 0.0);
    if (domain_vals) S->dom.assign(domain_vals, domain_vals + n_domain);
    for (double v : S->iface)
        if (!std::isfinite(v)) return api_fail(OCTMG_ERR_NONFINITE, "interface value is not finite");
    for (double v : S->dom)
        if (!std::isfinite(v)) return api_fail(OCTMG_ERR_NONFINITE, "domain value is not finite");
    SHIP(hipSetDevice(s->device));
    SHIP(hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking));
    SHIP(hipEventCreateWithFlags(&S->done, hipEventDisableTiming));
    std::lock_guard<std::mutex> lk(s->mu);
    *slot = (int)s->slots.size();
    s->slots.push_back(std::move(S));
    return OCTMG_OK;
}

octmg_status octmg_server_submit(octmg_server s, int slot, const double *rhs, int rhs_on_device, double *solution,
                                 int solution_on_device, double rtol, uint64_t *id) {
    if (!s || !rhs || !solution || !id) return api_fail(OCTMG_ERR_INVALID, "null argument");
    if (!(rtol > 0.0)) return api_fail(OCTMG_ERR_INVALID, "rtol must be positive");
    std::lock_guard<std::mutex> g(s->mu);
    if (!s->worker_error.empty()) return api_fail(OCTMG_ERR_HIP, "server stopped: " + s->worker_error);
    if (slot < 0 || slot >= (int)s->slots.size()) return api_fail(OCTMG_ERR_INVALID, "unknown geometry slot");
    Request r;
    r.id = s->next_id++;
    r.slot = slot;
    r.rhs = rhs;
    r.rhs_dev = rhs_on_device;
    r.out = solution;
    r.out_dev = solution_on_device;
    r.rtol = rtol;
    r.t_submit = s->now();
    s->incoming.push_back(r);
    s->stats.submitted++;
    *id = r.id;
    s->cv.notify_one();
    return OCTMG_OK;
}

octmg_status octmg_server_poll(octmg_server s, octmg_result *done, int cap, int *n_done) {
    if (!s || !n_done || (cap > 0 && !done)) return api_fail(OCTMG_ERR_INVALID, "null argument");
    std::lock_guard<std::mutex> g(s->mu);
    const int n = std::min<int>(cap, (int)s->finished.size());
    std::copy(s->finished.begin(), s->finished.begin() + n, done);
    s->finished.erase(s->finished.begin(), s->finished.begin() + n);
    *n_done = n;
    if (n == 0 && !s->worker_error.empty()) return api_fail(OCTMG_ERR_HIP, "server stopped: " + s->worker_error);
    return OCTMG_OK;
}

octmg_status octmg_server_get_stats(octmg_server s, octmg_server_stats *out) {
    if (!s || !out) return api_fail(OCTMG_ERR_INVALID, "null argument");
    std::lock_guard<std::mutex> g(s->mu);
    *out = s->stats;
    out->bytes_in_use = s->used;
    out->now = s->now();
    return OCTMG_OK;
}

void octmg_server_destroy(octmg_server s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
        s->cv.notify_one();
    }
    // the worker finishes what is queued or running before it exits
    if (s->worker.joinable()) s->worker.join();
    (void)hipSetDevice(s->device);
    for (auto &p : s->slots) {
        if (p->state) octmg_state_destroy(p->state);
        if (p->done) (void)hipEventDestroy(p->done);
        if (p->stream) (void)hipStreamDestroy(p->stream);
    }
    delete s;
}

}  // extern "C"
