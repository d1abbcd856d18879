// Serving: continuous batching of solve requests over hierarchies cached on
// the device, admitted by an HBM budget.
//
// A request names a registered problem (mesh, order, lambda, options) and a
// right-hand side.  Every problem with resident memory owns one group: its
// hierarchy and a session of `slots` columns on a stream of its own, so the
// groups' work overlaps on the device.  Requests join free slots of their
// group between chunks of CG iterations and leave as soon as their column
// converges.  A problem without a resident hierarchy is set up on a worker
// thread once the budget allows, evicting idle groups in least-recently-used
// order.  Latency is measured from submission to the moment the solution is
// back in the caller's array.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>

#include "internal.h"

namespace giamg {

void build_hierarchy(Handle& H, const double* coords, const int32_t* l2g);
int64_t handle_device_bytes(const Handle& H);
struct Session;
Session* session_create(Handle& H, int k, double tol);
void session_destroy(Session* S);
void session_admit(Session* S, const int* slot, const double* const* b, int count);
void session_step(Session* S, int iters);
bool session_ready(Session* S);
void session_states(Session* S, int* state, giamg_info* infos);
void session_retire_async(Session* S, int slot, double* x);
hipStream_t session_stream(Session* S);
int64_t session_device_bytes(const Session* S);

namespace {
using Clock = std::chrono::steady_clock;

struct Problem {
    std::vector<double> coords;
    std::vector<int32_t> l2g;
    int64_t n_nodes = 0, n_elem = 0;
    int p = 1;
    double lambda = 0.0;
    giamg_opts opts{};
    int group = -1;          // resident group, or -1
    int64_t known_bytes = -1;  // device bytes measured at its last setup
    int64_t reserved = 0;      // bytes reserved while its setup runs
    bool setting_up = false;
    int failed = 0;          // error code of a failed setup
    std::string fail_msg;
};

struct Request {
    int64_t id = 0;
    int problem = 0;
    std::vector<double> b;
    double* x = nullptr;
    Clock::time_point submit, admitted, done;
    giamg_info info{};
    bool finished = false;
    bool counted = false;    // cache hit/miss recorded
    std::string msg;         // error message of a failed request
};

// A resident hierarchy with its session.  Slot s holds request slot_req[s]
// (-1: free).  A right-hand side enters through stretch s of the pinned input
// staging and of the device staging; a finished column drains (gathered into
// the device staging, copied to stretch s of the pinned output staging)
// behind the `drained` event, and its request completes once that event has
// passed.  A slot is free for a new request as soon as its drain is queued:
// the group's stream runs the drain before the next admission's copies.
struct Group {
    int problem = -1;
    std::unique_ptr<Handle> H;
    Session* S = nullptr;
    hipStream_t stream = nullptr;
    std::vector<int64_t> slot_req;   // request id per slot, -1 free
    std::vector<char> running;       // the column iterates (as of the last completed step)
    std::vector<std::pair<int, int64_t>> draining;   // (slot, request) on their way to the host
    std::vector<giamg_info> info;    // per slot: the state of its column when it finished
    hipEvent_t drained = nullptr;
    bool inflight = false;           // a step is queued and not yet complete
    Clock::time_point last_used;
    double solve_ms = 0.0;           // admission to completion of its last finished request
    int64_t bytes = 0;
    DevBuf<double> stage;            // [slots][n] right-hand sides / results
    double* pin_in = nullptr;        // [slots][n] host staging of right-hand sides
    double* pin_out = nullptr;       // [slots][n] host staging of solutions
    bool idle() const {
        return !inflight && draining.empty() &&
               std::none_of(slot_req.begin(), slot_req.end(), [](int64_t v) { return v >= 0; });
    }
    ~Group() {
        if (S) session_destroy(S);   // waits for the session's stream
        H.reset();
        if (stream) (void)hipStreamDestroy(stream);
        if (drained) (void)hipEventDestroy(drained);
        if (pin_in) (void)hipHostFree(pin_in);
        if (pin_out) (void)hipHostFree(pin_out);
    }
};
}  // namespace

struct Server {
    giamg_server_opts o{};
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done, cv_setup;
    std::deque<Problem> problems;                     // stable references
    std::map<int64_t, Request> requests;
    std::deque<int64_t> pending;
    std::vector<std::unique_ptr<Group>> groups;      // slot in this vector = group id
    std::deque<int> setup_jobs;
    std::vector<std::unique_ptr<Group>> setup_done;
    int64_t next_id = 1;
    int64_t resident = 0, reserved = 0;
    giamg_server_statistics st{};
    bool stop = false;
    int dead = 0;            // error code once the loop has died
    std::string dead_msg;
    int worker_dead = 0;     // error code once the setup worker has died
    std::string worker_msg;
    std::thread loop, setup;
    ~Server() {
        // the groups wait for their streams before freeing
        groups.clear();
        setup_done.clear();
    }

    // Device bytes of a problem's group: measured after its first setup,
    // before that an estimate (mean row length (p+2)^3 on hexahedral meshes;
    // coarse levels, transfers and work vectors add ~25 %).
    int64_t need(const Problem& P) const {
        if (P.known_bytes >= 0) return P.known_bytes;
        const double rows = (double)P.n_nodes;
        const double nnz = rows * (P.p + 2.0) * (P.p + 2.0) * (P.p + 2.0);
        const double vb = P.opts.precision == GIAMG_PREC_MIXED ? 16.0 : 12.0;
        return (int64_t)(1.25 * (vb * nnz + 150.0 * rows + 80.0 * rows * o.slots));
    }

    void setup_main() {
        GIAMG_HIP(hipSetDevice(device));
        while (true) {
            int pid;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_setup.wait(lk, [&] { return stop || !setup_jobs.empty(); });
                if (stop) return;
                pid = setup_jobs.front();
                setup_jobs.pop_front();
            }
            const Problem& P = problems[pid];
            std::unique_ptr<Group> g(new Group());
            int err = GIAMG_OK;
            std::string msg;
            try {
                g->problem = pid;
                GIAMG_HIP(hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking));
                g->H.reset(new Handle());
                Handle& H = *g->H;
                H.stream = g->stream;
                H.opts = P.opts;
                H.porder = P.p;
                H.lambda = P.lambda;
                H.n_nodes = P.n_nodes;
                H.n_elem = P.n_elem;
                build_hierarchy(H, P.coords.data(), P.l2g.data());
                g->S = session_create(H, o.slots, o.tol);
                g->stage.alloc((size_t)o.slots * P.n_nodes);
                GIAMG_HIP(hipHostMalloc(reinterpret_cast<void**>(&g->pin_in),
                                        (size_t)o.slots * P.n_nodes * sizeof(double)));
                GIAMG_HIP(hipHostMalloc(reinterpret_cast<void**>(&g->pin_out),
                                        (size_t)o.slots * P.n_nodes * sizeof(double)));
                GIAMG_HIP(hipEventCreateWithFlags(&g->drained, hipEventDisableTiming));
                g->slot_req.assign(o.slots, -1);
                g->running.assign(o.slots, 0);
                g->info.assign(o.slots, giamg_info{});
                g->bytes = handle_device_bytes(H) + session_device_bytes(g->S) +
                           (int64_t)g->stage.n * 8;
            } catch (const Error& e) {
                err = e.code;
                msg = e.what();
            } catch (const std::exception& e) {
                err = GIAMG_ENOMEM;
                msg = e.what();
            }
            std::lock_guard<std::mutex> lk(mu);
            if (err != GIAMG_OK) {
                problems[pid].failed = err;
                problems[pid].fail_msg = "setup failed: " + msg;
                problems[pid].setting_up = false;
                reserved -= problems[pid].reserved;
                problems[pid].reserved = 0;
                g.reset();
            } else {
                setup_done.push_back(std::move(g));
            }
            cv_work.notify_all();
        }
    }

    // the setup worker died outside a setup: the loop ends every request
    void worker_died(int code, const std::string& msg) {
        std::lock_guard<std::mutex> lk(mu);
        worker_dead = code;
        worker_msg = "setup worker: " + msg;
        cv_work.notify_all();
    }

    // the loop died: every unfinished request ends with `code`
    void fail_all(int code, const std::string& msg) {
        std::lock_guard<std::mutex> lk(mu);
        dead_msg = "server loop stopped: " + msg;
        for (auto& kv : requests)
            if (!kv.second.finished) {
                kv.second.msg = dead_msg;
                finish(kv.second, code);
            }
        pending.clear();
        dead = code;
    }

    // requires mu held
    void finish(Request& r, int status) {
        r.info.status = status;
        r.finished = true;
        r.done = Clock::now();
        st.completed += 1;
        cv_done.notify_all();
    }

    // requires mu held: evict idle groups (LRU) until `bytes` more fit; a
    // group larger than the budget is admitted only into an empty cache
    bool make_room(int64_t bytes, const std::map<int, std::vector<Request*>>& queued) {
        while (resident + reserved + bytes > o.hbm_budget) {
            if (resident == 0 && reserved == 0) return true;
            int victim = -1;
            for (size_t i = 0; i < groups.size(); ++i) {
                Group* g = groups[i].get();
                if (!g || !g->idle() || queued.count((int)i)) continue;
                if (victim < 0 || g->last_used < groups[victim]->last_used) victim = (int)i;
            }
            if (victim < 0) return false;
            resident -= groups[victim]->bytes;
            problems[groups[victim]->problem].group = -1;
            {
                std::lock_guard<std::mutex> cap(capture_mutex());
                groups[victim].reset();
            }
            st.evictions += 1;
        }
        return true;
    }

    // requires mu held: up to `room` pending requests for `problem`, in
    // arrival order, taken off the pending list
    std::vector<Request*> take_pending(int problem, int room) {
        std::vector<Request*> out;
        for (auto it = pending.begin(); it != pending.end() && (int)out.size() < room;) {
            Request& r = requests[*it];
            if (r.problem == problem) {
                out.push_back(&r);
                it = pending.erase(it);
            } else {
                ++it;
            }
        }
        return out;
    }

    // One pass over a group at a chunk boundary (no step in flight): drain
    // the columns that finished, admit pending requests into free slots,
    // queue the next chunk of iterations.  Every call here is asynchronous.
    // With hold_ms > 0 pending requests enter a group only once they fill its
    // free slots or the oldest of them has waited the group's hold: hold_ms,
    // or less once a request has finished there, the time that request took
    // from admission to completion (a hold longer than a solve costs more
    // latency than the batching gains).  An admission runs a start sequence
    // for the columns it brings, and a product costs the same for one
    // running column as for all, so admitting in batches gives fuller steps
    // at the price of latency.
    bool group_boundary(Group& g, int n_waiting, Clock::time_point oldest, std::vector<int>& state,
                        std::vector<giamg_info>& infos) {
        bool progress = false;
        const int64_t n = problems[g.problem].n_nodes;
        hipStream_t st = session_stream(g.S);
        if (g.inflight) {   // the step completed: read the column states it copied out
            g.inflight = false;
            state.assign(o.slots, 0);
            infos.assign(o.slots, giamg_info{});
            session_states(g.S, state.data(), infos.data());
            for (int sl = 0; sl < o.slots; ++sl) {
                if (g.running[sl] && !state[sl]) g.info[sl] = infos[sl];
                g.running[sl] = g.running[sl] && state[sl];
            }
            progress = true;
        }
        // finished columns drain (one drain in flight per group)
        if (g.draining.empty()) {
            for (int sl = 0; sl < o.slots; ++sl) {
                if (g.slot_req[sl] < 0 || g.running[sl]) continue;
                double* dev = g.stage.get() + (size_t)sl * n;
                session_retire_async(g.S, sl, dev);
                GIAMG_HIP(hipMemcpyAsync(g.pin_out + (size_t)sl * n, dev, n * sizeof(double),
                                         hipMemcpyDeviceToHost, st));
                g.draining.emplace_back(sl, g.slot_req[sl]);
                g.slot_req[sl] = -1;
            }
            if (!g.draining.empty()) {
                GIAMG_HIP(hipEventRecord(g.drained, st));
                progress = true;
            }
        }
        // admissions into the free slots
        const int room = (int)std::count(g.slot_req.begin(), g.slot_req.end(), (int64_t)-1);
        const bool admit =
            room > 0 && n_waiting > 0 &&
            (o.hold_ms <= 0 || n_waiting >= room ||
             std::chrono::duration<double, std::milli>(Clock::now() - oldest).count() >=
                 (g.solve_ms > 0.0 ? std::min<double>(o.hold_ms, g.solve_ms) : (double)o.hold_ms));
        std::vector<Request*> adm;
        if (admit) {
            std::lock_guard<std::mutex> lk(mu);
            adm = take_pending(g.problem, room);
        }
        if (!adm.empty()) {
            std::vector<int> slots;
            std::vector<const double*> ptrs;
            for (Request* rp : adm) {
                const int sl =
                    (int)(std::find(g.slot_req.begin(), g.slot_req.end(), (int64_t)-1) - g.slot_req.begin());
                g.slot_req[sl] = rp->id;
                g.running[sl] = 1;
                rp->admitted = Clock::now();
                double* dst = g.stage.get() + (size_t)sl * n;
                double* src = g.pin_in + (size_t)sl * n;
                std::memcpy(src, rp->b.data(), n * sizeof(double));
                GIAMG_HIP(hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyHostToDevice, st));
                slots.push_back(sl);
                ptrs.push_back(dst);
            }
            session_admit(g.S, slots.data(), ptrs.data(), (int)slots.size());
            progress = true;
        }
        // the next chunk for the running columns
        if (std::any_of(g.running.begin(), g.running.end(), [](char v) { return v != 0; })) {
            session_step(g.S, o.chunk);
            g.inflight = true;
            progress = true;
        }
        if (progress) g.last_used = Clock::now();
        return progress;
    }

    void loop_main() {
        GIAMG_HIP(hipSetDevice(device));
        std::vector<int> state;
        std::vector<giamg_info> infos;
        while (true) {
            bool progress = false;
            std::map<int, std::vector<Request*>> wanted;   // groups with requests waiting
            {
                std::unique_lock<std::mutex> lk(mu);
                if (stop) break;
                if (worker_dead) throw Error(worker_dead, worker_msg);
                // finished setups become resident groups
                while (!setup_done.empty()) {
                    std::unique_ptr<Group> g = std::move(setup_done.back());
                    setup_done.pop_back();
                    Problem& P = problems[g->problem];
                    reserved -= P.reserved;
                    P.reserved = 0;
                    P.known_bytes = g->bytes;
                    resident += g->bytes;
                    st.peak_bytes = std::max(st.peak_bytes, resident);
                    P.setting_up = false;
                    size_t slot = 0;
                    while (slot < groups.size() && groups[slot]) ++slot;
                    if (slot == groups.size()) groups.emplace_back();
                    P.group = (int)slot;
                    g->last_used = Clock::now();
                    groups[slot] = std::move(g);
                    st.setups += 1;
                    progress = true;
                }
                // requests of failed problems end; problems without a
                // resident hierarchy are set up when the budget allows
                for (auto it = pending.begin(); it != pending.end();) {
                    Request& r = requests[*it];
                    Problem& P = problems[r.problem];
                    if (P.failed) {
                        r.msg = P.fail_msg;
                        finish(r, P.failed);
                        it = pending.erase(it);
                        progress = true;
                        continue;
                    }
                    if (!r.counted) {
                        r.counted = true;
                        if (P.group >= 0) st.cache_hits += 1;
                    }
                    if (P.group >= 0) {
                        wanted[P.group].push_back(&r);
                    } else if (!P.setting_up) {
                        const int64_t est = need(P);
                        if (make_room(est, wanted)) {
                            P.setting_up = true;
                            P.reserved = est;
                            reserved += est;
                            setup_jobs.push_back(r.problem);
                            cv_setup.notify_one();
                            progress = true;
                        }
                    }
                    ++it;
                }
            }
            for (size_t gi = 0; gi < groups.size(); ++gi) {
                if (!groups[gi]) continue;
                Group& g = *groups[gi];
                // drains that reached the host: their requests complete
                if (!g.draining.empty()) {
                    const hipError_t e = hipEventQuery(g.drained);
                    if (e != hipSuccess && e != hipErrorNotReady) GIAMG_HIP(e);
                    if (e == hipSuccess) {
                        const int64_t n = problems[g.problem].n_nodes;
                        std::lock_guard<std::mutex> lk(mu);
                        for (const auto& d : g.draining) {
                            Request& r = requests[d.second];
                            std::memcpy(r.x, g.pin_out + (size_t)d.first * n, n * sizeof(double));
                            r.info = g.info[d.first];
                            finish(r, g.info[d.first].status);
                            g.solve_ms = std::chrono::duration<double, std::milli>(r.done - r.admitted).count();
                        }
                        g.draining.clear();
                        g.last_used = Clock::now();
                        progress = true;
                    }
                }
                if (g.inflight && !session_ready(g.S)) continue;
                const auto w = wanted.find((int)gi);
                const int n_waiting = w == wanted.end() ? 0 : (int)w->second.size();
                const Clock::time_point oldest = n_waiting ? w->second.front()->submit : Clock::now();
                if (group_boundary(g, n_waiting, oldest, state, infos)) progress = true;
            }
            if (!progress) {
                std::unique_lock<std::mutex> lk3(mu);
                if (stop) break;
                cv_work.wait_for(lk3, std::chrono::microseconds(100));
            }
        }
    }
};

}  // namespace giamg

struct giamg_server_s {
    giamg::Server srv;
};

namespace giamg {
std::string& last_error();
}

namespace {
template <typename F>
int sguard(F&& f) {
    try {
        giamg::last_error().clear();
        return f();
    } catch (const giamg::Error& e) {
        giamg::last_error() = e.what();
        return e.code;
    } catch (const std::exception& e) {
        giamg::last_error() = e.what();
        return GIAMG_EINVAL;
    }
}
}  // namespace

extern "C" {

int giamg_server_create(const giamg_server_opts* o, giamg_server* out) {
    return sguard([&]() -> int {
        GIAMG_REQUIRE(o && out, "null argument");
        GIAMG_REQUIRE(o->hbm_budget > 0 && o->slots >= 1 && o->slots <= 1024 && o->chunk >= 1 &&
                          o->tol >= 0.0 && o->hold_ms >= 0 && o->hold_ms <= 60000,
                      "bad server options");
        std::unique_ptr<giamg_server_s> own(new giamg_server_s());
        giamg_server_s* s = own.get();
        s->srv.o = *o;
        GIAMG_HIP(hipGetDevice(&s->srv.device));
        s->srv.loop = std::thread([s] {
            try {
                s->srv.loop_main();
            } catch (const giamg::Error& e) {
                s->srv.fail_all(e.code, e.what());
            } catch (const std::exception& e) {
                s->srv.fail_all(GIAMG_EHIP, e.what());
            }
        });
        try {
            s->srv.setup = std::thread([s] {
                try {
                    s->srv.setup_main();
                } catch (const giamg::Error& e) {
                    s->srv.worker_died(e.code, e.what());
                } catch (const std::exception& e) {
                    s->srv.worker_died(GIAMG_EHIP, e.what());
                }
            });
        } catch (...) {   // no setup worker: stop the loop before the server goes
            {
                std::lock_guard<std::mutex> lk(s->srv.mu);
                s->srv.stop = true;
            }
            s->srv.cv_work.notify_all();
            s->srv.loop.join();
            throw;
        }
        *out = own.release();
        return GIAMG_OK;
    });
}

int giamg_server_add_problem(giamg_server s, const double* coords, int64_t n_nodes, const int32_t* l2g,
                             int64_t n_elem, int32_t p, double lambda, const giamg_opts* opts,
                             int32_t* problem) {
    return sguard([&]() -> int {
        GIAMG_REQUIRE(s && problem, "null argument");
        giamg::Problem P;
        giamg_default_opts(&P.opts);
        if (opts) P.opts = *opts;
        giamg::check_setup_args(coords, n_nodes, l2g, n_elem, p, lambda, P.opts);
        const int64_t nl = (int64_t)(p + 1) * (p + 1) * (p + 1);
        P.coords.assign(coords, coords + n_nodes * 3);
        P.l2g.assign(l2g, l2g + n_elem * nl);
        P.n_nodes = n_nodes;
        P.n_elem = n_elem;
        P.p = p;
        P.lambda = lambda;
        std::lock_guard<std::mutex> lk(s->srv.mu);
        s->srv.problems.push_back(std::move(P));
        *problem = (int32_t)s->srv.problems.size() - 1;
        return GIAMG_OK;
    });
}

int giamg_server_submit(giamg_server s, int32_t problem, const double* b, double* x, int64_t* request) {
    return sguard([&]() -> int {
        GIAMG_REQUIRE(s && b && x && request, "null argument");
        std::lock_guard<std::mutex> lk(s->srv.mu);
        if (s->srv.dead) throw giamg::Error(s->srv.dead, s->srv.dead_msg);
        GIAMG_REQUIRE(problem >= 0 && problem < (int)s->srv.problems.size(), "unknown problem");
        const int64_t n = s->srv.problems[problem].n_nodes;
        giamg::Request r;
        r.id = s->srv.next_id++;
        r.problem = problem;
        r.b.assign(b, b + n);
        r.x = x;
        r.submit = giamg::Clock::now();
        s->srv.requests[r.id] = std::move(r);
        s->srv.pending.push_back(s->srv.next_id - 1);
        s->srv.st.submitted += 1;
        *request = s->srv.next_id - 1;
        s->srv.cv_work.notify_all();
        return GIAMG_OK;
    });
}

int giamg_server_wait(giamg_server s, int64_t request, giamg_info* info, double* latency_ms) {
    return sguard([&]() -> int {
        GIAMG_REQUIRE(s, "null server");
        std::unique_lock<std::mutex> lk(s->srv.mu);
        auto it = s->srv.requests.find(request);
        GIAMG_REQUIRE(it != s->srv.requests.end(), "unknown request");
        s->srv.cv_done.wait(lk, [&] { return it->second.finished || s->srv.stop; });
        giamg::Request& r = it->second;
        if (!r.finished) throw giamg::Error(GIAMG_EINVAL, "server stopped before the request finished");
        if (info) *info = r.info;
        if (latency_ms)
            *latency_ms = std::chrono::duration<double, std::milli>(r.done - r.submit).count();
        const int status = r.info.status;
        if (status < 0) giamg::last_error() = r.msg;
        s->srv.requests.erase(it);
        return status;
    });
}

int giamg_server_stats(giamg_server s, giamg_server_statistics* out) {
    return sguard([&]() -> int {
        GIAMG_REQUIRE(s && out, "null argument");
        std::lock_guard<std::mutex> lk(s->srv.mu);
        *out = s->srv.st;
        out->resident_bytes = s->srv.resident;
        int g = 0;
        for (auto& p : s->srv.groups) g += p ? 1 : 0;
        out->groups_resident = g;
        return GIAMG_OK;
    });
}

void giamg_server_free(giamg_server s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->srv.mu);
        s->srv.stop = true;
    }
    s->srv.cv_work.notify_all();
    s->srv.cv_setup.notify_all();
    s->srv.cv_done.notify_all();
    if (s->srv.loop.joinable()) s->srv.loop.join();
    if (s->srv.setup.joinable()) s->srv.setup.join();
    (void)hipSetDevice(s->srv.device);
    delete s;   // groups synchronise their own streams before freeing
}

}  // extern "C"
