// Serving loop: continuous batching of solve requests (include/fm.h, fm_server_*).
//
// A dispatcher thread admits submitted requests by device-memory footprint and
// routes each to a lane: one lane per (problem description, precision,
// restart length), each with its own HIP stream, its own Krylov workspace
// (a Batch with one slot per request of that shape waiting when the lane is
// made, at least 2 and at most max_batch) and its own host thread, so the
// lanes' kernels overlap on the device.  An idle lane keeps its workspace
// until a new lane needs the memory; then the longest idle lanes give it back,
// as many as needed.  Problems (the energy-independent factors) are cached by
// description.  A request joins its lane at the lane's next restart
// boundary; a lane with waiting requests and free slots ends its cycle early
// (after at least a minimum number of Arnoldi steps) so that they can join.
// Finished requests leave their slot, their solution is copied to the caller's
// host buffer, and a result is queued for fm_poll.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>

#include "batch.h"

namespace fm {

namespace {

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// Problems are cached by every field of the description except the device.
std::string desc_key(const fm_problem_desc &d) {
    std::string k;
    auto put = [&k](const void *v, size_t n) { k.append(static_cast<const char *>(v), n); };
    put(d.mass, sizeof d.mass);
    put(d.charge, sizeof d.charge);
    put(&d.J, sizeof d.J);
    put(&d.tau, sizeof d.tau);
    for (const fm_dim *dims : {d.x, d.y, d.z})
        for (int a = 0; a < 3; ++a) {
            put(&dims[a].degree, sizeof(int));
            put(&dims[a].n, sizeof(int));
            put(&dims[a].R, sizeof(double));
            put(&dims[a].map, sizeof(int));
        }
    put(&d.x0, sizeof d.x0);
    put(&d.y0, sizeof d.y0);
    put(&d.nu, sizeof d.nu);
    put(&d.vhat, sizeof d.vhat);
    const int pv = d.precond == FM_PREC_COUPLED ? 2 : 1;
    put(&pv, sizeof pv);
    put(&d.exchange, sizeof d.exchange);
    put(&d.zhalf, sizeof d.zhalf);
    const double tol = d.precond == FM_PREC_COUPLED ? (d.mode_fit_tol > 0 ? d.mode_fit_tol : FM_DEFAULT_MODE_FIT_TOL) : 0.0;
    put(&tol, sizeof tol);
    return k;
}

long long unknowns_of(const fm_problem_desc &d) {
    int M0 = (1 - d.tau) / 2;
    long long nM = d.J - M0 + 1, s = 0;
    for (int a = 0; a < 3; ++a)
        if (!(d.exchange != 0 && (a == 1 || (d.exchange == 3 && a == 2)))) {
            long long nz = d.z[a].n;
            if (a == 2 && d.zhalf) {     // component 3 on z in [0, 1] (fm_problem_desc.zhalf)
                const int sigma = d.exchange * ((M0 & 1) ? -1 : 1);
                nz = d.z[a].degree == 3 ? d.z[a].n / 2 : 3 * (d.z[a].n / 3 - 1) / 2 + (sigma == 1 ? 2 : 1);
            }
            s += (long long)d.x[a].n * d.y[a].n * nz;
        }
    return nM * s;
}

}  // namespace

struct ServeReq {
    uint64_t tag = 0;
    fm_problem_desc desc{};
    double E = 0;
    std::vector<double> b;
    double *x_host = nullptr;
    fm_solve_opts opts{};
    double t_submit = 0, t_start = 0, t_done = 0;
    int status = FM_OK, iters = 0;
    // restart escalation: steps taken in lanes of shorter restarts, and the
    // true residual at the end of the last full cycle in this lane
    int iters_before = 0;
    double prev_rel = 1.0;
    double rel = 0;
};

struct Lane {
    std::string key;
    fm_problem *prob = nullptr;
    Batch batch;
    double *B = nullptr, *X = nullptr;
    std::vector<ServeReq *> slot;
    std::deque<ServeReq *> joinq;      // guarded by the server mutex
    std::thread th;
    hipStream_t st = nullptr;
    bool finished = false;             // thread has exited
    size_t bytes = 0;
    // guarded by the server mutex: waiting for work since idle_since, and
    // chosen to give its memory back
    bool idle = false, evict = false;
    double idle_since = 0;
};

}  // namespace fm

struct fm_server {
    size_t budget = 0;
    int max_batch = 1;
    int device = 0;
    std::mutex mu;
    std::condition_variable cv;        // dispatcher and lanes wait here
    std::condition_variable done_cv;   // fm_poll waits here
    std::deque<fm::ServeReq *> pending;
    std::deque<fm::ServeReq *> finished;
    std::map<std::string, fm_problem *> cache;
    std::map<std::string, int> setting_up;   // problem keys being built (value unused)
    int setups_running = 0;
    std::vector<std::thread> setup_threads;  // joined when the dispatcher ends
    std::vector<fm::Lane *> lanes;
    size_t in_use = 0;
    long long outstanding = 0;         // submitted and not yet finished
    bool stop = false;
    std::thread dispatcher;
    std::string error;
};

namespace fm {

namespace {

constexpr double STALL_FACTOR = 0.1;   // least residual reduction per full cycle before a restart escalation

void finish(fm_server *S, ServeReq *r) {
    r->t_done = now_s();
    S->finished.push_back(r);
    S->outstanding -= 1;
    S->done_cv.notify_all();
}

void lane_loop(fm_server *S, Lane *L) {
    (void)hipSetDevice(S->device);
    const long long N = L->prob->N;
    const int cap = L->batch.cap;
    for (;;) {
        std::vector<std::pair<int, ServeReq *>> joiners;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            for (;;) {
                for (int s = 0; s < cap && !L->joinq.empty(); ++s)
                    if (!L->slot[s]) {
                        L->slot[s] = L->joinq.front();
                        L->joinq.pop_front();
                        joiners.push_back({s, L->slot[s]});
                    }
                bool busy = L->batch.any_running() || !joiners.empty();
                if (busy) {
                    L->idle = false;
                    break;
                }
                if (S->stop || L->evict) {
                    L->finished = true;
                    S->cv.notify_all();
                    return;
                }
                // idle: keep the workspace for the next request of this shape
                // until the dispatcher picks this lane to make room for another
                if (!L->idle) {
                    L->idle = true;
                    L->idle_since = now_s();
                }
                S->cv.wait_for(lk, std::chrono::milliseconds(50));
            }
        }
        std::vector<int> js;
        for (auto &pr : joiners) {
            ServeReq *r = pr.second;
            r->t_start = now_s();
            (void)hipMemcpyAsync(L->B + (long long)pr.first * N, r->b.data(), sizeof(double) * N,
                                 hipMemcpyHostToDevice, L->st);
            L->batch.E[pr.first] = r->E;
            L->batch.limit[pr.first] = r->opts.max_iters;
            js.push_back(pr.first);
        }
        std::vector<int> was(L->batch.run);
        fm_status st = L->batch.boundary(js, 0);
        std::vector<int> done;
        for (int s = 0; s < cap; ++s)
            if (L->slot[s] && (was[s] || std::find(js.begin(), js.end(), s) != js.end()) &&
                (!L->batch.run[s] || st != FM_OK))
                done.push_back(s);
        if (!done.empty()) {
            std::vector<double> rel, md;
            std::vector<int> fl;
            if (L->batch.read_results(rel, md, fl) != FM_OK) st = FM_E_HIP;
            for (int s : done) {
                ServeReq *r = L->slot[s];
                (void)hipMemcpyAsync(r->x_host, L->X + (long long)s * N, sizeof(double) * N, hipMemcpyDeviceToHost,
                                     L->st);
                (void)hipStreamSynchronize(L->st);
                r->iters = r->iters_before + L->batch.iters[s];
                r->rel = rel.empty() ? 0.0 : rel[s];
                if (st != FM_OK) r->status = st;
                else if (fl[s]) r->status = FM_E_NONFINITE;
                else r->status = r->rel <= r->opts.rtol ? FM_OK : FM_E_NOT_CONVERGED;
                std::lock_guard<std::mutex> lk(S->mu);
                L->slot[s] = nullptr;
                finish(S, r);
            }
        }
        if (st != FM_OK) {
            // a failed device call ends the lane: report every occupant
            std::lock_guard<std::mutex> lk(S->mu);
            for (int s = 0; s < cap; ++s)
                if (L->slot[s]) {
                    L->slot[s]->status = st;
                    finish(S, L->slot[s]);
                    L->slot[s] = nullptr;
                }
            for (auto *r : L->joinq) {
                r->status = st;
                finish(S, r);
            }
            L->joinq.clear();
            std::fill(L->batch.run.begin(), L->batch.run.end(), 0);
            L->finished = true;
            S->error = "lane stopped after a HIP error";
            S->cv.notify_all();
            return;
        }
        if (st == FM_OK) {
            // a request whose true residual fell by less than STALL_FACTOR over a
            // full cycle has stalled at this restart length (GMRES(m) can stagnate
            // high in the continuum): it leaves the lane and is queued again with
            // twice the restart length, from x = 0, with the steps it has left
            std::vector<int> full;
            for (int s = 0; s < cap; ++s)
                if (L->slot[s] && was[s] && L->batch.run[s] && L->batch.last_steps[s] >= L->batch.m) full.push_back(s);
            std::vector<int> up;
            if (!full.empty()) {
                std::vector<double> rel, md;
                std::vector<int> fl;
                if (L->batch.read_results(rel, md, fl) == FM_OK)
                    for (int s : full) {
                        ServeReq *r = L->slot[s];
                        const bool stalled = rel[s] > STALL_FACTOR * r->prev_rel;
                        r->prev_rel = rel[s];
                        fm_problem one;
                        one.N = N;
                        const int m2 = 2 * L->batch.m;
                        if (stalled && m2 <= MAX_RESTART &&
                            Batch::footprint(&one, 1, m2) + 2 * size_t(N) * 8 <= S->budget / 4)
                            up.push_back(s);
                    }
            }
            if (!up.empty() && L->batch.stop(up) == FM_OK) {
                std::lock_guard<std::mutex> lk(S->mu);
                for (int s : up) {
                    ServeReq *r = L->slot[s];
                    const int used = L->batch.iters[s];
                    r->iters_before += used;
                    r->opts.max_iters = std::max(r->opts.max_iters - used, 2 * L->batch.m);
                    r->opts.restart = 2 * L->batch.m;
                    r->prev_rel = 1.0;
                    L->slot[s] = nullptr;
                    S->pending.push_back(r);
                }
                S->cv.notify_all();
            }
        }
        if (L->batch.any_running()) {
            auto want_cut = [S, L, cap]() {
                std::lock_guard<std::mutex> lk(S->mu);
                if (L->joinq.empty()) return false;
                for (int s = 0; s < cap; ++s)
                    if (!L->slot[s]) return true;
                return false;
            };
            if (L->batch.cycle(want_cut, 24) != FM_OK) {
                std::lock_guard<std::mutex> lk(S->mu);
                S->error = "lane cycle failed";
            }
        }
    }
}

void reap_lanes(fm_server *S) {
    // called with the mutex held
    for (size_t i = 0; i < S->lanes.size();) {
        Lane *L = S->lanes[i];
        if (L->finished) {
            if (L->th.joinable()) L->th.join();
            std::lock_guard<std::recursive_mutex> hl(hip_setup_mutex());
            L->batch.release();
            (void)hipFree(L->B);
            (void)hipFree(L->X);
            (void)hipStreamDestroy(L->st);
            S->in_use -= L->bytes;
            delete L;
            S->lanes.erase(S->lanes.begin() + i);
        } else {
            ++i;
        }
    }
}

// Builds a problem off the dispatcher thread; the result goes to the cache (or
// its failure to every pending request of that description).
void setup_problem_async(fm_server *S, std::string pkey, fm_problem_desc d) {
    (void)hipSetDevice(S->device);
    d.device = S->device;
    fm_problem *prob = nullptr;
    fm_status st = fm_create_problem(&d, &prob);
    std::lock_guard<std::mutex> lk(S->mu);
    S->setting_up.erase(pkey);
    S->setups_running -= 1;
    if (st == FM_OK) {
        S->cache[pkey] = prob;
        size_t res = 0;
        fm_problem_info(prob, nullptr, &res, 1, nullptr);
        S->in_use += res;
    } else {
        for (auto it = S->pending.begin(); it != S->pending.end();) {
            if (desc_key((*it)->desc) == pkey) {
                (*it)->status = st;
                finish(S, *it);
                it = S->pending.erase(it);
            } else {
                ++it;
            }
        }
    }
    S->cv.notify_all();
}

constexpr int MAX_SETUPS = 2;          // problem builds in flight (each is multi-threaded)

void dispatch_loop(fm_server *S) {
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        reap_lanes(S);
        if (S->stop && S->pending.empty() && S->setups_running == 0) {
            bool all = true;
            for (auto *L : S->lanes) all &= L->finished;
            if (all) {
                reap_lanes(S);
                std::vector<std::thread> th;
                th.swap(S->setup_threads);
                lk.unlock();
                for (auto &t : th) t.join();
                return;
            }
            S->cv.notify_all();
            S->cv.wait_for(lk, std::chrono::milliseconds(20));
            continue;
        }
        bool progressed = false;
        // first every request whose lane exists, then at most one new lane (its
        // problem set-up can take a while and must not hold up the others)
        for (auto it = S->pending.begin(); it != S->pending.end();) {
            ServeReq *r = *it;
            std::string lkey = desc_key(r->desc) + std::to_string(r->opts.prec) + ":" + std::to_string(r->opts.restart);
            Lane *lane = nullptr;
            for (auto *L : S->lanes)
                if (L->key == lkey && !L->finished) lane = L;
            if (lane) {
                lane->evict = false;       // wanted again
                lane->joinq.push_back(r);
                it = S->pending.erase(it);
                progressed = true;
                S->cv.notify_all();
            } else {
                ++it;
            }
        }
        for (auto it = S->pending.begin(); it != S->pending.end();) {
            ServeReq *r = *it;
            std::string pkey = desc_key(r->desc);
            std::string lkey = pkey + std::to_string(r->opts.prec) + ":" + std::to_string(r->opts.restart);
            bool has_lane = false;
            for (auto *L : S->lanes)
                if (L->key == lkey && !L->finished) has_lane = true;
            if (has_lane) {
                ++it;                      // attached on the next pass
                continue;
            }
            // a new lane: problem (cached, else built off this thread) plus a batch
            {
                fm_problem one;
                one.N = unknowns_of(r->desc);
                if (Batch::footprint(&one, 1, r->opts.restart) + 2 * size_t(one.N) * 8 > S->budget) {
                    r->status = FM_E_REJECTED;
                    it = S->pending.erase(it);
                    finish(S, r);
                    continue;
                }
            }
            auto c = S->cache.find(pkey);
            if (c == S->cache.end()) {
                if (!S->setting_up.count(pkey) && S->setups_running < MAX_SETUPS) {
                    S->setting_up[pkey] = 1;
                    S->setups_running += 1;
                    S->setup_threads.emplace_back(setup_problem_async, S, pkey, r->desc);
                }
                ++it;                      // the lane is made once the problem exists
                continue;
            }
            fm_problem *prob = c->second;
            long long N = unknowns_of(r->desc);
            // slots: max_batch, fewer when one slot's workspace is large (a lane
            // takes at most a quarter of the budget unless one slot needs more)
            fm_problem tmp;
            tmp.N = N;
            const size_t per_slot = Batch::footprint(&tmp, 1, r->opts.restart) + 2 * size_t(N) * 8;
            // as many slots as requests of this shape are waiting (at least 2, so
            // that a request arriving during a solve can join it), capped by
            // max_batch and by memory
            int want = 0;
            for (auto *q : S->pending)
                if (desc_key(q->desc) + std::to_string(q->opts.prec) + ":" + std::to_string(q->opts.restart) == lkey)
                    ++want;
            const int slots = int(std::max<size_t>(
                1, std::min<size_t>({size_t(S->max_batch), size_t(std::max(2, want)), (S->budget / 4) / per_slot})));
            size_t need = Batch::footprint(&tmp, slots, r->opts.restart) + 2 * size_t(N) * 8 * slots;
            if (need > S->budget) {
                r->status = FM_E_REJECTED;
                it = S->pending.erase(it);
                finish(S, r);
                continue;
            }
            if (S->in_use + need > S->budget) {
                // idle lanes give their memory back, the longest idle first,
                // as many as this lane needs
                size_t freeing = 0;
                std::vector<Lane *> idle;
                for (auto *L : S->lanes)
                    if (!L->finished) {
                        if (L->evict) freeing += L->bytes;
                        else if (L->idle && L->joinq.empty()) idle.push_back(L);
                    }
                std::sort(idle.begin(), idle.end(), [](Lane *a, Lane *b) { return a->idle_since < b->idle_since; });
                for (auto *L : idle) {
                    if (S->in_use - std::min(S->in_use, freeing) + need <= S->budget) break;
                    L->evict = true;
                    freeing += L->bytes;
                }
                S->cv.notify_all();
                ++it;
                continue;
            }
            Lane *L = new Lane();
            L->key = lkey;
            L->prob = prob;
            L->slot.assign(slots, nullptr);
            std::unique_lock<std::recursive_mutex> hl(hip_setup_mutex());
            // non-blocking: a lane's stream has no implicit order with the null stream
            bool ok = hipStreamCreateWithFlags(&L->st, hipStreamNonBlocking) == hipSuccess;
            ok = ok && hipMalloc(reinterpret_cast<void **>(&L->B), sizeof(double) * N * slots) == hipSuccess;
            ok = ok && hipMalloc(reinterpret_cast<void **>(&L->X), sizeof(double) * N * slots) == hipSuccess;
            ok = ok && L->batch.create(prob, slots, r->opts.restart, L->st) == FM_OK;
            hl.unlock();
            if (!ok) {
                hl.lock();
                if (L->B) (void)hipFree(L->B);
                if (L->X) (void)hipFree(L->X);
                if (L->st) (void)hipStreamDestroy(L->st);
                L->batch.release();
                delete L;
                r->status = FM_E_NOMEM;
                it = S->pending.erase(it);
                finish(S, r);
                continue;
            }
            L->batch.B = L->B;
            L->batch.X = L->X;
            L->batch.prec = r->opts.prec;
            L->batch.graphs = r->opts.graphs;
            L->batch.rtol = r->opts.rtol;
            L->bytes = L->batch.bytes + 2 * sizeof(double) * N * slots;
            S->in_use += L->bytes;
            L->joinq.push_back(r);
            it = S->pending.erase(it);
            S->lanes.push_back(L);
            L->th = std::thread(lane_loop, S, L);
            progressed = true;
            break;                         // back to the attach pass
        }
        if (!progressed) S->cv.wait_for(lk, std::chrono::milliseconds(5));
    }
}

}  // namespace

}  // namespace fm

using namespace fm;

extern "C" {

fm_status fm_server_create(size_t hbm_budget_bytes, int max_batch, int device, fm_server **out) {
    if (!out || max_batch < 1 || max_batch > 4096 || hbm_budget_bytes == 0) {
        set_error("bad argument");
        return FM_E_INVALID;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        set_error("no such HIP device");
        return FM_E_HIP;
    }
    fm_server *S = new (std::nothrow) fm_server();
    if (!S) {
        set_error("host allocation failed");
        return FM_E_NOMEM;
    }
    S->budget = hbm_budget_bytes;
    S->max_batch = max_batch;
    S->device = device;
    S->dispatcher = std::thread(dispatch_loop, S);
    *out = S;
    return FM_OK;
}

fm_status fm_submit(fm_server *S, const fm_problem_desc *desc, double E, const double *b_host, double *x_host,
                    const fm_solve_opts *opts, uint64_t tag) {
    if (!S || !desc || !b_host || !x_host || !opts || !std::isfinite(E) || opts->restart < 1 || opts->restart > MAX_RESTART ||
        !(opts->rtol > 0) || opts->max_iters < 1 ||
        (opts->prec != FM_FP64 && opts->prec != FM_FP32 && opts->prec != FM_BF16X3)) {
        set_error("bad argument");
        return FM_E_INVALID;
    }
    long long N = unknowns_of(*desc);
    if (N <= 0 || N > (1LL << 31)) {
        set_error("bad problem size");
        return FM_E_INVALID;
    }
    ServeReq *r = new (std::nothrow) ServeReq();
    if (!r) {
        set_error("host allocation failed");
        return FM_E_NOMEM;
    }
    r->tag = tag;
    r->desc = *desc;
    r->E = E;
    r->b.assign(b_host, b_host + N);
    r->x_host = x_host;
    r->opts = *opts;
    r->t_submit = now_s();
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) {
        delete r;
        set_error("server is shutting down");
        return FM_E_INVALID;
    }
    S->pending.push_back(r);
    S->outstanding += 1;
    S->cv.notify_all();
    return FM_OK;
}

fm_status fm_poll(fm_server *S, fm_request_result *results, int max, int *n_done, int block) {
    if (!S || !results || max < 1 || !n_done) {
        set_error("bad argument");
        return FM_E_INVALID;
    }
    std::unique_lock<std::mutex> lk(S->mu);
    if (block)
        S->done_cv.wait(lk, [S] { return !S->finished.empty() || S->outstanding == 0; });
    int n = 0;
    while (n < max && !S->finished.empty()) {
        ServeReq *r = S->finished.front();
        S->finished.pop_front();
        fm_request_result &o = results[n++];
        o.tag = r->tag;
        o.status = r->status;
        o.iters = r->iters;
        o.rel_residual = r->rel;
        o.t_submit = r->t_submit;
        o.t_start = r->t_start;
        o.t_done = r->t_done;
        o.restart = r->opts.restart;
        delete r;
    }
    *n_done = n;
    return FM_OK;
}

fm_status fm_server_stats(fm_server *S, size_t *bytes_in_use, int *lanes, long long *outstanding) {
    if (!S) {
        set_error("null server");
        return FM_E_INVALID;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    if (bytes_in_use) *bytes_in_use = S->in_use;
    if (lanes) *lanes = int(S->lanes.size());
    if (outstanding) *outstanding = S->outstanding;
    return FM_OK;
}

fm_status fm_server_destroy(fm_server *S) {
    if (!S) return FM_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        S->cv.notify_all();
    }
    if (S->dispatcher.joinable()) S->dispatcher.join();
    for (auto &kv : S->cache) fm_destroy_problem(kv.second);
    for (auto *r : S->finished) delete r;
    for (auto *r : S->pending) delete r;
    delete S;
    return FM_OK;
}

}  // extern "C"
