// Continuous batching of many Newton-Krylov solves on one GPU.
//
// A worker thread owns one stream.  Requests wait in a FIFO queue and are
// admitted while the number of active solves is below max_slots and their
// device footprint (task vectors, state, preconditioner) fits the HBM budget.
// Every step advances all active solves together: each solve enqueues the
// work that produces its next residual request, the requests of all solves
// are evaluated by shared all-pairs launches (shipwave_residual_batched), each
// solve enqueues the work that consumes its result, the stream is synchronised
// once, and each solve's host logic runs.  Finished solves retire (their slot
// and memory are released) and waiting requests are admitted between steps,
// so requests that arrive while others run join the running batch.
//
// A solve's arithmetic does not depend on which other solves share its
// launches (the batched residual is bitwise equal to a lone one and every
// other kernel works on one solve's vectors), so a request gives the same
// result alone and in any mix.  Preconditioners are cached per (mesh, domain,
// F rounded to 0.025, q); the rounding changes only how fast GMRES converges.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <vector>

#include "solve_task.hpp"

namespace sw {

// Preconditioner half-bandwidth chosen by mesh when the caller leaves it to the server:
// the wider band pays for its set-up on the larger meshes (measured on the serving mix).
int mesh_q(const Geo& g) { return g.N <= 200 ? 5 : 8; }

namespace {

double clock_s(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// F bucket of the cached preconditioners.  On the serving mix (F uniform in [0.5, 1]),
// 0.025 gave the lowest latency: 0.05 cost 1.8 more GMRES iterations per solve and
// 30% on p99, 0.1 cost 25% of the throughput, and 0.0125 or exact F spent more on
// set-ups than they saved.
constexpr double kFBucket = 0.025;

}  // namespace
}  // namespace sw

using namespace sw;

struct sw_server {
    sw_server_opts opts{};
    int device = -1;
    hipStream_t stream = nullptr;
    std::chrono::steady_clock::time_point t0;
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    uint64_t next_ticket = 1;
    size_t outstanding = 0;

    struct Pending {
        uint64_t ticket;
        sw_request req;
        double t_submit;
    };
    std::deque<Pending> queue;
    struct Finished {
        sw_result res;
        std::vector<double> zeta;
    };
    std::map<uint64_t, Finished> done;

    // worker-owned
    struct Active {
        uint64_t ticket = 0;
        sw_request req{};
        Geo g{};
        SolveParams prm;
        void* mem = nullptr;
        size_t bytes = 0;
        double* u = nullptr;
        double* zeta = nullptr;
        double* pin = nullptr;
        size_t npin = 0;
        const sw_precond* P = nullptr;
        std::unique_ptr<SolveTask> task;
        double t_submit = 0, t_admit = 0;
        int used_fallback = 0;
        int evals = 0, newton = 0, gmres = 0;
    };
    std::vector<std::unique_ptr<Active>> active;
    size_t hbm_used = 0;
    struct CachedP {
        sw_precond* P;
        size_t bytes;
        int users;
        uint64_t last_use;
    };
    std::map<std::tuple<int, int, double, double, double, long, int>, CachedP> pcache;
    uint64_t use_clock = 0;

    void run();
    bool admit_one(std::unique_lock<std::mutex>& lk);
    void start_task(Active& a, int precision);
    void retire(Active& a, int status);
    const sw_precond* get_precond(const Geo& g, size_t& charged);
    void release_precond(const Geo& g);
    int q_of(const Geo& g) const { return opts.q_blocks >= 0 ? opts.q_blocks : mesh_q(g); }
    std::tuple<int, int, double, double, double, long, int> pkey(const Geo& g) const {
        return std::make_tuple(g.N, g.M, g.x1, g.xN, g.yM, std::lround(g.F / kFBucket), q_of(g));
    }
};

const sw_precond* sw_server::get_precond(const Geo& g, size_t& charged) {
    auto key = pkey(g);
    auto it = pcache.find(key);
    if (it != pcache.end()) {
        it->second.users++;
        it->second.last_use = ++use_clock;
        charged = 0;
        return it->second.P;
    }
    Geo gr = g;
    gr.F = std::lround(g.F / kFBucket) * kFBucket;
    sw_precond* P = precond_build(gr, q_of(g), stream);
    charged = precond_bytes(P);
    pcache[key] = CachedP{P, charged, 1, ++use_clock};
    return P;
}

void sw_server::release_precond(const Geo& g) {
    auto it = pcache.find(pkey(g));
    if (it != pcache.end() && it->second.users > 0) it->second.users--;
}

void sw_server::start_task(Active& a, int precision) {
    a.prm = SolveParams{};
    a.prm.tol = opts.tol;
    a.prm.precision = precision;
    a.prm.init_flat = true;
    Carve c(a.mem);
    a.u = c.take<double>(2 * (size_t)a.g.NM);
    a.zeta = c.take<double>((size_t)a.g.NM);
    void* tmem = c.p + ((c.off + 255) & ~size_t(255));
    a.task.reset(new SolveTask(a.g, a.prm, a.P, a.u, tmem, a.pin));
    a.task->deferred = true;
}

namespace {
Geo request_geo(const sw_request& req) {
    sw_problem p{};
    p.mesh = req.mesh;
    p.domain = req.domain;
    p.params.F = req.F;
    p.params.eps = req.eps;
    p.params.nu = 0.05;
    p.params.precision = SW_PREC_FP64;
    const Geo g = make_geo(p);
    SW_REQUIRE(g.N <= kMaxN, "a request needs a preconditioner, which needs N <= 1024");
    return g;
}

// device bytes of one admitted request, besides its preconditioner: its solve state, its
// share of the stream's batched-residual scratch (the FP32 layout, the larger one) and
// its spline operator (kept per M by the residual)
size_t task_bytes_of(const Geo& g) {
    const int m = SolveParams{}.m;
    Geo g32 = g;
    g32.precision = SW_PREC_FP32;
    return carve_size({2 * (size_t)g.NM * 8, (size_t)g.NM * 8}) + SolveTask::device_bytes(g, m) +
           256 + residual_scratch_bytes(g32, choose_chunks(g32)) + (size_t)g.M * g.M * 8;
}
}  // namespace

bool sw_server::admit_one(std::unique_lock<std::mutex>& lk) {
    if (queue.empty() || (int)active.size() >= opts.max_slots) return false;
    Pending pd = queue.front();
    Geo g;
    try {
        g = request_geo(pd.req);
    } catch (const Error& e) {
        queue.pop_front();
        Finished f{};
        f.res.status = e.code;
        f.res.t_submit_s = pd.t_submit;
        f.res.t_admit_s = f.res.t_done_s = clock_s(t0);
        done[pd.ticket] = std::move(f);
        outstanding--;
        cv_done.notify_all();
        return true;
    }
    const size_t task_bytes = task_bytes_of(g);
    const bool cached = pcache.count(pkey(g)) > 0;
    const size_t p_bytes = cached ? 0 : precond_bytes_estimate(g, q_of(g));
    const double budget = opts.hbm_budget_bytes;
    if ((double)(task_bytes + p_bytes) > budget) {
        queue.pop_front();
        Finished f{};
        f.res.status = SW_ENOMEM;
        f.res.t_submit_s = pd.t_submit;
        f.res.t_admit_s = f.res.t_done_s = clock_s(t0);
        done[pd.ticket] = std::move(f);
        outstanding--;
        cv_done.notify_all();
        return true;
    }
    if ((double)(hbm_used + task_bytes + p_bytes) > budget) {
        // evict unused cached preconditioners, least recently used first
        while ((double)(hbm_used + task_bytes + p_bytes) > budget) {
            auto victim = pcache.end();
            for (auto it = pcache.begin(); it != pcache.end(); ++it)
                if (it->second.users == 0 &&
                    (victim == pcache.end() || it->second.last_use < victim->second.last_use))
                    victim = it;
            if (victim == pcache.end()) return false;  // wait for running solves to finish
            hbm_used -= victim->second.bytes;
            precond_destroy(victim->second.P, false);  // freed: the budget counts it gone
            pcache.erase(victim);
        }
    }
    queue.pop_front();
    lk.unlock();
    auto a = std::make_unique<Active>();
    a->ticket = pd.ticket;
    a->req = pd.req;
    a->g = g;
    a->t_submit = pd.t_submit;
    a->t_admit = clock_s(t0);
    a->bytes = task_bytes;
    try {
        size_t charged = 0;
        a->P = get_precond(g, charged);
        hbm_used += charged;
        if (hipMalloc(&a->mem, task_bytes) != hipSuccess) {
            (void)hipGetLastError();
            release_precond(g);
            throw Error{SW_ENOMEM, "server: task allocation failed"};
        }
        hbm_used += task_bytes;
        a->npin = SolveTask::pinned_doubles(SolveParams{}.m);
        a->pin = pinned_get(a->npin);
        start_task(*a, opts.precision);
    } catch (const Error& e) {
        lk.lock();
        if (a->mem) {
            (void)hipFree(a->mem);
            hbm_used -= task_bytes;
        }
        Finished f{};
        f.res.status = e.code;
        f.res.t_submit_s = a->t_submit;
        f.res.t_admit_s = a->t_admit;
        f.res.t_done_s = clock_s(t0);
        done[pd.ticket] = std::move(f);
        outstanding--;
        cv_done.notify_all();
        return true;
    }
    lk.lock();
    active.push_back(std::move(a));
    return true;
}

void sw_server::retire(Active& a, int status) {
    Finished f{};
    f.res.status = status;
    f.res.newton_iters = a.newton;
    f.res.gmres_iters = a.gmres;
    f.res.residual_evals = a.evals;
    f.res.used_fallback = a.used_fallback;
    f.res.final_norm = a.task ? a.task->final_norm : 0.0;
    f.res.fp32_error = a.task ? a.task->fp32_error : -1.0;
    f.res.t_submit_s = a.t_submit;
    f.res.t_admit_s = a.t_admit;
    f.zeta.assign((size_t)a.g.NM, 0.0);
    if (a.task) {
        zeta_enqueue(a.g, a.u, a.zeta, stream);
        SW_HIP(hipMemcpyAsync(f.zeta.data(), a.zeta, (size_t)a.g.NM * sizeof(double),
                              hipMemcpyDeviceToHost, stream));
        SW_HIP(hipStreamSynchronize(stream));
    }
    (void)hipFree(a.mem);
    pinned_put(a.pin, a.npin);
    release_precond(a.g);
    std::lock_guard<std::mutex> lk(mu);
    hbm_used -= a.bytes;
    f.res.t_done_s = clock_s(t0);
    done[a.ticket] = std::move(f);
    outstanding--;
    cv_done.notify_all();
}

void sw_server::run() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
        while (admit_one(lk)) {
        }
        if (active.empty()) {
            if (stop && queue.empty()) break;
            cv_work.wait(lk, [&] { return stop || !queue.empty(); });
            continue;
        }
        lk.unlock();
        try {
            std::vector<Geo> geos;
            std::vector<const double*> xs;
            std::vector<double*> Es;
            // Krylov steps stop at their preconditioner applies, which run together
            std::vector<const sw_precond*> aP;
            std::vector<const double*> ab;
            std::vector<double*> ax;
            std::vector<ScaleArgs> scales;
            for (auto& a : active) {
                SolveTask& t = *a->task;
                t.pre(stream);
                if (t.scale_pending) {
                    scales.push_back(t.scale_req);
                    t.scale_pending = false;
                }
                if (t.apply_pending) {
                    aP.push_back(t.apply_P);
                    ab.push_back(t.apply_b);
                    ax.push_back(t.apply_x);
                }
            }
            if (!scales.empty()) scale_copy_batched((int)scales.size(), scales.data(), stream);
            if (!aP.empty())
                precond_apply_batched((int)aP.size(), aP.data(), ab.data(), ax.data(), stream);
            std::vector<ShiftArgs> shifts;
            for (auto& a : active) {
                SolveTask& t = *a->task;
                if (t.apply_pending) t.pre_rest(stream);
                if (t.shift_pending) {
                    shifts.push_back(t.shift_req);
                    t.shift_pending = false;
                }
                if (t.done()) continue;
                geos.push_back(*t.req_g);
                xs.push_back(t.req_x);
                Es.push_back(t.req_E);
            }
            if (!shifts.empty()) shift_auto_batched((int)shifts.size(), shifts.data(), stream);
            if (!geos.empty())
                residual_batched_enqueue((int)geos.size(), geos.data(), xs.data(), Es.data(),
                                         stream);
            // Krylov steps leave their Gram-Schmidt passes, which run together
            std::vector<Cgs2Args> cgs;
            for (auto& a : active) {
                SolveTask& t = *a->task;
                if (t.done()) continue;
                t.post(stream);
                if (t.cgs_pending) cgs.push_back(t.cgs_req);
            }
            if (!cgs.empty()) cgs2_norm_batched((int)cgs.size(), cgs.data(), stream);
            for (auto& a : active)
                if (a->task->cgs_pending) a->task->post_tail(stream);
            SW_HIP(hipStreamSynchronize(stream));
            for (auto& a : active) a->task->host(stream);
            std::vector<std::unique_ptr<Active>> keep;
            for (auto& a : active) {
                SolveTask& t = *a->task;
                if (!t.done()) {
                    keep.push_back(std::move(a));
                    continue;
                }
                a->evals += t.evals;
                a->newton += t.newton;
                a->gmres += t.gmres_total;
                if (t.status != SW_OK && a->prm.precision == SW_PREC_FP32 && opts.fallback_fp64) {
                    a->used_fallback = 1;
                    start_task(*a, SW_PREC_FP64);
                    keep.push_back(std::move(a));
                    continue;
                }
                retire(*a, t.status);
            }
            active.swap(keep);
        } catch (const Error& e) {
            set_error(e.msg);
            (void)hipStreamSynchronize(stream);
            for (auto& a : active) {
                try {
                    retire(*a, e.code);
                } catch (...) {
                }
            }
            active.clear();
        } catch (...) {
            (void)hipStreamSynchronize(stream);
            for (auto& a : active) {
                try {
                    retire(*a, SW_EHIP);
                } catch (...) {
                }
            }
            active.clear();
        }
        lk.lock();
    }
}

extern "C" {

int32_t shipwave_server_create(const sw_server_opts* opts, sw_server** out) {
    return guard([&]() -> int32_t {
        SW_REQUIRE(opts && out, "null pointer");
        SW_REQUIRE(opts->max_slots >= 1, "max_slots must be >= 1");
        SW_REQUIRE(opts->hbm_budget_bytes > 0.0, "hbm_budget_bytes must be > 0");
        SW_REQUIRE(opts->precision == SW_PREC_FP64 || opts->precision == SW_PREC_FP32,
                   "precision must be 0 or 1");
        auto* s = new sw_server();
        s->opts = *opts;
        if (!(s->opts.tol > 0.0)) s->opts.tol = 1e-10;
        s->t0 = std::chrono::steady_clock::now();
        if (hipGetDevice(&s->device) != hipSuccess ||
            hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
            delete s;
            throw Error{SW_EHIP, "server: stream creation failed"};
        }
        s->worker = std::thread([s] { s->run(); });
        *out = s;
        return SW_OK;
    });
}

int32_t shipwave_server_request_bytes(const sw_server_opts* opts, const sw_request* req,
                                      uint64_t* bytes) {
    return guard([&]() -> int32_t {
        SW_REQUIRE(opts && req && bytes, "null pointer");
        const Geo g = request_geo(*req);
        const int q = opts->q_blocks >= 0 ? opts->q_blocks : mesh_q(g);
        *bytes = (uint64_t)(task_bytes_of(g) + precond_bytes_estimate(g, q));
        return SW_OK;
    });
}

int32_t shipwave_server_submit(sw_server* s, const sw_request* req, uint64_t* ticket) {
    return guard([&]() -> int32_t {
        SW_REQUIRE(s && req && ticket, "null pointer");
        std::lock_guard<std::mutex> lk(s->mu);
        SW_REQUIRE(!s->stop, "server is stopping");
        const uint64_t t = s->next_ticket++;
        s->queue.push_back(sw_server::Pending{t, *req, clock_s(s->t0)});
        s->outstanding++;
        *ticket = t;
        s->cv_work.notify_all();
        return SW_OK;
    });
}

int32_t shipwave_server_poll(sw_server* s, uint64_t ticket, sw_result* res, double* zeta_host) {
    return guard([&]() -> int32_t {
        SW_REQUIRE(s && res, "null pointer");
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->done.find(ticket);
        if (it == s->done.end()) {
            SW_REQUIRE(ticket > 0 && ticket < s->next_ticket, "unknown ticket");
            return SW_EBUSY;
        }
        *res = it->second.res;
        if (zeta_host)
            std::copy(it->second.zeta.begin(), it->second.zeta.end(), zeta_host);
        s->done.erase(it);
        return SW_OK;
    });
}

int32_t shipwave_server_drain(sw_server* s) {
    return guard([&]() -> int32_t {
        SW_REQUIRE(s, "null pointer");
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv_done.wait(lk, [&] { return s->outstanding == 0; });
        return SW_OK;
    });
}

void shipwave_server_destroy(sw_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    (void)hipSetDevice(s->device);
    for (auto& kv : s->pcache) precond_destroy(kv.second.P);
    (void)hipStreamDestroy(s->stream);
    delete s;
}

}  // extern "C"
