// Jacobian-free Newton-Krylov solve of E(u) = 0 (Jacobian-free Newton-Krylov
// section): damped Newton u <- u + lambda du (eq. newtonstep0) with a
// backtracking line search on ||E||_2; the Newton step J du = -E (eq.
// newtonstep) from restarted right-preconditioned GMRES whose Krylov vectors
// stay on the device and whose Jacobian-vector products are first-order
// difference quotients (eq. JvApprox); inexact-Newton forcing terms
// (Eisenstat-Walker, second choice, gamma = 0.9, alpha = 2).
//
// In mixed precision (inner precision FP32) every JVP uses the FP32-Kahan
// all-pairs sum on both u + h z and its base point u; the Newton residual, the
// line search, the closed-form I and the preconditioner stay FP64.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <map>
#include <mutex>
#include <vector>

#include "solve_task.hpp"

namespace sw {

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

std::mutex g_pin_mu;
std::multimap<size_t, double*> g_pin_free;

std::atomic<int> g_inject_mask{0}, g_inject_nth{0};

__global__ void k_poison(double* E) { E[0] = __builtin_nan(""); }

}  // namespace

void inject_get(int* mask, int* nth) {
    *mask = g_inject_mask.load();
    *nth = g_inject_nth.load();
}

double* pinned_get(size_t doubles) {
    {
        std::lock_guard<std::mutex> lk(g_pin_mu);
        auto it = g_pin_free.lower_bound(doubles);
        if (it != g_pin_free.end() && it->first < 4 * doubles + 64) {
            double* p = it->second;
            g_pin_free.erase(it);
            return p;
        }
    }
    double* p = nullptr;
    SW_HIP(hipHostMalloc(reinterpret_cast<void**>(&p), (doubles + 8) * sizeof(double)));
    p[0] = static_cast<double>(doubles);  // size tag in the first slot
    return p + 8;
}

void pinned_put(double* p, size_t /*doubles*/) {
    if (!p) return;
    const size_t tag = static_cast<size_t>((p - 8)[0]);
    std::lock_guard<std::mutex> lk(g_pin_mu);
    g_pin_free.emplace(tag, p);
}

// ---- device layout of one task ---------------------------------------------------------
// hd (3m + 16 doubles): [0, m+1) first Gram-Schmidt pass, [m+1, 2m+2) second pass,
// [2m+2, 2m+4) norms of the new Krylov vector, [2m+4, 2m+6) norms of u,
// [2m+6, 2m+8) norms of the JVP direction, [2m+8, 2m+10) step h and 1/h,
// [2m+10, 3m+10) GMRES coefficients y, [3m+12, 3m+14) norms of a residual.
size_t SolveTask::device_bytes(const Geo& g, int m) {
    const size_t n = 2 * (size_t)g.NM;
    return carve_size({(size_t)(m + 1) * n * 8, n * 8, n * 8, n * 8, n * 8, n * 8, n * 8, n * 8,
                       n * 8, n * 8, (size_t)(3 * m + 16) * 8,
                       reduce_work_doubles((int)n, m + 1) * 8});
}

size_t SolveTask::pinned_doubles(int m) { return (size_t)(2 * m + 8) + (size_t)(m + 2); }

SolveTask::SolveTask(const Geo& g64, const SolveParams& prm, const sw_precond* P, double* u,
                     void* dev_mem, double* pin)
    : g64_(g64), gin_(g64), prm_(prm), P_(P), u_(u) {
    g64_.precision = SW_PREC_FP64;
    gin_.precision = prm.precision;
    g32_ = g64;
    g32_.precision = SW_PREC_FP32;
    inject_get(&inj_mask_, &inj_nth_);
    n_ = 2 * g64.NM;
    m_ = prm.m;
    const double macheps =
        (prm.precision == SW_PREC_FP32) ? 1.1920928955078125e-07 : 2.220446049250313e-16;
    sqrt_eps_in_ = std::sqrt(macheps);
    sqrt_n_ = std::sqrt((double)n_);
    Carve c(dev_mem);
    const size_t n = n_;
    V_ = c.take<double>((size_t)(m_ + 1) * n);
    E_ = c.take<double>(n);
    Et_ = c.take<double>(n);
    E32_ = c.take<double>(n);
    Ejv_ = c.take<double>(n);
    du_ = c.take<double>(n);
    ut_ = c.take<double>(n);
    xs_ = c.take<double>(n);
    z_ = c.take<double>(n);
    w_ = c.take<double>(n);
    hd_ = c.take<double>(3 * m_ + 16);
    red_ = c.take<double>(reduce_work_doubles(n_, m_ + 1));
    pin_out_ = pin;
    pin_y_ = pin + (2 * m_ + 8);
    H_.assign((size_t)(m_ + 1) * m_, 0.0);
    cs_.assign(m_, 0.0);
    sn_.assign(m_, 0.0);
    gv_.assign(m_ + 1, 0.0);
    y_.assign(m_, 0.0);
}

void SolveTask::pre(hipStream_t s) {
    const int m = m_;
    if (fin_pending_) {
        // the apply of the last cycle's update comes first; pre_rest() continues
        apply_pending = true;
        apply_P = P_;
        apply_b = w_;
        apply_x = z_;
        req_x = nullptr;
        req_E = nullptr;
        req_g = nullptr;
        return;
    }
    switch (ph_) {
        case Phase::E0:
            if (prm_.init_flat) flat_state(g64_.NM, u_, s);
            req_x = u_;
            req_E = E_;
            req_g = &g64_;
            break;
        case Phase::Ein:
            req_x = u_;
            req_E = E32_;
            req_g = &gin_;
            break;
        case Phase::Krylov: {
            double* vj = V_ + (size_t)j_ * n_;
            ScaleArgs sc{0, 0.0, nullptr, nullptr};
            if (j_ == 0)
                sc = restart_mode_ ? ScaleArgs{n_, 1.0 / beta_, w_, V_}
                                   : ScaleArgs{n_, -1.0 / beta_, E_, V_};
            else if (pending_scale_ > 0.0)
                sc = ScaleArgs{n_, 1.0 / pending_scale_, vj, vj};
            if (sc.x && deferred) {
                scale_req = sc;
                scale_pending = true;
            } else if (sc.x) {
                scale_copy(sc.n, sc.a, sc.x, sc.out, s);
            }
            if (deferred) {
                apply_pending = true;
                apply_P = P_;
                apply_b = vj;
                apply_x = z_;
                req_x = nullptr;
                req_E = nullptr;
                req_g = nullptr;
                return;
            }
            precond_apply(P_, vj, z_, s);
            pre_rest(s);
            break;
        }
        case Phase::Restart: {
            const ShiftArgs a{n_, u_, du_, hd_ + 2 * m + 4, sqrt_eps_in_, sqrt_n_,
                              hd_ + 2 * m + 6, hd_ + 2 * m + 8, xs_, red_};
            if (deferred) {
                shift_req = a;
                shift_pending = true;
            } else {
                shift_auto(a.n, a.u, a.z, a.norms_u, a.sqrt_eps, a.sqrt_n, a.norms_z, a.h,
                           a.out, a.work, s);
            }
            req_x = xs_;
            req_E = Ejv_;
            req_g = &gin_;
            break;
        }
        case Phase::Line:
            axpby(n_, 1.0, u_, lam_, du_, ut_, s);
            req_x = ut_;
            req_E = Et_;
            req_g = &g64_;
            break;
        case Phase::Check:
            req_x = u_;
            req_E = E32_;
            req_g = &g32_;
            break;
        case Phase::Done:
            req_x = nullptr;
            req_E = nullptr;
            req_g = nullptr;
            break;
    }
}

// the rest of pre() once its apply z = P^{-1} b is enqueued: after a Krylov step's apply,
// the shifted state; after a cycle-update apply, du (+)= z and then the Line or Restart
// state's pre()
void SolveTask::pre_rest(hipStream_t s) {
    const int m = m_;
    apply_pending = false;
    if (fin_pending_) {
        fin_pending_ = false;
        axpby(n_, 1.0, z_, fin_first_ ? 0.0 : 1.0, fin_first_ ? z_ : du_, du_, s);
        pre(s);  // the Line or Restart state
        return;
    }
    const ShiftArgs a{n_, u_, z_, hd_ + 2 * m + 4, sqrt_eps_in_, sqrt_n_, hd_ + 2 * m + 6,
                      hd_ + 2 * m + 8, xs_, red_};
    if (deferred) {
        shift_req = a;
        shift_pending = true;
    } else {
        shift_auto(a.n, a.u, a.z, a.norms_u, a.sqrt_eps, a.sqrt_n, a.norms_z, a.h, a.out, a.work,
                   s);
    }
    req_x = xs_;
    req_E = Ejv_;
    req_g = &gin_;
}

void SolveTask::maybe_inject(int kind, hipStream_t s) {
    if (!(inj_mask_ & kind) || inj_nth_ <= 0) return;
    const int slot = (kind == kInjectNewton) ? 0 : (kind == kInjectLine) ? 1
                     : (kind == kInjectJvp64) ? 2 : 3;
    if (++inj_count_[slot] == inj_nth_) k_poison<<<1, 1, 0, s>>>(req_E);
}

void SolveTask::post(hipStream_t s) {
    const int m = m_;
    switch (ph_) {
        case Phase::E0:
            maybe_inject(kInjectNewton, s);
            norm_inf_2(n_, req_E, hd_ + 3 * m + 12, red_, s);
            SW_HIP(hipMemcpyAsync(pin_out_, hd_ + 3 * m + 12, 2 * sizeof(double),
                                  hipMemcpyDeviceToHost, s));
            break;
        case Phase::Line:
            maybe_inject(kInjectLine, s);
            norm_inf_2(n_, req_E, hd_ + 3 * m + 12, red_, s);
            SW_HIP(hipMemcpyAsync(pin_out_, hd_ + 3 * m + 12, 2 * sizeof(double),
                                  hipMemcpyDeviceToHost, s));
            break;
        case Phase::Ein:
            break;
        case Phase::Krylov: {
            maybe_inject(gin_.precision == SW_PREC_FP32 ? kInjectJvp32 : kInjectJvp64, s);
            double* vn = V_ + (size_t)(j_ + 1) * n_;
            // vn = J z by the difference quotient, then two Gram-Schmidt passes
            const Cgs2Args a{n_, j_ + 1, V_, (size_t)n_, Ejv_, Ein_, hd_ + 2 * m + 8, vn,
                             hd_, hd_ + (m + 1), hd_ + 2 * m + 2, red_};
            if (deferred) {
                cgs_req = a;
                cgs_pending = true;
                break;
            }
            cgs_pass(n_, a.k, V_, a.ldv, a.Ep, a.Eu, a.h, vn, a.hout1, red_, s);
            cgs_pass(n_, a.k, V_, a.ldv, nullptr, nullptr, nullptr, vn, a.hout2, red_, s);
            norm_inf_2(n_, vn, a.norms, red_, s);
            post_tail(s);
            break;
        }
        case Phase::Restart:
            maybe_inject(gin_.precision == SW_PREC_FP32 ? kInjectJvp32 : kInjectJvp64, s);
            quotient(n_, Ejv_, Ein_, hd_ + 2 * m + 8, w_, s);
            axpby(n_, -1.0, E_, -1.0, w_, w_, s);
            norm_inf_2(n_, w_, hd_ + 3 * m + 12, red_, s);
            SW_HIP(hipMemcpyAsync(pin_out_, hd_ + 3 * m + 12, 2 * sizeof(double),
                                  hipMemcpyDeviceToHost, s));
            break;
        case Phase::Check:
            // E_ holds E64 at the returned u
            axpby(n_, 1.0, E32_, -1.0, E_, w_, s);
            norm_inf_2(n_, w_, hd_ + 3 * m + 12, red_, s);
            SW_HIP(hipMemcpyAsync(pin_out_, hd_ + 3 * m + 12, 2 * sizeof(double),
                                  hipMemcpyDeviceToHost, s));
            break;
        case Phase::Done:
            break;
    }
}

// the copy of a Krylov step's scalars (Gram-Schmidt coefficients and norms) to the host
void SolveTask::post_tail(hipStream_t s) {
    cgs_pending = false;
    SW_HIP(hipMemcpyAsync(pin_out_, hd_, (2 * m_ + 4) * sizeof(double), hipMemcpyDeviceToHost,
                          s));
}

void SolveTask::finish(int st) {
    status = st;
    final_norm = nr_[0];
    // u_ is the returned iterate and E_ = E64(u_) in every case that reaches here with a
    // finite norm (the initial state, an accepted step, or a rejected line search that
    // left u_ and E_ unchanged): one FP32 evaluation at u_ measures the FP32 error there
    ph_ = (std::isfinite(nr_[0]) && std::isfinite(nr_[1])) ? Phase::Check : Phase::Done;
}

void SolveTask::newton_top(hipStream_t s) {
    if (!std::isfinite(nr_[0]) || !std::isfinite(nr_[1])) return finish(SW_ENONFINITE);
    if (nr_[0] <= prm_.tol) return finish(SW_OK);
    if (newton >= prm_.max_newton) return finish(SW_ENOCONV);
    norm_inf_2(n_, u_, hd_ + 2 * m_ + 4, red_, s);
    if (prm_.precision == SW_PREC_FP32)
        ph_ = Phase::Ein;
    else
        start_gmres(s);
}

void SolveTask::start_gmres(hipStream_t) {
    Ein_ = (prm_.precision == SW_PREC_FP32) ? E32_ : E_;
    const double eta_floor = (prm_.precision == SW_PREC_FP32) ? 1e-4 : 0.0;
    const double eta_use =
        std::min(prm_.eta_max, std::max({eta_, eta_floor, 0.5 * prm_.tol / nr_[0]}));
    target_ = eta_use * nr_[1];
    its_ = 0;
    first_cycle_ = true;
    restart_mode_ = false;
    beta_ = nr_[1];
    std::fill(H_.begin(), H_.end(), 0.0);
    std::fill(gv_.begin(), gv_.end(), 0.0);
    gv_[0] = beta_;
    j_ = 0;
    pending_scale_ = 0.0;
    ph_ = Phase::Krylov;
}

void SolveTask::finish_cycle(hipStream_t s, bool converged) {
    const int m = m_;
    const int k = j_ + 1;
    for (int i = k - 1; i >= 0; --i) {
        double t = gv_[i];
        for (int c = i + 1; c < k; ++c) t -= H_[(size_t)i * m + c] * y_[c];
        const double hii = H_[(size_t)i * m + i];
        y_[i] = (hii != 0.0) ? t / hii : 0.0;
    }
    for (int i = 0; i < k; ++i) pin_y_[i] = y_[i];
    SW_HIP(hipMemcpyAsync(hd_ + 2 * m + 10, pin_y_, k * sizeof(double), hipMemcpyHostToDevice, s));
    gemv_acc(n_, k, V_, n_, hd_ + 2 * m + 10, w_, s);
    if (deferred) {
        fin_pending_ = true;
        fin_first_ = first_cycle_;
    } else {
        precond_apply(P_, w_, z_, s);
        if (first_cycle_)
            axpby(n_, 1.0, z_, 0.0, z_, du_, s);
        else
            axpby(n_, 1.0, z_, 1.0, du_, du_, s);
    }
    first_cycle_ = false;
    if (converged || its_ >= prm_.max_gmres) {
        lam_ = 1.0;
        ph_ = Phase::Line;
    } else {
        ph_ = Phase::Restart;
    }
}

void SolveTask::host(hipStream_t s) {
    const int m = m_;
    if (ph_ == Phase::Done) return;
    if (ph_ == Phase::Check) {
        fp32_error = pin_out_[0] / std::max(1.0, nr_[0]);
        if (!std::isfinite(fp32_error)) fp32_error = -1.0;
        ph_ = Phase::Done;
        return;
    }
    ++evals;
    switch (ph_) {
        case Phase::E0:
            nr_[0] = pin_out_[0];
            nr_[1] = pin_out_[1];
            prev2_ = nr_[1];
            eta_ = 0.1;
            newton_top(s);
            break;
        case Phase::Ein:
            start_gmres(s);
            break;
        case Phase::Krylov: {
            const int j = j_;
            double* col = &H_[(size_t)j];  // column j, row stride m
            for (int i = 0; i <= j; ++i) col[(size_t)i * m] = pin_out_[i] + pin_out_[(m + 1) + i];
            const double hn = pin_out_[2 * m + 3];
            if (!std::isfinite(hn)) return finish(SW_ENONFINITE);
            col[(size_t)(j + 1) * m] = hn;
            for (int i = 0; i < j; ++i) {
                const double a = col[(size_t)i * m], b = col[(size_t)(i + 1) * m];
                col[(size_t)i * m] = cs_[i] * a + sn_[i] * b;
                col[(size_t)(i + 1) * m] = -sn_[i] * a + cs_[i] * b;
            }
            const double a = col[(size_t)j * m], b = col[(size_t)(j + 1) * m];
            const double d = std::hypot(a, b);
            cs_[j] = (d > 0.0) ? a / d : 1.0;
            sn_[j] = (d > 0.0) ? b / d : 0.0;
            col[(size_t)j * m] = d;
            col[(size_t)(j + 1) * m] = 0.0;
            gv_[j + 1] = -sn_[j] * gv_[j];
            gv_[j] = cs_[j] * gv_[j];
            ++its_;
            ++gmres_total;
            pending_scale_ = hn;
            const bool conv = std::fabs(gv_[j + 1]) <= target_ || hn == 0.0;
            if (conv || j + 1 == m || its_ >= prm_.max_gmres)
                finish_cycle(s, conv);
            else
                ++j_;
            break;
        }
        case Phase::Restart: {
            beta_ = pin_out_[1];
            if (!(beta_ > target_)) {
                lam_ = 1.0;
                ph_ = Phase::Line;
            } else {
                restart_mode_ = true;
                std::fill(H_.begin(), H_.end(), 0.0);
                std::fill(gv_.begin(), gv_.end(), 0.0);
                gv_[0] = beta_;
                j_ = 0;
                pending_scale_ = 0.0;
                ph_ = Phase::Krylov;
            }
            break;
        }
        case Phase::Line: {
            const double nt0 = pin_out_[0], nt1 = pin_out_[1];
            if (std::isfinite(nt1) && nt1 <= (1.0 - 1e-4 * lam_) * nr_[1]) {
                axpby(n_, 1.0, ut_, 0.0, ut_, u_, s);
                std::swap(E_, Et_);
                ++newton;
                const double ratio = nt1 / prev2_;
                double eta_new = 0.9 * ratio * ratio;
                if (0.9 * eta_ * eta_ > 0.1) eta_new = std::max(eta_new, 0.9 * eta_ * eta_);
                eta_ = std::min(prm_.eta_max, eta_new);
                prev2_ = nt1;
                nr_[0] = nt0;
                nr_[1] = nt1;
                newton_top(s);
            } else {
                lam_ *= 0.5;
                ++backtracks;
                if (lam_ < 1e-4) return finish(SW_ENOCONV);
            }
            break;
        }
        case Phase::Done:
            break;
    }
}

// ---- single solve ------------------------------------------------------------------------
int32_t solve_impl(double F, double eps, const sw_mesh* mesh, const sw_domain* dom,
                   const sw_solve_opts* opts_in, double* u, double* zeta_out, sw_solve_info* info,
                   hipStream_t s) {
    const double t0 = now_s();
    sw_solve_opts o;
    shipwave_solve_opts_default(&o);
    if (opts_in) o = *opts_in;
    SW_REQUIRE(mesh && dom && u, "null pointer");
    SW_REQUIRE(o.tol > 0.0 && std::isfinite(o.tol), "tol must be positive");
    SW_REQUIRE(o.max_newton >= 1 && o.gmres_restart >= 1 && o.max_gmres >= 1,
               "iteration limits must be >= 1");
    SW_REQUIRE(o.gmres_restart <= 200, "gmres_restart must be <= 200");
    SW_REQUIRE(o.init >= 0 && o.init <= 2, "init must be 0, 1 or 2");
    sw_problem p{};
    p.mesh = *mesh;
    p.domain = *dom;
    p.params.F = F;
    p.params.eps = eps;
    p.params.nu = (o.nu > 0.0) ? o.nu : 0.05;
    p.params.weights = o.weights;
    p.params.spline_bc = o.spline_bc;
    p.params.precision = o.precision;
    const Geo g = make_geo(p);  // validates the inner precision too
    SW_REQUIRE(g.N <= kMaxN, "a solve needs a preconditioner, which needs N <= 1024");
    SolveParams prm;
    prm.tol = o.tol;
    prm.max_newton = o.max_newton;
    prm.m = o.gmres_restart;
    prm.max_gmres = o.max_gmres;
    prm.precision = o.precision;
    prm.eta_max = (o.eta_max > 0.0) ? std::min(o.eta_max, 0.9999) : 0.9;
    prm.init_flat = (o.init == 0);
    sw_solve_info inf{};
    Scratch& sc = scratch_for(s, 2);
    sc.ensure(SolveTask::device_bytes(g, prm.m));
    const size_t npin = SolveTask::pinned_doubles(prm.m);
    double* pin = pinned_get(npin);
    sw_precond* own = nullptr;
    int32_t status = SW_ENOCONV;
    try {
        Geo g64 = g;
        g64.precision = SW_PREC_FP64;
        if (o.precond)
            SW_REQUIRE(precond_matches(o.precond, g64),
                       "the preconditioner was built for another mesh or domain");
        bool need_build = !o.precond;
        const sw_precond* P0 = o.precond;
        if (o.init == 2) {
            // Linear-solution initial guess u = u_flat - eps P^{-1} s: the root of the
            // linear system when P is the full linear Jacobian (q >= M - 1, built for this F).
            // P is needed before the first evaluation, so it is built here, on `s`.
            if (need_build) {
                const double tp0 = now_s();
                own = precond_build(g64, o.q_blocks >= 0 ? o.q_blocks : 1, s);
                inf.time_precond_s = now_s() - tp0;
                P0 = own;
                need_build = false;
            }
            const size_t n = 2 * (size_t)g64.NM;
            double* w = static_cast<double*>(sc.base);  // the task's memory, not yet in use
            double* z = w + n;
            flat_state(g64.NM, u, s);
            source_vector(g64, w, s);
            precond_apply(P0, w, z, s);
            axpby((int)n, 1.0, u, -eps, z, u, s);
        }
        SolveTask task(g64, prm, P0, u, sc.base, pin);
        while (!task.done()) {
            task.pre(s);
            if (task.done()) break;
            residual_one(*task.req_g, task.req_x, task.req_E, s);
            task.post(s);
            if (need_build) {
                // The first step evaluates E(u) only; the preconditioner is built beside it
                // on a helper stream (it reads nothing of the solve) and is complete when
                // precond_build returns, before the first Krylov step is enqueued.
                need_build = false;
                const double tp0 = now_s();
                hipStream_t ps = side_stream_take();
                try {
                    own = precond_build(g64, o.q_blocks >= 0 ? o.q_blocks : 1, ps ? ps : s);
                } catch (...) {
                    side_stream_give(ps);
                    throw;
                }
                side_stream_give(ps);
                inf.time_precond_s = now_s() - tp0;
                task.set_precond(own);
            }
            SW_HIP(hipStreamSynchronize(s));
            task.host(s);
        }
        if (zeta_out) zeta_enqueue(task.geo(), u, zeta_out, s);
        SW_HIP(hipStreamSynchronize(s));
        status = task.status;
        inf.newton_iters = task.newton;
        inf.gmres_iters = task.gmres_total;
        inf.residual_evals = task.evals;
        inf.final_norm = task.final_norm;
        inf.fp32_error = task.fp32_error;
        inf.linesearch_backtracks = task.backtracks;
    } catch (...) {
        (void)hipStreamSynchronize(s);
        if (own) precond_destroy(own);
        pinned_put(pin, npin);
        throw;
    }
    if (own) precond_destroy(own);
    pinned_put(pin, npin);
    inf.status = status;
    inf.time_total_s = now_s() - t0;
    if (info) *info = inf;
    return status;
}

}  // namespace sw

using namespace sw;

extern "C" {

void shipwave_solve_opts_default(sw_solve_opts* o) {
    if (!o) return;
    o->tol = 1e-10;
    o->max_newton = 50;
    o->gmres_restart = 30;
    o->max_gmres = 200;
    o->q_blocks = 5;
    o->precision = SW_PREC_FP64;
    o->weights = SW_WEIGHTS_TRAPEZOID;
    o->spline_bc = SW_SPLINE_CLAMPED0;
    o->init = 0;
    o->nu = 0.05;
    o->eta_max = 0.9;
    o->precond = nullptr;
}

int32_t shipwave_debug_inject_nonfinite(int32_t kinds, int32_t nth) {
    return guard([&]() -> int32_t {
        SW_REQUIRE(kinds >= 0 && kinds <= 15 && nth >= 0, "kinds must be in [0, 15], nth >= 0");
        sw::g_inject_nth.store(kinds ? nth : 0);
        sw::g_inject_mask.store(nth ? kinds : 0);
        return SW_OK;
    });
}

int32_t shipwave_solve(double F, double eps, const sw_mesh* mesh, const sw_domain* domain,
                       const sw_solve_opts* opts, double* u_inout, double* zeta_out,
                       sw_solve_info* info_out, hipStream_t stream) {
    if (info_out) *info_out = sw_solve_info{};
    int32_t st = guard([&]() -> int32_t {
        return solve_impl(F, eps, mesh, domain, opts, u_inout, zeta_out, info_out, stream);
    });
    if (info_out && st != SW_OK && info_out->status == SW_OK) info_out->status = st;
    return st;
}

}  // extern "C"
