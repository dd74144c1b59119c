// A Newton-Krylov solve written as a state machine whose every residual
// evaluation is an explicit request.  A driver calls, per step,
//   pre(s)   enqueue the device work that produces the next state to evaluate
//            (req_x) and names the output (req_E) and the precision (req_g);
//            with `deferred` set, a Krylov step leaves the scaling of its basis
//            vector in scale_req (scale_pending), stops at its preconditioner apply
//            (as does the first pre() after a GMRES cycle, whose solution update
//            needs an apply) and names it in apply_P/apply_b/apply_x (apply_pending); the driver
//            runs it, alone or batched with other tasks', then calls pre_rest(s),
//            which leaves the shifted state's kernels in shift_req (shift_pending);
//   <evaluate E(req_x) -> req_E, alone or batched with other tasks>;
//   post(s)  enqueue the device work that consumes req_E and copies the
//            scalars the host needs into pinned memory (deferred Krylov steps
//            leave their Gram-Schmidt passes and norm in cgs_req (cgs_pending);
//            the driver runs them, then calls post_tail(s) for the copy);
//   <synchronise the stream>;
//   host(s)  read those scalars and advance (Givens rotations, convergence
//            tests, line-search decisions), possibly enqueueing device work.
// shipwave_solve drives one task; the server drives many, with one shared
// residual launch and one stream synchronisation per step for all of them.
#pragma once

#include <vector>

#include "sw_internal.hpp"

namespace sw {

sw_precond* precond_build(const Geo& g, int q, hipStream_t s);
void precond_apply(const sw_precond* P, const double* b, double* x, hipStream_t s);
// x_i = P_i^{-1} b_i for n requests in shared launches; bitwise precond_apply on each
void precond_apply_batched(int n, const sw_precond* const* P, const double* const* b,
                           double* const* x, hipStream_t s);
// keep_block: the device block may be kept for the next set-up of a similar size
// (otherwise it is freed at once)
void precond_destroy(sw_precond* P, bool keep_block = true);
size_t precond_bytes(const sw_precond* P);  // device bytes the preconditioner holds
size_t precond_bytes_estimate(const Geo& g, int q);
bool precond_matches(const sw_precond* P, const Geo& g);
// A non-blocking stream of the current device from a pool kept for the process (nullptr
// if none can be created), and its return once the caller has synchronised its work.
hipStream_t side_stream_take();
void side_stream_give(hipStream_t st);

struct SolveParams {
    double tol = 1e-10;
    int max_newton = 50;
    int m = 30;          // GMRES restart length
    int max_gmres = 200; // Krylov iterations per Newton step
    int precision = SW_PREC_FP64;
    double eta_max = 0.9;
    bool init_flat = true;
};

// Host-forced non-finite residuals for tests of the failure paths: the nth evaluation
// (1-based, counted per task) of each kind in the mask gets a NaN written into the first
// entry of its output by a one-thread kernel, after the residual kernels have finished.
enum : int {
    kInjectNewton = 1,  // E(u) at the initial state
    kInjectLine = 2,    // E at a line-search trial point
    kInjectJvp64 = 4,   // shifted-point evaluation of an FP64 JVP
    kInjectJvp32 = 8    // shifted-point evaluation of an FP32 JVP (mixed precision)
};
void inject_get(int* mask, int* nth);

class SolveTask {
   public:
    // u: device state (2NM doubles, initial guess unless init_flat); dev_mem:
    // device_bytes(g, m) bytes; pin: pinned_doubles(m) doubles of pinned host memory.
    SolveTask(const Geo& g64, const SolveParams& prm, const sw_precond* P, double* u,
              void* dev_mem, double* pin);
    static size_t device_bytes(const Geo& g, int m);
    static size_t pinned_doubles(int m);

    bool done() const { return ph_ == Phase::Done; }
    // the preconditioner may be supplied after construction, before the first Krylov step
    void set_precond(const sw_precond* P) { P_ = P; }
    void pre(hipStream_t s);
    void pre_rest(hipStream_t s);
    void post(hipStream_t s);
    void post_tail(hipStream_t s);
    void host(hipStream_t s);

    const double* req_x = nullptr;
    double* req_E = nullptr;
    const Geo* req_g = nullptr;

    bool deferred = false;
    bool scale_pending = false;
    ScaleArgs scale_req{};
    bool apply_pending = false;
    const sw_precond* apply_P = nullptr;
    const double* apply_b = nullptr;
    double* apply_x = nullptr;
    bool shift_pending = false;
    ShiftArgs shift_req{};
    bool cgs_pending = false;
    Cgs2Args cgs_req{};

    int status = SW_ENOCONV;
    int newton = 0;
    int gmres_total = 0;
    int evals = 0;         // evaluations of the solve (the closing FP32 check not included)
    int backtracks = 0;    // line-search halvings of lambda
    double final_norm = 0.0;
    // max |E32(u) - E64(u)| / max(1, ||E64(u)||_inf) at the returned u (one FP32-Kahan
    // evaluation after the solve ends); -1 when the solve ended on a non-finite value
    double fp32_error = -1.0;
    double* u() const { return u_; }
    const Geo& geo() const { return g64_; }

   private:
    enum class Phase { E0, Ein, Krylov, Restart, Line, Check, Done };
    void newton_top(hipStream_t s);
    void start_gmres(hipStream_t s);
    void finish_cycle(hipStream_t s, bool converged);
    void finish(int st);
    void maybe_inject(int kind, hipStream_t s);

    Geo g64_, gin_, g32_;
    int inj_mask_ = 0, inj_nth_ = 0;
    int inj_count_[4] = {0, 0, 0, 0};
    SolveParams prm_;
    const sw_precond* P_;
    int n_, m_;
    double sqrt_eps_in_, sqrt_n_;
    double *u_, *V_, *E_, *Et_, *E32_, *Ejv_, *du_, *ut_, *xs_, *z_, *w_, *hd_, *red_;
    double *pin_out_, *pin_y_;
    const double* Ein_ = nullptr;
    Phase ph_ = Phase::E0;
    // Newton state
    double nr_[2] = {0, 0};
    double prev2_ = 0.0, eta_ = 0.1, lam_ = 1.0;
    // GMRES state
    std::vector<double> H_, cs_, sn_, gv_, y_;
    int j_ = 0, its_ = 0;
    double beta_ = 0.0, target_ = 0.0, pending_scale_ = 0.0;
    bool first_cycle_ = true, restart_mode_ = false;
    // deferred: a GMRES cycle's update du (+)= P^{-1} w is left to the next pre()
    bool fin_pending_ = false, fin_first_ = false;
};

// Pinned host blocks for task scalars, reused across tasks.
double* pinned_get(size_t doubles);
void pinned_put(double* p, size_t doubles);

}  // namespace sw
