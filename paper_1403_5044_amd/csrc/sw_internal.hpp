// Internal declarations shared by the translation units of libshipwave.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/shipwave.h"

namespace sw {

// ---- errors ---------------------------------------------------------------
void set_error(const std::string& msg);
struct Error {
    int32_t code;
    std::string msg;
};

#define SW_HIP(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            throw ::sw::Error{SW_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)

#define SW_REQUIRE(cond, msg)                                      \
    do {                                                           \
        if (!(cond)) throw ::sw::Error{SW_EINVAL, std::string(msg)}; \
    } while (0)

// Runs f, converting exceptions into a return code and a thread-local message.
template <class Fn>
int32_t guard(Fn&& f) {
    try {
        return f();
    } catch (const Error& e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc&) {
        set_error("host allocation failed");
        return SW_ENOMEM;
    } catch (const std::exception& e) {
        set_error(e.what());
        return SW_EHIP;
    } catch (...) {
        set_error("unknown error");
        return SW_EHIP;
    }
}

// ---- problem geometry as seen by kernels ------------------------------------
struct Geo {
    int N, M, Nc, NM, ncol;  // ncol = (N-1) M collocation points
    int weights, bc, precision;
    double x1, xN, yM, dx, dy;
    double F, eps, nu;
};

// Mesh widths: the residual, JVP and zeta calls stage source rows through LDS in
// segments, so any N up to kMaxGridN works there; the preconditioner's apply kernels
// hold a block row in LDS and its wide-block inversion at most four panel rows per
// thread, so preconditioners (and hence solves and server requests) need N <= kMaxN.
constexpr int kMaxN = 1024;
constexpr int kMaxGridN = 1 << 16;

Geo make_geo(const sw_problem& p);  // validates, throws SW_EINVAL

// ---- device scratch ----------------------------------------------------------
// A growable device buffer carved into named regions.  One per (device,
// stream); growth synchronises the stream before freeing the old buffer.
struct Scratch {
    void* base = nullptr;
    size_t bytes = 0;
    int device = -1;
    hipStream_t stream = nullptr;
    void ensure(size_t need);
    ~Scratch();
};

// Scratch of the current device for `stream` (created on first use).
Scratch& scratch_for(hipStream_t stream, int slot = 0);

struct Carve {
    char* p;
    size_t off = 0;
    explicit Carve(void* base) : p(static_cast<char*>(base)) {}
    template <class T>
    T* take(size_t n) {
        off = (off + 255) & ~size_t(255);
        T* r = reinterpret_cast<T*>(p + off);
        off += n * sizeof(T);
        return r;
    }
};
inline size_t carve_size(std::initializer_list<size_t> byte_counts) {
    size_t off = 0;
    for (size_t b : byte_counts) off = ((off + 255) & ~size_t(255)) + b;
    return off + 256;
}

// ---- residual ------------------------------------------------------------------
// Per-problem device state for one residual evaluation.
struct ResidualBufs {
    double* psi;      // [M][N] grid potential perturbation psi = phi - x
    double* zeta;     // [M][N]
    double* psiy;     // [M][N]
    double* zetay;    // [M][N]
    double* src64;    // [NM][8] source records (FP64)
    float* src32;     // [NM][8] source records (FP32), precision == FP32 only
    double* col;      // [ncol][8] collocation records
    double* partial;  // [G][ncol] partial pair sums
    double* spl;      // [2][M] spline elimination coefficients
    int G;            // source-row chunks of the pair sum
};

size_t residual_scratch_bytes(const Geo& g, int G);
ResidualBufs carve_residual(Carve& c, const Geo& g, int G);
int choose_chunks(const Geo& g);

// Enqueue E(u) for one problem on `stream` using bufs (already carved).
void residual_enqueue(const Geo& g, const double* u, double* E, const ResidualBufs& b,
                      hipStream_t stream);
// The same residual with nothing allocated or created on the way (for the entry point
// that takes no memory of its own): spline slopes by the per-column sweep, no timing.
void residual_enqueue_fixed(const Geo& g, const double* u, double* E, const ResidualBufs& b,
                            hipStream_t stream);
// Batched form: shared launches over nb problems.
void residual_batched_enqueue(int nb, const Geo* g, const double* const* u, double* const* E,
                              hipStream_t stream);

// Simple device vector helpers (krylov.hip).
void axpby(int n, double a, const double* x, double b, const double* y, double* out,
           hipStream_t s);  // out = a x + b y
void scale_copy(int n, double a, const double* x, double* out, hipStream_t s);
// Deterministic reductions; results land in device memory `out`.
void dots(int n, int k, const double* V, size_t ldv, const double* w, double* out,
          double* work, hipStream_t s);  // out[i] = V_i . w, i < k
void gemv_sub(int n, int k, const double* V, size_t ldv, const double* h, double* w,
              hipStream_t s);  // w -= sum_i h[i] V_i (h on device)
void gemv_acc(int n, int k, const double* V, size_t ldv, const double* y, double* out,
              hipStream_t s);  // out = sum_i y[i] V_i (y on device)
void norm_inf_2(int n, const double* x, double* out2, double* work,
                hipStream_t s);  // out2[0] = max|x|, out2[1] = ||x||_2
// Difference-quotient JVP pieces: h = [step, 1/step] computed on the device from
// the 2-norms in norms_u[1], norms_z[1]; out = u + step z; out = (Ep - Eu) / step.
void jvp_step(const double* norms_u, const double* norms_z, double sqrt_eps, double sqrt_n,
              double* h, hipStream_t s);
void set_step(double h, double* out, hipStream_t s);
void shift(int n, const double* u, const double* z, const double* h, double* out, hipStream_t s);
void quotient(int n, const double* Ep, const double* Eu, const double* h, double* out,
              hipStream_t s);
void flat_state(int NM, double* u, hipStream_t s);  // phi_x = 1, zeta_x = 0
// w = s, the source term of E2 at the flat surface per unit eps (linear system's right side)
void source_vector(const Geo& g, double* w, hipStream_t s);
// norm_inf_2(z) into norms_z, jvp_step(norms_u, norms_z) into h and shift(u, z, h) into
// out, in two launches (work as for norm_inf_2).
void shift_auto(int n, const double* u, const double* z, const double* norms_u, double sqrt_eps,
                double sqrt_n, double* norms_z, double* h, double* out, double* work,
                hipStream_t s);
// One classical Gram-Schmidt pass against V_0..V_{k-1}: hout = V^T w, w -= V hout.  With
// Ep != nullptr, w is first set to (Ep - Eu) / h[0] (quotient()).  Two launches while
// the reduction partials are few, three otherwise; the results equal those of
// quotient(), dots() and gemv_sub().
void cgs_pass(int n, int k, const double* V, size_t ldv, const double* Ep, const double* Eu,
              const double* h, double* w, double* hout, double* work, hipStream_t s);
// Batched forms for several independent solves (the server): every job's results are
// bitwise those of its own scale_copy, shift_auto, or cgs_pass with Ep, cgs_pass
// without, then norm_inf_2(w) into norms; the jobs share the launches.
struct ScaleArgs {
    int n;
    double a;
    const double* x;
    double* out;
};
void scale_copy_batched(int nj, const ScaleArgs* a, hipStream_t s);
struct ShiftArgs {
    int n;
    const double* u;
    const double* z;
    const double* norms_u;
    double sqrt_eps, sqrt_n;
    double* norms_z;
    double* h;
    double* out;
    double* work;
};
void shift_auto_batched(int nj, const ShiftArgs* a, hipStream_t s);
struct Cgs2Args {
    int n, k;
    const double* V;
    size_t ldv;
    const double* Ep;
    const double* Eu;
    const double* h;
    double* w;
    double* hout1;
    double* hout2;
    double* norms;
    double* work;
};
void cgs2_norm_batched(int nj, const Cgs2Args* a, hipStream_t s);
void residual_one(const Geo& g, const double* u, double* E, hipStream_t s);
// work doubles for dots() with up to k vectors and for norm_inf_2()
size_t reduce_work_doubles(int n, int k);

// Event timing of all-pairs launches (diagnostics).
struct ProfileMark {
    hipEvent_t a = nullptr, b = nullptr;
};
ProfileMark profile_begin(hipStream_t s);
void profile_end(const ProfileMark& m, hipStream_t s, double pairs);

// zeta on the grid from u (trapezoid integration of zeta_x)
void zeta_enqueue(const Geo& g, const double* u, double* zeta, hipStream_t s);

}  // namespace sw
