// Memory-bound vector kernels for the Krylov solver: axpby, blocked dot
// products (classical Gram-Schmidt), multi-vector updates and norms.
// Reductions are two-pass with a grid size that depends only on n, so every
// result is bitwise reproducible.
#include "sw_internal.hpp"

#include <algorithm>
#include <vector>

namespace sw {

namespace {

constexpr int kThreads = 256;

__host__ __device__ inline int red_blocks(int n) {
    int b = (n + kThreads * 4 - 1) / (kThreads * 4);
    return b < 1 ? 1 : (b > 512 ? 512 : b);
}

__global__ __launch_bounds__(kThreads) void k_axpby(int n, double a, const double* __restrict__ x,
                                                    double b, const double* __restrict__ y,
                                                    double* __restrict__ out) {
    for (int t = blockIdx.x * kThreads + threadIdx.x; t < n; t += gridDim.x * kThreads)
        out[t] = fma(a, x[t], b * y[t]);
}

__device__ __forceinline__ void scale_body(int n, double a, const double* __restrict__ x,
                                           double* __restrict__ out, int bx, int nbx) {
    for (int t = bx * kThreads + threadIdx.x; t < n; t += nbx * kThreads) out[t] = a * x[t];
}

__global__ __launch_bounds__(kThreads) void k_scale(int n, double a, const double* __restrict__ x,
                                                    double* __restrict__ out) {
    scale_body(n, a, x, out, blockIdx.x, gridDim.x);
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kThreads / 64; ++i) r += sh[i];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double block_max(double v, double* sh) {
    for (int d = 32; d >= 1; d >>= 1) v = fmax(v, __shfl_xor(v, d, 64));
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kThreads / 64; ++i) r = fmax(r, sh[i]);
    __syncthreads();
    return r;
}

// work[i * B + b] = partial dot of V_i and w over the block's grid-stride range
__device__ __forceinline__ void dots1_body(int n, const double* __restrict__ V, size_t ldv,
                                           const double* __restrict__ w,
                                           double* __restrict__ work, int bx, int i, int nbx,
                                           double* sh) {
    const double* v = V + (size_t)i * ldv;
    double s = 0.0;
    for (int t = bx * kThreads + threadIdx.x; t < n; t += nbx * kThreads)
        s = fma(v[t], w[t], s);
    s = block_sum(s, sh);
    if (threadIdx.x == 0) work[(size_t)i * nbx + bx] = s;
}

__global__ __launch_bounds__(kThreads) void k_dots1(int n, const double* __restrict__ V,
                                                    size_t ldv, const double* __restrict__ w,
                                                    double* __restrict__ work) {
    __shared__ double sh[kThreads / 64];
    dots1_body(n, V, ldv, w, work, blockIdx.x, blockIdx.y, gridDim.x, sh);
}

__global__ void k_dots2(int k, int B, const double* __restrict__ work, double* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= k) return;
    double s = 0.0;
    for (int b = 0; b < B; ++b) s += work[(size_t)i * B + b];
    out[i] = s;
}

__global__ __launch_bounds__(kThreads) void k_gemv_sub(int n, int k, const double* __restrict__ V,
                                                       size_t ldv, const double* __restrict__ h,
                                                       double* __restrict__ w) {
    for (int t = blockIdx.x * kThreads + threadIdx.x; t < n; t += gridDim.x * kThreads) {
        double s = w[t];
        for (int i = 0; i < k; ++i) s = fma(-h[i], V[(size_t)i * ldv + t], s);
        w[t] = s;
    }
}

__global__ __launch_bounds__(kThreads) void k_gemv_acc(int n, int k, const double* __restrict__ V,
                                                       size_t ldv, const double* __restrict__ y,
                                                       double* __restrict__ out) {
    for (int t = blockIdx.x * kThreads + threadIdx.x; t < n; t += gridDim.x * kThreads) {
        double s = 0.0;
        for (int i = 0; i < k; ++i) s = fma(y[i], V[(size_t)i * ldv + t], s);
        out[t] = s;
    }
}

// The kernels below are written as bodies over block bx of nbx blocks, so that the
// batched launches (several independent vectors, each over its own range of blocks)
// run the same arithmetic in the same order as the single launches.
__device__ __forceinline__ void norm1_body(int n, const double* __restrict__ x,
                                           double* __restrict__ work, int bx, int nbx,
                                           double* sh) {
    double m = 0.0, s = 0.0;
    for (int t = bx * kThreads + threadIdx.x; t < n; t += nbx * kThreads) {
        const double v = x[t];
        // NaN propagates through the sum of squares; fmax would drop it
        m = fmax(m, fabs(v));
        s = fma(v, v, s);
    }
    m = block_max(m, sh);
    s = block_sum(s, sh);
    if (threadIdx.x == 0) {
        work[bx] = m;
        work[nbx + bx] = s;
    }
}

__global__ __launch_bounds__(kThreads) void k_norm1(int n, const double* __restrict__ x,
                                                    double* __restrict__ work) {
    __shared__ double sh[kThreads / 64];
    norm1_body(n, x, work, blockIdx.x, gridDim.x, sh);
}

// thread 0 only
__device__ __forceinline__ void norm2_body(int B, const double* __restrict__ work,
                                           double* __restrict__ out2) {
    double m = 0.0, s = 0.0;
    for (int b = 0; b < B; ++b) {
        m = fmax(m, work[b]);
        s += work[B + b];
    }
    // a non-finite sum of squares marks the max norm as non-finite too
    out2[0] = (s == s && s <= 1.7976931348623157e308) ? m : s;
    out2[1] = sqrt(s);
}

__global__ void k_norm2(int B, const double* __restrict__ work, double* __restrict__ out2) {
    if (threadIdx.x != 0) return;
    norm2_body(B, work, out2);
}

__global__ void k_jvp_h(const double* norms_u, const double* norms_z, double sqrt_eps,
                        double sqrt_n, double* h) {
    // h[0] = step, h[1] = 1/step (both 0 if z == 0); the step moves each entry of u by
    // about sqrt(macheps) (1 + rms(u)).
    const double nz = norms_z[1];
    if (nz > 0.0) {
        const double st = sqrt_eps * (sqrt_n + norms_u[1]) / nz;
        h[0] = st;
        h[1] = 1.0 / st;
    } else {
        h[0] = 0.0;
        h[1] = 0.0;
    }
}

__global__ void k_set_h(double h, double* out) {
    out[0] = h;
    out[1] = 1.0 / h;
}

__global__ __launch_bounds__(kThreads) void k_shift(int n, const double* __restrict__ u,
                                                    const double* __restrict__ z,
                                                    const double* __restrict__ h,
                                                    double* __restrict__ out) {
    const double st = h[0];
    for (int t = blockIdx.x * kThreads + threadIdx.x; t < n; t += gridDim.x * kThreads)
        out[t] = fma(st, z[t], u[t]);
}

__global__ __launch_bounds__(kThreads) void k_quot(int n, const double* __restrict__ Ep,
                                                   const double* __restrict__ Eu,
                                                   const double* __restrict__ h,
                                                   double* __restrict__ out) {
    const double r = h[1];
    for (int t = blockIdx.x * kThreads + threadIdx.x; t < n; t += gridDim.x * kThreads)
        out[t] = (Ep[t] - Eu[t]) * r;
}

// Fused forms for the Krylov step; each finishes a two-pass reduction in the same order
// as k_norm2 / k_dots2, so their results are bitwise those of the separate launches.

// Final pass of norm_inf_2 on z (partials in work), the JVP step from it (as k_jvp_h),
// and out = u + step z.  Workgroup 0 stores the norms of z and h = [step, 1/step].
__device__ __forceinline__ void shift_auto_body(int n, int B, const double* __restrict__ work,
                                                const double* __restrict__ norms_u,
                                                double sqrt_eps, double sqrt_n,
                                                double* __restrict__ norms_z,
                                                double* __restrict__ h,
                                                const double* __restrict__ u,
                                                const double* __restrict__ z,
                                                double* __restrict__ out, int bx, int nbx) {
    __shared__ double st_s;
    if (threadIdx.x == 0) {
        double m = 0.0, s = 0.0;
        for (int b = 0; b < B; ++b) {
            m = fmax(m, work[b]);
            s += work[B + b];
        }
        const double nz = sqrt(s);
        double st = 0.0, inv = 0.0;
        if (nz > 0.0) {
            st = sqrt_eps * (sqrt_n + norms_u[1]) / nz;
            inv = 1.0 / st;
        }
        st_s = st;
        if (bx == 0) {
            norms_z[0] = (s == s && s <= 1.7976931348623157e308) ? m : s;
            norms_z[1] = nz;
            h[0] = st;
            h[1] = inv;
        }
    }
    __syncthreads();
    const double st = st_s;
    for (int t = bx * kThreads + threadIdx.x; t < n; t += nbx * kThreads)
        out[t] = fma(st, z[t], u[t]);
}

__global__ __launch_bounds__(kThreads) void k_shift_auto(int n, int B,
                                                         const double* __restrict__ work,
                                                         const double* __restrict__ norms_u,
                                                         double sqrt_eps, double sqrt_n,
                                                         double* __restrict__ norms_z,
                                                         double* __restrict__ h,
                                                         const double* __restrict__ u,
                                                         const double* __restrict__ z,
                                                         double* __restrict__ out) {
    shift_auto_body(n, B, work, norms_u, sqrt_eps, sqrt_n, norms_z, h, u, z, out, blockIdx.x,
                    gridDim.x);
}

// w = (Ep - Eu) / step (as k_quot; stored by the blocks of V_0) and the partial dots of
// V_i with it (as k_dots1).
__device__ __forceinline__ void dots1_quot_body(int n, const double* __restrict__ V, size_t ldv,
                                                const double* __restrict__ Ep,
                                                const double* __restrict__ Eu,
                                                const double* __restrict__ h,
                                                double* __restrict__ w,
                                                double* __restrict__ work, int bx, int i,
                                                int nbx, double* sh) {
    const double* v = V + (size_t)i * ldv;
    const double r = h[1];
    double s = 0.0;
    for (int t = bx * kThreads + threadIdx.x; t < n; t += nbx * kThreads) {
        const double wt = (Ep[t] - Eu[t]) * r;
        if (i == 0) w[t] = wt;
        s = fma(v[t], wt, s);
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) work[(size_t)i * nbx + bx] = s;
}

__global__ __launch_bounds__(kThreads) void k_dots1_quot(int n, const double* __restrict__ V,
                                                         size_t ldv, const double* __restrict__ Ep,
                                                         const double* __restrict__ Eu,
                                                         const double* __restrict__ h,
                                                         double* __restrict__ w,
                                                         double* __restrict__ work) {
    __shared__ double sh[kThreads / 64];
    dots1_quot_body(n, V, ldv, Ep, Eu, h, w, work, blockIdx.x, blockIdx.y, gridDim.x, sh);
}

// Final pass of dots (partials in work, B per vector) in every block, then
// w -= sum_i h[i] V_i (as k_gemv_sub).  Block 0 stores h.
__device__ __forceinline__ void gemv_sub_dots_body(int n, int k, int B,
                                                   const double* __restrict__ V, size_t ldv,
                                                   const double* __restrict__ work,
                                                   double* __restrict__ hout,
                                                   double* __restrict__ w, int bx, int nbx,
                                                   double* hs) {
    for (int i = threadIdx.x; i < k; i += kThreads) {
        double s = 0.0;
        for (int b = 0; b < B; ++b) s += work[(size_t)i * B + b];
        hs[i] = s;
        if (bx == 0) hout[i] = s;
    }
    __syncthreads();
    for (int t = bx * kThreads + threadIdx.x; t < n; t += nbx * kThreads) {
        double s = w[t];
        for (int i = 0; i < k; ++i) s = fma(-hs[i], V[(size_t)i * ldv + t], s);
        w[t] = s;
    }
}

__global__ __launch_bounds__(kThreads) void k_gemv_sub_dots(int n, int k, int B,
                                                            const double* __restrict__ V,
                                                            size_t ldv,
                                                            const double* __restrict__ work,
                                                            double* __restrict__ hout,
                                                            double* __restrict__ w) {
    extern __shared__ double hs[];
    gemv_sub_dots_body(n, k, B, V, ldv, work, hout, w, blockIdx.x, gridDim.x, hs);
}

// ---- batched forms: job p takes blocks [first[p], first[p + 1]) of a 1-D grid ----
constexpr int kMaxKJobs = 32;

__device__ __forceinline__ int job_of(const int* first, int nj) {
    int p = 0;
    while (p + 1 < nj && (int)blockIdx.x >= first[p + 1]) ++p;
    return p;
}

struct NormJob {
    int n;
    const double* x;
    double* work;
    double* out2;
};
struct NormBatch {
    NormJob j[kMaxKJobs];
    int first[kMaxKJobs + 1];
    int nj;
};

struct ShiftJob {
    int n, B;
    const double* work;
    const double* norms_u;
    double* norms_z;
    double* h;
    const double* u;
    const double* z;
    double* out;
    double sqrt_eps, sqrt_n;
};
struct ShiftBatch {
    ShiftJob j[kMaxKJobs];
    int first[kMaxKJobs + 1];
    int nj;
};

struct CgsJob {
    int n, k, B;
    const double* V;
    size_t ldv;
    const double* Ep;  // first pass: w = (Ep - Eu) / h[0]; nullptr: w as it is
    const double* Eu;
    const double* h;
    double* w;
    double* hout;
    double* work;
};
struct CgsBatch {
    CgsJob j[kMaxKJobs];
    int first[kMaxKJobs + 1];
    int nj;
};
static_assert(sizeof(NormBatch) <= 4096 && sizeof(ShiftBatch) <= 4096 &&
                  sizeof(CgsBatch) <= 4096,
              "kernel argument block");

struct ScaleBatch {
    ScaleArgs j[kMaxKJobs];
    int first[kMaxKJobs + 1];
    int nj;
};
static_assert(sizeof(ScaleBatch) <= 4096, "kernel argument block");

// blocks per job: ew_blocks(n)
__global__ __launch_bounds__(kThreads) void k_scale_batched(const ScaleBatch b) {
    const int p = job_of(b.first, b.nj);
    const ScaleArgs& J = b.j[p];
    scale_body(J.n, J.a, J.x, J.out, blockIdx.x - b.first[p], b.first[p + 1] - b.first[p]);
}

// blocks per job: red_blocks(n)
__global__ __launch_bounds__(kThreads) void k_norm1_batched(const NormBatch b) {
    __shared__ double sh[kThreads / 64];
    const int p = job_of(b.first, b.nj);
    const NormJob& J = b.j[p];
    norm1_body(J.n, J.x, J.work, blockIdx.x - b.first[p], b.first[p + 1] - b.first[p], sh);
}

// one block per job
__global__ void k_norm2_batched(const NormBatch b) {
    if (threadIdx.x != 0) return;
    const NormJob& J = b.j[blockIdx.x];
    norm2_body(red_blocks(J.n), J.work, J.out2);
}

// blocks per job: ew_blocks(n)
__global__ __launch_bounds__(kThreads) void k_shift_auto_batched(const ShiftBatch b) {
    const int p = job_of(b.first, b.nj);
    const ShiftJob& J = b.j[p];
    shift_auto_body(J.n, J.B, J.work, J.norms_u, J.sqrt_eps, J.sqrt_n, J.norms_z, J.h, J.u, J.z,
                    J.out, blockIdx.x - b.first[p], b.first[p + 1] - b.first[p]);
}

// blocks per job: B k, block l of the job is (l % B, vector l / B)
__global__ __launch_bounds__(kThreads) void k_dots1_batched(const CgsBatch b) {
    __shared__ double sh[kThreads / 64];
    const int p = job_of(b.first, b.nj);
    const CgsJob& J = b.j[p];
    const int l = blockIdx.x - b.first[p];
    const int i = l / J.B, bx = l - i * J.B;
    if (J.Ep)
        dots1_quot_body(J.n, J.V, J.ldv, J.Ep, J.Eu, J.h, J.w, J.work, bx, i, J.B, sh);
    else
        dots1_body(J.n, J.V, J.ldv, J.w, J.work, bx, i, J.B, sh);
}

// blocks per job: ew_blocks(n); dynamic LDS: the largest k
__global__ __launch_bounds__(kThreads) void k_gemv_sub_dots_batched(const CgsBatch b) {
    extern __shared__ double hs[];
    const int p = job_of(b.first, b.nj);
    const CgsJob& J = b.j[p];
    gemv_sub_dots_body(J.n, J.k, J.B, J.V, J.ldv, J.work, J.hout, J.w, blockIdx.x - b.first[p],
                       b.first[p + 1] - b.first[p], hs);
}

__global__ void k_flat(int NM, double* u) {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < 2 * NM; t += gridDim.x * blockDim.x)
        u[t] = (t < NM) ? 1.0 : 0.0;
}

// Source vector of the linear system (linear-problem section): the submerged-source term
// of E2 at the flat surface, 1 / sqrt(x*^2 + y*^2 + 1) on the E2 rows, zero elsewhere.
__global__ void k_source(Geo g, double* w) {
    const int NM = g.NM;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < 2 * NM; t += gridDim.x * blockDim.x) {
        double v = 0.0;
        if (t >= NM) {
            const int l = (t - NM) / g.N, r = (t - NM) - l * g.N;
            if (r > 0) {
                const double xs = g.x1 + (r - 0.5) * g.dx, ys = l * g.dy;
                v = 1.0 / sqrt(xs * xs + ys * ys + 1.0);
            }
        }
        w[t] = v;
    }
}

inline int ew_blocks(int n) {
    int b = (n + kThreads - 1) / kThreads;
    return b < 1 ? 1 : (b > 4096 ? 4096 : b);
}

}  // namespace

size_t reduce_work_doubles(int n, int k) { return (size_t)(k + 2) * red_blocks(n) + 64; }

void axpby(int n, double a, const double* x, double b, const double* y, double* out,
           hipStream_t s) {
    k_axpby<<<ew_blocks(n), kThreads, 0, s>>>(n, a, x, b, y, out);
}

void scale_copy(int n, double a, const double* x, double* out, hipStream_t s) {
    k_scale<<<ew_blocks(n), kThreads, 0, s>>>(n, a, x, out);
}

void dots(int n, int k, const double* V, size_t ldv, const double* w, double* out, double* work,
          hipStream_t s) {
    const int B = red_blocks(n);
    k_dots1<<<dim3(B, k), kThreads, 0, s>>>(n, V, ldv, w, work);
    k_dots2<<<(k + 63) / 64, 64, 0, s>>>(k, B, work, out);
}

void gemv_sub(int n, int k, const double* V, size_t ldv, const double* h, double* w,
              hipStream_t s) {
    k_gemv_sub<<<ew_blocks(n), kThreads, 0, s>>>(n, k, V, ldv, h, w);
}

void gemv_acc(int n, int k, const double* V, size_t ldv, const double* y, double* out,
              hipStream_t s) {
    k_gemv_acc<<<ew_blocks(n), kThreads, 0, s>>>(n, k, V, ldv, y, out);
}

void norm_inf_2(int n, const double* x, double* out2, double* work, hipStream_t s) {
    const int B = red_blocks(n);
    k_norm1<<<B, kThreads, 0, s>>>(n, x, work);
    k_norm2<<<1, 64, 0, s>>>(B, work, out2);
}

void jvp_step(const double* norms_u, const double* norms_z, double sqrt_eps, double sqrt_n,
              double* h, hipStream_t s) {
    k_jvp_h<<<1, 1, 0, s>>>(norms_u, norms_z, sqrt_eps, sqrt_n, h);
}

void set_step(double h, double* out, hipStream_t s) { k_set_h<<<1, 1, 0, s>>>(h, out); }

void shift(int n, const double* u, const double* z, const double* h, double* out,
           hipStream_t s) {
    k_shift<<<ew_blocks(n), kThreads, 0, s>>>(n, u, z, h, out);
}

void quotient(int n, const double* Ep, const double* Eu, const double* h, double* out,
              hipStream_t s) {
    k_quot<<<ew_blocks(n), kThreads, 0, s>>>(n, Ep, Eu, h, out);
}

void flat_state(int NM, double* u, hipStream_t s) { k_flat<<<256, 256, 0, s>>>(NM, u); }

void source_vector(const Geo& g, double* w, hipStream_t s) {
    k_source<<<ew_blocks(2 * g.NM), kThreads, 0, s>>>(g, w);
}

void shift_auto(int n, const double* u, const double* z, const double* norms_u, double sqrt_eps,
                double sqrt_n, double* norms_z, double* h, double* out, double* work,
                hipStream_t s) {
    const int B = red_blocks(n);
    k_norm1<<<B, kThreads, 0, s>>>(n, z, work);
    k_shift_auto<<<ew_blocks(n), kThreads, 0, s>>>(n, B, work, norms_u, sqrt_eps, sqrt_n, norms_z,
                                                    h, u, z, out);
}

// Every block of the subtraction re-reads the k B partials; beyond this many the separate
// final-pass launch is cheaper.
constexpr int kFusedPartials = 2048;

void cgs_pass(int n, int k, const double* V, size_t ldv, const double* w_in_Ep,
              const double* Eu, const double* h, double* w, double* hout, double* work,
              hipStream_t s) {
    const int B = red_blocks(n);
    if (w_in_Ep)
        k_dots1_quot<<<dim3(B, k), kThreads, 0, s>>>(n, V, ldv, w_in_Ep, Eu, h, w, work);
    else
        k_dots1<<<dim3(B, k), kThreads, 0, s>>>(n, V, ldv, w, work);
    if ((size_t)k * B <= (size_t)kFusedPartials) {
        k_gemv_sub_dots<<<ew_blocks(n), kThreads, (size_t)k * sizeof(double), s>>>(
            n, k, B, V, ldv, work, hout, w);
    } else {
        k_dots2<<<(k + 63) / 64, 64, 0, s>>>(k, B, work, hout);
        k_gemv_sub<<<ew_blocks(n), kThreads, 0, s>>>(n, k, V, ldv, hout, w);
    }
}

void scale_copy_batched(int nj, const ScaleArgs* a, hipStream_t s) {
    for (int o = 0; o < nj; o += kMaxKJobs) {
        const int c = std::min(kMaxKJobs, nj - o);
        ScaleBatch b{};
        int eb = 0;
        for (int q = 0; q < c; ++q) {
            b.j[q] = a[o + q];
            b.first[q] = eb;
            eb += ew_blocks(a[o + q].n);
        }
        b.first[c] = eb;
        b.nj = c;
        k_scale_batched<<<eb, kThreads, 0, s>>>(b);
    }
}

void shift_auto_batched(int nj, const ShiftArgs* a, hipStream_t s) {
    for (int o = 0; o < nj; o += kMaxKJobs) {
        const int c = std::min(kMaxKJobs, nj - o);
        NormBatch nb{};
        ShiftBatch sb{};
        int rb = 0, eb = 0;
        for (int q = 0; q < c; ++q) {
            const ShiftArgs& A = a[o + q];
            nb.j[q] = NormJob{A.n, A.z, A.work, nullptr};
            nb.first[q] = rb;
            rb += red_blocks(A.n);
            sb.j[q] = ShiftJob{A.n, red_blocks(A.n), A.work, A.norms_u, A.norms_z, A.h,
                               A.u, A.z, A.out, A.sqrt_eps, A.sqrt_n};
            sb.first[q] = eb;
            eb += ew_blocks(A.n);
        }
        nb.first[c] = rb;
        nb.nj = c;
        sb.first[c] = eb;
        sb.nj = c;
        k_norm1_batched<<<rb, kThreads, 0, s>>>(nb);
        k_shift_auto_batched<<<eb, kThreads, 0, s>>>(sb);
    }
}

void cgs2_norm_batched(int nj, const Cgs2Args* a, hipStream_t s) {
    std::vector<const Cgs2Args*> fused;
    for (int q = 0; q < nj; ++q) {
        const Cgs2Args& A = a[q];
        if ((size_t)A.k * red_blocks(A.n) <= (size_t)kFusedPartials) {
            fused.push_back(&A);
            continue;
        }
        // many partials: the separate final-pass launches of cgs_pass
        cgs_pass(A.n, A.k, A.V, A.ldv, A.Ep, A.Eu, A.h, A.w, A.hout1, A.work, s);
        cgs_pass(A.n, A.k, A.V, A.ldv, nullptr, nullptr, nullptr, A.w, A.hout2, A.work, s);
        norm_inf_2(A.n, A.w, A.norms, A.work, s);
    }
    const int nf = (int)fused.size();
    for (int o = 0; o < nf; o += kMaxKJobs) {
        const int c = std::min(kMaxKJobs, nf - o);
        CgsBatch cb{};
        NormBatch nb{};
        int db = 0, eb = 0, rb = 0, kmax = 1;
        std::vector<int> efirst(c + 1);
        for (int q = 0; q < c; ++q) {
            const Cgs2Args& A = *fused[o + q];
            const int B = red_blocks(A.n);
            cb.j[q] = CgsJob{A.n, A.k, B, A.V, A.ldv, A.Ep, A.Eu, A.h, A.w, A.hout1, A.work};
            cb.first[q] = db;
            db += B * A.k;
            efirst[q] = eb;
            eb += ew_blocks(A.n);
            kmax = std::max(kmax, A.k);
            nb.j[q] = NormJob{A.n, A.w, A.work, A.norms};
            nb.first[q] = rb;
            rb += B;
        }
        cb.first[c] = db;
        cb.nj = c;
        nb.first[c] = rb;
        nb.nj = c;
        CgsBatch eb1 = cb;
        for (int q = 0; q <= c; ++q) eb1.first[q] = efirst[q];
        efirst[c] = eb;
        eb1.first[c] = eb;
        const size_t lds = (size_t)kmax * sizeof(double);
        // first pass: w = (Ep - Eu) / step, hout1 = V^T w, w -= V hout1
        k_dots1_batched<<<db, kThreads, 0, s>>>(cb);
        k_gemv_sub_dots_batched<<<eb, kThreads, lds, s>>>(eb1);
        // second pass on w: hout2
        for (int q = 0; q < c; ++q) {
            cb.j[q].Ep = nullptr;
            cb.j[q].Eu = nullptr;
            cb.j[q].h = nullptr;
            cb.j[q].hout = fused[o + q]->hout2;
            eb1.j[q] = cb.j[q];
        }
        k_dots1_batched<<<db, kThreads, 0, s>>>(cb);
        k_gemv_sub_dots_batched<<<eb, kThreads, lds, s>>>(eb1);
        k_norm1_batched<<<rb, kThreads, 0, s>>>(nb);
        k_norm2_batched<<<c, 64, 0, s>>>(nb);
    }
}

}  // namespace sw
