// Memory-bound vector kernels for the Krylov solver: axpby, blocked dot
// products (classical Gram-Schmidt), multi-vector updates and norms.
// Reductions are two-pass with a grid size that depends only on n, so every
// result is bitwise reproducible.
#include "sw_internal.hpp"

namespace sw {

namespace {

constexpr int kThreads = 256;

inline int red_blocks(int n) {
    int b = (n + kThreads * 4 - 1) / (kThreads * 4);
    return b < 1 ? 1 : (b > 512 ? 512 : b);
}

__global__ __launch_bounds__(kThreads) void k_axpby(int n, double a, const double* __restrict__ x,
                                                    double b, const double* __restrict__ y,
                                                    double* __restrict__ out) {
    for (int t = blockIdx.x * kThreads + threadIdx.x; t < n; t += gridDim.x * kThreads)
        out[t] = fma(a, x[t], b * y[t]);
}

__global__ __launch_bounds__(kThreads) void k_scale(int n, double a, const double* __restrict__ x,
                                                    double* __restrict__ out) {
    for (int t = blockIdx.x * kThreads + threadIdx.x; t < n; t += gridDim.x * kThreads)
        out[t] = a * x[t];
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
__global__ __launch_bounds__(kThreads) void k_dots1(int n, const double* __restrict__ V,
                                                    size_t ldv, const double* __restrict__ w,
                                                    double* __restrict__ work) {
    __shared__ double sh[kThreads / 64];
    const int i = blockIdx.y;
    const double* v = V + (size_t)i * ldv;
    double s = 0.0;
    for (int t = blockIdx.x * kThreads + threadIdx.x; t < n; t += gridDim.x * kThreads)
        s = fma(v[t], w[t], s);
    s = block_sum(s, sh);
    if (threadIdx.x == 0) work[(size_t)i * gridDim.x + blockIdx.x] = s;
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

__global__ __launch_bounds__(kThreads) void k_norm1(int n, const double* __restrict__ x,
                                                    double* __restrict__ work) {
    __shared__ double sh[kThreads / 64];
    double m = 0.0, s = 0.0;
    for (int t = blockIdx.x * kThreads + threadIdx.x; t < n; t += gridDim.x * kThreads) {
        const double v = x[t];
        // NaN propagates through the sum of squares; fmax would drop it
        m = fmax(m, fabs(v));
        s = fma(v, v, s);
    }
    m = block_max(m, sh);
    s = block_sum(s, sh);
    if (threadIdx.x == 0) {
        work[blockIdx.x] = m;
        work[gridDim.x + blockIdx.x] = s;
    }
}

__global__ void k_norm2(int B, const double* __restrict__ work, double* __restrict__ out2) {
    if (threadIdx.x != 0) return;
    double m = 0.0, s = 0.0;
    for (int b = 0; b < B; ++b) {
        m = fmax(m, work[b]);
        s += work[B + b];
    }
    // a non-finite sum of squares marks the max norm as non-finite too
    out2[0] = (s == s && s <= 1.7976931348623157e308) ? m : s;
    out2[1] = sqrt(s);
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
__global__ __launch_bounds__(kThreads) void k_shift_auto(int n, int B,
                                                         const double* __restrict__ work,
                                                         const double* __restrict__ norms_u,
                                                         double sqrt_eps, double sqrt_n,
                                                         double* __restrict__ norms_z,
                                                         double* __restrict__ h,
                                                         const double* __restrict__ u,
                                                         const double* __restrict__ z,
                                                         double* __restrict__ out) {
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
        if (blockIdx.x == 0) {
            norms_z[0] = (s == s && s <= 1.7976931348623157e308) ? m : s;
            norms_z[1] = nz;
            h[0] = st;
            h[1] = inv;
        }
    }
    __syncthreads();
    const double st = st_s;
    for (int t = blockIdx.x * kThreads + threadIdx.x; t < n; t += gridDim.x * kThreads)
        out[t] = fma(st, z[t], u[t]);
}

// w = (Ep - Eu) / step (as k_quot; stored by the blocks of V_0) and the partial dots of
// V_i with it (as k_dots1).
__global__ __launch_bounds__(kThreads) void k_dots1_quot(int n, const double* __restrict__ V,
                                                         size_t ldv, const double* __restrict__ Ep,
                                                         const double* __restrict__ Eu,
                                                         const double* __restrict__ h,
                                                         double* __restrict__ w,
                                                         double* __restrict__ work) {
    __shared__ double sh[kThreads / 64];
    const int i = blockIdx.y;
    const double* v = V + (size_t)i * ldv;
    const double r = h[1];
    double s = 0.0;
    for (int t = blockIdx.x * kThreads + threadIdx.x; t < n; t += gridDim.x * kThreads) {
        const double wt = (Ep[t] - Eu[t]) * r;
        if (i == 0) w[t] = wt;
        s = fma(v[t], wt, s);
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) work[(size_t)i * gridDim.x + blockIdx.x] = s;
}

// Final pass of dots (partials in work, B per vector) in every block, then
// w -= sum_i h[i] V_i (as k_gemv_sub).  Block 0 stores h.
__global__ __launch_bounds__(kThreads) void k_gemv_sub_dots(int n, int k, int B,
                                                            const double* __restrict__ V,
                                                            size_t ldv,
                                                            const double* __restrict__ work,
                                                            double* __restrict__ hout,
                                                            double* __restrict__ w) {
    extern __shared__ double hs[];
    for (int i = threadIdx.x; i < k; i += kThreads) {
        double s = 0.0;
        for (int b = 0; b < B; ++b) s += work[(size_t)i * B + b];
        hs[i] = s;
        if (blockIdx.x == 0) hout[i] = s;
    }
    __syncthreads();
    for (int t = blockIdx.x * kThreads + threadIdx.x; t < n; t += gridDim.x * kThreads) {
        double s = w[t];
        for (int i = 0; i < k; ++i) s = fma(-hs[i], V[(size_t)i * ldv + t], s);
        w[t] = s;
    }
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

}  // namespace sw
