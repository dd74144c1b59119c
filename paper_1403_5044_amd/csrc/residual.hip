// Nonlinear residual E(u) on gfx950.
//
// Steps (numerical discretisation section and Appendix A):
//   k_scan      unknowns -> psi, zeta on the grid by trapezoidal integration in x
//               (eq. zetaapprox), psi_1 and zeta_1 from the eliminated radiation
//               rows E3/E5; the radiation rows E4/E6 (eq. numUpRadiation).
//   k_spline    psi_y, zeta_y: slopes of the cubic spline through each column.
//   k_points    source records of every grid point (fields pre-multiplied by the
//               quadrature weight) and collocation records of every half-mesh
//               point: two-point interpolation, Bernoulli E1 (eq. freeSurfCond),
//               A, B, C, the closed form of I (eq. IS2), the submerged-source term.
//   k_pairs_*   the all-pairs sum over every (collocation, grid) pair of
//               w [(psi - psi*) K1 + zeta_x K2 - zeta_x* S2] (eq. IntegroEqn, S2),
//               split over chunks of source rows; FP64 or FP32 + Kahan.
//   k_finish    E2 = 2 pi psi* + source term - zeta_x* I - (sum over chunks).
//
// The all-pairs sum is bound by FP64 vector arithmetic, not memory: each lane
// owns CP collocation points and sweeps a row of source records staged in LDS
// (every lane reads the same record: an LDS broadcast).  The per-row terms
// (y offsets and their products with B, C) are hoisted out of the source loop.
#include "sw_internal.hpp"
#include "sw_device.hpp"

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

namespace sw {

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr int kMaxDenseSplineM = 512;

// ---- a1-a2: trapezoid integration in x, radiation rows -------------------------
// One wavefront per (row l, field f): f = 0 -> psi from phi_x - 1, f = 1 -> zeta.
// The bodies of this and the other prelude and finish kernels take their block index
// as arguments, so that the batched launches below run them unchanged.
__device__ __forceinline__ void scan_body(const Geo& g, const double* __restrict__ u,
                                          double* __restrict__ psi, double* __restrict__ zeta,
                                          double* __restrict__ E, int l, int f) {
    const int lane = threadIdx.x;
    const int N = g.N;
    const double* in = u + (size_t)f * g.NM + (size_t)l * N;
    double* out = (f == 0 ? psi : zeta) + (size_t)l * N;
    const double off = (f == 0) ? 1.0 : 0.0;
    const double hdx = 0.5 * g.dx;
    const int K = (N + 63) / 64;
    const int a = min(lane * K, N);
    const int b = min(a + K, N);
    double tot = 0.0;
    for (int m = a; m < b && m < N - 1; ++m) tot += hdx * ((in[m] - off) + (in[m + 1] - off));
    double incl = tot;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const double t = __shfl_up(incl, d, 64);
        if (lane >= d) incl += t;
    }
    double excl = __shfl_up(incl, 1, 64);
    if (lane == 0) excl = 0.0;
    const double fx0 = in[0] - off;
    const double f1 = (-g.x1 / g.nu) * fx0;  // eliminated E3 / E5
    double val = f1 + excl;
    for (int k = a; k < b; ++k) {
        out[k] = val;
        if (k < N - 1) val += hdx * ((in[k] - off) + (in[k + 1] - off));
    }
    if (lane == 0) {
        const double fx1 = in[1] - off;
        E[(size_t)f * g.NM + (size_t)l * N] = g.x1 * (fx1 - fx0) / g.dx + g.nu * fx0;
    }
}

__global__ __launch_bounds__(64) void k_scan(Geo g, const double* __restrict__ u,
                                             double* __restrict__ psi,
                                             double* __restrict__ zeta,
                                             double* __restrict__ E) {
    scan_body(g, u, psi, zeta, E, blockIdx.x, blockIdx.y);
}

// ---- a3: cubic-spline slopes in y ----------------------------------------------------
// Tridiagonal form of the spline conditions (uniform knots, spacing h, slopes s):
//   first knot:  clamped0: s_0 = 0;  not-a-knot: s_0 + 2 s_1 = (5 d_0 + d_1) / (2h)
//   interior:    s_{j-1} + 4 s_j + s_{j+1} = 3 (f_{j+1} - f_{j-1}) / h
//   last knot:   not-a-knot: 2 s_{M-2} + s_{M-1} = (d_{M-3} + 5 d_{M-2}) / (2h)
// (d_j = f_{j+1} - f_j; the not-a-knot rows are the third-derivative
// continuity conditions with the neighbouring interior row eliminated).
// The elimination coefficients depend only on M and the end condition.
__global__ void k_spline_setup(int M, int bc, double* __restrict__ spl) {
    double* cp = spl;
    double* minv = spl + M;
    double c0 = (bc == SW_SPLINE_CLAMPED0) ? 0.0 : 2.0;
    double m = 1.0;
    minv[0] = 1.0 / m;
    cp[0] = c0 / m;
    for (int j = 1; j < M; ++j) {
        const double aj = (j == M - 1) ? 2.0 : 1.0;
        const double bj = (j == M - 1) ? 1.0 : 4.0;
        const double cj = (j == M - 1) ? 0.0 : 1.0;
        m = bj - aj * cp[j - 1];
        minv[j] = 1.0 / m;
        cp[j] = cj / m;
    }
}

__global__ __launch_bounds__(128) void k_spline(Geo g, const double* __restrict__ spl,
                                                const double* __restrict__ psi,
                                                const double* __restrict__ zeta,
                                                double* __restrict__ psiy,
                                                double* __restrict__ zetay) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * g.N) return;
    const int f = t / g.N;
    const int k = t - f * g.N;
    const int N = g.N, M = g.M;
    const double* F = (f == 0 ? psi : zeta) + k;
    double* S = (f == 0 ? psiy : zetay) + k;
    const double* cp = spl;
    const double* minv = spl + M;
    const double h = g.dy;
    const double r3h = 3.0 / h;
    const double r2h = 0.5 / h;
    double f0 = F[0], f1 = F[(size_t)N], f2 = F[(size_t)2 * N];
    double d0 = (g.bc == SW_SPLINE_CLAMPED0) ? 0.0 : r2h * (5.0 * (f1 - f0) + (f2 - f1));
    double dp = d0 * minv[0];
    S[0] = dp;
    double fm = f0, fc = f1;
    for (int j = 1; j < M - 1; ++j) {
        const double fp = F[(size_t)(j + 1) * N];
        dp = (r3h * (fp - fm) - dp) * minv[j];
        S[(size_t)j * N] = dp;
        fm = fc;
        fc = fp;
    }
    {
        // fm = f_{M-3}... after the loop fm = f_{M-2}, fc = f_{M-1}
        const double fmm = F[(size_t)(M - 3) * N];
        const double dlast = r2h * ((fm - fmm) + 5.0 * (fc - fm));
        dp = (dlast - 2.0 * dp) * minv[M - 1];
    }
    double s = dp;
    S[(size_t)(M - 1) * N] = s;
    for (int j = M - 2; j >= 0; --j) {
        s = S[(size_t)j * N] - cp[j] * s;
        S[(size_t)j * N] = s;
    }
}

// Slope operator of the spline for h = 1: slopes = (1/h) Q f, one column of Q per
// thread (the slopes of the unit vector e_m), same elimination as k_spline.
__global__ void k_spline_operator(int M, int bc, double* __restrict__ Q) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    auto f = [m](int j) { return (j == m) ? 1.0 : 0.0; };
    double* S = Q + m;  // column m, stride M
    double cp = (bc == SW_SPLINE_CLAMPED0) ? 0.0 : 2.0;
    double d0 = (bc == SW_SPLINE_CLAMPED0) ? 0.0 : 0.5 * (5.0 * (f(1) - f(0)) + (f(2) - f(1)));
    double dp = d0;
    S[0] = dp;
    double* cps = nullptr;  // cp_j is recomputed on the way back
    (void)cps;
    for (int j = 1; j < M - 1; ++j) {
        const double mj = 4.0 - cp;
        dp = (3.0 * (f(j + 1) - f(j - 1)) - dp) / mj;
        cp = 1.0 / mj;
        S[(size_t)j * M] = dp;
    }
    {
        const double mj = 1.0 - 2.0 * cp;
        const double dl = 0.5 * ((f(M - 2) - f(M - 3)) + 5.0 * (f(M - 1) - f(M - 2)));
        dp = (dl - 2.0 * dp) / mj;
    }
    S[(size_t)(M - 1) * M] = dp;
    // back substitution needs cp_j: rebuild the forward sequence into a local recurrence
    double s = dp;
    for (int j = M - 2; j >= 0; --j) {
        double c = (bc == SW_SPLINE_CLAMPED0) ? 0.0 : 2.0;
        for (int i = 1; i <= j; ++i) c = 1.0 / (4.0 - c);
        s = S[(size_t)j * M] - c * s;
        S[(size_t)j * M] = s;
    }
}

// psi_y, zeta_y = (1/h) Q f for every column at once: block (x-tile, row j, field).
__device__ __forceinline__ void spline_dense_body(const Geo& g, const double* __restrict__ Q,
                                                  const double* __restrict__ psi,
                                                  const double* __restrict__ zeta,
                                                  double* __restrict__ psiy,
                                                  double* __restrict__ zetay, int bx, int j,
                                                  int f) {
    const int k = bx * 128 + threadIdx.x;
    if (k >= g.N) return;
    const double* F = (f == 0 ? psi : zeta) + k;
    const double* q = Q + (size_t)j * g.M;
    double s[8] = {};  // eight independent chains: eight loads in flight
    int m = 0;
    for (; m + 7 < g.M; m += 8)
#pragma unroll
        for (int e = 0; e < 8; ++e) s[e] = fma(q[m + e], F[(size_t)(m + e) * g.N], s[e]);
    for (; m < g.M; ++m) s[0] = fma(q[m], F[(size_t)m * g.N], s[0]);
    const double t = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
    (f == 0 ? psiy : zetay)[(size_t)j * g.N + k] = t / g.dy;
}

__global__ __launch_bounds__(128) void k_spline_dense(Geo g, const double* __restrict__ Q,
                                                      const double* __restrict__ psi,
                                                      const double* __restrict__ zeta,
                                                      double* __restrict__ psiy,
                                                      double* __restrict__ zetay) {
    spline_dense_body(g, Q, psi, zeta, psiy, zetay, blockIdx.x, blockIdx.y, blockIdx.z);
}

// Source record (64 B): x, zeta, zeta_x, zeta_y, w psi, w, w zeta_x, -
// FP32 source record (32 B): i (exact), zeta, zeta_x, zeta_y, w psi, w, w zeta_x, -
// Collocation record (64 B): x*, y*, zeta*, psi*, zeta_x*, zeta_y*, E2 local part, -
// Eight lanes per grid point: lane 0 writes the source record and, for a collocation
// point, E1 and the collocation record; the eight log integrals of the closed-form I
// are spread over the eight lanes and added by shuffles.
__device__ __forceinline__ void points_body(const Geo& g, const double* __restrict__ u,
                                            const double* __restrict__ psi,
                                            const double* __restrict__ zeta,
                                            const double* __restrict__ psiy,
                                            const double* __restrict__ zetay,
                                            double* __restrict__ src64, float* __restrict__ src32,
                                            double* __restrict__ col, double* __restrict__ E,
                                            int bx) {
    const int tid = bx * 256 + threadIdx.x;
    const int gi = tid >> 3, sub = tid & 7;
    const bool live = gi < g.NM;  // no early exit: the eight lanes shuffle below
    const int gs = live ? gi : 0;
    const int l = gs / g.N;
    const int k = gs - l * g.N;
    const double* phx = u;
    const double* zx = u + g.NM;
    const double w = g.dx * g.dy * weight1d(k, g.N, g.weights) * weight1d(l, g.M, g.weights);
    const double ps = psi[gs], ze = zeta[gs], zxv = zx[gs], zyv = zetay[gs];
    if (live && sub == 0) {
        double* r = src64 + (size_t)gs * 8;
        const double x = g.x1 + k * g.dx;
        reinterpret_cast<double4*>(r)[0] = make_double4(x, ze, zxv, zyv);
        reinterpret_cast<double4*>(r)[1] = make_double4(w * ps, w, w * zxv, 0.0);
        if (g.precision == SW_PREC_FP32) {
            float* sp = src32 + (size_t)gs * 8;
            reinterpret_cast<float4*>(sp)[0] =
                make_float4((float)k, (float)ze, (float)zxv, (float)zyv);
            reinterpret_cast<float4*>(sp)[1] =
                make_float4((float)(w * ps), (float)w, (float)(w * zxv), 0.0f);
        }
    }
    const bool colpt = live && k < g.N - 1;
    const int g1 = colpt ? gs + 1 : gs;
    const double zs = 0.5 * (ze + zeta[g1]);
    const double zxs = 0.5 * (zxv + zx[g1]);
    const double zys = 0.5 * (zyv + zetay[g1]);
    const double den = 1.0 + zxs * zxs + zys * zys;
    // singular-part quadratic form and its exact integral
    const double A = 1.0 + zxs * zxs, B = 2.0 * zxs * zys, C = 1.0 + zys * zys;
    const double xs = g.x1 + (k + 0.5) * g.dx;
    const double ys = l * g.dy;
    double part = colpt ? closed_form_I_part(sub >> 1, sub & 1, A, B, C, 4.0 * den, xs - g.x1,
                                             g.xN - xs, ys, g.yM)
                        : 0.0;
    part += __shfl_xor(part, 1, 8);
    part += __shfl_xor(part, 2, 8);
    part += __shfl_xor(part, 4, 8);
    if (!colpt || sub != 0) return;
    const double I = part;
    const int c = l * g.Nc + k;
    const double pxs = 0.5 * ((phx[gs] - 1.0) + (phx[g1] - 1.0));
    const double pss = 0.5 * (ps + psi[g1]);
    const double pys = 0.5 * (psiy[gs] + psiy[g1]);
    // E1: Bernoulli condition with phi_x* = 1 + psi_x*, phi_y* = psi_y*
    const double fx = 1.0 + pxs, fy = pys;
    const double num = (1.0 + zxs * zxs) * fy * fy + (1.0 + zys * zys) * fx * fx -
                       2.0 * zxs * zys * fx * fy;
    E[(size_t)l * g.N + k + 1] = 0.5 * num / den + zs / (g.F * g.F) - 0.5;
    const double zp1 = zs + 1.0;
    const double srcterm = g.eps / sqrt(xs * xs + ys * ys + zp1 * zp1);
    const double base = kTwoPi * pss + srcterm - zxs * I;
    double* r = col + (size_t)c * 8;
    reinterpret_cast<double4*>(r)[0] = make_double4(xs, ys, zs, pss);
    reinterpret_cast<double4*>(r)[1] = make_double4(zxs, zys, base, 0.0);
}

__global__ __launch_bounds__(256) void k_points(Geo g, const double* __restrict__ u,
                                                const double* __restrict__ psi,
                                                const double* __restrict__ zeta,
                                                const double* __restrict__ psiy,
                                                const double* __restrict__ zetay,
                                                double* __restrict__ src64,
                                                float* __restrict__ src32,
                                                double* __restrict__ col,
                                                double* __restrict__ E) {
    points_body(g, u, psi, zeta, psiy, zetay, src64, src32, col, E, blockIdx.x);
}

// ---- a5: the all-pairs sum ----------------------------------------------------------
// 2/sqrt(x) in FP64: hardware estimate y0 plus one Newton-Raphson step written as
// y0 (3 - x y0^2), which is twice the refined 1/sqrt(x) (relative error 1.5 e0^2 for
// an estimate error e0) in three operations; the factors of 2 are taken out of the
// row sums once per collocation point.
__device__ __forceinline__ double rsq2_64(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    return y * fma(-x * y, y, 3.0);
}

constexpr int kPairThreads = 256;
// source records staged in LDS at a time (64 KB of FP64 records, 32 KB of FP32 ones)
constexpr int kPairSeg = 1024;
#ifndef SW_UNROLL64
#define SW_UNROLL64 2  // source points per FP64 inner-loop iteration
#endif
#ifndef SW_PAIR_TARGET
#define SW_PAIR_TARGET 2048  // blocks per pair launch
#endif
#ifndef SW_WPE64
#define SW_WPE64 1  // minimum waves per SIMD asked of the FP64 pair kernels' register use
#endif

template <int CP>
__device__ __forceinline__ void pairs_f64_body(const Geo& g, const double* __restrict__ src,
                                               const double* __restrict__ col,
                                               double* __restrict__ partial, int tile, int chunk,
                                               int G, double* lds) {
    const int tid = threadIdx.x;
    const int N = g.N;
    // this chunk's sources: a contiguous range of the row-major source index
    const int s0 = (int)((long long)chunk * g.NM / G);
    const int s1 = (int)((long long)(chunk + 1) * g.NM / G);
    double xs[CP], zs[CP], ps[CP], zxs[CP], A[CP], B[CP], C[CP];
    double acc1[CP], acc2[CP], acc3[CP];
    int idx[CP], lrow[CP];
#pragma unroll
    for (int c = 0; c < CP; ++c) {
        idx[c] = tile * kPairThreads * CP + c * kPairThreads + tid;
        const int li = min(idx[c], g.ncol - 1);
        lrow[c] = li / g.Nc;
        const double4 r0 = reinterpret_cast<const double4*>(col + (size_t)li * 8)[0];
        const double4 r1 = reinterpret_cast<const double4*>(col + (size_t)li * 8)[1];
        xs[c] = r0.x;
        zs[c] = r0.z;
        ps[c] = r0.w;
        zxs[c] = r1.x;
        const double zy = r1.y;
        A[c] = 1.0 + r1.x * r1.x;
        B[c] = 2.0 * r1.x * zy;
        C[c] = 1.0 + zy * zy;
        acc1[c] = acc2[c] = acc3[c] = 0.0;
    }
    for (int j = s0 / N; j * N < s1; ++j) {
        const int i0 = max(0, s0 - j * N), i1 = min(N, s1 - j * N);
        double dy[CP], dyp[CP], dy2[CP], ddy[CP], Bdy[CP], mBdyp[CP], Cdy2[CP], Cdyp2[CP];
#pragma unroll
        for (int c = 0; c < CP; ++c) {
            dy[c] = (double)(j - lrow[c]) * g.dy;
            dyp[c] = (double)(j + lrow[c]) * g.dy;
            dy2[c] = dy[c] * dy[c];
            // (y + y*)^2 - (y - y*)^2 = 4 j l dy^2: the image distance from the direct one
            ddy[c] = (double)(4 * j * lrow[c]) * (g.dy * g.dy);
            Bdy[c] = B[c] * dy[c];
            mBdyp[c] = -B[c] * dyp[c];
            Cdy2[c] = C[c] * dy2[c];
            Cdyp2[c] = C[c] * (dyp[c] * dyp[c]);
        }
        // the row's sources in segments of at most kPairSeg records (one segment for
        // N <= kPairSeg)
        for (int a = i0; a < i1; a += kPairSeg) {
        const int b = min(i1, a + kPairSeg);
        __syncthreads();
        {
            const double2* srow =
                reinterpret_cast<const double2*>(src + ((size_t)j * N + a) * 8);
            double2* dst = reinterpret_cast<double2*>(lds);
            for (int t = tid; t < (b - a) * 4; t += kPairThreads) dst[t] = srow[t];
        }
        __syncthreads();
#pragma unroll SW_UNROLL64
        for (int i = a; i < b; ++i) {
            const double4 r0 = reinterpret_cast<const double4*>(lds + (i - a) * 8)[0];
            const double4 r1 = reinterpret_cast<const double4*>(lds + (i - a) * 8)[1];
            const double sx = r0.x, sz = r0.y, szx = r0.z, szy = r0.w;
            const double swp = r1.x, sw = r1.y, swzx = r1.z;
#pragma unroll
            for (int c = 0; c < CP; ++c) {
                const double dx = sx - xs[c];
                const double dz = sz - zs[c];
                const double rr = fma(dx, dx, fma(dz, dz, dy2[c]));
                // doubled reciprocal distances: i = 2/r, and the sum j1s + j2s of the
                // doubled 2/sqrt(q), whose last Newton products share one fma
                const double i1 = rsq2_64(rr);
                const double i2 = rsq2_64(rr + ddy[c]);
                const double q1 = fma(dx, fma(A[c], dx, Bdy[c]), Cdy2[c]);
                const double q2 = fma(dx, fma(A[c], dx, mBdyp[c]), Cdyp2[c]);
                const double y1 = __builtin_amdgcn_rsq(q1);
                const double y2 = __builtin_amdgcn_rsq(q2);
                const double f1 = fma(-q1 * y1, y1, 3.0);
                const double f2 = fma(-q2 * y2, y2, 3.0);
                const double js = fma(y1, f1, y2 * f2);
                const double n0 = fma(-dx, szx, dz);
                const double n1 = fma(-dy[c], szy, n0);
                const double n2 = fma(-dyp[c], szy, n0);
                const double K1 = fma(n1, i1 * i1 * i1, n2 * (i2 * i2 * i2));
                const double wd = fma(-sw, ps[c], swp);
                acc1[c] = fma(wd, K1, acc1[c]);
                acc2[c] = fma(swzx, i1 + i2, acc2[c]);
                acc3[c] = fma(sw, js, acc3[c]);
            }
        }
        }
    }
#pragma unroll
    for (int c = 0; c < CP; ++c)
        if (idx[c] < g.ncol)
            partial[(size_t)chunk * g.ncol + idx[c]] =
                fma(0.125, acc1[c], 0.5 * fma(-zxs[c], acc3[c], acc2[c]));
}

template <int CP>
__global__ __launch_bounds__(kPairThreads) __attribute__((amdgpu_waves_per_eu(SW_WPE64))) void k_pairs_f64(Geo g, const double* __restrict__ src,
                                                            const double* __restrict__ col,
                                                            double* __restrict__ partial,
                                                            int ntiles, int G) {
    extern __shared__ double lds[];
    const int w = xcd_remap(blockIdx.x, gridDim.x);
    pairs_f64_body<CP>(g, src, col, partial, w % ntiles, w / ntiles, G, lds);
}

// FP32 pair sum: the same terms in single precision.  Offsets come from exact
// integers (i - k - 1/2 and j -+ l are exact in FP32), so the nearest pairs
// keep full relative accuracy.  Each source row is summed in FP32 and the row
// sums are added with Kahan compensation.
__device__ __forceinline__ void kahan_add(float& s, float& comp, float v) {
    const float y = __fsub_rn(v, comp);
    const float t = __fadd_rn(s, y);
    comp = __fsub_rn(__fsub_rn(t, s), y);
    s = t;
}

template <int CP>
__device__ __forceinline__ void pairs_f32_body(const Geo& g, const float* __restrict__ src,
                                               const double* __restrict__ col,
                                               double* __restrict__ partial, int tile, int chunk,
                                               int G, float* lds) {
    const int tid = threadIdx.x;
    const int N = g.N;
    const int lo = (int)((long long)chunk * g.NM / G);
    const int hi = (int)((long long)(chunk + 1) * g.NM / G);
    const float fdx = (float)g.dx;
    float t0[CP], zs[CP], ps[CP], zxs[CP], A[CP], B[CP], C[CP];
    float S[CP], comp[CP];
    int idx[CP], lrow[CP];
#pragma unroll
    for (int c = 0; c < CP; ++c) {
        idx[c] = tile * kPairThreads * CP + c * kPairThreads + tid;
        const int li = min(idx[c], g.ncol - 1);
        lrow[c] = li / g.Nc;
        const int kc = li - lrow[c] * g.Nc;
        t0[c] = -((float)kc + 0.5f);
        const double4 r0 = reinterpret_cast<const double4*>(col + (size_t)li * 8)[0];
        const double4 r1 = reinterpret_cast<const double4*>(col + (size_t)li * 8)[1];
        zs[c] = (float)r0.z;
        ps[c] = (float)r0.w;
        zxs[c] = (float)r1.x;
        A[c] = (float)(1.0 + r1.x * r1.x);
        B[c] = (float)(2.0 * r1.x * r1.y);
        C[c] = (float)(1.0 + r1.y * r1.y);
        S[c] = comp[c] = 0.0f;
    }
    for (int j = lo / N; j * N < hi; ++j) {
        const int i0 = max(0, lo - j * N), i1 = min(N, hi - j * N);
        float dy[CP], dyp[CP], dy2[CP], ddy[CP], Bdy[CP], mBdyp[CP], Cdy2[CP], Cdyp2[CP];
        float r1[CP], r2[CP], r3[CP];
#pragma unroll
        for (int c = 0; c < CP; ++c) {
            dy[c] = (float)(j - lrow[c]) * (float)g.dy;
            dyp[c] = (float)(j + lrow[c]) * (float)g.dy;
            dy2[c] = dy[c] * dy[c];
            ddy[c] = (float)(4 * j * lrow[c]) * ((float)g.dy * (float)g.dy);
            Bdy[c] = B[c] * dy[c];
            mBdyp[c] = -B[c] * dyp[c];
            Cdy2[c] = C[c] * dy2[c];
            Cdyp2[c] = C[c] * (dyp[c] * dyp[c]);
            r1[c] = r2[c] = r3[c] = 0.0f;
        }
        for (int a = i0; a < i1; a += kPairSeg) {
        const int b = min(i1, a + kPairSeg);
        __syncthreads();
        {
            const float4* srow = reinterpret_cast<const float4*>(src + ((size_t)j * N + a) * 8);
            float4* dst = reinterpret_cast<float4*>(lds);
            for (int t = tid; t < (b - a) * 2; t += kPairThreads) dst[t] = srow[t];
        }
        __syncthreads();
#pragma unroll 2
        for (int i = a; i < b; ++i) {
            const float4 s0 = reinterpret_cast<const float4*>(lds + (i - a) * 8)[0];
            const float4 s1 = reinterpret_cast<const float4*>(lds + (i - a) * 8)[1];
#pragma unroll
            for (int c = 0; c < CP; ++c) {
                const float dx = (s0.x + t0[c]) * fdx;
                const float dz = s0.y - zs[c];
                const float rr = fmaf(dx, dx, fmaf(dz, dz, dy2[c]));
                const float i1 = __builtin_amdgcn_rsqf(rr);
                const float i2 = __builtin_amdgcn_rsqf(rr + ddy[c]);
                const float q1 = fmaf(dx, fmaf(A[c], dx, Bdy[c]), Cdy2[c]);
                const float q2 = fmaf(dx, fmaf(A[c], dx, mBdyp[c]), Cdyp2[c]);
                const float j1s = __builtin_amdgcn_rsqf(q1);
                const float j2s = __builtin_amdgcn_rsqf(q2);
                const float n0 = fmaf(-dx, s0.z, dz);
                const float n1 = fmaf(-dy[c], s0.w, n0);
                const float n2 = fmaf(-dyp[c], s0.w, n0);
                const float K1 = fmaf(n1, i1 * i1 * i1, n2 * (i2 * i2 * i2));
                const float wd = fmaf(-s1.y, ps[c], s1.x);
                r1[c] = fmaf(wd, K1, r1[c]);
                r2[c] = fmaf(s1.z, i1 + i2, r2[c]);
                r3[c] = fmaf(s1.y, j1s + j2s, r3[c]);
            }
        }
        }
#pragma unroll
        for (int c = 0; c < CP; ++c) kahan_add(S[c], comp[c], (r1[c] + r2[c]) - zxs[c] * r3[c]);
    }
#pragma unroll
    for (int c = 0; c < CP; ++c)
        if (idx[c] < g.ncol)
            partial[(size_t)chunk * g.ncol + idx[c]] = (double)S[c] - (double)comp[c];
}

template <int CP>
__global__ __launch_bounds__(kPairThreads) void k_pairs_f32(Geo g, const float* __restrict__ src,
                                                            const double* __restrict__ col,
                                                            double* __restrict__ partial,
                                                            int ntiles, int G) {
    extern __shared__ float ldsf[];
    const int w = xcd_remap(blockIdx.x, gridDim.x);
    pairs_f32_body<CP>(g, src, col, partial, w % ntiles, w / ntiles, G, ldsf);
}

// Batched all-pairs launch: a work list of (problem, collocation tile, source
// chunk) items over several problems, each problem with its own geometry and
// buffers.  Every item runs the same body as the single-problem launch with
// the same tile/chunk split, so each problem's partial sums are bitwise those
// of its own launch.
struct PairProb {
    Geo g;
    const void* src;
    const double* col;
    double* partial;
    int ntiles;
    int G;
    int first_block;  // first work-list index of this problem
    int pad;
};
constexpr int kMaxBatch = 24;  // keeps the kernel argument block under 4 KB
struct PairBatch {
    PairProb p[kMaxBatch];
    int nprob;
    int total;
};

template <int CP>
__global__ __launch_bounds__(kPairThreads) __attribute__((amdgpu_waves_per_eu(SW_WPE64))) void k_pairs_f64_batched(PairBatch b) {
    extern __shared__ double lds[];
    const int w = xcd_remap(blockIdx.x, gridDim.x);
    int q = 0;
    while (q + 1 < b.nprob && w >= b.p[q + 1].first_block) ++q;
    const PairProb& pp = b.p[q];
    const int local = w - pp.first_block;
    pairs_f64_body<CP>(pp.g, static_cast<const double*>(pp.src), pp.col, pp.partial,
                       local % pp.ntiles, local / pp.ntiles, pp.G, lds);
}

template <int CP>
__global__ __launch_bounds__(kPairThreads) void k_pairs_f32_batched(PairBatch b) {
    extern __shared__ float ldsf[];
    const int w = xcd_remap(blockIdx.x, gridDim.x);
    int q = 0;
    while (q + 1 < b.nprob && w >= b.p[q + 1].first_block) ++q;
    const PairProb& pp = b.p[q];
    const int local = w - pp.first_block;
    pairs_f32_body<CP>(pp.g, static_cast<const float*>(pp.src), pp.col, pp.partial,
                       local % pp.ntiles, local / pp.ntiles, pp.G, ldsf);
}

// ---- a6: E2 assembly ---------------------------------------------------------------------
__device__ __forceinline__ void finish_body(const Geo& g, const double* __restrict__ col,
                                            const double* __restrict__ partial, int G,
                                            double* __restrict__ E, int bx) {
    const int c = bx * 256 + threadIdx.x;
    if (c >= g.ncol) return;
    double t[8] = {};  // eight independent chains: eight loads in flight
    int q = 0;
    for (; q + 7 < G; q += 8)
#pragma unroll
        for (int e = 0; e < 8; ++e) t[e] += partial[(size_t)(q + e) * g.ncol + c];
    for (; q < G; ++q) t[0] += partial[(size_t)q * g.ncol + c];
    const double s = ((t[0] + t[1]) + (t[2] + t[3])) + ((t[4] + t[5]) + (t[6] + t[7]));
    const int l = c / g.Nc;
    const int k = c - l * g.Nc;
    E[(size_t)g.NM + (size_t)l * g.N + k + 1] = col[(size_t)c * 8 + 6] - s;
}

__global__ __launch_bounds__(256) void k_finish(Geo g, const double* __restrict__ col,
                                                const double* __restrict__ partial, int G,
                                                double* __restrict__ E) {
    finish_body(g, col, partial, G, E, blockIdx.x);
}

// The prelude and finish of several residuals in one launch each: block b runs block
// b - first[kind] of the problem it falls in, with the single launch's block shape.
struct PreProb {
    Geo g;
    const double* u;
    double* E;
    double* psi;
    double* zeta;
    double* psiy;
    double* zetay;
    double* src64;
    float* src32;
    double* col;
    const double* Q;  // dense spline operator
    const double* partial;
    int G;
    int first[4];  // first block in the scan, spline, points and finish launches
};
constexpr int kMaxPre = 18;  // keeps the kernel argument block under 4 KB
struct PreBatch {
    PreProb p[kMaxPre];
    int nprob;
};
static_assert(sizeof(PreBatch) <= 4096, "kernel argument block");

__device__ __forceinline__ int pre_find(const PreBatch& b, int kind, int blk) {
    int q = 0;
    while (q + 1 < b.nprob && blk >= b.p[q + 1].first[kind]) ++q;
    return q;
}

__global__ __launch_bounds__(64) void k_scan_batched(PreBatch b) {
    const PreProb& P = b.p[pre_find(b, 0, blockIdx.x)];
    const int local = blockIdx.x - P.first[0];
    scan_body(P.g, P.u, P.psi, P.zeta, P.E, local % P.g.M, local / P.g.M);
}

__global__ __launch_bounds__(128) void k_spline_dense_batched(PreBatch b) {
    const PreProb& P = b.p[pre_find(b, 1, blockIdx.x)];
    const int local = blockIdx.x - P.first[1];
    const int nbx = (P.g.N + 127) / 128;
    spline_dense_body(P.g, P.Q, P.psi, P.zeta, P.psiy, P.zetay, local % nbx,
                      (local / nbx) % P.g.M, local / (nbx * P.g.M));
}

__global__ __launch_bounds__(256) void k_points_batched(PreBatch b) {
    const PreProb& P = b.p[pre_find(b, 2, blockIdx.x)];
    points_body(P.g, P.u, P.psi, P.zeta, P.psiy, P.zetay, P.src64, P.src32, P.col, P.E,
                blockIdx.x - P.first[2]);
}

__global__ __launch_bounds__(256) void k_finish_batched(PreBatch b) {
    const PreProb& P = b.p[pre_find(b, 3, blockIdx.x)];
    finish_body(P.g, P.col, P.partial, P.G, P.E, blockIdx.x - P.first[3]);
}

// zeta on the grid from the zeta_x half of u: one wavefront per row, the same scan (and
// summation order) as the zeta half of k_scan, so the result equals the zeta that the
// residual uses.
__global__ __launch_bounds__(64) void k_zeta_rows(Geo g, const double* __restrict__ u,
                                                  double* __restrict__ zeta) {
    const int l = blockIdx.x;
    const int lane = threadIdx.x;
    const int N = g.N;
    const double* in = u + g.NM + (size_t)l * N;
    double* out = zeta + (size_t)l * N;
    const double hdx = 0.5 * g.dx;
    const int K = (N + 63) / 64;
    const int a = min(lane * K, N);
    const int b = min(a + K, N);
    double tot = 0.0;
    for (int m = a; m < b && m < N - 1; ++m) tot += hdx * (in[m] + in[m + 1]);
    double incl = tot;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const double t = __shfl_up(incl, d, 64);
        if (lane >= d) incl += t;
    }
    double excl = __shfl_up(incl, 1, 64);
    if (lane == 0) excl = 0.0;
    double val = (-g.x1 / g.nu) * in[0] + excl;
    for (int k = a; k < b; ++k) {
        out[k] = val;
        if (k < N - 1) val += hdx * (in[k] + in[k + 1]);
    }
}

// Collocation points per lane (register blocking of the pair loop).
#ifndef SW_CP64
#define SW_CP64 2
#endif
#ifndef SW_CP32
#define SW_CP32 2
#endif
constexpr int kCP64 = SW_CP64;
constexpr int kCP32 = SW_CP32;

}  // namespace

// Dense spline slope operators, cached per (device, M, end condition); NULL for
// M above kMaxDenseSplineM (then the tridiagonal sweep per column is used).
const double* spline_operator(int M, int bc, hipStream_t s) {
    if (M > kMaxDenseSplineM) return nullptr;
    static std::mutex mu;
    static std::map<std::tuple<int, int, int>, double*> cache;
    int dev = -1;
    SW_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    auto key = std::make_tuple(dev, M, bc);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    double* Q = nullptr;
    if (hipMalloc(&Q, (size_t)M * M * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        throw Error{SW_ENOMEM, "device allocation of the spline operator failed"};
    }
    k_spline_operator<<<(M + 63) / 64, 64, 0, s>>>(M, bc, Q);
    SW_HIP(hipGetLastError());
    SW_HIP(hipStreamSynchronize(s));  // other streams may read it right away
    cache[key] = Q;
    return Q;
}

int choose_chunks(const Geo& g) {
    const int cp = (g.precision == SW_PREC_FP32) ? kCP32 : kCP64;
    const int ntiles = (g.ncol + kPairThreads * cp - 1) / (kPairThreads * cp);
    // About 2048 equal blocks (two full rounds at four 256-thread blocks per CU), twice
    // that once there are many collocation tiles (finer chunks balance better there:
    // measured 4-5% at 361x121 and 721x241, 3% slower at 181x61).  A chunk keeps at
    // least 64 sources so that staging it in LDS pays off.
    const int target = (ntiles >= 64) ? 2 * SW_PAIR_TARGET : SW_PAIR_TARGET;
    const int G = (target + ntiles / 2) / ntiles;
    return std::max(1, std::min(G, g.NM / 64));
}

size_t residual_scratch_bytes(const Geo& g, int G) {
    const size_t NM = g.NM, nc = g.ncol;
    return carve_size({4 * NM * 8, NM * 64, (g.precision == SW_PREC_FP32 ? NM * 32 : 0), nc * 64,
                       (size_t)G * nc * 8, (size_t)2 * g.M * 8});
}

ResidualBufs carve_residual(Carve& c, const Geo& g, int G) {
    ResidualBufs b{};
    const size_t NM = g.NM, nc = g.ncol;
    double* grid = c.take<double>(4 * NM);
    b.psi = grid;
    b.zeta = grid + NM;
    b.psiy = grid + 2 * NM;
    b.zetay = grid + 3 * NM;
    b.src64 = c.take<double>(NM * 8);
    b.src32 = c.take<float>(g.precision == SW_PREC_FP32 ? NM * 8 : 0);
    b.col = c.take<double>(nc * 8);
    b.partial = c.take<double>((size_t)G * nc);
    b.spl = c.take<double>((size_t)2 * g.M);
    b.G = G;
    return b;
}

namespace {
void prelude(const Geo& g, const double* u, double* E, const ResidualBufs& b, hipStream_t s,
             bool dense_spline = true);
}

void residual_enqueue(const Geo& g, const double* u, double* E, const ResidualBufs& b,
                      hipStream_t s) {
    prelude(g, u, E, b, s);
    const ProfileMark pm = profile_begin(s);
    if (g.precision == SW_PREC_FP32) {
        const int ntiles = (g.ncol + kPairThreads * kCP32 - 1) / (kPairThreads * kCP32);
        k_pairs_f32<kCP32><<<ntiles * b.G, kPairThreads, (size_t)std::min(g.N, kPairSeg) * 32, s>>>(
            g, b.src32, b.col, b.partial, ntiles, b.G);
    } else {
        const int ntiles = (g.ncol + kPairThreads * kCP64 - 1) / (kPairThreads * kCP64);
        k_pairs_f64<kCP64><<<ntiles * b.G, kPairThreads, (size_t)std::min(g.N, kPairSeg) * 64, s>>>(
            g, b.src64, b.col, b.partial, ntiles, b.G);
    }
    profile_end(pm, s, (double)g.ncol * (double)g.NM);
    k_finish<<<(g.ncol + 255) / 256, 256, 0, s>>>(g, b.col, b.partial, b.G, E);
    SW_HIP(hipGetLastError());
}

void residual_enqueue_fixed(const Geo& g, const double* u, double* E, const ResidualBufs& b,
                            hipStream_t s) {
    // the same kernels as residual_enqueue, except that the spline slopes come from the
    // per-column sweep (its coefficients live in b.spl), not the cached dense operator,
    // and the launches are not timed: nothing is allocated or created
    prelude(g, u, E, b, s, false);
    if (g.precision == SW_PREC_FP32) {
        const int ntiles = (g.ncol + kPairThreads * kCP32 - 1) / (kPairThreads * kCP32);
        k_pairs_f32<kCP32><<<ntiles * b.G, kPairThreads, (size_t)std::min(g.N, kPairSeg) * 32, s>>>(
            g, b.src32, b.col, b.partial, ntiles, b.G);
    } else {
        const int ntiles = (g.ncol + kPairThreads * kCP64 - 1) / (kPairThreads * kCP64);
        k_pairs_f64<kCP64><<<ntiles * b.G, kPairThreads, (size_t)std::min(g.N, kPairSeg) * 64, s>>>(
            g, b.src64, b.col, b.partial, ntiles, b.G);
    }
    k_finish<<<(g.ncol + 255) / 256, 256, 0, s>>>(g, b.col, b.partial, b.G, E);
    SW_HIP(hipGetLastError());
}

namespace {
void prelude(const Geo& g, const double* u, double* E, const ResidualBufs& b, hipStream_t s,
             bool dense_spline) {
    k_scan<<<dim3(g.M, 2), 64, 0, s>>>(g, u, b.psi, b.zeta, E);
    if (const double* Q = dense_spline ? spline_operator(g.M, g.bc, s) : nullptr) {
        k_spline_dense<<<dim3((g.N + 127) / 128, g.M, 2), 128, 0, s>>>(g, Q, b.psi, b.zeta,
                                                                       b.psiy, b.zetay);
    } else {
        k_spline_setup<<<1, 1, 0, s>>>(g.M, g.bc, b.spl);
        k_spline<<<(2 * g.N + 127) / 128, 128, 0, s>>>(g, b.spl, b.psi, b.zeta, b.psiy, b.zetay);
    }
    k_points<<<(unsigned)((8 * (size_t)g.NM + 255) / 256), 256, 0, s>>>(
        g, u, b.psi, b.zeta, b.psiy, b.zetay, b.src64,
                                                 b.src32, b.col, E);
}
}  // namespace

void residual_batched_enqueue(int nb, const Geo* g, const double* const* u, double* const* E,
                              hipStream_t s) {
    // scratch for all problems
    std::vector<int> G(nb);
    std::vector<size_t> off(nb + 1, 0);
    for (int i = 0; i < nb; ++i) {
        G[i] = choose_chunks(g[i]);
        off[i + 1] = off[i] + residual_scratch_bytes(g[i], G[i]);
    }
    Scratch& sc = scratch_for(s, 3);
    sc.ensure(off[nb] + 256);
    std::vector<ResidualBufs> bufs(nb);
    std::vector<const double*> Q(nb, nullptr);
    bool batch_pre = true;  // every problem has the dense spline operator
    for (int i = 0; i < nb; ++i) {
        Carve c(static_cast<char*>(sc.base) + off[i]);
        bufs[i] = carve_residual(c, g[i], G[i]);
        Q[i] = spline_operator(g[i].M, g[i].bc, s);
        batch_pre = batch_pre && Q[i];
    }
    // the preludes of up to kMaxPre problems per launch of each of their three kernels
    // (a lone residual's launches, run as one), else one problem at a time
    auto pre_batches = [&](auto&& launch) {
        for (int i0 = 0; i0 < nb; i0 += kMaxPre) {
            PreBatch pb{};
            int tot[4] = {0, 0, 0, 0};
            for (int i = i0; i < std::min(nb, i0 + kMaxPre); ++i) {
                PreProb& pp = pb.p[pb.nprob++];
                pp = PreProb{g[i], u[i], E[i], bufs[i].psi, bufs[i].zeta, bufs[i].psiy,
                             bufs[i].zetay, bufs[i].src64, bufs[i].src32, bufs[i].col, Q[i],
                             bufs[i].partial, G[i], {tot[0], tot[1], tot[2], tot[3]}};
                tot[0] += 2 * g[i].M;
                tot[1] += ((g[i].N + 127) / 128) * g[i].M * 2;
                tot[2] += (int)((8 * (size_t)g[i].NM + 255) / 256);
                tot[3] += (g[i].ncol + 255) / 256;
            }
            launch(pb, tot);
        }
    };
    if (batch_pre) {
        pre_batches([&](const PreBatch& pb, const int* tot) {
            k_scan_batched<<<tot[0], 64, 0, s>>>(pb);
            k_spline_dense_batched<<<tot[1], 128, 0, s>>>(pb);
            k_points_batched<<<tot[2], 256, 0, s>>>(pb);
        });
    } else {
        for (int i = 0; i < nb; ++i) prelude(g[i], u[i], E[i], bufs[i], s);
    }
    const ProfileMark pm = profile_begin(s);
    double pairs = 0.0;
    for (int prec = 0; prec < 2; ++prec) {
        const int cp = (prec == SW_PREC_FP32) ? kCP32 : kCP64;
        PairBatch batch{};
        int maxN = 0;
        auto flush = [&]() {
            if (batch.nprob == 0) return;
            const size_t lds = (size_t)std::min(maxN, kPairSeg) * (prec == SW_PREC_FP32 ? 32 : 64);
            if (prec == SW_PREC_FP32)
                k_pairs_f32_batched<kCP32><<<batch.total, kPairThreads, lds, s>>>(batch);
            else
                k_pairs_f64_batched<kCP64><<<batch.total, kPairThreads, lds, s>>>(batch);
            batch = PairBatch{};
            maxN = 0;
        };
        for (int i = 0; i < nb; ++i) {
            if (g[i].precision != prec) continue;
            if (batch.nprob == kMaxBatch) flush();
            PairProb& pp = batch.p[batch.nprob++];
            pp.g = g[i];
            pp.src = (prec == SW_PREC_FP32) ? static_cast<const void*>(bufs[i].src32)
                                             : static_cast<const void*>(bufs[i].src64);
            pp.col = bufs[i].col;
            pp.partial = bufs[i].partial;
            pp.ntiles = (g[i].ncol + kPairThreads * cp - 1) / (kPairThreads * cp);
            pp.G = G[i];
            pp.first_block = batch.total;
            batch.total += pp.ntiles * pp.G;
            maxN = std::max(maxN, g[i].N);
            pairs += (double)g[i].ncol * (double)g[i].NM;
        }
        flush();
    }
    profile_end(pm, s, pairs);
    if (batch_pre) {
        pre_batches([&](const PreBatch& pb, const int* tot) {
            k_finish_batched<<<tot[3], 256, 0, s>>>(pb);
        });
    } else {
        for (int i = 0; i < nb; ++i)
            k_finish<<<(g[i].ncol + 255) / 256, 256, 0, s>>>(g[i], bufs[i].col,
                                                            bufs[i].partial, G[i], E[i]);
    }
    SW_HIP(hipGetLastError());
}

void zeta_enqueue(const Geo& g, const double* u, double* zeta, hipStream_t s) {
    k_zeta_rows<<<g.M, 64, 0, s>>>(g, u, zeta);
    SW_HIP(hipGetLastError());
}

}  // namespace sw
