// Device helpers shared by the residual and preconditioner kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/shipwave.h"

namespace sw {

// Workgroups are dispatched round-robin over the 8 XCDs of the chip.  Map the
// hardware block id to a work id such that each XCD receives a contiguous
// range of work ids (and hence a contiguous range of source chunks, which then
// share that XCD's L2).  Bijective on [0, nblocks).
__device__ __forceinline__ int xcd_remap(int b, int nblocks) {
    constexpr int kXcd = 8;
    const int xcd = b % kXcd;
    const int idx = b / kXcd;
    const int base = nblocks / kXcd;
    const int rem = nblocks % kXcd;
    return xcd * base + min(xcd, rem) + idx;
}

__device__ __forceinline__ double weight1d(int i, int n, int rule) {
    if (rule == SW_WEIGHTS_TRAPEZOID) return (i == 0 || i == n - 1) ? 0.5 : 1.0;
    if (i == 0 || i == n - 1) return 1.0 / 3.0;
    return (i & 1) ? 4.0 / 3.0 : 2.0 / 3.0;
}

// ---- a4: closed form of I -----------------------------------------------------------
// L(P,B,R;t) = int_0^t ds / sqrt(P s^2 + B s + R) = P^{-1/2} ln((2 sqrt(P) q(t) + 2Pt + B) /
// (2 sqrt(PR) + B)), q(t) = sqrt(P t^2 + B t + R); a negative 2Pt + B (or B) is
// handled through the conjugate (4PR - B^2) / (2 sqrt(P) q - 2Pt - B).
__device__ inline double lint(double P, double B, double R, double disc, double t) {
    const double sP = sqrt(P);
    const double q = sqrt(fma(fma(P, t, B), t, R));
    const double lin = fma(2.0 * P, t, B);
    const double top = (lin >= 0.0) ? fma(2.0 * sP, q, lin) : disc / fma(2.0 * sP, q, -lin);
    const double s0 = 2.0 * sqrt(P * R);
    const double bot = (B >= 0.0) ? s0 + B : disc / (s0 - B);
    return log(top / bot) / sP;
}

// G(a,b) = int_0^a int_0^b dY dX / sqrt(A X^2 + B X Y + C Y^2): the rectangle split on
// its diagonal, Y = tX below and X = sY above.
__device__ inline double grect(double A, double B, double C, double disc, double a, double b) {
    if (!(a > 0.0) || !(b > 0.0)) return 0.0;
    return a * lint(C, B, A, disc, b / a) + b * lint(A, B, C, disc, a / b);
}

// I = integral of the linearised kernel over the truncated domain plus its image.
// The direct part is four quadrants about the collocation point (x lengths a1 behind,
// a2 ahead; y lengths ys below, yM - ys above).  The image strip covers distances ys to
// ys + yM below, so its lower quadrants extend the direct ones from ys to yM + ys: the
// two lower direct quadrants cancel against the subtracted part of the image, leaving
// four rectangles.  Term m of closed_form_I is grect(A, sB_m B, C, disc, a_m, b_m) with
//   m = 0: (+, a2, yM - ys), 1: (-, a1, yM - ys), 2: (-, a2, yM + ys), 3: (+, a1, yM + ys).
__device__ inline double closed_form_I(double A, double B, double C, double disc, double a1, double a2,
                                double ys, double yM) {
    const double b2 = yM - ys, yt = yM + ys;
    return (grect(A, B, C, disc, a2, b2) + grect(A, -B, C, disc, a1, b2)) +
           (grect(A, -B, C, disc, a2, yt) + grect(A, B, C, disc, a1, yt));
}

// Half h (0 or 1) of rectangle term m of closed_form_I: grect's two log integrals
// are split over two lanes.
__device__ inline double closed_form_I_part(int m, int h, double A, double B, double C, double disc,
                                            double a1, double a2, double ys, double yM) {
    const double a = (m == 0 || m == 2) ? a2 : a1;
    const double b = (m < 2) ? yM - ys : yM + ys;
    const double sB = (m == 0 || m == 3) ? B : -B;
    if (!(a > 0.0) || !(b > 0.0)) return 0.0;
    return h == 0 ? a * lint(C, sB, A, disc, b / a) : b * lint(A, sB, C, disc, a / b);
}

// In-place inclusive prefix sum of arr[0..n) in LDS by one 64-lane wavefront
// (block of 64 threads): each lane sums a contiguous chunk, the chunk totals
// are scanned across the wave, then each lane rewrites its chunk.
__device__ inline void lds_prefix_sum(double* arr, int n) {
    const int lane = threadIdx.x;
    const int K = (n + 63) / 64;
    const int a = min(lane * K, n), b = min(a + K, n);
    double tot = 0.0;
    for (int i = a; i < b; ++i) tot += arr[i];
    double incl = tot;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const double t = __shfl_up(incl, d, 64);
        if (lane >= d) incl += t;
    }
    double run = __shfl_up(incl, 1, 64);
    if (lane == 0) run = 0.0;
    for (int i = a; i < b; ++i) {
        run += arr[i];
        arr[i] = run;
    }
    __syncthreads();
}

}  // namespace sw
