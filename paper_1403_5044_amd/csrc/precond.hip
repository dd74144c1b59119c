// Preconditioner from the linear Jacobian (preconditioning section, Appendix B
// entries PreA-PreD), stored, factorised and applied as in Appendix C.
//
//   P = [[A, B], [C, D_q]],  A = I (x) A-hat, B = I (x) T/F^2, C = I (x) 2 pi T,
//   A-hat: row 0 (E4) = (nu - x_1/dx, x_1/dx), row r >= 1 (E1) = 1/2 on columns r-1, r;
//   T[r][n] = d zeta*_{r-1} / d zeta_x,n (trapezoid integration from zeta_1 =
//   -(x_1/nu) zeta_x,1, then two-point averaging); T is applied as a scan, never stored.
//   D_q: the D blocks (l, m) with |l - m| <= q; row 0 of a diagonal block is the
//   E6 row, rows r >= 1 are -w(n,m) K3(n,m; k=r-1, l), plus (sum w K3 - I_lin)/2 on
//   columns k, k+1 of the diagonal block.
//   Schur complement S = D_q - I (x) Wc with Wc = (2 pi / F^2) T A-hat^{-1} T (one N x N
//   block, the same for every row l).
//
// S is factorised by block LU without pivoting between blocks (partial
// pivoting inside each N x N diagonal block, by Gauss-Jordan), eliminating the
// block rows in an order that starts at both ends of the band (make_order).
// Stored per block row l (2q+1 slots of N x N; slot q + c - l holds column c):
//   slot q:                       Dinv_l    = (updated diagonal block)^{-1}
//   column c eliminated before l: L_{l,c} = S~_{l,c} Dinv_c
//   column c eliminated after l:  G_{l,c} = Dinv_l S~_{l,c}
// so that, in elimination order,  forward  y_l = t_l - sum L_{l,c} y_c
//                  and in reverse, backward x_l = Dinv_l y_l - sum G_{l,c} x_c
// are block GEMVs.  q = 0 (block bandwidth 1) makes every block independent.
#include "band_plan.hpp"
#include "sw_device.hpp"
#include "sw_internal.hpp"

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <functional>
#include <mutex>
#include <vector>

namespace sw {
// One step of the super-row substitution: out rows of block row i are
//   out_i[r] = sum over t in [first[i], first[i+1]) of blk[t][r][:] . vec[t][:]
// (blk: N x N row-major operator blocks, vec: input blocks of length N).
struct SuperStep {
    int nrow;
    int first[kMaxSuperRows + 1];
    double* out[kMaxSuperRows];  // output block (N doubles) of each row
    const double* blk[kMaxSuperTerms];
    const double* vec[kMaxSuperTerms];
};

// One step of the block substitution with one block row per step (super rows of height 1):
// one or two independent block rows (a top-chain row and the bottom-chain row eliminated in
// the same factorisation step), out_i = add_i + sum over the row's terms of
// sign_t blk_t vec_t, the operator blocks read in place from the band factors.
constexpr int kMaxBandTerms = 64;
struct BandStep {
    int nrow;
    int first[3];
    const double* add[2];  // t_l (forward) or nullptr (backward)
    double* out[2];
    const double* blk[kMaxBandTerms];
    const double* vec[kMaxBandTerms];
    double sign[kMaxBandTerms];
};
}  // namespace sw

struct sw_precond {
    sw::Geo g;
    int q;
    int nb;
    double* base = nullptr;  // one allocation
    double* S = nullptr;     // [M][nb][N][N]
    double* Wc = nullptr;    // [N][N]
    double* k3 = nullptr;    // [ncol] sum w K3
    double* work = nullptr;  // [4][NM]
    double* tmp = nullptr;   // workspace of the diagonal-block inversion
    double* tmp2 = nullptr;  // [2q][N][N] products of one factorisation step
    int* info = nullptr;     // [2M] zero pivots seen, two per factorisation step
    void* terms = nullptr;   // device GemvTerm lists of the band substitution steps
    hipGraphExec_t subst = nullptr;  // the substitution launches, captured once
    std::vector<int> fwd_off, fwd_cnt, bwd_off, bwd_cnt;
    int sb = 0;                      // block rows per super row (0: one block row per step)
    double* W = nullptr;             // super-row operators (nonzero N x N blocks)
    std::vector<sw::SuperStep> fsteps, bsteps;  // kernel arguments of the super-row steps
    sw::SuperStep* dsteps = nullptr;            // device copy: fsteps, then bsteps
    std::vector<sw::BandStep> band_steps;       // forward then backward steps when sb <= 1
    std::vector<int> ord;                       // elimination order of the block rows
    size_t bytes = 0;
    size_t block = 0;  // size of the device block at base (>= bytes)
    int device = -1;
};

namespace sw {

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;

__device__ __forceinline__ double rsq_exact(double x) {
    // hardware estimate + two Newton steps: about 1 ulp
    double y = __builtin_amdgcn_rsq(x);
    double e = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    e = fma(-x * y, y, 1.0);
    return fma(0.5 * y, e, y);
}

// Wc[:, n] = (2 pi / F^2) T A-hat^{-1} T e_n; one thread per column.  The three sweeps
// down the column are recurrences and run together in registers:
//   t = T e_n:        z_0 = -(x_1/nu) [n = 0], z_r = z_{r-1} + dx/2 (e_{r-1} + e_r),
//                     t_0 = 0, t_r = (z_{r-1} + z_r)/2;
//   s = A-hat^{-1} t: s_0 = (t_0 - 2 a01 t_1) / (a00 - a01), s_r = 2 t_r - s_{r-1};
//   w = T s:          the same trapezoid recurrence on s, from -(x_1/nu) s_0.
__global__ void k_wmat(Geo g, double* __restrict__ Wc) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    const int N = g.N;
    const double hdx = 0.5 * g.dx;
    const double a01 = g.x1 / g.dx, a00 = g.nu - a01;
    const double scale = kTwoPi / (g.F * g.F);
    auto e = [n](int r) { return (r == n) ? 1.0 : 0.0; };
    // t_0 = 0 and t_1 from the first step of the T recurrence
    double z1 = (n == 0) ? (-g.x1 / g.nu) : 0.0;
    const double t1 = 0.5 * (z1 + (z1 + hdx * (e(0) + e(1))));
    // s_0 = (t_0 - 2 a01 t_1) / (a00 - a01), then s_r = 2 t_r - s_{r-1}
    double sp = (0.0 - 2.0 * a01 * t1) / (a00 - a01);
    double z3 = (-g.x1 / g.nu) * sp;
    Wc[n] = 0.0;
    for (int r = 1; r < N; ++r) {
        const double z1n = z1 + hdx * (e(r - 1) + e(r));
        const double t = 0.5 * (z1 + z1n);
        z1 = z1n;
        const double sr = 2.0 * t - sp;
        const double z3n = z3 + hdx * (sp + sr);
        Wc[(size_t)r * N + n] = scale * 0.5 * (z3 + z3n);
        z3 = z3n;
        sp = sr;
    }
}

// sum_{i,j} w(i,j) K3(i,j; k,l) for each collocation point (k, l).  The sum over i at
// a fixed row offset depends only on k and that offset, so it is formed once per offset:
//   R[o][k] = sum_i w_i / sqrt(((i - k) - 1/2)^2 dx^2 + (o dy)^2),   o = 0 .. 2M-2,
// and then k3(k, l) = dx dy sum_j w_j (R[|j - l|][k] + R[j + l][k]).
__global__ __launch_bounds__(256) void k_k3_rows(Geo g, double* __restrict__ R) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    const int o = blockIdx.y;
    if (k >= g.Nc) return;
    const double dy = (double)o * g.dy, dy2 = dy * dy;
    double row = 0.0;
    for (int i = 0; i < g.N; ++i) {
        const double dx = ((double)(i - k) - 0.5) * g.dx;
        row = fma(weight1d(i, g.N, g.weights), rsq_exact(dx * dx + dy2), row);
    }
    R[(size_t)o * g.Nc + k] = row;
}

__global__ __launch_bounds__(256) void k_k3_sum(Geo g, const double* __restrict__ R,
                                                double* __restrict__ k3) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= g.ncol) return;
    const int l = c / g.Nc;
    const int k = c - l * g.Nc;
    double s = 0.0;
    for (int j = 0; j < g.M; ++j) {
        const int o = j >= l ? j - l : l - j;
        s = fma(weight1d(j, g.M, g.weights),
                R[(size_t)o * g.Nc + k] + R[(size_t)(j + l) * g.Nc + k], s);
    }
    k3[c] = g.dx * g.dy * s;
}

// Entries of the banded Schur complement before factorisation: grid x over the N x N
// entries of one band block, grid y over the blocks (l, d) (block b = l (2q+1) + d).
__global__ __launch_bounds__(256) void k_assemble(Geo g, int q, const double* __restrict__ k3,
                                                  const double* __restrict__ Wc,
                                                  double* __restrict__ S) {
    const int nb = 2 * q + 1;
    const unsigned N = g.N, NN = N * N;
    for (int b = blockIdx.y; b < g.M * nb; b += gridDim.y) {
        const int l = b / nb;
        const int m = l + (b - l * nb) - q;
        double* Sb = S + (size_t)b * NN;
        const bool inside = m >= 0 && m < g.M;
        const double dy = (double)(m - l) * g.dy, dyp = (double)(m + l) * g.dy;
        const double dy2 = dy * dy, dyp2 = dyp * dyp;
        const double wm = g.dx * g.dy * weight1d(inside ? m : 0, g.M, g.weights);
        for (unsigned e = blockIdx.x * 256 + threadIdx.x; e < NN; e += gridDim.x * 256) {
            const int r = (int)(e / N), n = (int)(e - (unsigned)r * N);
            double v = 0.0;
            if (inside) {
                if (r == 0) {
                    if (m == l) {
                        if (n == 0) v = g.nu - g.x1 / g.dx;
                        if (n == 1) v = g.x1 / g.dx;
                    }
                } else {
                    const int k = r - 1;
                    const double dx = ((double)(n - k) - 0.5) * g.dx;
                    const double dx2 = dx * dx;
                    const double K3 = rsq_exact(dx2 + dy2) + rsq_exact(dx2 + dyp2);
                    v = -(wm * weight1d(n, g.N, g.weights)) * K3;
                    if (m == l) {
                        if (n == k || n == k + 1) {
                            const double xs = g.x1 + (k + 0.5) * g.dx;
                            const double ys = l * g.dy;
                            const double Il =
                                closed_form_I(1.0, 0.0, 1.0, 4.0, xs - g.x1, g.xN - xs, ys, g.yM);
                            v += 0.5 * (k3[(size_t)l * g.Nc + k] - Il);
                        }
                        v -= Wc[(size_t)r * g.N + n];
                    }
                }
            }
            Sb[e] = v;
        }
    }
}

// ---- inverses of the diagonal blocks ----------------------------------------------------
// Gauss-Jordan with partial pivoting done implicitly: rows are never swapped.
// Step p eliminates column p with the unused row rp of largest |B[rp][p]| and
// stores the inverse's column in place of the eliminated one.  With
// rowpiv[p] = rp and step_of[rp] = p the inverse is
//     A^{-1}[step_of[r]][rowpiv[c]] = B[r][c],
// written by one scatter at the end.
//
// Blocked form.  The columns are taken in panels of w.  The panel alone (all
// rows, w columns) is eliminated first; its pivot rows R_0..R_{w-1} and new
// columns Pn follow (rows R_t of Pn hold W = (B[R][panel])^{-1}, any other row r
// holds -B[r][panel] W).  Every column outside the panel then receives the w
// steps at once through the old pivot rows Z_t = B[R_t]:
//     B[r][j] <- base_r[j] + sum_t Pn[r][t] Z_t[j],   base_r = 0 if r is in R, else B[r],
// which is the Schur complement B - B[:,panel] W B[R,:] on the other rows and
// W B[R,:] on the pivot rows, i.e. the same as taking the w steps one by one.

// Pivot key of a candidate: the high word of |v|, which orders non-negative doubles
// (NaN above infinity, so a NaN column is taken and reported).  Values that agree in
// the high word (20 mantissa bits) tie and the lowest lane wins: partial pivoting
// needs a large pivot, not the exact maximum.
__device__ __forceinline__ int pivot_key(double v) {
    return (int)((unsigned long long)__double_as_longlong(v) >> 32) & 0x7fffffff;
}

template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Maximum over each row of 16 lanes, left in every lane of that row
// (quad swaps, then half-row and row mirrors).
__device__ __forceinline__ int row16_max_i32(int v) {
    v = max(v, dpp_i32<0xB1>(v));   // quad_perm [1,0,3,2]
    v = max(v, dpp_i32<0x4E>(v));   // quad_perm [2,3,0,1]
    v = max(v, dpp_i32<0x141>(v));  // row_half_mirror
    v = max(v, dpp_i32<0x140>(v));  // row_mirror
    return v;
}

__device__ __forceinline__ int wave_max_i32(int v) {
    v = row16_max_i32(v);
    return max(max(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
               max(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}

// 1/x: hardware estimate and two Newton steps; 0 and NaN give NaN (counted as a zero pivot)
__device__ __forceinline__ double rcp64(double x) {
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

// ---- N <= 192: the whole block in registers, one workgroup ----
// Wavefront 0 eliminates the panels (rows lane + 64 i in registers; pivot search by DPP
// and readlane, no block barrier inside a panel).  Wavefronts 1..7 hold the block: thread
// (tr = t' / 32, tc = t' % 32), t' = t - 64, holds B[tr + 14 i][tc + 32 c].  The two roles
// run separate loops whose barriers pair one to one (two per panel), so the block's
// registers are not live in wavefront 0's code.  Iteration k:
//   wavefront 0: applies panel k (its multipliers, kept in registers) to panel k+1's
//     columns, which the tile waves staged before panel k's update; barrier E;
//     eliminates panel k+1; barrier X.
//   tile waves: copy panel k's pivot rows to Zr (their base becomes zero); barrier E;
//     apply panel k's rank-kPW update to the whole block; stage panel k+2's columns;
//     barrier X.
constexpr int kGT = 512;
constexpr int kPW = 8;

// Steps of one W-column panel held in pv (rows lane + 64 i, columns 0..kb-1), in place.  A
// candidate carries its row in the pivot key: (high word of |v|, low TB bits cleared) |
// tag, tag = 2^TB - 1 - row while the row is a candidate and -1 (key -1) once pivoted or
// padding (64 RW <= 2^TB).  One integer maximum then yields the pivot row: the largest
// candidate to 20 - TB mantissa bits (partial pivoting needs a large pivot, not the exact
// maximum; a NaN is taken and reported), the lowest row among ties.  Lane s of rps
// receives the pivot row of step s.
template <int RW, int W, int TB, bool FULL>
__device__ __forceinline__ void gj_panel_steps(int kb, int lane, double (&pv)[RW][W],
                                               int (&tag)[RW], int& rps, int& zeros) {
    static_assert(64 * RW <= (1 << TB), "row tags need TB bits");
    constexpr int kTagMask = (1 << TB) - 1;
#pragma unroll
    for (int s = 0; s < W; ++s) {
        if (!FULL && s >= kb) continue;  // uniform; a constant trip count unrolls fully
        int key = -1;
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            const int hi = (int)((unsigned long long)__double_as_longlong(pv[i][s]) >> 32);
            key = max(key, (hi & (0x7fffffff & ~kTagMask)) | tag[i]);
        }
        const int wt = wave_max_i32(key) & kTagMask;
        const int rp = kTagMask - wt;
        const int pl = rp & 63, pi = rp >> 6;
        double prow[W];
#pragma unroll
        for (int u = 0; u < W; ++u) prow[u] = 0.0;
#pragma unroll
        for (int i = 0; i < RW; ++i)
            if (i == pi)
#pragma unroll
                for (int u = 0; u < W; ++u) prow[u] = readlane_f64(pv[i][u], pl);
        const double piv = prow[s];
        if (!(fabs(piv) > 0.0)) ++zeros;
        const double d = rcp64(piv);
        double pd[W];
#pragma unroll
        for (int u = 0; u < W; ++u) pd[u] = (u == s) ? d : prow[u] * d;
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            const double m = pv[i][s];
#pragma unroll
            for (int u = 0; u < W; ++u) pv[i][u] = (u == s) ? -m * d : fma(-m, pd[u], pv[i][u]);
        }
        if (lane == pl) {
#pragma unroll
            for (int i = 0; i < RW; ++i)
                if (i == pi)
#pragma unroll
                    for (int u = 0; u < W; ++u) pv[i][u] = pd[u];
        }
#pragma unroll
        for (int i = 0; i < RW; ++i) tag[i] = (tag[i] == wt) ? -1 : tag[i];
        rps = (lane == s) ? rp : rps;
    }
}

// Eliminates panel k0 .. k0 + kb - 1 held in pv and records its pivots in rowpiv / step_of.
template <int RW>
__device__ __forceinline__ void gj_panel(int N, int k0, int kb, int lane, double (&pv)[RW][kPW],
                                         int* rowpiv, int* step_of, int& zeros) {
    int tag[RW];
#pragma unroll
    for (int i = 0; i < RW; ++i) {
        const int r = lane + 64 * i;
        tag[i] = (r < N && step_of[r] < 0) ? 255 - r : -1;
    }
    int rps = 0;
    if (kb == kPW)
        gj_panel_steps<RW, kPW, 8, true>(kb, lane, pv, tag, rps, zeros);
    else
        gj_panel_steps<RW, kPW, 8, false>(kb, lane, pv, tag, rps, zeros);
    if (lane < kb) {
        rowpiv[k0 + lane] = rps;
        step_of[rps] = k0 + lane;
    }
}

// Panel k (multipliers pk, pivot rows rowpiv[k0 ..]) applied to the next panel's columns
// staged in Pin before panel k's update, for rows lane + 64 i: the base (zero on panel k's
// pivot rows) plus the sum over t of multiplier t times the staged pivot row t.
template <int RW, bool FULL>
__device__ __forceinline__ void gj_stage(int lane, int k0, int kb, const double (&pk)[RW][kPW],
                                         double (&pv)[RW][kPW], const double (*Pin)[kPW],
                                         const int* rowpiv, const int* step_of) {
    int r[kPW];
#pragma unroll
    for (int s = 0; s < kPW; ++s) r[s] = (FULL || s < kb) ? rowpiv[k0 + s] : 0;
    bool pr[RW];
#pragma unroll
    for (int i = 0; i < RW; ++i) {
        const int st = step_of[lane + 64 * i] - k0;
        pr[i] = st >= 0 && st < kb;
    }
#pragma unroll
    for (int i = 0; i < RW; ++i)
#pragma unroll
        for (int u = 0; u < kPW; ++u) pv[i][u] = pr[i] ? 0.0 : Pin[lane + 64 * i][u];
#pragma unroll
    for (int s = 0; s < kPW; ++s) {
        if (!FULL && s >= kb) break;
        double z[kPW];
#pragma unroll
        for (int u = 0; u < kPW; ++u) z[u] = Pin[r[s]][u];
#pragma unroll
        for (int i = 0; i < RW; ++i)
#pragma unroll
            for (int u = 0; u < kPW; ++u) pv[i][u] = fma(pk[i][s], z[u], pv[i][u]);
    }
}

// RB x CB block per tile thread (14 RB >= N, 32 CB >= N), RW panel rows per lane (64 RW >= N)
template <int RB, int CB, int RW>
__global__ __launch_bounds__(kGT) void k_gj_tile(int N, double* __restrict__ base, size_t stride,
                                                 int* __restrict__ info) {
    __builtin_amdgcn_s_setprio(3);  // the inversion chain is the set-up's critical path
    constexpr int R = 14 * RB, C = 32 * CB;
    constexpr int RP = (R > 64 * RW) ? R : 64 * RW;  // rows of the panel buffers
    double* A = base + (size_t)blockIdx.x * stride;
    __shared__ double Pn[2][RP][kPW];  // eliminated panels k (k even / odd)
    __shared__ double Pin[RP][kPW];    // next panel's columns, staged before the update
    __shared__ double Zr[kPW][C];      // pivot rows before the update
    __shared__ int rowpiv[C], step_of[RP];
    const int t = threadIdx.x;
    const int lane = t & 63;
    for (int e = t; e < RP * kPW; e += kGT) {
        (&Pn[0][0][0])[e] = 0.0;
        (&Pn[1][0][0])[e] = 0.0;
        (&Pin[0][0])[e] = 0.0;
    }
    for (int r = t; r < RP; r += kGT) step_of[r] = -1;
    for (int r = t; r < C; r += kGT) rowpiv[r] = -1;
    const int npan = (N + kPW - 1) / kPW;
    if (__builtin_amdgcn_readfirstlane(t) < 64) {
        // wavefront 0 (a uniform branch: each wavefront runs one of the two loops)
        int zeros = 0;
        double pk[RW][kPW];  // multipliers of the last eliminated panel
        __syncthreads();     // B0: panel 0 staged
        {
            double pv[RW][kPW];
#pragma unroll
            for (int i = 0; i < RW; ++i)
#pragma unroll
                for (int u = 0; u < kPW; ++u) pv[i][u] = Pin[lane + 64 * i][u];
            __syncthreads();  // B1: Pin free for panel 1
            gj_panel<RW>(N, 0, min(kPW, N), lane, pv, rowpiv, step_of, zeros);
#pragma unroll
            for (int i = 0; i < RW; ++i)
#pragma unroll
                for (int u = 0; u < kPW; ++u) {
                    Pn[0][lane + 64 * i][u] = pv[i][u];
                    pk[i][u] = pv[i][u];
                }
        }
        __syncthreads();  // X(-1)
        for (int k = 0; k < npan; ++k) {
            const int k0 = k * kPW, kb = min(kPW, N - k0);
            const int k1 = k0 + kPW, kb1 = min(kPW, N - k1);
            double pv[RW][kPW];
            if (k + 1 < npan) {
                if (kb == kPW)
                    gj_stage<RW, true>(lane, k0, kb, pk, pv, Pin, rowpiv, step_of);
                else
                    gj_stage<RW, false>(lane, k0, kb, pk, pv, Pin, rowpiv, step_of);
            }
            __syncthreads();  // E(k)
            if (k + 1 < npan) {
                gj_panel<RW>(N, k1, kb1, lane, pv, rowpiv, step_of, zeros);
#pragma unroll
                for (int i = 0; i < RW; ++i)
#pragma unroll
                    for (int u = 0; u < kPW; ++u) {
                        Pn[(k + 1) & 1][lane + 64 * i][u] = pv[i][u];
                        pk[i][u] = pv[i][u];
                    }
            }
            __syncthreads();  // X(k)
        }
        if (t == 0 && info) info[blockIdx.x] = zeros;
        return;
    }
    const int tt = t - 64;  // tile thread
    const int tc = tt & 31, tr = tt >> 5;
    double a[RB][CB];
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const int r = tr + 14 * i, j = tc + 32 * c;
            a[i][c] = (r < N && j < N) ? A[(size_t)r * N + j] : 0.0;
        }
    if (tc < kPW) {
#pragma unroll
        for (int i = 0; i < RB; ++i) Pin[tr + 14 * i][tc] = a[i][0];
    }
    __syncthreads();  // B0
    __syncthreads();  // B1
    if (npan > 1 && tc >= kPW && tc < 2 * kPW) {
#pragma unroll
        for (int i = 0; i < RB; ++i) Pin[tr + 14 * i][tc - kPW] = a[i][0];
    }
    __syncthreads();  // X(-1)
    for (int k = 0; k < npan; ++k) {
        const int k0 = k * kPW, kb = min(kPW, N - k0);
        const int buf = k & 1;
        const int c0 = k0 >> 5, t0 = k0 & 31;  // kPW divides 32: a panel never straddles c
        const int k2 = k0 + 2 * kPW;
        const int c2 = k2 >> 5, t2 = k2 & 31;
        {
            // panel k's pivot rows to Zr; their base becomes zero
            int st[RB];
#pragma unroll
            for (int i = 0; i < RB; ++i) st[i] = step_of[tr + 14 * i] - k0;
#pragma unroll
            for (int i = 0; i < RB; ++i) {
                if (st[i] >= 0 && st[i] < kb) {
#pragma unroll
                    for (int c = 0; c < CB; ++c) {
                        Zr[st[i]][tc + 32 * c] = a[i][c];
                        a[i][c] = 0.0;
                    }
                }
            }
        }
        __syncthreads();  // E(k)
        {
            // rank-kb update of the whole block, operands of step u + 1 loaded while u is applied
            double z[CB], p[RB];
#pragma unroll
            for (int c = 0; c < CB; ++c) z[c] = Zr[0][tc + 32 * c];
#pragma unroll
            for (int i = 0; i < RB; ++i) p[i] = Pn[buf][tr + 14 * i][0];
#pragma unroll
            for (int u = 0; u < kPW; ++u) {
                if (u >= kb) break;
                double zn[CB], pn[RB];
                const int un = (u + 1 < kPW) ? u + 1 : u;
#pragma unroll
                for (int c = 0; c < CB; ++c) zn[c] = Zr[un][tc + 32 * c];
#pragma unroll
                for (int i = 0; i < RB; ++i) pn[i] = Pn[buf][tr + 14 * i][un];
#pragma unroll
                for (int i = 0; i < RB; ++i)
#pragma unroll
                    for (int c = 0; c < CB; ++c) a[i][c] = fma(p[i], z[c], a[i][c]);
#pragma unroll
                for (int c = 0; c < CB; ++c) z[c] = zn[c];
#pragma unroll
                for (int i = 0; i < RB; ++i) p[i] = pn[i];
            }
            // the panel's own columns take the eliminated values
            if (tc >= t0 && tc < t0 + kPW) {
#pragma unroll
                for (int c = 0; c < CB; ++c)
                    if (c == c0)
#pragma unroll
                        for (int i = 0; i < RB; ++i) a[i][c] = Pn[buf][tr + 14 * i][tc - t0];
            }
            // panel k+2's columns, before panel k+1's update
            if (k2 < N && tc >= t2 && tc < t2 + kPW) {
#pragma unroll
                for (int c = 0; c < CB; ++c)
                    if (c == c2)
#pragma unroll
                        for (int i = 0; i < RB; ++i) Pin[tr + 14 * i][tc - t2] = a[i][c];
            }
        }
        __syncthreads();  // X(k)
    }
    // The inverse: row step_of[r], column rowpiv[j] takes B[r][j].  Output column o comes
    // from column step_of[o]; each half-wave passes its row through LDS (the panel buffers
    // are free now) and reads it back permuted, so that its stores are contiguous.
    static_assert(14 * C <= 2 * RP * kPW, "row buffers exceed the panel buffers");
    double* rowbuf = &Pn[0][0][0] + (size_t)tr * C;
    int src[CB];
#pragma unroll
    for (int c = 0; c < CB; ++c) {
        const int o = tc + 32 * c;
        src[c] = (o < N) ? step_of[o] : -1;
    }
#pragma unroll
    for (int i = 0; i < RB; ++i) {
        const int r = tr + 14 * i;
#pragma unroll
        for (int c = 0; c < CB; ++c) rowbuf[tc + 32 * c] = a[i][c];
        double v[CB];
#pragma unroll
        for (int c = 0; c < CB; ++c) v[c] = (src[c] >= 0 && src[c] < N) ? rowbuf[src[c]] : 0.0;
        const int sr = (r < N) ? step_of[r] : -1;
        if (sr >= 0 && sr < N) {
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                const int o = tc + 32 * c;
                if (src[c] >= 0 && src[c] < N) A[(size_t)sr * N + o] = v[c];
            }
        }
    }
}

// ---- N > 192: the block in global memory, one panel and one update launch per panel ----
// Panel kernel: one NT-thread workgroup per block; thread t holds panel rows
// t + NT i (i < RW, N <= NT RW).  One block barrier per step: every wavefront posts
// its best candidate (key, row, and the row already scaled by the candidate's
// reciprocal) in a double-buffered LDS slot; after the barrier every thread takes the
// best of the 4 posts.  It writes the new panel columns pn[N][kPWG], the old pivot rows
// z[kPWG][N], step_of[N] and rowpiv[N] (per block, in the workspace).
// The step loop is not unrolled (an unrolled one is ~9K instructions, far beyond the
// instruction cache, and ran at ~90 us per panel): instead each step works on register
// column 0 and writes its results shifted down by one column, so that the panel
// columns rotate through the registers and are back in place after kPWG steps.
constexpr int kGP = 256;
constexpr int kPWG = 16;

struct GjWork {
    double* pn;   // [nblocks][N][kPWG]
    double* z;    // [nblocks][kPWG][N]; for N <= 256 the second Pn buffer, [nblocks][N][kPWG]
    int* piv;     // [nblocks][2][N]: step_of, rowpiv
};

template <int RW, int NT>
__global__ __launch_bounds__(NT) void k_gjp_panel(int N, const double* __restrict__ base,
                                                   size_t stride, GjWork w, int k0,
                                                   int* __restrict__ info) {
    __builtin_amdgcn_s_setprio(3);  // the inversion chain is the set-up's critical path
    constexpr int NW = NT / 64;
    const double* B = base + (size_t)blockIdx.x * stride;
    double* pn = w.pn + (size_t)blockIdx.x * N * kPWG;
    double* z = w.z + (size_t)blockIdx.x * kPWG * N;
    int* step_of = w.piv + (size_t)blockIdx.x * 2 * N;
    int* rowpiv = step_of + N;
    __shared__ double rec[2][NW][kPWG + 1];  // scaled candidate row (rotated), then its pivot
    __shared__ int ckey[2][NW], crow[2][NW], rp_s[kPWG];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int kb = min(kPWG, N - k0);
    int st[RW];
    double pv[RW][kPWG];
#pragma unroll
    for (int i = 0; i < RW; ++i) {
        const int r = t + NT * i;
        const bool valid = r < N;
        st[i] = valid ? ((k0 > 0) ? step_of[r] : -1) : N;  // N marks padding
#pragma unroll
        for (int u = 0; u < kPWG; ++u)
            pv[i][u] = (valid && u < kb) ? B[(size_t)r * N + k0 + u] : 0.0;
    }
    int zeros = 0;
    // step s: register column 0 holds panel column s; register column u holds panel
    // column (s + u) mod kPWG
#pragma unroll 1
    for (int s = 0; s < kb; ++s) {
        const int buf = s & 1;
        int key = -1, bi = -1;
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            const int kk = pivot_key(pv[i][0]);
            if (st[i] < 0 && kk > key) {
                key = kk;
                bi = i;
            }
        }
        const int wm = wave_max_i32(key);
        const unsigned long long mask = __ballot(bi >= 0 && key == wm);
        const int wl = mask ? __builtin_ctzll(mask) : -1;
        if (lane == wl) {
            double row[kPWG];
#pragma unroll
            for (int u = 0; u < kPWG; ++u) row[u] = pv[0][u];
#pragma unroll
            for (int i = 1; i < RW; ++i)
                if (i == bi)
#pragma unroll
                    for (int u = 0; u < kPWG; ++u) row[u] = pv[i][u];
            const double d = rcp64(row[0]);
            rec[buf][wv][0] = d;
#pragma unroll
            for (int u = 1; u < kPWG; ++u) rec[buf][wv][u] = row[u] * d;
            rec[buf][wv][kPWG] = row[0];
        }
        // read the candidate's row slot with every lane active: inside the lane-0 branch
        // below the other lanes of bi need not hold a value
        const int bsel = __builtin_amdgcn_readlane(bi, max(wl, 0));
        if (lane == 0) {
            ckey[buf][wv] = mask ? wm : -1;
            crow[buf][wv] = mask ? wv * 64 + wl + NT * max(0, bsel) : -1;
        }
        __syncthreads();
        int gw = 0, gk = ckey[buf][0];
#pragma unroll
        for (int q = 1; q < NW; ++q) {
            const int kq = ckey[buf][q];
            if (kq > gk) {
                gk = kq;
                gw = q;
            }
        }
        const int rp = max(0, min(N - 1, crow[buf][gw]));
        double pd[kPWG];
#pragma unroll
        for (int u = 0; u < kPWG; ++u) pd[u] = rec[buf][gw][u];
        const double d = pd[0];
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            if (t + NT * i == rp) {
                // the pivot row becomes the scaled row; column s takes 1/pivot
#pragma unroll
                for (int u = 0; u + 1 < kPWG; ++u) pv[i][u] = pd[u + 1];
                pv[i][kPWG - 1] = d;
                st[i] = k0 + s;
            } else {
                const double m = pv[i][0];
#pragma unroll
                for (int u = 0; u + 1 < kPWG; ++u) pv[i][u] = fma(-m, pd[u + 1], pv[i][u + 1]);
                pv[i][kPWG - 1] = -m * d;
            }
        }
        if (t == 0) {
            rp_s[s] = rp;
            rowpiv[k0 + s] = rp;
            if (!(fabs(rec[buf][gw][kPWG]) > 0.0)) ++zeros;
        }
    }
    // a short last panel: kb rotations done, kPWG - kb more put the columns back in place
#pragma unroll 1
    for (int s = kb; s < kPWG; ++s) {
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            const double c0 = pv[i][0];
#pragma unroll
            for (int u = 0; u + 1 < kPWG; ++u) pv[i][u] = pv[i][u + 1];
            pv[i][kPWG - 1] = c0;
        }
    }
#pragma unroll
    for (int i = 0; i < RW; ++i) {
        const int r = t + NT * i;
        if (r < N) {
#pragma unroll
            for (int u = 0; u < kPWG; ++u) pn[(size_t)r * kPWG + u] = pv[i][u];
            step_of[r] = st[i];
        }
    }
    __syncthreads();
    // the old pivot rows: every load issued before the first store (a load-store loop
    // would wait out one memory latency per element)
#pragma unroll
    for (int tt = 0; tt < kPWG; ++tt) {
        const double* src = B + (size_t)rp_s[min(tt, kb - 1)] * N;
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            const int j = t + NT * i;
            pv[i][tt] = (tt < kb && j < N) ? src[j] : 0.0;
        }
    }
#pragma unroll
    for (int tt = 0; tt < kPWG; ++tt)
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            const int j = t + NT * i;
            if (tt < kb && j < N) z[(size_t)tt * N + j] = pv[i][tt];
        }
    if (t == 0 && info) info[blockIdx.x] = (k0 == 0 ? 0 : info[blockIdx.x]) + zeros;
}

// ---- 192 < N <= 256: one launch per panel, column strips ----
// Launch k (k = -1 .. npan - 1): workgroup s owns columns [16 s, 16 s + 16) of every row,
// one row per thread.  If panel k exists (first column kp), the workgroup applies it to
// its strip, B[r] <- base_r + sum_t Pn_k[r][t] Z_t with base_r = 0 on panel k's pivot
// rows (panel k's own strip takes Pn_k), reading the old pivot rows Z_t of its strip
// before any of its writes: no other workgroup touches these columns, so no copy of the
// pivot rows is needed.  The workgroup holding panel k+1 (first column kn) then
// eliminates it from its updated strip (wavefront 0, rows lane + 64 i, the register-tile
// pivot steps) and writes Pn_{k+1} and the pivots; Pn alternates between two buffers by
// panel parity.  It does not store its strip: launch k+1 gives those columns Pn_{k+1}.
__global__ __launch_bounds__(kGP) void k_gjs_step(int N, double* __restrict__ base, size_t stride,
                                                  GjWork w, int kp, int kn,
                                                  int* __restrict__ info) {
    __builtin_amdgcn_s_setprio(3);  // the inversion chain is the set-up's critical path
    constexpr int RW = kGP / 64;  // panel rows per lane: 64 RW >= N
    double* B = base + (size_t)blockIdx.y * stride;
    int* step_of = w.piv + (size_t)blockIdx.y * 2 * N;
    int* rowpiv = step_of + N;
    auto pnbuf = [&](int k0) {
        return (((k0 / kPWG) & 1) ? w.z : w.pn) + (size_t)blockIdx.y * N * kPWG;
    };
    const int c0 = blockIdx.x * kPWG;
    const int nc = min(kPWG, N - c0);
    const bool panel = kn >= 0 && c0 == kn;
    if (kp < 0 && !panel) return;
    __shared__ double Zs[kPWG][kPWG];
    __shared__ double strip[kGP][kPWG + 1];
    const int t = threadIdx.x;
    const int r = t;  // this thread's row
    double v[kPWG];
#pragma unroll
    for (int u = 0; u < kPWG; ++u) v[u] = (r < N && u < nc) ? B[(size_t)r * N + c0 + u] : 0.0;
    if (kp >= 0) {
        const int kb = min(kPWG, N - kp);
        const double* pk = pnbuf(kp);
        {
            const int tt = t / kPWG, u = t % kPWG;
            Zs[tt][u] = (tt < kb && u < nc) ? B[(size_t)rowpiv[kp + tt] * N + c0 + u] : 0.0;
        }
        __syncthreads();
        if (r < N) {
            if (c0 == kp) {
#pragma unroll
                for (int u = 0; u < kPWG; ++u) v[u] = (u < nc) ? pk[(size_t)r * kPWG + u] : 0.0;
            } else {
                const int st = step_of[r] - kp;
                const bool isp = st >= 0 && st < kb;
                double pr[kPWG];
#pragma unroll
                for (int tt = 0; tt < kPWG; ++tt) pr[tt] = (tt < kb) ? pk[(size_t)r * kPWG + tt] : 0.0;
#pragma unroll
                for (int u = 0; u < kPWG; ++u) v[u] = isp ? 0.0 : v[u];
#pragma unroll
                for (int tt = 0; tt < kPWG; ++tt)
#pragma unroll
                    for (int u = 0; u < kPWG; ++u) v[u] = fma(pr[tt], Zs[tt][u], v[u]);
            }
            if (!panel) {
#pragma unroll
                for (int u = 0; u < kPWG; ++u)
                    if (u < nc) B[(size_t)r * N + c0 + u] = v[u];
            }
        }
    }
    if (!panel) return;
    if (kp < 0)
        for (int q = t; q < N; q += kGP) step_of[q] = -1;
#pragma unroll
    for (int u = 0; u < kPWG; ++u) strip[t][u] = (r < N) ? v[u] : 0.0;
    __syncthreads();
    if (__builtin_amdgcn_readfirstlane(t) < 64) {
        const int lane = t;
        const int kb = min(kPWG, N - kn);
        double pv[RW][kPWG];
        int tag[RW];
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            const int rr = lane + 64 * i;
            tag[i] = (rr < N && step_of[rr] < 0) ? 511 - rr : -1;
#pragma unroll
            for (int u = 0; u < kPWG; ++u) pv[i][u] = strip[rr][u];
        }
        int zeros = 0, rps = 0;
        if (kb == kPWG)
            gj_panel_steps<RW, kPWG, 9, true>(kb, lane, pv, tag, rps, zeros);
        else
            gj_panel_steps<RW, kPWG, 9, false>(kb, lane, pv, tag, rps, zeros);
        double* pn = pnbuf(kn);
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            const int rr = lane + 64 * i;
            if (rr < N)
#pragma unroll
                for (int u = 0; u < kPWG; ++u) pn[(size_t)rr * kPWG + u] = pv[i][u];
        }
        if (lane < kb) {
            rowpiv[kn + lane] = rps;
            step_of[rps] = kn + lane;
        }
        if (lane == 0 && info) info[blockIdx.y] = (kn == 0 ? 0 : info[blockIdx.y]) + zeros;
    }
}

// Rank-kb update of every column outside the panel; the panel columns take pn.
// Tile of 16 rows x 64 columns per 256-thread workgroup; grid (cols, rows, blocks).
__global__ __launch_bounds__(256) void k_gjp_update(int N, double* __restrict__ base,
                                                    size_t stride, GjWork w, int k0) {
    __builtin_amdgcn_s_setprio(3);  // the inversion chain is the set-up's critical path
    double* B = base + (size_t)blockIdx.z * stride;
    const double* pn = w.pn + (size_t)blockIdx.z * N * kPWG;
    const double* z = w.z + (size_t)blockIdx.z * kPWG * N;
    const int* step_of = w.piv + (size_t)blockIdx.z * 2 * N;
    const int kb = min(kPWG, N - k0);
    __shared__ double ps[16][kPWG], zs[kPWG][64];
    __shared__ int isp[16];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int row0 = blockIdx.y * 16, col0 = blockIdx.x * 64;
    {
        const int rr = threadIdx.x >> 4, u = threadIdx.x & 15;
        const int gr = row0 + rr;
        ps[rr][u] = (gr < N && u < kb) ? pn[(size_t)gr * kPWG + u] : 0.0;
        if (u == 0) {
            const int st = (gr < N) ? step_of[gr] : -1;
            isp[rr] = (st >= k0 && st < k0 + kb);
        }
    }
    for (int e = threadIdx.x; e < kPWG * 64; e += 256) {
        const int u = e >> 6, c = e & 63, gc = col0 + c;
        zs[u][c] = (u < kb && gc < N) ? z[(size_t)u * N + gc] : 0.0;
    }
    __syncthreads();
    const int j = col0 + tx;
    if (j >= N) return;
    const bool inpanel = j >= k0 && j < k0 + kb;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int rr = ty + 4 * i, gr = row0 + rr;
        if (gr >= N) break;
        double* p = B + (size_t)gr * N + j;
        if (inpanel) {
            *p = ps[rr][j - k0];
        } else {
            double v = isp[rr] ? 0.0 : *p;
#pragma unroll
            for (int u = 0; u < kPWG; ++u) v = fma(ps[rr][u], zs[u][tx], v);
            *p = v;
        }
    }
}

// out[step_of[r]][rowpiv[c]] = B[r][c]; grid (elements, blocks)
__global__ void k_gjp_scatter(int N, const double* __restrict__ base, size_t stride,
                              double* __restrict__ outbase, size_t out_stride, GjWork w) {
    const double* B = base + (size_t)blockIdx.y * stride;
    double* O = outbase + (size_t)blockIdx.y * out_stride;
    const int* step_of = w.piv + (size_t)blockIdx.y * 2 * N;
    const int* rowpiv = step_of + N;
    const size_t NN = (size_t)N * N;
    // output (o, p) = B[rowpiv[o]][step_of[p]]: contiguous stores, gathered loads
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < NN;
         e += (size_t)gridDim.x * blockDim.x) {
        const int o = (int)(e / N), p = (int)(e - (size_t)o * N);
        const int r = rowpiv[o], c = step_of[p];
        if (r >= 0 && r < N && c >= 0 && c < N) O[e] = B[(size_t)r * N + c];
    }
}

__global__ void k_copy_blocks(int N, const double* __restrict__ a, size_t a_stride,
                              double* __restrict__ b, size_t b_stride) {
    const size_t NN = (size_t)N * N;
    const double* src = a + (size_t)blockIdx.y * a_stride;
    double* dst = b + (size_t)blockIdx.y * b_stride;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < NN;
         e += (size_t)gridDim.x * blockDim.x)
        dst[e] = src[e];
}

size_t gj_work_doubles(int N, int nblocks) {
    return N > 192 ? (size_t)nblocks * (2 * kPWG + 1) * N : 0;
}

// Inverts nblocks blocks in place.  For N > 192: tmp holds nblocks x N x N
// doubles (the scattered inverses) and work gj_work_doubles(N, nblocks).
void gj_inverse(int N, double* base, size_t stride, int nblocks, int* info, double* tmp,
                double* work, hipStream_t s) {
    if (N <= 64) {
        k_gj_tile<5, 2, 1><<<nblocks, kGT, 0, s>>>(N, base, stride, info);
    } else if (N <= 128) {
        k_gj_tile<10, 4, 2><<<nblocks, kGT, 0, s>>>(N, base, stride, info);
    } else if (N <= 182) {
        k_gj_tile<13, 6, 3><<<nblocks, kGT, 0, s>>>(N, base, stride, info);
    } else if (N <= 192) {
        k_gj_tile<14, 6, 3><<<nblocks, kGT, 0, s>>>(N, base, stride, info);
    } else {
        const size_t NN = (size_t)N * N;
        GjWork w;
        w.pn = work;
        w.z = work + (size_t)nblocks * N * kPWG;
        w.piv = reinterpret_cast<int*>(work + (size_t)nblocks * 2 * kPWG * N);
        if (N <= kGP) {
            const int npan = (N + kPWG - 1) / kPWG;
            for (int k = -1; k < npan; ++k) {
                const int kp = (k >= 0) ? k * kPWG : -1;
                const int kn = (k + 1 < npan) ? (k + 1) * kPWG : -1;
                k_gjs_step<<<dim3(npan, nblocks), kGP, 0, s>>>(N, base, stride, w, kp, kn, info);
            }
        } else {
            const dim3 ug((N + 63) / 64, (N + 15) / 16, nblocks);
            for (int k0 = 0; k0 < N; k0 += kPWG) {
                // four wavefronts with two to four panel rows per thread (one row per thread
                // in 8-16 wavefronts measured 2.5x slower per panel at N = 721)
                if (N <= 2 * kGP)
                    k_gjp_panel<2, kGP><<<nblocks, kGP, 0, s>>>(N, base, stride, w, k0, info);
                else if (N <= 3 * kGP)
                    k_gjp_panel<3, kGP><<<nblocks, kGP, 0, s>>>(N, base, stride, w, k0, info);
                else
                    k_gjp_panel<4, kGP><<<nblocks, kGP, 0, s>>>(N, base, stride, w, k0, info);
                k_gjp_update<<<ug, 256, 0, s>>>(N, base, stride, w, k0);
            }
        }
        const unsigned ge = (unsigned)std::min<size_t>((NN + 255) / 256, 2048);
        k_gjp_scatter<<<dim3(ge, nblocks), 256, 0, s>>>(N, base, stride, tmp, NN, w);
        k_copy_blocks<<<dim3(ge, nblocks), 256, 0, s>>>(N, tmp, NN, base, stride);
    }
}
// C = Cin + alpha A B for N x N row-major blocks (C may equal Cin, not A or B);
// blockIdx.z selects one of a list of such products.  A job with B = nullptr copies A
// to C instead.
struct GemmJob {
    const double* A;
    const double* B;
    const double* Cin;
    double* C;
};
constexpr int kMaxGemmJobs = 64;
struct GemmBatch {
    GemmJob j[kMaxGemmJobs];
};

// FP64 matrix cores (v_mfma_f64_16x16x4f64): four wavefronts per workgroup in a 2 x 2
// arrangement, each computing WM x WN MFMA tiles of 16 x 16 (a (32 WM) x (32 WN) tile of C
// per workgroup; 64 x 64 for blocks with N > 256), K staged through LDS kGK at a time with
// the next slice prefetched into registers.  Operand layout of the instruction: lane l
// holds A[l % 16][l / 16] and B[l / 16][l % 16]; result register r of lane l is
// C[l / 16 + 4 r][l % 16].
typedef double dbl4 __attribute__((ext_vector_type(4)));

template <int WM, int WN, int kGK>
__global__ __launch_bounds__(256) void k_gemm(int n, double alpha, GemmBatch batch) {
    constexpr int TM = 32 * WM, TN = 32 * WN;
    constexpr int EA = TM * kGK / 256, EB = TN * kGK / 256;  // slice elements per thread
    const GemmJob job = batch.j[blockIdx.z];
    const double* __restrict__ A = job.A;
    const double* __restrict__ B = job.B;
    if (B == nullptr) {
        // a copy job (C = A over this block's tile), riding along with the products
        const int r0 = blockIdx.y * TM, c0 = blockIdx.x * TN;
        for (int e = threadIdx.x; e < TM * TN; e += 256) {
            const int gr = r0 + e / TN, gc = c0 + e % TN;
            if (gr < n && gc < n) job.C[(size_t)gr * n + gc] = A[(size_t)gr * n + gc];
        }
        return;
    }
    __shared__ double As[TM][kGK + 1];
    __shared__ double Bs[kGK][TN + 2];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int row0 = blockIdx.y * TM, col0 = blockIdx.x * TN;
    const int wr = (w >> 1) * 16 * WM, wc = (w & 1) * 16 * WN;
    dbl4 acc[WM][WN];
#pragma unroll
    for (int a = 0; a < WM; ++a)
#pragma unroll
        for (int b = 0; b < WN; ++b) acc[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};
    const int ar = t / (kGK / EA), ak = (t % (kGK / EA)) * EA;  // A slice TM x 16
    const int bk = t / (TN / EB), bc = (t % (TN / EB)) * EB;    // B slice 16 x TN
    double ra[EA], rb[EB];
    auto load = [&](int k0) {
#pragma unroll
        for (int e = 0; e < EA; ++e) {
            const int gr = row0 + ar, gk = k0 + ak + e;
            ra[e] = (gr < n && gk < n) ? A[(size_t)gr * n + gk] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < EB; ++e) {
            const int gk = k0 + bk, gc = col0 + bc + e;
            rb[e] = (gk < n && gc < n) ? B[(size_t)gk * n + gc] : 0.0;
        }
    };
    load(0);
    for (int k0 = 0; k0 < n; k0 += kGK) {
        __syncthreads();
#pragma unroll
        for (int e = 0; e < EA; ++e) As[ar][ak + e] = ra[e];
#pragma unroll
        for (int e = 0; e < EB; ++e) Bs[bk][bc + e] = rb[e];
        __syncthreads();
        if (k0 + kGK < n) load(k0 + kGK);
#pragma unroll
        for (int k4 = 0; k4 < kGK; k4 += 4) {
            double fa[WM], fb[WN];
#pragma unroll
            for (int a = 0; a < WM; ++a) fa[a] = As[wr + a * 16 + (lane & 15)][k4 + (lane >> 4)];
#pragma unroll
            for (int b = 0; b < WN; ++b) fb[b] = Bs[k4 + (lane >> 4)][wc + b * 16 + (lane & 15)];
#pragma unroll
            for (int a = 0; a < WM; ++a)
#pragma unroll
                for (int b = 0; b < WN; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fb[b], acc[a][b], 0, 0, 0);
        }
    }
    const double* Cin = job.Cin;
    double* C = job.C;
#pragma unroll
    for (int a = 0; a < WM; ++a)
#pragma unroll
        for (int b = 0; b < WN; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gr = row0 + wr + a * 16 + (lane >> 4) + 4 * r;
                const int gc = col0 + wc + b * 16 + (lane & 15);
                if (gr < n && gc < n) {
                    const size_t o = (size_t)gr * n + gc;
                    C[o] = (Cin ? Cin[o] : 0.0) + alpha * acc[a][b][r];
                }
            }
}

// Products of one eliminated block row l, each as a single product whose rows run over
// (a, i) and columns over (b, j): C(a, b) = [C(a, b) +] alpha A_a B_b for a < na, b < nb.
//   Schur update: A_a = S(nbr[a], l), B_b = G_{l, nbr[b]}, C(a, b) = S(nbr[a], nbr[b]),
//                 accumulated, alpha = -1 (na = nb = number of coupled rows);
//   L = S(nbr[a], l) Dinv_l: nb = 1, B_0 = Dinv_l;   G = Dinv_l S(l, nbr[b]): na = 1.
// As one (na N) x (nb N) x N product only its last tile row and column are padded, where
// a 721^3 block product alone pads 721 to 768 in both dimensions (13% of its
// matrix-core work).  A pair that is not in the mask is neither updated nor, where a
// whole tile lies in such pairs, computed.
constexpr int kMaxRowNbr = 32;
struct RowProd {
    const double* A[kMaxRowNbr];  // A_a, N x N row-major
    double* Crow[kMaxRowNbr];     // C(a, b) = Crow[a] + b N^2
    const double* B;              // B_b = B + b N^2
    unsigned mask[kMaxRowNbr];    // bit b of word a: pair (a, b) is computed
    int na, nb;
    int accumulate;               // C += alpha A B, else C = alpha A B
};
constexpr int kMaxRowProds = 4;
struct RowProdArgs {
    RowProd p[kMaxRowProds];
    int first[kMaxRowProds];  // first tile of each problem in the grid
    int np;
};
static_assert(sizeof(RowProdArgs) <= 4096, "kernel argument block");

// 64 x 64 tile per 256-thread workgroup, 2 x 2 wavefronts of 2 x 2 v_mfma_f64_16x16x4f64
// tiles, K in slices of 16 double-buffered in LDS through a register prefetch (one
// barrier per slice).  Loads are unconditional: rows and columns past the product are
// read clamped (they reach only outputs that are not stored) and the K padding is zeroed
// on B's side with a bit mask, so that no load waits on a branch.  Tiles are taken
// eight tile rows at a time, column by column, and consecutive tiles stay on one XCD.
// Each element's K sum runs in the same order as in k_gemm, so the two give the same
// bits.
__global__ __launch_bounds__(256) void k_row_products(int N, double alpha, RowProdArgs args) {
    constexpr int T = 64, KS = 16, RA = 4, RB = 4, AR = 16, BKP = 4, kGroup = 8;
    const int lin = xcd_remap(blockIdx.x, gridDim.x);
    int pi = 0;
    while (pi + 1 < args.np && lin >= args.first[pi + 1]) ++pi;
    const RowProd& P = args.p[pi];
    const int tile = lin - args.first[pi];
    const int ntr = P.na * N, ntc = P.nb * N;
    const int tpm = (ntr + T - 1) / T, tpn = (ntc + T - 1) / T;
    const int grp = tile / (kGroup * tpn);
    const int gsz = min(kGroup, tpm - grp * kGroup);
    const int within = tile - grp * kGroup * tpn;
    const int row0 = (grp * kGroup + within % gsz) * T, col0 = (within / gsz) * T;
    {
        const int a0 = row0 / N, a1 = (min(row0 + T, ntr) - 1) / N;
        const int b0 = col0 / N, b1 = (min(col0 + T, ntc) - 1) / N;
        unsigned any = 0;
        for (int a = a0; a <= a1; ++a) any |= P.mask[a] >> b0 & ((2u << (b1 - b0)) - 1u);
        if (!any) return;
    }
    __shared__ double As[2][T][KS + 1];
    __shared__ double Bs[2][KS][T + 2];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    dbl4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};
    // A slice T x 16: thread t takes k = t % 16 of rows t / 16 + 16 e; B slice 16 x T:
    // column t % T of k-rows t / T + 4 e
    const int ak = t % KS, ar = t / KS;
    const double* arow[RA];
#pragma unroll
    for (int e = 0; e < RA; ++e) {
        const int r = min(row0 + ar + AR * e, ntr - 1);
        const int a = r / N;
        arow[e] = P.A[a] + (size_t)(r - a * N) * N;
    }
    const int bcl = t % T, bk0 = t / T;
    const double* bcolp;
    {
        const int c = min(col0 + bcl, ntc - 1);
        const int b = c / N;
        bcolp = P.B + (size_t)b * N * N + (c - b * N);
    }
    double ra[RA], rb[RB];
    unsigned bmask[RB];
    auto load = [&](int k0) {
        const int gk = min(k0 + ak, N - 1);
#pragma unroll
        for (int e = 0; e < RA; ++e) ra[e] = arow[e][gk];
#pragma unroll
        for (int e = 0; e < RB; ++e) {
            const int gkb = k0 + bk0 + BKP * e;
            bmask[e] = (gkb < N) ? ~0u : 0u;
            rb[e] = bcolp[(size_t)min(gkb, N - 1) * N];
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int e = 0; e < RA; ++e) As[buf][ar + AR * e][ak] = ra[e];
#pragma unroll
        for (int e = 0; e < RB; ++e) {
            const unsigned long long m = ((unsigned long long)bmask[e] << 32) | bmask[e];
            Bs[buf][bk0 + BKP * e][bcl] =
                __builtin_bit_cast(double, __builtin_bit_cast(unsigned long long, rb[e]) & m);
        }
    };
    const int ns = (N + KS - 1) / KS;
    load(0);
    store(0);
    __syncthreads();
    for (int s = 0; s < ns; ++s) {
        const int buf = s & 1;
        const int k0 = s * KS;
        if (s + 1 < ns) load(k0 + KS);
#pragma unroll
        for (int k4 = 0; k4 < KS; k4 += 4) {
            if (k0 + k4 < N) {
                double fa[2], fb[2];
#pragma unroll
                for (int a = 0; a < 2; ++a) fa[a] = As[buf][wr + a * 16 + (lane & 15)][k4 + (lane >> 4)];
#pragma unroll
                for (int b = 0; b < 2; ++b) fb[b] = Bs[buf][k4 + (lane >> 4)][wc + b * 16 + (lane & 15)];
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fb[b], acc[a][b], 0, 0, 0);
            }
        }
        if (s + 1 < ns) store(buf ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const int c = col0 + wc + b * 16 + (lane & 15);
        const int bb = c / N, j = c - bb * N;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int rr = row0 + wr + a * 16 + (lane >> 4) + 4 * r;
                const int aa = rr / N, i = rr - aa * N;
                if (rr < ntr && c < ntc && ((P.mask[aa] >> bb) & 1u)) {
                    double* o = P.Crow[aa] + (size_t)bb * N * N + (size_t)i * N + j;
                    *o = (P.accumulate ? *o : 0.0) + alpha * acc[a][b][r];
                }
            }
    }
}

// Small blocks (N <= 256): one 32 x 32 output tile per 256-thread workgroup.  The four
// wavefronts take interleaved quarters of K (wavefront w: k-steps of 4 numbered w, w + 4,
// ...; KS steps each, 16 KS >= n), load all their MFMA operands straight from global
// memory first (one memory round trip instead of a staged K loop), accumulate 2 x 2
// v_mfma_f64_16x16x4f64 tiles, and the four partial tiles are added in LDS in a fixed
// order.  A job with B = nullptr copies A to C over the tile.
template <int KS>
__global__ __launch_bounds__(256) void k_gemm_ks(int n, double alpha, GemmBatch batch) {
    const GemmJob job = batch.j[blockIdx.z];
    const double* __restrict__ A = job.A;
    const double* __restrict__ B = job.B;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
    if (B == nullptr) {
        for (int e = t; e < 32 * 32; e += 256) {
            const int gr = r0 + (e >> 5), gc = c0 + (e & 31);
            if (gr < n && gc < n) job.C[(size_t)gr * n + gc] = A[(size_t)gr * n + gc];
        }
        return;
    }
    __shared__ double part[4][32][33];
    const int kl = lane >> 4, l16 = lane & 15;
    const int nsteps = (n + 3) >> 2;
    double fa[KS][2], fb[KS][2];
#pragma unroll
    for (int i = 0; i < KS; ++i) {
        const int k = 4 * (w + 4 * i) + kl;
        const bool ok = k < n;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int ar = r0 + 16 * h + l16, bc = c0 + 16 * h + l16;
            fa[i][h] = (ok && ar < n) ? A[(size_t)ar * n + k] : 0.0;
            fb[i][h] = (ok && bc < n) ? B[(size_t)k * n + bc] : 0.0;
        }
    }
    dbl4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < KS; ++i)
        if (w + 4 * i < nsteps) {
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i][a], fb[i][b], acc[a][b], 0, 0, 0);
        }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) part[w][16 * a + kl + 4 * r][16 * b + l16] = acc[a][b][r];
    __syncthreads();
    for (int e = t; e < 32 * 32; e += 256) {
        const int row = e >> 5, col = e & 31;
        const int gr = r0 + row, gc = c0 + col;
        if (gr < n && gc < n) {
            const double v = (part[0][row][col] + part[1][row][col]) + (part[2][row][col] + part[3][row][col]);
            const size_t o = (size_t)gr * n + gc;
            job.C[o] = (job.Cin ? job.Cin[o] : 0.0) + alpha * v;
        }
    }
}

// ---- apply ----------------------------------------------------------------------------
// One 64-lane workgroup per row l; the row lives in LDS.  Both sequential
// operators are prefix sums:
//   A-hat^{-1} b:  y_r = (-1)^r x_r obeys y_r = y_{r-1} + (-1)^r 2 b_r, y_0 = x_0
//                  = (b_0 - 2 a01 b_1) / (a00 - a01);
//   T v:           z_i = z_0 + sum_{m<i} dx/2 (v_m + v_{m+1}), z_0 = -(x_1/nu) v_0,
//                  (T v)_r = (z_{r-1} + z_r) / 2 for r >= 1, 0 for r = 0.
__device__ void lds_ahat_solve(const Geo& g, const double* b, double* x) {
    const int N = g.N;
    const double a01 = g.x1 / g.dx;
    const double a00 = g.nu - a01;
    const double x0 = (b[0] - 2.0 * a01 * b[1]) / (a00 - a01);
    __syncthreads();
    for (int i = threadIdx.x; i < N; i += 64) x[i] = (i == 0) ? x0 : ((i & 1) ? -2.0 : 2.0) * b[i];
    __syncthreads();
    lds_prefix_sum(x, N);
    for (int i = threadIdx.x; i < N; i += 64)
        if (i & 1) x[i] = -x[i];
    __syncthreads();
}

// z = grid values of the trapezoid integral of v (z may not alias v)
__device__ void lds_trapezoid(const Geo& g, const double* v, double* z) {
    const int N = g.N;
    const double hdx = 0.5 * g.dx;
    for (int i = threadIdx.x; i < N; i += 64)
        z[i] = (i == 0) ? (-g.x1 / g.nu) * v[0] : hdx * (v[i - 1] + v[i]);
    __syncthreads();
    lds_prefix_sum(z, N);
}

// s1 = A-hat^{-1} b1, t2 = b2 - 2 pi T s1 (row l)
__device__ __forceinline__ void apply_first_row(const Geo& g, const double* __restrict__ b,
                                                double* __restrict__ s1,
                                                double* __restrict__ t2, int l) {
    __shared__ double B[kMaxN], X[kMaxN], Z[kMaxN];
    const int N = g.N;
    const size_t o = (size_t)l * N;
    for (int i = threadIdx.x; i < N; i += 64) B[i] = b[o + i];
    __syncthreads();
    lds_ahat_solve(g, B, X);
    for (int i = threadIdx.x; i < N; i += 64) s1[o + i] = X[i];
    lds_trapezoid(g, X, Z);
    const double* b2 = b + g.NM + o;
    for (int i = threadIdx.x; i < N; i += 64)
        t2[o + i] = b2[i] - ((i == 0) ? 0.0 : kTwoPi * 0.5 * (Z[i - 1] + Z[i]));
}

// r1 = s1 - A-hat^{-1} (T s2 / F^2), r2 = s2 (row l)
__device__ __forceinline__ void apply_last_row(const Geo& g, const double* __restrict__ s1,
                                               const double* __restrict__ s2,
                                               double* __restrict__ x, int l) {
    __shared__ double V[kMaxN], Z[kMaxN], X[kMaxN];
    const int N = g.N;
    const size_t o = (size_t)l * N;
    for (int i = threadIdx.x; i < N; i += 64) V[i] = s2[o + i];
    __syncthreads();
    lds_trapezoid(g, V, Z);
    const double rF2 = 1.0 / (g.F * g.F);
    // reuse V for T s2 / F^2 (V is still needed for r2: write r2 first)
    for (int i = threadIdx.x; i < N; i += 64) x[(size_t)g.NM + o + i] = V[i];
    __syncthreads();
    for (int i = threadIdx.x; i < N; i += 64) V[i] = (i == 0) ? 0.0 : rF2 * 0.5 * (Z[i - 1] + Z[i]);
    __syncthreads();
    lds_ahat_solve(g, V, X);
    for (int i = threadIdx.x; i < N; i += 64) x[o + i] = s1[o + i] - X[i];
}

__global__ __launch_bounds__(64) void k_apply_first(Geo g, const double* __restrict__ b,
                                                    double* __restrict__ s1,
                                                    double* __restrict__ t2) {
    apply_first_row(g, b, s1, t2, blockIdx.x);
}

__global__ __launch_bounds__(64) void k_apply_last(Geo g, const double* __restrict__ s1,
                                                   const double* __restrict__ s2,
                                                   double* __restrict__ x) {
    apply_last_row(g, s1, s2, x, blockIdx.x);
}

// First or last step of several applies in one launch: workgroups [first[p], first[p+1])
// take the block rows of request p, whose temporaries are work[p] (the handle's [4][NM]).
constexpr int kMaxApplyBatch = 32;
struct ApplyBatch {
    Geo g[kMaxApplyBatch];
    double* work[kMaxApplyBatch];
    const double* in[kMaxApplyBatch];  // b (first step)
    double* out[kMaxApplyBatch];       // x (last step)
    int first[kMaxApplyBatch + 1];
    int n;
};
static_assert(sizeof(ApplyBatch) <= 4096, "kernel argument block");

__device__ __forceinline__ int batch_member(const int* first, int n) {
    int p = 0;
    while (p + 1 < n && (int)blockIdx.x >= first[p + 1]) ++p;
    return p;
}

__global__ __launch_bounds__(64) void k_apply_first_batched(const ApplyBatch ab) {
    const int p = batch_member(ab.first, ab.n);
    const Geo& g = ab.g[p];
    apply_first_row(g, ab.in[p], ab.work[p], ab.work[p] + g.NM, blockIdx.x - ab.first[p]);
}

__global__ __launch_bounds__(64) void k_apply_last_batched(const ApplyBatch ab) {
    const int p = batch_member(ab.first, ab.n);
    const Geo& g = ab.g[p];
    apply_last_row(g, ab.work[p], ab.work[p] + 2 * (size_t)g.NM, ab.out[p],
                   blockIdx.x - ab.first[p]);
}

// One wavefront per output row r of one block row:
//   out[r] = add[r] + sum over terms (sign * block[r][:] . vec[:])
struct GemvTerm {
    const double* blk;
    const double* vec;
    double sign;
    double pad;
};

constexpr int kMaxTerms = 16;

__global__ __launch_bounds__(256) void k_band_step(int N, const GemvTerm* __restrict__ terms,
                                                   int nterms, const double* __restrict__ add,
                                                   double* __restrict__ out) {
    const int wid = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (wid >= N) return;
    // term pointers in registers (uniform), then one pass over the columns with the
    // loads of every term issued together
    const double* rows[kMaxTerms];
    const double* vecs[kMaxTerms];
    double sg[kMaxTerms];
    const int nt = min(nterms, kMaxTerms);
#pragma unroll
    for (int q = 0; q < kMaxTerms; ++q) {
        if (q < nt) {
            const GemvTerm tm = terms[q];
            rows[q] = tm.blk + (size_t)wid * N;
            vecs[q] = tm.vec;
            sg[q] = tm.sign;
        } else {
            rows[q] = nullptr;
            vecs[q] = nullptr;
            sg[q] = 0.0;
        }
    }
    double s = 0.0;
    for (int n = lane; n < N; n += 64) {
#pragma unroll
        for (int q = 0; q < kMaxTerms; ++q)
            if (q < nt) s = fma(sg[q] * rows[q][n], vecs[q][n], s);
    }
    // terms beyond kMaxTerms (q > 15) in a second sweep
    for (int q = kMaxTerms; q < nterms; ++q) {
        const GemvTerm tm = terms[q];
        const double* row = tm.blk + (size_t)wid * N;
        double p = 0.0;
        for (int n = lane; n < N; n += 64) p = fma(row[n], tm.vec[n], p);
        s = fma(tm.sign, p, s);
    }
    for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
    if (lane == 0) out[wid] = (add ? add[wid] : 0.0) + s;
}

#ifndef SW_BAND_WAVES
#define SW_BAND_WAVES 4   // wavefronts per output row of a band step
#endif
#ifndef SW_BAND_UNROLL
#define SW_BAND_UNROLL 4  // columns per lane whose loads are issued together
#endif

// One workgroup per output row of a band step: its kWaves wavefronts take the row's terms
// in turn, two at a time, so that each lane has several rows of operator blocks in flight;
// the per-wave dot products are added in a fixed order.
template <int kWaves>
__global__ __launch_bounds__(64 * kWaves) void k_band_pair(int N, const BandStep st) {
    const int row = blockIdx.x;
    const int i = row / N, r = row - i * N;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int t0 = st.first[i], t1 = st.first[i + 1];
    double s = 0.0;
    for (int t = t0 + w; t < t1; t += 2 * kWaves) {
        const bool two = t + kWaves < t1;
        const double* b0 = st.blk[t] + (size_t)r * N;
        const double* v0 = st.vec[t];
        const double* b1 = two ? st.blk[t + kWaves] + (size_t)r * N : b0;
        const double* v1 = two ? st.vec[t + kWaves] : v0;
        double p0 = 0.0, p1 = 0.0;
#pragma unroll SW_BAND_UNROLL
        for (int n = lane; n < N; n += 64) {
            p0 = fma(b0[n], v0[n], p0);
            p1 = fma(b1[n], v1[n], p1);
        }
        s = fma(st.sign[t], p0, s);
        if (two) s = fma(st.sign[t + kWaves], p1, s);
    }
    for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
    __shared__ double part[kWaves];
    if (lane == 0) part[w] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double sum = st.add[i] ? st.add[i][r] : 0.0;
        for (int k = 0; k < kWaves; ++k) sum += part[k];
        st.out[i][r] = sum;
    }
}

// The same step with the whole workgroup on each term: a workgroup computes kR
// consecutive output rows of one block row; thread t takes columns t + 256 c of each
// term (c < kCols, 256 kCols >= N), so that a term is one round of loads for all kR rows
// instead of N / 64 dependent ones per row, the term's vector is read once for the kR
// rows, and kTU terms are in flight together.  The per-thread sums are added across the
// workgroup in a fixed order.
template <int kCols, int kTU, int kR>
__global__ __launch_bounds__(256) void k_band_row(int N, const BandStep st) {
    const int nrb = (N + kR - 1) / kR;  // row groups per block row
    const int i = blockIdx.x / nrb;
    const int r0 = (blockIdx.x - i * nrb) * kR;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int t0 = st.first[i], t1 = st.first[i + 1];
    double s[kR];
#pragma unroll
    for (int rr = 0; rr < kR; ++rr) s[rr] = 0.0;
    for (int u = t0; u < t1; u += kTU) {
        double p[kTU][kR];
#pragma unroll
        for (int k = 0; k < kTU; ++k) {
#pragma unroll
            for (int rr = 0; rr < kR; ++rr) p[k][rr] = 0.0;
            if (u + k < t1) {
                const double* b = st.blk[u + k];
                const double* v = st.vec[u + k];
#pragma unroll
                for (int c = 0; c < kCols; ++c) {
                    const int n = t + 256 * c;
                    if (n < N) {
                        const double vn = v[n];
#pragma unroll
                        for (int rr = 0; rr < kR; ++rr)
                            if (r0 + rr < N)
                                p[k][rr] = fma(b[(size_t)(r0 + rr) * N + n], vn, p[k][rr]);
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < kTU; ++k)
            if (u + k < t1)
#pragma unroll
                for (int rr = 0; rr < kR; ++rr) s[rr] = fma(st.sign[u + k], p[k][rr], s[rr]);
    }
    __shared__ double part[kR][4];
#pragma unroll
    for (int rr = 0; rr < kR; ++rr) {
        double x = s[rr];
        for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
        if (lane == 0) part[rr][w] = x;
    }
    __syncthreads();
    if (t < kR && r0 + t < N) {
        const double sum = (part[t][0] + part[t][1]) + (part[t][2] + part[t][3]);
        st.out[i][r0 + t] = (st.add[i] ? st.add[i][r0 + t] : 0.0) + sum;
    }
}

// At 721 x 241, q = 16, one apply takes 8.2 ms with k_band_row (2 terms in flight, one
// output row per workgroup) against 10.4 ms with k_band_pair; two or four rows per
// workgroup (fewer workgroups) took 13.1 and 23.1 ms.
#ifndef SW_BAND_ROW_TU
#define SW_BAND_ROW_TU 2  // terms in flight per thread in k_band_row (0: k_band_pair)
#endif
#ifndef SW_BAND_ROW_R
#define SW_BAND_ROW_R 1   // output rows per workgroup in k_band_row
#endif

// q = 0: x_l = Dinv_l t_l for all l at once (wavefront per output row).
__global__ __launch_bounds__(256) void k_blockdiag_gemv(int N, int M, const double* __restrict__ S,
                                                        const double* __restrict__ t,
                                                        double* __restrict__ x) {
    const int wid = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (wid >= N * M) return;
    const int l = wid / N;
    const double* row = S + (size_t)l * N * N + (size_t)(wid - l * N) * N;
    const double* v = t + (size_t)l * N;
    double p = 0.0;
    for (int n = lane; n < N; n += 64) p = fma(row[n], v[n], p);
    for (int d = 32; d >= 1; d >>= 1) p += __shfl_xor(p, d, 64);
    if (lane == 0) x[wid] = p;
}

// One workgroup per output row of a super-row step (SuperStep): its four wavefronts
// take every fourth term, so that each has few dependent load rounds, and the four
// partial dot products are added in a fixed order.
__device__ __forceinline__ void super_step_row(int N, const SuperStep& st, int row) {
    const int i = row / N, r = row - i * N;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int t0 = st.first[i], t1 = st.first[i + 1];
    double s0 = 0.0, s1 = 0.0;
    int t = t0 + w;
    for (; t + 4 < t1; t += 8) {
        const double* b0 = st.blk[t] + (size_t)r * N;
        const double* b1 = st.blk[t + 4] + (size_t)r * N;
        const double* v0 = st.vec[t];
        const double* v1 = st.vec[t + 4];
        for (int n = lane; n < N; n += 64) {
            s0 = fma(b0[n], v0[n], s0);
            s1 = fma(b1[n], v1[n], s1);
        }
    }
    if (t < t1) {
        const double* b0 = st.blk[t] + (size_t)r * N;
        const double* v0 = st.vec[t];
        for (int n = lane; n < N; n += 64) s0 = fma(b0[n], v0[n], s0);
    }
    double sum = s0 + s1;
    for (int d = 32; d >= 1; d >>= 1) sum += __shfl_xor(sum, d, 64);
    __shared__ double part[4];
    if (lane == 0) part[w] = sum;
    __syncthreads();
    if (threadIdx.x == 0) st.out[i][r] = (part[0] + part[1]) + (part[2] + part[3]);
}

__global__ __launch_bounds__(256) void k_super_step(int N, const SuperStep st) {
    super_step_row(N, st, blockIdx.x);
}

// Step k of several applies in one launch: request p's step descriptor is st[p] (device
// copy of the handle's kernel arguments), its nrow N rows workgroups [first[p], first[p+1]).
struct StepBatch {
    const SuperStep* st[kMaxApplyBatch];
    int N[kMaxApplyBatch];
    int first[kMaxApplyBatch + 1];
    int n;
};
static_assert(sizeof(StepBatch) <= 4096, "kernel argument block");

__global__ __launch_bounds__(256) void k_super_step_batched(const StepBatch sb) {
    const int p = batch_member(sb.first, sb.n);
    super_step_row(sb.N[p], *sb.st[p], blockIdx.x - sb.first[p]);
}

// dst = 0, I, src or -src for a batch of N x N blocks; grid (chunks, jobs)
struct FillJob {
    double* dst;
    const double* src;
    int mode;  // 0 zero, 1 identity, 2 copy, 3 negated copy
    int pad;
};
struct FillBatch {
    FillJob j[64];
};
__global__ void k_fill_blocks(int N, FillBatch b) {
    const FillJob job = b.j[blockIdx.y];
    const size_t NN = (size_t)N * N;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < NN;
         e += (size_t)gridDim.x * blockDim.x) {
        double v = 0.0;
        if (job.mode == 1) {
            const size_t r = e / N;
            v = (e - r * N == r) ? 1.0 : 0.0;
        } else if (job.mode == 2) {
            v = job.src[e];
        } else if (job.mode == 3) {
            v = -job.src[e];
        }
        job.dst[e] = v;
    }
}

size_t blk_off(const sw_precond* P, int l, int slot) {
    return ((size_t)l * P->nb + slot) * (size_t)P->g.N * P->g.N;
}

void gemm_batched(int n, double alpha, const std::vector<GemmJob>& jobs, hipStream_t s) {
    for (size_t b = 0; b < jobs.size(); b += kMaxGemmJobs) {
        GemmBatch batch{};
        const int cnt = (int)std::min<size_t>(kMaxGemmJobs, jobs.size() - b);
        for (int i = 0; i < cnt; ++i) batch.j[i] = jobs[b + i];
        if (n <= 256) {
            dim3 grid((n + 31) / 32, (n + 31) / 32, cnt);
            if (n <= 192)
                k_gemm_ks<12><<<grid, 256, 0, s>>>(n, alpha, batch);
            else
                k_gemm_ks<16><<<grid, 256, 0, s>>>(n, alpha, batch);
        } else {
            dim3 grid((n + 63) / 64, (n + 63) / 64, cnt);
            k_gemm<2, 2, 16><<<grid, 256, 0, s>>>(n, alpha, batch);
        }
    }
}

// Row products (k_row_products), up to four per launch; problems whose mask is empty are
// dropped.
void row_products(int N, double alpha, const RowProd* rp, int np, hipStream_t s) {
    RowProdArgs args{};
    int total = 0;
    for (int i = 0; i < np; ++i) {
        unsigned any = 0;
        for (int a = 0; a < rp[i].na; ++a) any |= rp[i].mask[a];
        if (!any) continue;
        if (args.np == kMaxRowProds) {
            k_row_products<<<total, 256, 0, s>>>(N, alpha, args);
            args = RowProdArgs{};
            total = 0;
        }
        args.p[args.np] = rp[i];
        args.first[args.np++] = total;
        total += ((rp[i].na * N + 63) / 64) * ((rp[i].nb * N + 63) / 64);
    }
    if (args.np > 0) k_row_products<<<total, 256, 0, s>>>(N, alpha, args);
}


}  // namespace

namespace {
// scratch blocks: the output blocks of two inversions at once (N > 192) and, per chain of
// the elimination, 2q products for steps of either parity; or M inverses at once (q = 0,
// N > 192)
size_t tmp2_blocks(const Geo& g, int q) {
    if (q == 0) return (size_t)(g.N > 192 ? g.M : 1);
    return (size_t)(8 * q + 2);
}

// workspace of the diagonal-block inversions (N > 192), at least one N x N block
size_t gj_work_size(const Geo& g, int q) {
    const size_t NN = (size_t)g.N * g.N;
    return std::max(NN, gj_work_doubles(g.N, q == 0 ? g.M : 2));
}

// row sums of the K3 sum, one per row offset
size_t k3_rows_doubles(const Geo& g) { return (size_t)(2 * g.M - 1) * g.Nc; }
}  // namespace

// The elimination order and the super-row plan are in band_plan.hpp.
namespace {
#ifndef SW_SUPER_TARGET
#define SW_SUPER_TARGET 1000.0
#endif
constexpr double kSuperTarget = SW_SUPER_TARGET;  // b N: super-row height in grid rows

void fill_batched(int N, const std::vector<FillJob>& jobs, hipStream_t s) {
    const size_t NN = (size_t)N * N;
    const unsigned gx = (unsigned)std::min<size_t>((NN + 255) / 256, 64);
    for (size_t b = 0; b < jobs.size(); b += 64) {
        FillBatch fb{};
        const int cnt = (int)std::min<size_t>(64, jobs.size() - b);
        for (int i = 0; i < cnt; ++i) fb.j[i] = jobs[b + i];
        k_fill_blocks<<<dim3(gx, cnt), 256, 0, s>>>(N, fb);
    }
}

// Form W and W' of the given super rows from the band factors in P->S.  Only the
// factor blocks stored in the super rows' own block rows are read.  The forward and
// backward levels of one depth share a launch.
void super_operators(sw_precond* P, const SuperPlan& plan, const std::vector<int>& rows_of,
                     hipStream_t s) {
    const Geo& g = P->g;
    const int q = P->q, N = g.N;
    const size_t NN = (size_t)N * N;
    auto Wb = [&](int id) { return P->W + (size_t)id * NN; };
    auto Sb = [&](int r, int c) { return P->S + blk_off(P, r, c - r + q); };
    std::vector<FillJob> fills;
    for (int gi : rows_of) {
        const SuperRow& R = plan.fwd[gi];
        const int nb = (int)R.rows.size(), ne = (int)R.ext.size();
        for (int i = 0; i < nb; ++i)
            for (int c = 0; c < nb + ne; ++c) {
                if (R.id[i][c] < 0) continue;
                FillJob j{Wb(R.id[i][c]), nullptr, 0, 0};
                if (c < ne && coupled(R.rows[i], R.ext[c], q)) {
                    j.src = Sb(R.rows[i], R.ext[c]);  // L_{r,c}
                    j.mode = 3;
                } else if (c == ne + i) {
                    j.mode = 1;
                }
                fills.push_back(j);
            }
    }
    for (int gi : rows_of) {
        const SuperRow& R = plan.bwd[gi];
        const int nb = (int)R.rows.size(), ne = (int)R.ext.size();
        for (int i = 0; i < nb; ++i)
            for (int c = 0; c < nb + ne; ++c) {
                if (R.id[i][c] < 0) continue;
                FillJob j{Wb(R.id[i][c]), nullptr, 0, 0};
                if (c == i) {
                    j.src = Sb(R.rows[i], R.rows[i]);  // Dinv_r
                    j.mode = 2;
                } else if (c >= nb && coupled(R.rows[i], R.ext[c - nb], q)) {
                    j.src = Sb(R.rows[i], R.ext[c - nb]);  // G_{r,c}
                    j.mode = 3;
                }
                fills.push_back(j);
            }
    }
    fill_batched(N, fills, s);
    // level e, depth d: forward W_e -= L_{R_e, R_{e-d}} W_{e-d}; backward (i = nb - 1 - e)
    // W'_i -= G_{R_i, R_{i+d}} W'_{i+d}
    for (int e = 1; e < plan.b; ++e)
        for (int d = 1; d <= std::min(q, e); ++d) {
            std::vector<GemmJob> jobs;
            for (int gi : rows_of) {
                const SuperRow& R = plan.fwd[gi];
                if (e >= (int)R.rows.size() || !coupled(R.rows[e], R.rows[e - d], q)) continue;
                for (size_t c = 0; c < R.id[e].size(); ++c) {
                    const int src = R.id[e - d][c];
                    if (src < 0) continue;
                    double* dst = Wb(R.id[e][c]);
                    jobs.push_back(GemmJob{Sb(R.rows[e], R.rows[e - d]), Wb(src), dst, dst});
                }
            }
            for (int gi : rows_of) {
                const SuperRow& R = plan.bwd[gi];
                const int i = (int)R.rows.size() - 1 - e;
                if (i < 0 || !coupled(R.rows[i], R.rows[i + d], q)) continue;
                for (size_t c = 0; c < R.id[i].size(); ++c) {
                    const int src = R.id[i + d][c];
                    if (src < 0) continue;
                    double* dst = Wb(R.id[i][c]);
                    jobs.push_back(GemmJob{Sb(R.rows[i], R.rows[i + d]), Wb(src), dst, dst});
                }
            }
            gemm_batched(N, -1.0, jobs, s);
        }
}

// Kernel arguments of the super-row steps: forward inputs y (= work + 3 NM) and t2
// (= work + NM), output y; backward inputs y and x (= work + 2 NM), output x.  Backward
// steps are stored in launch order.
void super_steps(sw_precond* P, const SuperPlan& plan) {
    const Geo& g = P->g;
    const int N = g.N;
    const size_t NN = (size_t)N * N, NM = g.NM;
    auto Wb = [&](int id) { return P->W + (size_t)id * NN; };
    double* t2 = P->work + NM;
    double* xv = P->work + 2 * NM;
    double* yv = P->work + 3 * NM;
    auto make = [&](const std::vector<int>& stage, bool fwd) {
        SuperStep st{};
        int t = 0, row = 0;
        for (int gi : stage) {
            const SuperRow& R = fwd ? plan.fwd[gi] : plan.bwd[gi];
            const int nb = (int)R.rows.size(), ne = (int)R.ext.size();
            for (int i = 0; i < nb; ++i, ++row) {
                st.first[row] = t;
                st.out[row] = (fwd ? yv : xv) + (size_t)R.rows[i] * N;
                for (int c = 0; c < nb + ne; ++c) {
                    if (R.id[i][c] < 0) continue;
                    const double* v;
                    if (fwd)
                        v = (c < ne) ? yv + (size_t)R.ext[c] * N : t2 + (size_t)R.rows[c - ne] * N;
                    else
                        v = (c < nb) ? yv + (size_t)R.rows[c] * N : xv + (size_t)R.ext[c - nb] * N;
                    if (t >= kMaxSuperTerms)
                        throw Error{SW_EINVAL, "super-row step has too many terms"};
                    st.blk[t] = Wb(R.id[i][c]);
                    st.vec[t] = v;
                    ++t;
                }
            }
        }
        st.nrow = row;
        st.first[row] = t;
        return st;
    };
    P->fsteps.clear();
    P->bsteps.clear();
    for (const auto& stage : plan.stages) P->fsteps.push_back(make(stage, true));
    for (size_t k = plan.stages.size(); k-- > 0;) P->bsteps.push_back(make(plan.stages[k], false));
}

// Block LU of the band in the elimination order of make_order.  Step s < max(k, nB)
// eliminates top row s and bottom row M-1-s together: one inversion launch for both
// diagonal blocks, their products in the same GEMM launches.  The separator rows follow
// one per step.  For a row l and each later-eliminated row i, j coupled to it:
//   L_{i,l} = S_il Dinv_l,  G_{l,j} = Dinv_l S_lj,  S_ij -= S_il G_{l,j}.
// G replaces S_lj in the launch of the Schur updates (which do not read it); L replaces
// S_il in the next step's first launch (the Schur updates read S_il).  Products go to the
// scratch of their chain and step parity.  The two chains meet only on the separator's
// own blocks; a bottom update of a block that the top chain updates in the same step
// goes to a launch of its own.
//
// With a second stream s2 (new_event gives it events), only the Schur updates of the
// next step's diagonal blocks stay on s: the next inversion needs nothing else, and the
// other updates and the G copies run on s2 beside it.  s waits for them before the next
// step's products (which read those blocks and overwrite S_il).  done(step) runs once a
// step's work is ordered before anything later enqueued on s, and done(INT_MAX) after
// the last.
// Blocks wider than this take the second stream: there an inversion (strip launches,
// about 330 us at N = 241) hides the other updates, and the split paid 17% of the set-up at
// 241x81; with the register-tile inversion (about 115 us at N = 181) the waits between the
// streams cost more than the overlap saved.
constexpr int kSplitSchurN = 192;

void factor_band(sw_precond* P, const Order& o, hipStream_t s, hipStream_t s2,
                 const std::function<hipEvent_t()>& new_event,
                 const std::function<void(int)>& done) {
    const Geo& g = P->g;
    const int q = P->q, M = g.M;
    const size_t NN = (size_t)g.N * g.N;
    auto Sb = [&](int r, int c) { return P->S + blk_off(P, r, c - r + q); };
    double* gjt = P->tmp2;  // output blocks of an N > 192 inversion (two)
    auto half = [&](int ch, int par) {
        return P->tmp2 + NN * (2 + (size_t)(2 * ch + par) * 2 * q);
    };
    const int ns = std::max(o.k, o.nB), nsteps = ns + q;
    auto rows_of = [&](int step, int* rows) {
        int nr = 0;
        if (step < ns) {
            if (step < o.k) rows[nr++] = step;
            if (step < o.nB) rows[nr++] = M - 1 - step;
        } else if (step < nsteps) {
            rows[nr++] = o.k + (step - ns);
        }
        return nr;
    };
    std::vector<GemmJob> pendingL;
    hipEvent_t side_done = nullptr;  // the previous step's work on s2
    for (int step = 0; step < nsteps; ++step) {
        int rows[2], next[2];
        const int nr = rows_of(step, rows);
        const int nnext = rows_of(step + 1, next);
        // the bottom row's diagonal block is at a higher address than the top row's
        double* d0 = Sb(rows[0], rows[0]);
        const size_t stride = (nr == 2) ? (size_t)(Sb(rows[1], rows[1]) - d0) : 0;
        gj_inverse(g.N, d0, stride, nr, P->info + 2 * step, gjt, P->tmp, s);
        if (side_done) {
            SW_HIP(hipStreamWaitEvent(s, side_done, 0));
            side_done = nullptr;
            done(step - 1);
        }
        // wave a: top chain and non-conflicting bottom updates; wave b: bottom updates of
        // blocks that the top chain updates in this step
        std::vector<GemmJob> jobs1 = pendingL, diag_a, diag_b, rest_a, rest_b;
        pendingL.clear();
        std::vector<const double*> top_targets;
        // with N > 256 and consecutive coupled rows, a row's L and G run as two row
        // products (rp_lg) and its Schur updates outside the diagonal launches as one
        // (rp_rest, and rp_late for the bottom updates that must wait for the top chain's)
        RowProd rp_lg[4], rp_rest[2], rp_late[2];
        int nrp = 0, nlg = 0;
        for (int e = 0; e < nr; ++e) {
            const int l = rows[e];
            const int ch = (step < ns && l >= o.k) ? 1 : 0;
            const int pl = o.rank[l];
            std::vector<int> nbr;
            for (int c = std::max(0, l - q); c <= std::min(M - 1, l + q); ++c)
                if (c != l && o.rank[c] > pl) nbr.push_back(c);
            if (nbr.empty()) continue;
            double* sc = half(ch, step & 1);
            const int nn = (int)nbr.size();
            // the products address C(a, b) as C(a, 0) + b N^2 and G's right factors
            // S(l, nbr[b]) as S(l, nbr[0]) + b N^2: the coupled rows must be consecutive
            // band rows
            bool consecutive = g.N > 256 && nn <= kMaxRowNbr;
            for (int a = 0; a < nn && consecutive; ++a)
                for (int b = 0; b < nn && consecutive; ++b)
                    consecutive = Sb(nbr[a], nbr[b]) == Sb(nbr[a], nbr[0]) + (size_t)b * NN &&
                                  Sb(l, nbr[b]) == Sb(l, nbr[0]) + (size_t)b * NN;
            RowProd* rr = nullptr;
            RowProd* rl = nullptr;
            if (consecutive) {
                const unsigned all = (nn == 32) ? ~0u : ((1u << nn) - 1u);
                // L_{nbr[a], l} = S(nbr[a], l) Dinv_l into the scratch's first nn blocks
                RowProd& L = rp_lg[nlg++];
                L = RowProd{};
                L.B = Sb(l, l);
                L.na = nn;
                L.nb = 1;
                for (int a = 0; a < nn; ++a) {
                    L.A[a] = Sb(nbr[a], l);
                    L.Crow[a] = sc + (size_t)a * NN;
                    L.mask[a] = 1u;
                }
                // G_{l, nbr[b]} = Dinv_l S(l, nbr[b]) into blocks q, q + 1, ...
                RowProd& Gp = rp_lg[nlg++];
                Gp = RowProd{};
                Gp.A[0] = Sb(l, l);
                Gp.B = Sb(l, nbr[0]);
                Gp.Crow[0] = sc + (size_t)q * NN;
                Gp.mask[0] = all;
                Gp.na = 1;
                Gp.nb = nn;
                rr = &rp_rest[nrp];
                rl = &rp_late[nrp];
                ++nrp;
                *rr = RowProd{};
                rr->B = sc + (size_t)q * NN;
                rr->na = rr->nb = nn;
                rr->accumulate = 1;
                for (int a = 0; a < nn; ++a) {
                    rr->A[a] = Sb(nbr[a], l);
                    rr->Crow[a] = Sb(nbr[a], nbr[0]);
                }
                *rl = *rr;
            } else {
                for (int a = 0; a < nn; ++a)
                    jobs1.push_back(
                        GemmJob{Sb(nbr[a], l), Sb(l, l), nullptr, sc + (size_t)a * NN});
                for (int b = 0; b < nn; ++b)
                    jobs1.push_back(
                        GemmJob{Sb(l, l), Sb(l, nbr[b]), nullptr, sc + (size_t)(q + b) * NN});
            }
            for (int a = 0; a < nn; ++a)
                for (int b = 0; b < nn; ++b) {
                    double* Sij = Sb(nbr[a], nbr[b]);
                    const GemmJob j{Sb(nbr[a], l), sc + (size_t)(q + b) * NN, Sij, Sij};
                    const bool late = ch == 1 && std::find(top_targets.begin(), top_targets.end(),
                                                           Sij) != top_targets.end();
                    bool diag = false;
                    for (int x = 0; x < nnext; ++x) diag = diag || Sij == Sb(next[x], next[x]);
                    if (!s2) diag = false;  // one stream: everything in the rest launches
                    if (!diag && rr) {
                        (late ? rl : rr)->mask[a] |= 1u << b;
                    } else {
                        (diag ? (late ? diag_b : diag_a) : (late ? rest_b : rest_a)).push_back(j);
                    }
                    if (ch == 0) top_targets.push_back(Sij);
                }
            for (int b = 0; b < nn; ++b)
                rest_a.push_back(
                    GemmJob{sc + (size_t)(q + b) * NN, nullptr, nullptr, Sb(l, nbr[b])});
            for (int a = 0; a < nn; ++a)
                pendingL.push_back(GemmJob{sc + (size_t)a * NN, nullptr, nullptr, Sb(nbr[a], l)});
        }
        if (!jobs1.empty()) gemm_batched(g.N, 1.0, jobs1, s);
        row_products(g.N, 1.0, rp_lg, nlg, s);
        hipStream_t rs = s;
        if (s2 && (!rest_a.empty() || !rest_b.empty() || nrp > 0)) {
            hipEvent_t e = new_event();
            SW_HIP(hipEventRecord(e, s));
            SW_HIP(hipStreamWaitEvent(s2, e, 0));
            rs = s2;
        }
        if (!diag_a.empty()) gemm_batched(g.N, -1.0, diag_a, s);
        if (!diag_b.empty()) gemm_batched(g.N, -1.0, diag_b, s);
        row_products(g.N, -1.0, rp_rest, nrp, rs);
        if (!rest_a.empty()) gemm_batched(g.N, -1.0, rest_a, rs);
        row_products(g.N, -1.0, rp_late, nrp, rs);
        if (!rest_b.empty()) gemm_batched(g.N, -1.0, rest_b, rs);
        if (rs != s) {
            side_done = new_event();
            SW_HIP(hipEventRecord(side_done, rs));
        } else if (step + 1 < nsteps) {
            done(step);
        }
    }
    if (side_done) SW_HIP(hipStreamWaitEvent(s, side_done, 0));
    if (!pendingL.empty()) gemm_batched(g.N, 1.0, pendingL, s);
    done(INT_MAX);
}
}  // namespace

size_t precond_bytes_estimate(const Geo& g, int q_req) {
    const int q = std::max(0, std::min(q_req, g.M - 1));
    const int nb = 2 * q + 1;
    const size_t N = g.N, NN = N * N, NM = g.NM;
    const size_t nw = choose_super(g.N, make_order(g.M, q), q, kSuperTarget).nblocks;
    return carve_size({(size_t)g.M * nb * NN * 8, NN * 8, (size_t)g.ncol * 8, 4 * NM * 8,
                       gj_work_size(g, q) * 8, tmp2_blocks(g, q) * NN * 8, (size_t)g.M * 8,
                       k3_rows_doubles(g) * 8, nw * NN * 8});
}

size_t precond_bytes(const sw_precond* P) { return P ? P->block : 0; }

bool precond_matches(const sw_precond* P, const Geo& g) {
    return P && P->g.N == g.N && P->g.M == g.M && P->g.x1 == g.x1 && P->g.xN == g.xN &&
           P->g.yM == g.yM;
}

namespace {
void capture_substitution(sw_precond* P);
void band_steps(sw_precond* P, const Order& o, const std::vector<GemvTerm>& tv);
}

namespace {
// Helper streams and events are reused across builds: creating and destroying them
// costs the host about as much as a factorisation step.  They live until the process
// ends (one per concurrent build and device).
struct SidePool {
    std::mutex mu;
    std::vector<std::pair<int, hipStream_t>> streams;
    std::vector<std::pair<int, hipEvent_t>> events;
};
SidePool& side_pool() {
    static SidePool* p = new SidePool();  // never destroyed: used until exit
    return *p;
}

}  // namespace

hipStream_t side_stream_take() {
    int dev = 0;
    SW_HIP(hipGetDevice(&dev));
    {
        SidePool& p = side_pool();
        std::lock_guard<std::mutex> lk(p.mu);
        for (size_t i = 0; i < p.streams.size(); ++i)
            if (p.streams[i].first == dev) {
                hipStream_t st = p.streams[i].second;
                p.streams.erase(p.streams.begin() + i);
                return st;
            }
    }
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return st;
}

void side_stream_give(hipStream_t st) {
    if (!st) return;
    int dev = 0;
    SW_HIP(hipGetDevice(&dev));
    SidePool& p = side_pool();
    std::lock_guard<std::mutex> lk(p.mu);
    p.streams.emplace_back(dev, st);
}

namespace {
// A helper stream and the events that order it after s.  It goes back to the pool only
// once s (which waits for the helper at the end) has been synchronised, or after
// draining both.
struct SideStream {
    int dev = -1;
    hipStream_t aux = nullptr;
    std::vector<hipEvent_t> evs;
    SideStream() = default;
    SideStream(const SideStream&) = delete;
    SideStream& operator=(const SideStream&) = delete;
    void open() {  // without a helper stream the work stays on s
        if (aux) return;
        SW_HIP(hipGetDevice(&dev));
        aux = side_stream_take();
    }
    hipEvent_t event() {
        hipEvent_t e = nullptr;
        {
            SidePool& p = side_pool();
            std::lock_guard<std::mutex> lk(p.mu);
            for (size_t i = 0; i < p.events.size(); ++i)
                if (p.events[i].first == dev) {
                    e = p.events[i].second;
                    p.events.erase(p.events.begin() + i);
                    break;
                }
        }
        if (!e) SW_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        evs.push_back(e);
        return e;
    }
    ~SideStream() {
        if (!aux) return;
        (void)hipStreamSynchronize(aux);
        {
            SidePool& p = side_pool();
            std::lock_guard<std::mutex> lk(p.mu);
            for (hipEvent_t e : evs) p.events.emplace_back(dev, e);
        }
        side_stream_give(aux);
    }
};

// The band factorisation on s, and the super-row operators of each stage on the helper
// stream as soon as the step that eliminates the stage's last rows is enqueued: the
// chain of inversions leaves most of the device idle.  s then waits for the helper.
void factor_with_super(sw_precond* P, const Order& o, const SuperPlan& plan, SideStream& side,
                       SideStream& side2, hipStream_t s) {
    side.open();
    if (P->g.N > kSplitSchurN) side2.open();
    std::vector<int> ready(plan.stages.size(), 0);
    for (size_t k = 0; k < plan.stages.size(); ++k)
        for (int gi : plan.stages[k])
            for (int r : plan.fwd[gi].rows) ready[k] = std::max(ready[k], elim_step(o, r));
    std::vector<size_t> by_ready(plan.stages.size());
    for (size_t k = 0; k < by_ready.size(); ++k) by_ready[k] = k;
    std::stable_sort(by_ready.begin(), by_ready.end(),
                     [&](size_t a, size_t b) { return ready[a] < ready[b]; });
    size_t next = 0;
    factor_band(P, o, s, side2.aux, [&]() { return side2.event(); }, [&](int step) {
        while (next < by_ready.size() && ready[by_ready[next]] <= step) {
            const auto& stage = plan.stages[by_ready[next++]];
            if (!side.aux) continue;  // built on s after the factorisation
            hipEvent_t e = side.event();
            SW_HIP(hipEventRecord(e, s));
            SW_HIP(hipStreamWaitEvent(side.aux, e, 0));
            super_operators(P, plan, stage, side.aux);
        }
    });
    if (side.aux) {
        hipEvent_t e = side.event();
        SW_HIP(hipEventRecord(e, side.aux));
        SW_HIP(hipStreamWaitEvent(s, e, 0));
    } else {
        std::vector<int> all(plan.fwd.size());
        for (size_t i = 0; i < all.size(); ++i) all[i] = (int)i;
        super_operators(P, plan, all, s);
    }
}
}  // namespace

namespace {
// The device block of a destroyed preconditioner is kept for the next build of a
// similar size on the same device: allocating and freeing a few hundred MB costs the host
// a large share of a set-up, and hipFree waits for the whole device.  At most one block
// of up to kKeepBytes per device is kept, until the process ends or an allocation fails.
constexpr size_t kKeepBytes = (size_t)2 << 30;
struct KeptBlock {
    int dev;
    void* p;
    size_t bytes;
};
std::mutex& keep_mu() {
    static std::mutex* m = new std::mutex();
    return *m;
}
std::vector<KeptBlock>& kept() {
    static std::vector<KeptBlock>* v = new std::vector<KeptBlock>();
    return *v;
}

// A block of at least `bytes` on the current device, or nullptr; *got is its size.
void* precond_alloc(size_t bytes, size_t* got) {
    int dev = 0;
    SW_HIP(hipGetDevice(&dev));
    {
        std::lock_guard<std::mutex> lk(keep_mu());
        auto& v = kept();
        for (size_t i = 0; i < v.size(); ++i)
            if (v[i].dev == dev && v[i].bytes >= bytes && v[i].bytes <= bytes + bytes / 2) {
                void* p = v[i].p;
                *got = v[i].bytes;
                v.erase(v.begin() + i);
                return p;
            }
    }
    void* mem = nullptr;
    if (hipMalloc(&mem, bytes) != hipSuccess) {
        (void)hipGetLastError();
        std::vector<void*> drop;
        {
            std::lock_guard<std::mutex> lk(keep_mu());
            auto& v = kept();
            for (size_t i = v.size(); i-- > 0;)
                if (v[i].dev == dev) {
                    drop.push_back(v[i].p);
                    v.erase(v.begin() + i);
                }
        }
        for (void* p : drop) (void)hipFree(p);
        if (drop.empty() || hipMalloc(&mem, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
    }
    *got = bytes;
    return mem;
}

// Return a block no kernel uses any more (the caller has synchronised its work).
void precond_release(void* p, size_t bytes, int dev) {
    if (!p) return;
    if (bytes <= kKeepBytes) {
        std::lock_guard<std::mutex> lk(keep_mu());
        auto& v = kept();
        bool have = false;
        for (const KeptBlock& b : v) have = have || b.dev == dev;
        if (!have) {
            v.push_back(KeptBlock{dev, p, bytes});
            return;
        }
    }
    (void)hipFree(p);
}
}  // namespace

sw_precond* precond_build(const Geo& g0, int q_req, hipStream_t s) {
    SW_REQUIRE(g0.N <= kMaxN, "the preconditioner needs N <= 1024");
    Geo g = g0;
    g.precision = SW_PREC_FP64;
    const int q = std::max(0, std::min(q_req, g.M - 1));
    const int nb = 2 * q + 1;
    const size_t N = g.N, NN = N * N, NM = g.NM;
    const size_t bytes = precond_bytes_estimate(g, q);
    (void)N;
    auto* P = new sw_precond();
    P->g = g;
    P->q = q;
    P->nb = nb;
    SW_HIP(hipGetDevice(&P->device));
    void* mem = precond_alloc(bytes, &P->block);
    if (!mem) {
        delete P;
        throw Error{SW_ENOMEM, "device allocation of the preconditioner failed"};
    }
    P->base = static_cast<double*>(mem);
    P->bytes = bytes;
    Carve c(mem);
    P->S = c.take<double>((size_t)g.M * nb * NN);
    P->Wc = c.take<double>(NN);
    P->k3 = c.take<double>(g.ncol);
    P->work = c.take<double>(4 * NM);
    P->tmp = c.take<double>(gj_work_size(g, q));
    P->tmp2 = c.take<double>(tmp2_blocks(g, q) * NN);
    P->info = c.take<int>(2 * (size_t)g.M);
    double* k3rows = c.take<double>(k3_rows_doubles(g));
    const Order order = make_order(g.M, q);
    const SuperPlan plan = choose_super(g.N, order, q, kSuperTarget);
    P->sb = plan.b;
    P->W = c.take<double>(plan.nblocks * NN);
    try {
        k_wmat<<<(g.N + 63) / 64, 64, 0, s>>>(g, P->Wc);
        k_k3_rows<<<dim3((g.Nc + 255) / 256, 2 * g.M - 1), 256, 0, s>>>(g, k3rows);
        k_k3_sum<<<(g.ncol + 255) / 256, 256, 0, s>>>(g, k3rows, P->k3);
        const dim3 ag((unsigned)std::min<size_t>((NN + 1023) / 1024, 4096),
                      (unsigned)std::min(g.M * nb, 65535));
        k_assemble<<<ag, 256, 0, s>>>(g, q, P->k3, P->Wc, P->S);
        SW_HIP(hipMemsetAsync(P->info, 0, 2 * (size_t)g.M * sizeof(int), s));
        // declared before the synchronisation below, released after it
        SideStream side, side2;
        if (q == 0) {
            gj_inverse(g.N, P->S, NN, g.M, P->info, P->tmp2, P->tmp, s);
        } else if (P->sb > 1) {
            factor_with_super(P, order, plan, side, side2, s);
        } else {
            if (g.N > kSplitSchurN) side2.open();
            factor_band(P, order, s, side2.aux, [&]() { return side2.event(); }, [](int) {});
        }
        if (q > 0 && P->sb > 1) {
            super_steps(P, plan);
            capture_substitution(P);
            std::vector<SuperStep> all(P->fsteps);
            all.insert(all.end(), P->bsteps.begin(), P->bsteps.end());
            SW_HIP(hipMalloc(&P->dsteps, all.size() * sizeof(SuperStep)));
            SW_HIP(hipMemcpyAsync(P->dsteps, all.data(), all.size() * sizeof(SuperStep),
                                  hipMemcpyHostToDevice, s));
            SW_HIP(hipStreamSynchronize(s));
        } else if (q > 0) {
            std::vector<GemvTerm> tv;
            double* tmpv = P->work + 3 * NM;
            double* xv = P->work + 2 * NM;
            P->fwd_off.resize(g.M);
            P->fwd_cnt.resize(g.M);
            P->bwd_off.resize(g.M);
            P->bwd_cnt.resize(g.M);
            P->ord = order.ord;
            // position p of the elimination order, block row l = ord[p]:
            //   forward  y_l = t_l - sum L_{l,c} y_c over earlier c
            //   backward x_l = Dinv_l y_l - sum G_{l,c} x_c over later c
            for (int p = 0; p < g.M; ++p) {
                const int l = order.ord[p];
                P->fwd_off[p] = (int)tv.size();
                for (int c = std::max(0, l - q); c <= std::min(g.M - 1, l + q); ++c)
                    if (order.rank[c] < p)
                        tv.push_back(GemvTerm{P->S + blk_off(P, l, c - l + q),
                                              tmpv + (size_t)c * N, -1.0, 0.0});
                P->fwd_cnt[p] = (int)tv.size() - P->fwd_off[p];
            }
            for (int p = 0; p < g.M; ++p) {
                const int l = order.ord[p];
                P->bwd_off[p] = (int)tv.size();
                tv.push_back(GemvTerm{P->S + blk_off(P, l, q), tmpv + (size_t)l * N, 1.0, 0.0});
                for (int c = std::max(0, l - q); c <= std::min(g.M - 1, l + q); ++c)
                    if (order.rank[c] > p)
                        tv.push_back(GemvTerm{P->S + blk_off(P, l, c - l + q),
                                              xv + (size_t)c * N, -1.0, 0.0});
                P->bwd_cnt[p] = (int)tv.size() - P->bwd_off[p];
            }
            SW_HIP(hipMalloc(&P->terms, tv.size() * sizeof(GemvTerm)));
            SW_HIP(hipMemcpy(P->terms, tv.data(), tv.size() * sizeof(GemvTerm),
                             hipMemcpyHostToDevice));
            band_steps(P, order, tv);
            capture_substitution(P);
        }
        SW_HIP(hipGetLastError());
        std::vector<int> info(2 * (size_t)g.M);
        SW_HIP(hipMemcpyAsync(info.data(), P->info, info.size() * sizeof(int),
                              hipMemcpyDeviceToHost, s));
        SW_HIP(hipStreamSynchronize(s));
        for (int v : info)
            if (v != 0) throw Error{SW_ENONFINITE, "preconditioner: singular diagonal block"};
    } catch (...) {
        (void)hipStreamSynchronize(s);
        precond_release(P->base, P->block, P->device);
        if (P->terms) (void)hipFree(P->terms);
        if (P->dsteps) (void)hipFree(P->dsteps);
        if (P->subst) (void)hipGraphExecDestroy(P->subst);
        delete P;
        throw;
    }
    return P;
}

namespace {
// Kernel arguments of the paired band steps (one block row per super row): forward, the
// top-chain row and the bottom-chain row of each factorisation step together (they share
// no coupling), then the separator rows one by one; backward in the reverse order.  Left
// empty (one launch per block row from the device term lists) if a step has more terms
// than its argument block holds.
void band_steps(sw_precond* P, const Order& o, const std::vector<GemvTerm>& tv) {
    const Geo& g = P->g;
    const size_t NM = g.NM;
    const int N = g.N;
    double* t2 = P->work + NM;
    double* s2 = P->work + 2 * NM;
    double* tmp = P->work + 3 * NM;
    std::vector<BandStep> steps;
    auto add = [&](const std::vector<int>& ps, bool fwd) {
        BandStep st{};
        st.nrow = (int)ps.size();
        int nt = 0;
        for (int i = 0; i < st.nrow; ++i) {
            const int p = ps[i], l = o.ord[p];
            const int off = fwd ? P->fwd_off[p] : P->bwd_off[p];
            const int cnt = fwd ? P->fwd_cnt[p] : P->bwd_cnt[p];
            st.first[i] = nt;
            if (nt + cnt > kMaxBandTerms) return false;
            for (int t = 0; t < cnt; ++t, ++nt) {
                st.blk[nt] = tv[off + t].blk;
                st.vec[nt] = tv[off + t].vec;
                st.sign[nt] = tv[off + t].sign;
            }
            st.add[i] = fwd ? t2 + (size_t)l * N : nullptr;
            st.out[i] = (fwd ? tmp : s2) + (size_t)l * N;
        }
        st.first[st.nrow] = nt;
        steps.push_back(st);
        return true;
    };
    const int chain = std::max(o.k, o.nB), M = g.M;
    auto pair = [&](int j) {
        std::vector<int> ps;
        if (j < o.k) ps.push_back(j);
        if (j < o.nB) ps.push_back(o.k + j);
        return ps;
    };
    bool ok = true;
    for (int j = 0; j < chain && ok; ++j) ok = add(pair(j), true);
    for (int p = o.k + o.nB; p < M && ok; ++p) ok = add({p}, true);
    for (int p = M - 1; p >= o.k + o.nB && ok; --p) ok = add({p}, false);
    for (int j = chain - 1; j >= 0 && ok; --j) ok = add(pair(j), false);
    if (ok) P->band_steps.swap(steps);
}



// Block forward and backward substitution with the band factors (q >= 1); all
// pointers live in the preconditioner, so the sequence can be captured once.
void enqueue_substitution(const sw_precond* P, hipStream_t s) {
    const Geo& g = P->g;
    const size_t NM = g.NM;
    const int N = g.N;
    double* t2 = P->work + NM;
    double* s2 = P->work + 2 * NM;
    double* tmp = P->work + 3 * NM;
    if (P->sb > 1) {
        // y in tmp, x in s2 (the step arguments point there); backward steps are stored
        // in launch order
        for (const SuperStep& st : P->fsteps)
            k_super_step<<<(unsigned)(st.nrow * N), 256, 0, s>>>(N, st);
        for (const SuperStep& st : P->bsteps)
            k_super_step<<<(unsigned)(st.nrow * N), 256, 0, s>>>(N, st);
        return;
    }
    if (!P->band_steps.empty()) {
        for (const BandStep& st : P->band_steps) {
#if SW_BAND_ROW_TU > 0
            constexpr int kR = SW_BAND_ROW_R;
            const unsigned grid = (unsigned)(st.nrow * ((N + kR - 1) / kR));
            if (N <= 768)
                k_band_row<3, SW_BAND_ROW_TU, kR><<<grid, 256, 0, s>>>(N, st);
            else if (N <= 1024)
                k_band_row<4, SW_BAND_ROW_TU, kR><<<grid, 256, 0, s>>>(N, st);
            else
#endif
                k_band_pair<SW_BAND_WAVES>
                    <<<(unsigned)(st.nrow * N), 64 * SW_BAND_WAVES, 0, s>>>(N, st);
        }
        return;
    }
    const GemvTerm* terms = static_cast<const GemvTerm*>(P->terms);
    const unsigned blocks = (unsigned)((N * 64 + 255) / 256);
    // forward in elimination order (y in tmp), backward in reverse (x in s2)
    for (int p = 0; p < g.M; ++p) {
        const int l = P->ord[p];
        k_band_step<<<blocks, 256, 0, s>>>(N, terms + P->fwd_off[p], P->fwd_cnt[p],
                                           t2 + (size_t)l * N, tmp + (size_t)l * N);
    }
    for (int p = g.M - 1; p >= 0; --p) {
        const int l = P->ord[p];
        k_band_step<<<blocks, 256, 0, s>>>(N, terms + P->bwd_off[p], P->bwd_cnt[p], nullptr,
                                           s2 + (size_t)l * N);
    }
}

// Capture the substitution launches into an executable graph (kernel nodes only).
void capture_substitution(sw_precond* P) {
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    hipGraph_t graph = nullptr;
    bool ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
        enqueue_substitution(P, cs);
        ok = hipStreamEndCapture(cs, &graph) == hipSuccess && graph != nullptr;
    }
    if (ok) ok = hipGraphInstantiate(&P->subst, graph, nullptr, nullptr, 0) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        P->subst = nullptr;
    }
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipStreamDestroy(cs);
}
}  // namespace

void precond_apply(const sw_precond* P, const double* b, double* x, hipStream_t s) {
    const Geo& g = P->g;
    const size_t NM = g.NM;
    double* s1 = P->work;
    double* t2 = P->work + NM;
    double* s2 = P->work + 2 * NM;
    k_apply_first<<<g.M, 64, 0, s>>>(g, b, s1, t2);
    const int N = g.N;
    if (P->q == 0) {
        const int rows = N * g.M;
        k_blockdiag_gemv<<<(rows * 64 + 255) / 256, 256, 0, s>>>(N, g.M, P->S, t2, s2);
    } else if (P->subst) {
        SW_HIP(hipGraphLaunch(P->subst, s));
    } else {
        enqueue_substitution(P, s);
    }
    k_apply_last<<<g.M, 64, 0, s>>>(g, s1, s2, x);
    SW_HIP(hipGetLastError());
}

// Applies of several handles in shared launches.  Handles with super-row substitution
// go in rounds of distinct handles (a handle holds its apply's temporaries): one launch
// for the first step of every request in the round, then launch k runs step k of every
// request that has one (a request's steps: its forward steps, then its backward steps),
// then one launch for the last step.  Each request runs the same per-row arithmetic as
// precond_apply, so its result has the same bits.  A round of one request, and every
// other handle, goes through precond_apply.
void precond_apply_batched(int n, const sw_precond* const* P, const double* const* b,
                           double* const* x, hipStream_t s) {
    std::vector<int> pending;
    for (int i = 0; i < n; ++i) {
        if (P[i]->q > 0 && P[i]->sb > 1 && P[i]->dsteps)
            pending.push_back(i);
        else
            precond_apply(P[i], b[i], x[i], s);
    }
    while (!pending.empty()) {
        std::vector<int> round, later;
        for (int i : pending) {
            bool dup = (int)round.size() >= kMaxApplyBatch;
            for (int j : round) dup = dup || P[j] == P[i];
            (dup ? later : round).push_back(i);
        }
        pending.swap(later);
        if (round.size() == 1) {
            precond_apply(P[round[0]], b[round[0]], x[round[0]], s);
            continue;
        }
        const int nr = (int)round.size();
        ApplyBatch ab{};
        int rows = 0, nsteps = 0;
        for (int k = 0; k < nr; ++k) {
            const sw_precond* Q = P[round[k]];
            ab.g[k] = Q->g;
            ab.work[k] = Q->work;
            ab.in[k] = b[round[k]];
            ab.out[k] = x[round[k]];
            ab.first[k] = rows;
            rows += Q->g.M;
            nsteps = std::max(nsteps, (int)(Q->fsteps.size() + Q->bsteps.size()));
        }
        ab.first[nr] = rows;
        ab.n = nr;
        k_apply_first_batched<<<rows, 64, 0, s>>>(ab);
        for (int t = 0; t < nsteps; ++t) {
            StepBatch sb{};
            int wg = 0;
            for (int k = 0; k < nr; ++k) {
                const sw_precond* Q = P[round[k]];
                const int nf = (int)Q->fsteps.size();
                if (t >= nf + (int)Q->bsteps.size()) continue;
                const SuperStep& hs = (t < nf) ? Q->fsteps[t] : Q->bsteps[t - nf];
                sb.st[sb.n] = Q->dsteps + t;
                sb.N[sb.n] = Q->g.N;
                sb.first[sb.n] = wg;
                wg += hs.nrow * Q->g.N;
                ++sb.n;
            }
            sb.first[sb.n] = wg;
            k_super_step_batched<<<wg, 256, 0, s>>>(sb);
        }
        k_apply_last_batched<<<rows, 64, 0, s>>>(ab);
        SW_HIP(hipGetLastError());
    }
}

void precond_destroy(sw_precond* P, bool keep_block) {
    if (!P) return;
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (P->device >= 0 && P->device != cur) (void)hipSetDevice(P->device);
    (void)hipDeviceSynchronize();
    if (keep_block)
        precond_release(P->base, P->block, P->device);
    else
        (void)hipFree(P->base);
    if (P->terms) (void)hipFree(P->terms);
    if (P->dsteps) (void)hipFree(P->dsteps);
    if (P->subst) (void)hipGraphExecDestroy(P->subst);
    if (P->device >= 0 && P->device != cur) (void)hipSetDevice(cur);
    delete P;
}

}  // namespace sw

using namespace sw;

extern "C" {

int32_t shipwave_precond_build_banded(const sw_problem* prob, int32_t q_blocks, sw_precond** out,
                                      hipStream_t stream) {
    return guard([&]() -> int32_t {
        SW_REQUIRE(prob && out, "null pointer");
        SW_REQUIRE(q_blocks >= 0, "q_blocks must be >= 0");
        const Geo g = make_geo(*prob);
        *out = precond_build(g, q_blocks, stream);
        return SW_OK;
    });
}

int32_t shipwave_precond_apply(const sw_precond* P, const double* b, double* x,
                               hipStream_t stream) {
    return guard([&]() -> int32_t {
        SW_REQUIRE(P && b && x, "null pointer");
        precond_apply(P, b, x, stream);
        return SW_OK;
    });
}

int32_t shipwave_precond_apply_batched(int32_t n, const sw_precond* const* P,
                                       const double* const* b, double* const* x,
                                       hipStream_t stream) {
    return guard([&]() -> int32_t {
        SW_REQUIRE(n >= 0, "n must be >= 0");
        SW_REQUIRE(n == 0 || (P && b && x), "null pointer");
        for (int i = 0; i < n; ++i) SW_REQUIRE(P[i] && b[i] && x[i], "null pointer");
        precond_apply_batched(n, P, b, x, stream);
        return SW_OK;
    });
}

void shipwave_precond_destroy(sw_precond* P) { precond_destroy(P, true); }

}  // extern "C"
