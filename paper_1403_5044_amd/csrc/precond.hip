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
// pivoting inside each N x N diagonal block, by Gauss-Jordan).  Stored per
// block row l (2q+1 slots of N x N):
//   slot q:        Dinv_l   = (updated diagonal block)^{-1}
//   slot q-d (d>0): L_{l,l-d} = S~_{l,l-d} Dinv_{l-d}
//   slot q+d (d>0): G_{l,l+d} = Dinv_l U_{l,l+d}
// so that  forward  y_l = t_l - sum_d L_{l,l-d} y_{l-d}
//          backward x_l = Dinv_l y_l - sum_d G_{l,l+d} x_{l+d}
// are block GEMVs.  q = 0 (block bandwidth 1) makes every block independent.
#include "sw_internal.hpp"
#include "sw_device.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

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
    double* tmp2 = nullptr;  // [q][N][N] products of one factorisation step
    int* info = nullptr;     // [M] zero pivots seen
    void* terms = nullptr;   // device GemvTerm lists of the band substitution steps
    hipGraphExec_t subst = nullptr;  // the 2M substitution launches, captured once
    std::vector<int> fwd_off, fwd_cnt, bwd_off, bwd_cnt;
    size_t bytes = 0;
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

// A-hat^{-1} b in place along a strided vector: row r >= 1 gives x_r = 2 b_r - x_{r-1};
// row 0 then gives x_0 = (b_0 - 2 a01 b_1) / (a00 - a01).
__device__ void ahat_solve(const Geo& g, const double* b, double* x, size_t stride) {
    const double a01 = g.x1 / g.dx;
    const double a00 = g.nu - a01;
    double prev = (b[0] - 2.0 * a01 * b[stride]) / (a00 - a01);
    x[0] = prev;
    for (int r = 1; r < g.N; ++r) {
        prev = 2.0 * b[(size_t)r * stride] - prev;
        x[(size_t)r * stride] = prev;
    }
}

// out = T v (out_0 = 0): trapezoid integration of v from z_0 = -(x_1/nu) v_0, then
// averages of neighbouring grid values.
__device__ void apply_T(const Geo& g, const double* v, double* out, size_t stride, double scale) {
    const double hdx = 0.5 * g.dx;
    double z = (-g.x1 / g.nu) * v[0];
    double vp = v[0];
    out[0] = 0.0;
    for (int r = 1; r < g.N; ++r) {
        const double vr = v[(size_t)r * stride];
        const double zn = z + hdx * (vp + vr);
        out[(size_t)r * stride] = scale * 0.5 * (z + zn);
        z = zn;
        vp = vr;
    }
}

// Wc[:, n] = (2 pi / F^2) T A-hat^{-1} T e_n; one thread per column, scratch X [N][N].
__global__ void k_wmat(Geo g, double* __restrict__ X, double* __restrict__ Wc) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    const size_t st = g.N;
    // X[:, n] = T e_n
    {
        const double hdx = 0.5 * g.dx;
        double z = (n == 0) ? (-g.x1 / g.nu) : 0.0;
        X[n] = 0.0;
        for (int r = 1; r < g.N; ++r) {
            const double vp = (r - 1 == n) ? 1.0 : 0.0;
            const double vr = (r == n) ? 1.0 : 0.0;
            const double zn = z + hdx * (vp + vr);
            X[(size_t)r * st + n] = 0.5 * (z + zn);
            z = zn;
        }
    }
    ahat_solve(g, X + n, X + n, st);
    apply_T(g, X + n, Wc + n, st, kTwoPi / (g.F * g.F));
}

// sum_{i,j} w(i,j) K3(i,j; k,l) for each collocation point, split over row chunks.
__global__ __launch_bounds__(256) void k_k3_partial(Geo g, int G, double* __restrict__ part) {
    const int ntile = (g.ncol + 255) / 256;
    const int tile = blockIdx.x % ntile;
    const int chunk = blockIdx.x / ntile;
    const int c = tile * 256 + threadIdx.x;
    if (c >= g.ncol) return;
    const int l = c / g.Nc;
    const int k = c - l * g.Nc;
    const int j0 = (int)((long long)chunk * g.M / G), j1 = (int)((long long)(chunk + 1) * g.M / G);
    double s = 0.0;
    for (int j = j0; j < j1; ++j) {
        const double dy = (double)(j - l) * g.dy, dyp = (double)(j + l) * g.dy;
        const double dy2 = dy * dy, dyp2 = dyp * dyp;
        const double wy = g.dx * g.dy * weight1d(j, g.M, g.weights);
        double row = 0.0;
        for (int i = 0; i < g.N; ++i) {
            const double dx = ((double)(i - k) - 0.5) * g.dx;
            const double dx2 = dx * dx;
            row = fma(weight1d(i, g.N, g.weights), rsq_exact(dx2 + dy2) + rsq_exact(dx2 + dyp2),
                      row);
        }
        s = fma(wy, row, s);
    }
    part[(size_t)chunk * g.ncol + c] = s;
}

__global__ void k_k3_final(Geo g, int G, const double* __restrict__ part, double* __restrict__ k3) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.ncol) return;
    double s = 0.0;
    for (int q = 0; q < G; ++q) s += part[(size_t)q * g.ncol + c];
    k3[c] = s;
}

// Entries of the banded Schur complement before factorisation.
__global__ __launch_bounds__(256) void k_assemble(Geo g, int q, const double* __restrict__ k3,
                                                  const double* __restrict__ Wc,
                                                  double* __restrict__ S) {
    const int nb = 2 * q + 1;
    const size_t NN = (size_t)g.N * g.N;
    const size_t total = (size_t)g.M * nb * NN;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int n = (int)(e % g.N);
        const int r = (int)((e / g.N) % g.N);
        const int d = (int)((e / NN) % nb);
        const int l = (int)(e / (NN * nb));
        const int m = l + d - q;
        double v = 0.0;
        if (m >= 0 && m < g.M) {
            if (r == 0) {
                if (m == l) {
                    if (n == 0) v = g.nu - g.x1 / g.dx;
                    if (n == 1) v = g.x1 / g.dx;
                }
            } else {
                const int k = r - 1;
                const double dx = ((double)(n - k) - 0.5) * g.dx;
                const double dy = (double)(m - l) * g.dy, dyp = (double)(m + l) * g.dy;
                const double K3 = 1.0 / sqrt(dx * dx + dy * dy) + 1.0 / sqrt(dx * dx + dyp * dyp);
                const double w =
                    g.dx * g.dy * weight1d(n, g.N, g.weights) * weight1d(m, g.M, g.weights);
                v = -w * K3;
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
        S[e] = v;
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

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Maximum over each row of 16 lanes, left in every lane of that row
// (quad swaps, then half-row and row mirrors).  NaN operands are dropped by fmax.
__device__ __forceinline__ double row16_max_f64(double v) {
    v = fmax(v, dpp_f64<0xB1>(v));   // quad_perm [1,0,3,2]
    v = fmax(v, dpp_f64<0x4E>(v));   // quad_perm [2,3,0,1]
    v = fmax(v, dpp_f64<0x141>(v));  // row_half_mirror
    v = fmax(v, dpp_f64<0x140>(v));  // row_mirror
    return v;
}

__device__ __forceinline__ double wave_max_f64(double v) {
    v = row16_max_f64(v);
    return fmax(fmax(readlane_f64(v, 0), readlane_f64(v, 16)),
                fmax(readlane_f64(v, 32), readlane_f64(v, 48)));
}

// ---- N <= 192: the whole block in registers, one workgroup ----
// Thread (tr = t / 32, tc = t % 32) holds B[tr + 16 i][tc + 32 c].  Wavefront 0
// eliminates each panel of kPW columns with rows lane + 64 i in registers (pivot
// search by DPP and readlane, no block barrier); all threads then apply the
// rank-kPW update from LDS.
constexpr int kGT = 512;
constexpr int kPW = 8;

template <int RB, int CB>
__global__ __launch_bounds__(kGT) void k_gj_tile(int N, double* __restrict__ base, size_t stride,
                                                 int* __restrict__ info) {
    constexpr int R = 16 * RB, C = 32 * CB, RW = R / 64;
    static_assert(R == C && RW * 64 == R, "square tile, whole rows per lane of one wave");
    double* A = base + (size_t)blockIdx.x * stride;
    __shared__ double Pn[R][kPW];
    __shared__ double Zr[kPW][C];
    __shared__ int rowpiv[C], step_of[R];
    const int t = threadIdx.x;
    const int tc = t & 31, tr = t >> 5, lane = t & 63;
    const bool w0 = t < 64;
    double a[RB][CB];
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const int r = tr + 16 * i, j = tc + 32 * c;
            a[i][c] = (r < N && j < N) ? A[(size_t)r * N + j] : 0.0;
        }
    for (int r = t; r < R; r += kGT) {
        step_of[r] = -1;
        rowpiv[r] = -1;
    }
    unsigned usedm = 0;  // wavefront 0: bit i marks row lane + 64 i as pivoted or padding
#pragma unroll
    for (int i = 0; i < RW; ++i)
        if (lane + 64 * i >= N) usedm |= 1u << i;
    int zeros = 0;
    __syncthreads();
    for (int k0 = 0; k0 < N; k0 += kPW) {
        const int kb = min(kPW, N - k0);
        const int c0 = k0 >> 5, t0 = k0 & 31;  // kPW divides 32: a panel never straddles c
        const bool pcol = tc >= t0 && tc < t0 + kPW;
#pragma unroll
        for (int c = 0; c < CB; ++c)
            if (c == c0 && pcol)
#pragma unroll
                for (int i = 0; i < RB; ++i) Pn[tr + 16 * i][tc - t0] = a[i][c];
        __syncthreads();
        if (w0) {
            double pv[RW][kPW];
#pragma unroll
            for (int i = 0; i < RW; ++i)
#pragma unroll
                for (int u = 0; u < kPW; ++u) pv[i][u] = Pn[lane + 64 * i][u];
#pragma unroll
            for (int s = 0; s < kPW; ++s) {
                if (s >= kb) break;
                double best = -1.0;
                int bi = -1;
#pragma unroll
                for (int i = 0; i < RW; ++i) {
                    const double v = fabs(pv[i][s]);
                    if (!((usedm >> i) & 1u) && (bi < 0 || v > best)) {
                        best = v;
                        bi = i;
                    }
                }
                const double mx = wave_max_f64(best);
                unsigned long long mask = __ballot(bi >= 0 && best == mx);
                if (mask == 0) mask = __ballot(bi >= 0);  // the column holds NaN
                const int pl = mask ? __builtin_ctzll(mask) : 0;
                const int pi = max(0, __builtin_amdgcn_readlane(bi, pl));
                const int rp = pl + 64 * pi;
                double prow[kPW];
#pragma unroll
                for (int u = 0; u < kPW; ++u) prow[u] = 0.0;
#pragma unroll
                for (int i = 0; i < RW; ++i)
                    if (i == pi)
#pragma unroll
                        for (int u = 0; u < kPW; ++u) prow[u] = readlane_f64(pv[i][u], pl);
                const double piv = prow[s];
                if (!(fabs(piv) > 0.0)) ++zeros;
                const double d = 1.0 / piv;
                double pd[kPW];
#pragma unroll
                for (int u = 0; u < kPW; ++u) pd[u] = (u == s) ? d : prow[u] * d;
#pragma unroll
                for (int i = 0; i < RW; ++i) {
                    const double m = pv[i][s];
#pragma unroll
                    for (int u = 0; u < kPW; ++u)
                        pv[i][u] = (u == s) ? -m * d : fma(-m, pd[u], pv[i][u]);
                }
                if (lane == pl) {
#pragma unroll
                    for (int i = 0; i < RW; ++i)
                        if (i == pi) {
#pragma unroll
                            for (int u = 0; u < kPW; ++u) pv[i][u] = pd[u];
                            usedm |= 1u << i;
                        }
                }
                if (lane == 0) {
                    rowpiv[k0 + s] = rp;
                    step_of[rp] = k0 + s;
                }
            }
#pragma unroll
            for (int i = 0; i < RW; ++i)
#pragma unroll
                for (int u = 0; u < kPW; ++u) Pn[lane + 64 * i][u] = pv[i][u];
        }
        __syncthreads();
        // old pivot rows to Zr; their base becomes zero
#pragma unroll
        for (int i = 0; i < RB; ++i) {
            const int r = tr + 16 * i;
            const int st = step_of[r];
            if (st >= k0 && st < k0 + kb) {
#pragma unroll
                for (int c = 0; c < CB; ++c) {
                    Zr[st - k0][tc + 32 * c] = a[i][c];
                    a[i][c] = 0.0;
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kPW; ++u) {
            if (u >= kb) break;
            double z[CB];
#pragma unroll
            for (int c = 0; c < CB; ++c) z[c] = Zr[u][tc + 32 * c];
#pragma unroll
            for (int i = 0; i < RB; ++i) {
                const double p = Pn[tr + 16 * i][u];
#pragma unroll
                for (int c = 0; c < CB; ++c) a[i][c] = fma(p, z[c], a[i][c]);
            }
        }
#pragma unroll
        for (int c = 0; c < CB; ++c)
            if (c == c0 && pcol)
#pragma unroll
                for (int i = 0; i < RB; ++i) a[i][c] = Pn[tr + 16 * i][tc - t0];
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const int r = tr + 16 * i, j = tc + 32 * c;
            if (r < N && j < N) {
                const int sr = step_of[r], pj = rowpiv[j];
                if (sr >= 0 && sr < N && pj >= 0 && pj < N) A[(size_t)sr * N + pj] = a[i][c];
            }
        }
    if (t == 0 && info) info[blockIdx.x] = zeros;
}

// ---- N > 192: the block in global memory, one panel and one update launch per panel ----
// Panel kernel: one workgroup per block, thread r holds row r of the panel (N <= 1024).
// Pivot search: DPP maximum per wavefront, then over the 16 wavefront candidates.
// It writes the new panel columns pn[N][kPWG], the old pivot rows z[kPWG][N],
// step_of[N] and rowpiv[N] (per block, in the workspace gjw).
constexpr int kGP = 1024;
constexpr int kPWG = 16;

struct GjWork {
    double* pn;   // [nblocks][N][kPWG]
    double* z;    // [nblocks][kPWG][N]
    int* piv;     // [nblocks][2][N]: step_of, rowpiv
};

__global__ __launch_bounds__(kGP) void k_gjp_panel(int N, const double* __restrict__ base,
                                                   size_t stride, GjWork w, int k0,
                                                   int* __restrict__ info) {
    const double* B = base + (size_t)blockIdx.x * stride;
    double* pn = w.pn + (size_t)blockIdx.x * N * kPWG;
    double* z = w.z + (size_t)blockIdx.x * kPWG * N;
    int* step_of = w.piv + (size_t)blockIdx.x * 2 * N;
    int* rowpiv = step_of + N;
    __shared__ double candv[16], prow[kPWG];
    __shared__ int candr[16], rp_s[kPWG];
    const int r = threadIdx.x, lane = r & 63, wv = r >> 6;
    const int kb = min(kPWG, N - k0);
    const bool valid = r < N;
    int st = (valid && k0 > 0) ? step_of[r] : -1;
    double pv[kPWG];
#pragma unroll
    for (int u = 0; u < kPWG; ++u)
        pv[u] = (valid && u < kb) ? B[(size_t)r * N + k0 + u] : 0.0;
    int zeros = 0;
#pragma unroll
    for (int s = 0; s < kPWG; ++s) {
        if (s >= kb) break;
        const bool cand = valid && st < 0;
        const double v = cand ? fabs(pv[s]) : -1.0;
        const double wm = wave_max_f64(v);
        unsigned long long mask = __ballot(cand && v == wm);
        if (mask == 0) mask = __ballot(cand);
        if (lane == 0) {
            candv[wv] = mask ? wm : -2.0;
            candr[wv] = mask ? (wv * 64 + __builtin_ctzll(mask)) : -1;
        }
        __syncthreads();
        const double cv = (lane < 16) ? candv[lane] : -2.0;
        const int cr = (lane < 16) ? candr[lane] : -1;
        const double gm = readlane_f64(row16_max_f64(cv), 0);
        unsigned long long m2 = __ballot(cr >= 0 && cv == gm);
        if (m2 == 0) m2 = __ballot(cr >= 0);
        const int rp = m2 ? __builtin_amdgcn_readlane(cr, __builtin_ctzll(m2)) : 0;
        if (r == rp)
#pragma unroll
            for (int u = 0; u < kPWG; ++u) prow[u] = pv[u];
        __syncthreads();
        double pd[kPWG];
#pragma unroll
        for (int u = 0; u < kPWG; ++u) pd[u] = prow[u];
        const double piv = pd[s];
        const double d = 1.0 / piv;
#pragma unroll
        for (int u = 0; u < kPWG; ++u) pd[u] = (u == s) ? d : pd[u] * d;
        if (r == rp) {
#pragma unroll
            for (int u = 0; u < kPWG; ++u) pv[u] = pd[u];
            st = k0 + s;
        } else {
            const double m = pv[s];
#pragma unroll
            for (int u = 0; u < kPWG; ++u) pv[u] = (u == s) ? -m * d : fma(-m, pd[u], pv[u]);
        }
        if (r == 0) {
            rp_s[s] = rp;
            rowpiv[k0 + s] = rp;
            if (!(fabs(piv) > 0.0)) ++zeros;
        }
    }
    if (valid) {
#pragma unroll
        for (int u = 0; u < kPWG; ++u) pn[(size_t)r * kPWG + u] = pv[u];
        step_of[r] = st;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kb * N; e += kGP) {
        const int tt = e / N, j = e - tt * N;
        z[(size_t)tt * N + j] = B[(size_t)rp_s[tt] * N + j];
    }
    if (r == 0 && info) info[blockIdx.x] = (k0 == 0 ? 0 : info[blockIdx.x]) + zeros;
}

// Rank-kb update of every column outside the panel; the panel columns take pn.
// Tile of 16 rows x 64 columns per 256-thread workgroup; grid (cols, rows, blocks).
__global__ __launch_bounds__(256) void k_gjp_update(int N, double* __restrict__ base,
                                                    size_t stride, GjWork w, int k0) {
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
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < NN;
         e += (size_t)gridDim.x * blockDim.x) {
        const int r = (int)(e / N), c = (int)(e - (size_t)r * N);
        const int sr = step_of[r], pc = rowpiv[c];
        if (sr >= 0 && sr < N && pc >= 0 && pc < N) O[(size_t)sr * N + pc] = B[e];
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
        k_gj_tile<4, 2><<<nblocks, kGT, 0, s>>>(N, base, stride, info);
    } else if (N <= 128) {
        k_gj_tile<8, 4><<<nblocks, kGT, 0, s>>>(N, base, stride, info);
    } else if (N <= 192) {
        k_gj_tile<12, 6><<<nblocks, kGT, 0, s>>>(N, base, stride, info);
    } else {
        const size_t NN = (size_t)N * N;
        GjWork w;
        w.pn = work;
        w.z = work + (size_t)nblocks * N * kPWG;
        w.piv = reinterpret_cast<int*>(work + (size_t)nblocks * 2 * kPWG * N);
        const dim3 ug((N + 63) / 64, (N + 15) / 16, nblocks);
        for (int k0 = 0; k0 < N; k0 += kPWG) {
            k_gjp_panel<<<nblocks, kGP, 0, s>>>(N, base, stride, w, k0, info);
            k_gjp_update<<<ug, 256, 0, s>>>(N, base, stride, w, k0);
        }
        const unsigned ge = (unsigned)std::min<size_t>((NN + 255) / 256, 2048);
        k_gjp_scatter<<<dim3(ge, nblocks), 256, 0, s>>>(N, base, stride, tmp, NN, w);
        k_copy_blocks<<<dim3(ge, nblocks), 256, 0, s>>>(N, tmp, NN, base, stride);
    }
}
// C = Cin + alpha A B for N x N row-major blocks (C may equal Cin, not A or B);
// blockIdx.z selects one of a list of such products.
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

__global__ __launch_bounds__(256) void k_gemm(int n, double alpha, GemmBatch batch) {
    const GemmJob job = batch.j[blockIdx.z];
    const double* __restrict__ A = job.A;
    const double* __restrict__ B = job.B;
    const double* Cin = job.Cin;
    double* C = job.C;
    __shared__ double As[16][65];
    __shared__ double Bs[16][64];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int row0 = blockIdx.y * 64, col0 = blockIdx.x * 64;
    double acc[4][4] = {};
    for (int k0 = 0; k0 < n; k0 += 16) {
        for (int e = threadIdx.x; e < 64 * 16; e += 256) {
            const int r = e / 16, kk = e % 16;
            const int gr = row0 + r, gk = k0 + kk;
            As[kk][r] = (gr < n && gk < n) ? A[(size_t)gr * n + gk] : 0.0;
        }
        for (int e = threadIdx.x; e < 16 * 64; e += 256) {
            const int kk = e / 64, c = e % 64;
            const int gk = k0 + kk, gc = col0 + c;
            Bs[kk][c] = (gk < n && gc < n) ? B[(size_t)gk * n + gc] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx * 4 + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = row0 + ty * 4 + i, c = col0 + tx * 4 + j;
            if (r < n && c < n) {
                const size_t o = (size_t)r * n + c;
                C[o] = (Cin ? Cin[o] : 0.0) + alpha * acc[i][j];
            }
        }
}

__global__ void k_copy(size_t n, const double* __restrict__ a, double* __restrict__ b) {
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (size_t)gridDim.x * blockDim.x)
        b[t] = a[t];
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

// s1 = A-hat^{-1} b1, t2 = b2 - 2 pi T s1 (per row l)
__global__ __launch_bounds__(64) void k_apply_first(Geo g, const double* __restrict__ b,
                                                    double* __restrict__ s1,
                                                    double* __restrict__ t2) {
    __shared__ double B[kMaxN], X[kMaxN], Z[kMaxN];
    const int l = blockIdx.x;
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

// r1 = s1 - A-hat^{-1} (T s2 / F^2), r2 = s2 (per row l)
__global__ __launch_bounds__(64) void k_apply_last(Geo g, const double* __restrict__ s1,
                                                   const double* __restrict__ s2,
                                                   double* __restrict__ x) {
    __shared__ double V[kMaxN], Z[kMaxN], X[kMaxN];
    const int l = blockIdx.x;
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

size_t blk_off(const sw_precond* P, int l, int slot) {
    return ((size_t)l * P->nb + slot) * (size_t)P->g.N * P->g.N;
}

void gemm_batched(int n, double alpha, const std::vector<GemmJob>& jobs, hipStream_t s) {
    for (size_t b = 0; b < jobs.size(); b += kMaxGemmJobs) {
        GemmBatch batch{};
        const int cnt = (int)std::min<size_t>(kMaxGemmJobs, jobs.size() - b);
        for (int i = 0; i < cnt; ++i) batch.j[i] = jobs[b + i];
        dim3 grid((n + 63) / 64, (n + 63) / 64, cnt);
        k_gemm<<<grid, 256, 0, s>>>(n, alpha, batch);
    }
}

void copy(size_t n, const double* a, double* b, hipStream_t s) {
    k_copy<<<(unsigned)std::min<size_t>((n + 255) / 256, 8192), 256, 0, s>>>(n, a, b);
}

}  // namespace

namespace {
// scratch blocks: q products per factorisation step, or M inverses at once (q = 0, N > 192)
size_t tmp2_blocks(const Geo& g, int q) {
    return (size_t)std::max({q, 1, (q == 0 && g.N > 192) ? g.M : 1});
}

// workspace of the diagonal-block inversion (N > 192), at least one N x N block
size_t gj_work_size(const Geo& g, int q) {
    const size_t NN = (size_t)g.N * g.N;
    return std::max(NN, gj_work_doubles(g.N, q == 0 ? g.M : 1));
}

int k3_chunks(const Geo& g) {
    const int ntile = (g.ncol + 255) / 256;
    return std::max(1, std::min(g.M, (4096 + ntile - 1) / ntile));
}
}  // namespace

size_t precond_bytes_estimate(const Geo& g, int q_req) {
    const int q = std::max(0, std::min(q_req, g.M - 1));
    const int nb = 2 * q + 1;
    const size_t N = g.N, NN = N * N, NM = g.NM;
    const int G = k3_chunks(g);
    return carve_size({(size_t)g.M * nb * NN * 8, NN * 8, (size_t)g.ncol * 8, 4 * NM * 8,
                       gj_work_size(g, q) * 8, tmp2_blocks(g, q) * NN * 8, (size_t)g.M * 4, (size_t)G * g.ncol * 8,
                       NN * 8});
}

size_t precond_bytes(const sw_precond* P) { return P ? P->bytes : 0; }

bool precond_matches(const sw_precond* P, const Geo& g) {
    return P && P->g.N == g.N && P->g.M == g.M && P->g.x1 == g.x1 && P->g.xN == g.xN &&
           P->g.yM == g.yM;
}

namespace {
void capture_substitution(sw_precond* P);
}

sw_precond* precond_build(const Geo& g0, int q_req, hipStream_t s) {
    Geo g = g0;
    g.precision = SW_PREC_FP64;
    const int q = std::max(0, std::min(q_req, g.M - 1));
    const int nb = 2 * q + 1;
    const size_t N = g.N, NN = N * N, NM = g.NM;
    const int G = k3_chunks(g);
    const size_t bytes = precond_bytes_estimate(g, q);
    (void)N;
    auto* P = new sw_precond();
    P->g = g;
    P->q = q;
    P->nb = nb;
    SW_HIP(hipGetDevice(&P->device));
    void* mem = nullptr;
    if (hipMalloc(&mem, bytes) != hipSuccess) {
        (void)hipGetLastError();
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
    P->info = c.take<int>(g.M);
    double* part = c.take<double>((size_t)G * g.ncol);
    double* X = c.take<double>(NN);
    try {
        k_wmat<<<(g.N + 63) / 64, 64, 0, s>>>(g, X, P->Wc);
        const int ntile = (g.ncol + 255) / 256;
        k_k3_partial<<<ntile * G, 256, 0, s>>>(g, G, part);
        k_k3_final<<<(g.ncol + 255) / 256, 256, 0, s>>>(g, G, part, P->k3);
        const size_t total = (size_t)g.M * nb * NN;
        k_assemble<<<(unsigned)std::min<size_t>((total + 255) / 256, 65536), 256, 0, s>>>(
            g, q, P->k3, P->Wc, P->S);
        if (q == 0) {
            gj_inverse(g.N, P->S, NN, g.M, P->info, P->tmp2, P->tmp, s);
        } else {
            double* scratchL = P->tmp2;  // q blocks for L_{i,l} and G_{l,j}
            for (int l = 0; l < g.M; ++l) {
                gj_inverse(g.N, P->S + blk_off(P, l, q), 0, 1, P->info + l, P->tmp2, P->tmp,
                           s);
                const int hi = std::min(g.M - 1, l + q);
                const int cnt = hi - l;
                if (cnt == 0) continue;
                std::vector<GemmJob> jobs;
                // L_{i,l} = S_{i,l} Dinv_l (into scratch, then copied back)
                for (int i = l + 1; i <= hi; ++i)
                    jobs.push_back(GemmJob{P->S + blk_off(P, i, l - i + q),
                                           P->S + blk_off(P, l, q), nullptr,
                                           scratchL + (size_t)(i - l - 1) * NN});
                gemm_batched(g.N, 1.0, jobs, s);
                for (int i = l + 1; i <= hi; ++i)
                    copy(NN, scratchL + (size_t)(i - l - 1) * NN, P->S + blk_off(P, i, l - i + q),
                         s);
                // S_{i,j} -= L_{i,l} U_{l,j}
                jobs.clear();
                for (int i = l + 1; i <= hi; ++i)
                    for (int j = l + 1; j <= hi; ++j) {
                        double* Sij = P->S + blk_off(P, i, j - i + q);
                        jobs.push_back(GemmJob{P->S + blk_off(P, i, l - i + q),
                                               P->S + blk_off(P, l, j - l + q), Sij, Sij});
                    }
                gemm_batched(g.N, -1.0, jobs, s);
                // G_{l,j} = Dinv_l U_{l,j}
                jobs.clear();
                for (int j = l + 1; j <= hi; ++j)
                    jobs.push_back(GemmJob{P->S + blk_off(P, l, q), P->S + blk_off(P, l, j - l + q),
                                           nullptr, scratchL + (size_t)(j - l - 1) * NN});
                gemm_batched(g.N, 1.0, jobs, s);
                for (int j = l + 1; j <= hi; ++j)
                    copy(NN, scratchL + (size_t)(j - l - 1) * NN, P->S + blk_off(P, l, j - l + q),
                         s);
            }
        }
        if (q > 0) {
            std::vector<GemvTerm> tv;
            double* tmpv = P->work + 3 * NM;
            double* xv = P->work + 2 * NM;
            P->fwd_off.resize(g.M);
            P->fwd_cnt.resize(g.M);
            P->bwd_off.resize(g.M);
            P->bwd_cnt.resize(g.M);
            for (int l = 0; l < g.M; ++l) {
                P->fwd_off[l] = (int)tv.size();
                for (int d = 1; d <= q && l - d >= 0; ++d)
                    tv.push_back(GemvTerm{P->S + blk_off(P, l, q - d), tmpv + (size_t)(l - d) * N,
                                          -1.0, 0.0});
                P->fwd_cnt[l] = (int)tv.size() - P->fwd_off[l];
            }
            for (int l = 0; l < g.M; ++l) {
                P->bwd_off[l] = (int)tv.size();
                tv.push_back(GemvTerm{P->S + blk_off(P, l, q), tmpv + (size_t)l * N, 1.0, 0.0});
                for (int d = 1; d <= q && l + d < g.M; ++d)
                    tv.push_back(GemvTerm{P->S + blk_off(P, l, q + d), xv + (size_t)(l + d) * N,
                                          -1.0, 0.0});
                P->bwd_cnt[l] = (int)tv.size() - P->bwd_off[l];
            }
            SW_HIP(hipMalloc(&P->terms, tv.size() * sizeof(GemvTerm)));
            SW_HIP(hipMemcpy(P->terms, tv.data(), tv.size() * sizeof(GemvTerm),
                             hipMemcpyHostToDevice));
            capture_substitution(P);
        }
        SW_HIP(hipGetLastError());
        std::vector<int> info(g.M);
        SW_HIP(hipMemcpyAsync(info.data(), P->info, g.M * sizeof(int), hipMemcpyDeviceToHost, s));
        SW_HIP(hipStreamSynchronize(s));
        for (int v : info)
            if (v != 0) throw Error{SW_ENONFINITE, "preconditioner: singular diagonal block"};
    } catch (...) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(P->base);
        if (P->terms) (void)hipFree(P->terms);
        if (P->subst) (void)hipGraphExecDestroy(P->subst);
        delete P;
        throw;
    }
    return P;
}

namespace {
// Block forward and backward substitution with the band factors (q >= 1); all
// pointers live in the preconditioner, so the sequence can be captured once.
void enqueue_substitution(const sw_precond* P, hipStream_t s) {
    const Geo& g = P->g;
    const size_t NM = g.NM;
    const int N = g.N;
    double* t2 = P->work + NM;
    double* s2 = P->work + 2 * NM;
    double* tmp = P->work + 3 * NM;
    const GemvTerm* terms = static_cast<const GemvTerm*>(P->terms);
    const unsigned blocks = (unsigned)((N * 64 + 255) / 256);
    // forward: y_l = t_l - sum_d L_{l,l-d} y_{l-d}   (y in tmp)
    for (int l = 0; l < g.M; ++l)
        k_band_step<<<blocks, 256, 0, s>>>(N, terms + P->fwd_off[l], P->fwd_cnt[l],
                                           t2 + (size_t)l * N, tmp + (size_t)l * N);
    // backward: x_l = Dinv_l y_l - sum_d G_{l,l+d} x_{l+d}   (x in s2)
    for (int l = g.M - 1; l >= 0; --l)
        k_band_step<<<blocks, 256, 0, s>>>(N, terms + P->bwd_off[l], P->bwd_cnt[l], nullptr,
                                           s2 + (size_t)l * N);
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

void precond_destroy(sw_precond* P) {
    if (!P) return;
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (P->device >= 0 && P->device != cur) (void)hipSetDevice(P->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(P->base);
    if (P->terms) (void)hipFree(P->terms);
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

void shipwave_precond_destroy(sw_precond* P) { precond_destroy(P); }

}  // extern "C"
