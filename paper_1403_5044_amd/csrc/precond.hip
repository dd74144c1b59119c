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
    double* tmp = nullptr;   // [N][N]
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

// Inverses of N x N blocks (row-major), one workgroup per block: Gauss-Jordan
// with partial pivoting done implicitly.  Rows are never swapped: step p
// eliminates column p with the unused physical row rp of largest |B[rp][p]|,
// storing the inverse's columns in place of the eliminated ones.  With
// rowpiv[p] = rp and step_of[rp] = p the inverse is
//     A^{-1}[step_of[r]][rowpiv[c]] = B[r][c],
// written by one scatter at the end.  The pivot search of step p+1 runs inside
// the update of step p (look-ahead), so each step needs two barriers.
constexpr int kGJ = 1024;

// Matrix in registers: thread (ty = t / 64, tx = t % 64) holds B[ty + 16 i][tx + 64 c].
template <int RB, int CB>
__global__ __launch_bounds__(kGJ) void k_gj_reg(int N, double* __restrict__ base, size_t stride,
                                                int* __restrict__ info) {
    double* A = base + (size_t)blockIdx.x * stride;
    __shared__ double rowp[64 * CB], colp[16 * RB];
    __shared__ double candv[2][16];
    __shared__ int candr[2][16];
    __shared__ int rowpiv[64 * CB], step_of[16 * RB];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    double a[RB][CB];
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const int r = ty + 16 * i, j = tx + 64 * c;
            a[i][c] = (r < N && j < N) ? A[(size_t)r * N + j] : 0.0;
        }
    unsigned used = 0;  // bit i: row ty + 16 i has been a pivot
    if (tx == 0) {
        double bv = -1.0;
        int br = N;
#pragma unroll
        for (int i = 0; i < RB; ++i) {
            const int r = ty + 16 * i;
            const double v = fabs(a[i][0]);
            if (r < N && v > bv) {
                bv = v;
                br = r;
            }
        }
        candv[0][ty] = bv;
        candr[0][ty] = br;
    }
    __syncthreads();
    int zero_pivots = 0;
    for (int p = 0; p < N; ++p) {
        const int buf = p & 1;
        double bv = -1.0;
        int rp = N;
#pragma unroll
        for (int w = 0; w < 16; ++w) {
            const double v = candv[buf][w];
            const int r = candr[buf][w];
            if (v > bv || (v == bv && r < rp)) {
                bv = v;
                rp = r;
            }
        }
        if (ty == (rp & 15)) used |= 1u << (rp >> 4);
        if (threadIdx.x == 0) {
            rowpiv[p] = rp;
            step_of[rp] = p;
        }
        const int pc = p >> 6, pt = p & 63;
#pragma unroll
        for (int i = 0; i < RB; ++i) {
            const int r = ty + 16 * i;
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                if (r == rp) rowp[tx + 64 * c] = a[i][c];
                if (c == pc && tx == pt) colp[r] = a[i][c];
            }
        }
        __syncthreads();
        const double piv = rowp[p];
        if (piv == 0.0) ++zero_pivots;
        const double d = 1.0 / piv;
        const int p1 = p + 1, p1c = p1 >> 6, p1t = p1 & 63;
        double nb = -1.0;
        int nr = N;
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const int j = tx + 64 * c;
            const double rpj = (j == p) ? d : rowp[j] * d;
#pragma unroll
            for (int i = 0; i < RB; ++i) {
                const int r = ty + 16 * i;
                if (r == rp)
                    a[i][c] = rpj;
                else
                    a[i][c] = fma(-colp[r], rpj, (j == p) ? 0.0 : a[i][c]);
                if (c == p1c && tx == p1t && r < N && !((used >> i) & 1u)) {
                    const double v = fabs(a[i][c]);
                    if (v > nb) {
                        nb = v;
                        nr = r;
                    }
                }
            }
        }
        if (tx == p1t) {
            candv[buf ^ 1][ty] = nb;
            candr[buf ^ 1][ty] = nr;
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const int r = ty + 16 * i, j = tx + 64 * c;
            if (r < N && j < N) A[(size_t)step_of[r] * N + rowpiv[j]] = a[i][c];
        }
    if (threadIdx.x == 0 && info) info[blockIdx.x] = zero_pivots;
}

// Blocked form of the same elimination for N <= 64 * CB (matrix in registers).
// Panels of kPB pivot columns: one wavefront eliminates the panel columns in
// LDS (pivot search by shuffles, no block barriers), recording for every row r
// and panel step t the multiplier m_t[r] (column p_t of row r just before step
// t).  The other columns then receive all kPB steps at once:
//   Z_t = d_t (B_{rp_t} - sum_{s<t} m_s[rp_t] Z_s)     (pivot rows, kPB x N)
//   B_r <- B_r - sum_t m_t[r] Z_t                       (other rows)
//   B_{rp_t} <- Z_t - sum_{s>t} m_s[rp_t] Z_s            (pivot rows)
// which equals applying the kPB elementary steps one after another.
constexpr int kPB = 8;

template <int RB, int CB>
__global__ __launch_bounds__(kGJ) void k_gj_blocked(int N, double* __restrict__ base,
                                                    size_t stride, int* __restrict__ info) {
    constexpr int R = 16 * RB, C = 64 * CB;
    double* A = base + (size_t)blockIdx.x * stride;
    __shared__ double Pn[R][kPB];   // panel columns
    __shared__ double Mt[R][kPB];   // multipliers m_t[r]
    __shared__ double Zr[kPB][C];   // pivot rows before the panel (non-panel columns)
    __shared__ double Zz[kPB][C];   // Z_t
    __shared__ double W[kPB][kPB];
    __shared__ int rowpiv[C], step_of[R];
    __shared__ int used[R];
    __shared__ int zero_s;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    double a[RB][CB];
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const int r = ty + 16 * i, j = tx + 64 * c;
            a[i][c] = (r < N && j < N) ? A[(size_t)r * N + j] : 0.0;
        }
    for (int r = threadIdx.x; r < R; r += kGJ) {
        step_of[r] = -1;
        used[r] = 0;
    }
    for (int e = threadIdx.x; e < kPB * C; e += kGJ) Zz[e / C][e % C] = 0.0;
    if (threadIdx.x == 0) zero_s = 0;
    __syncthreads();
    for (int k0 = 0; k0 < N; k0 += kPB) {
        const int kb = min(kPB, N - k0);
        const int c0 = k0 >> 6, t0 = k0 & 63;
        // ---- panel to LDS
#pragma unroll
        for (int c = 0; c < CB; ++c)
            if (c == c0 && tx >= t0 && tx < t0 + kb)
#pragma unroll
                for (int i = 0; i < RB; ++i) Pn[ty + 16 * i][tx - t0] = a[i][c];
        __syncthreads();
        // ---- panel elimination by wavefront 0
        if (ty == 0) {
            for (int t = 0; t < kb; ++t) {
                const int p = k0 + t;
                double bv = -1.0;
                int br = N;
                for (int r = tx; r < N; r += 64)
                    if (!used[r]) {
                        const double v = fabs(Pn[r][t]);
                        if (v > bv) {
                            bv = v;
                            br = r;
                        }
                    }
                for (int d = 32; d >= 1; d >>= 1) {
                    const double ov = __shfl_xor(bv, d, 64);
                    const int orr = __shfl_xor(br, d, 64);
                    if (ov > bv || (ov == bv && orr < br)) {
                        bv = ov;
                        br = orr;
                    }
                }
                const int rp = br;
                double prow[kPB];
#pragma unroll
                for (int u = 0; u < kPB; ++u) prow[u] = Pn[rp][u];
                const double piv = Pn[rp][t];
                const double dd = 1.0 / piv;
                __builtin_amdgcn_wave_barrier();
                if (tx == 0) {
                    rowpiv[p] = rp;
                    step_of[rp] = p;
                    used[rp] = 1;
                    if (piv == 0.0) zero_s++;
                }
                for (int r = tx; r < N; r += 64) {
                    const double m = Pn[r][t];
                    Mt[r][t] = m;
                    if (r == rp) {
#pragma unroll
                        for (int u = 0; u < kPB; ++u) Pn[r][u] = (u == t) ? dd : prow[u] * dd;
                    } else {
#pragma unroll
                        for (int u = 0; u < kPB; ++u)
                            Pn[r][u] = (u == t) ? -m * dd : fma(-m, prow[u] * dd, Pn[r][u]);
                    }
                }
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            }
        }
        __syncthreads();
        // W with Z = W B0p; the pivot value of step t is Mt[rp_t][t]
        if (threadIdx.x == 0) {
            for (int t = 0; t < kb; ++t) {
                const int rt = rowpiv[k0 + t];
                const double dt = 1.0 / Mt[rt][t];
                for (int u = 0; u < kPB; ++u) W[t][u] = 0.0;
                W[t][t] = dt;
                for (int s2 = 0; s2 < t; ++s2) {
                    const double ms = Mt[rt][s2];
                    for (int u = 0; u <= s2; ++u) W[t][u] -= dt * ms * W[s2][u];
                }
            }
        }
        // ---- panel back to registers; pivot rows' other columns to LDS
#pragma unroll
        for (int c = 0; c < CB; ++c)
            if (c == c0 && tx >= t0 && tx < t0 + kb)
#pragma unroll
                for (int i = 0; i < RB; ++i) {
                    const int r = ty + 16 * i;
                    if (r < N) a[i][c] = Pn[r][tx - t0];
                }
#pragma unroll
        for (int i = 0; i < RB; ++i) {
            const int r = ty + 16 * i;
            const int st = (r < N) ? step_of[r] : -1;
            if (st >= k0 && st < k0 + kb)
#pragma unroll
                for (int c = 0; c < CB; ++c) Zr[st - k0][tx + 64 * c] = a[i][c];
        }
        __syncthreads();
        // ---- Z = W Zr
        if (ty < kb) {
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                const int j = tx + 64 * c;
                double z = 0.0;
                for (int u = 0; u <= ty; ++u) z = fma(W[ty][u], Zr[u][j], z);
                Zz[ty][j] = z;
            }
        }
        __syncthreads();
        // ---- rank-kb update of the non-panel columns
#pragma unroll
        for (int i = 0; i < RB; ++i) {
            const int r = ty + 16 * i;
            if (r >= N) continue;
            const int st = step_of[r];
            const bool isp = (st >= k0 && st < k0 + kb);
            const int tp = isp ? st - k0 : -1;
            double coef[kPB];
#pragma unroll
            for (int u = 0; u < kPB; ++u) coef[u] = (u < kb && u > tp) ? Mt[r][u] : 0.0;
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                const int j = tx + 64 * c;
                const bool inpanel = (c == c0 && tx >= t0 && tx < t0 + kb);
                if (inpanel) continue;
                double v = isp ? Zz[tp][j] : a[i][c];
#pragma unroll
                for (int u = 0; u < kPB; ++u) v = fma(-coef[u], Zz[u][j], v);
                a[i][c] = v;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const int r = ty + 16 * i, j = tx + 64 * c;
            if (r < N && j < N) A[(size_t)step_of[r] * N + rowpiv[j]] = a[i][c];
        }
    if (threadIdx.x == 0 && info) info[blockIdx.x] = zero_s;
}

// Matrix in global memory (any N <= kMaxN): thread (ty, tx) updates rows ty, ty+16, ...
// and columns tx, tx+64, ...  The inverse is scattered into `out` (not `base`).
__global__ __launch_bounds__(kGJ) void k_gj_global(int N, double* __restrict__ base,
                                                   size_t stride, double* __restrict__ outbase,
                                                   size_t out_stride, int* __restrict__ info) {
    double* B = base + (size_t)blockIdx.x * stride;
    double* O = outbase + (size_t)blockIdx.x * out_stride;
    __shared__ double rowp[kMaxN], colp[kMaxN];
    __shared__ double candv[2][16];
    __shared__ int candr[2][16];
    __shared__ int rowpiv[kMaxN], step_of[kMaxN];
    __shared__ unsigned char used[kMaxN];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = threadIdx.x; r < N; r += kGJ) used[r] = 0;
    if (tx == 0) {
        double bv = -1.0;
        int br = N;
        for (int r = ty; r < N; r += 16) {
            const double v = fabs(B[(size_t)r * N]);
            if (v > bv) {
                bv = v;
                br = r;
            }
        }
        candv[0][ty] = bv;
        candr[0][ty] = br;
    }
    __syncthreads();
    int zero_pivots = 0;
    for (int p = 0; p < N; ++p) {
        const int buf = p & 1;
        double bv = -1.0;
        int rp = N;
        for (int w = 0; w < 16; ++w) {
            const double v = candv[buf][w];
            const int r = candr[buf][w];
            if (v > bv || (v == bv && r < rp)) {
                bv = v;
                rp = r;
            }
        }
        if (threadIdx.x == 0) {
            rowpiv[p] = rp;
            step_of[rp] = p;
            used[rp] = 1;
        }
        for (int j = threadIdx.x; j < N; j += kGJ) rowp[j] = B[(size_t)rp * N + j];
        for (int r = threadIdx.x; r < N; r += kGJ) colp[r] = B[(size_t)r * N + p];
        __syncthreads();
        const double piv = rowp[p];
        if (piv == 0.0) ++zero_pivots;
        const double d = 1.0 / piv;
        const int p1 = p + 1;
        double nb = -1.0;
        int nr = N;
        for (int r = ty; r < N; r += 16) {
            double* row = B + (size_t)r * N;
            const double cr = colp[r];
            const bool isp = (r == rp);
            const bool cand = !used[r];
            for (int j = tx; j < N; j += 64) {
                const double rpj = (j == p) ? d : rowp[j] * d;
                const double v = isp ? rpj : fma(-cr, rpj, (j == p) ? 0.0 : row[j]);
                row[j] = v;
                if (j == p1 && cand && fabs(v) > nb) {
                    nb = fabs(v);
                    nr = r;
                }
            }
        }
        if (tx == (p1 & 63)) {
            candv[buf ^ 1][ty] = nb;
            candr[buf ^ 1][ty] = nr;
        }
        __syncthreads();
    }
    for (int r = ty; r < N; r += 16) {
        const double* row = B + (size_t)r * N;
        double* orow = O + (size_t)step_of[r] * N;
        for (int j = tx; j < N; j += 64) orow[rowpiv[j]] = row[j];
    }
    if (threadIdx.x == 0 && info) info[blockIdx.x] = zero_pivots;
}

__global__ void k_copy_blocks(size_t n, const double* __restrict__ a, double* __restrict__ b) {
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (size_t)gridDim.x * blockDim.x)
        b[t] = a[t];
}

// Inverts nblocks blocks in place; tmp: nblocks x N x N doubles, used for N > 192.
void gj_inverse(int N, double* base, size_t stride, int nblocks, int* info, double* tmp,
                hipStream_t s) {
    if (N <= 64) {
        k_gj_blocked<4, 1><<<nblocks, kGJ, 0, s>>>(N, base, stride, info);
    } else if (N <= 128) {
        k_gj_blocked<8, 2><<<nblocks, kGJ, 0, s>>>(N, base, stride, info);
    } else if (N <= 192) {
        k_gj_blocked<12, 3><<<nblocks, kGJ, 0, s>>>(N, base, stride, info);
    } else {
        const size_t NN = (size_t)N * N;
        k_gj_global<<<nblocks, kGJ, 0, s>>>(N, base, stride, tmp, NN, info);
        for (int b = 0; b < nblocks; ++b)
            k_copy_blocks<<<(unsigned)std::min<size_t>((NN + 255) / 256, 4096), 256, 0, s>>>(
                NN, tmp + (size_t)b * NN, base + (size_t)b * stride);
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
    return carve_size({(size_t)g.M * nb * NN * 8, NN * 8, (size_t)g.ncol * 8, 4 * NM * 8, NN * 8,
                       tmp2_blocks(g, q) * NN * 8, (size_t)g.M * 4, (size_t)G * g.ncol * 8,
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
    P->tmp = c.take<double>(NN);
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
            gj_inverse(g.N, P->S, NN, g.M, P->info, P->tmp2, s);
        } else {
            double* scratchL = P->tmp2;  // q blocks for L_{i,l} and G_{l,j}
            for (int l = 0; l < g.M; ++l) {
                gj_inverse(g.N, P->S + blk_off(P, l, q), 0, 1, P->info + l, P->tmp2, s);
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
