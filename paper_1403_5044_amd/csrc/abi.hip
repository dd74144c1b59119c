// C ABI entry points: validation, scratch management, residual, JVP, zeta.
#include <cmath>
#include <map>
#include <memory>
#include <tuple>

#include "sw_internal.hpp"

namespace sw {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }

Geo make_geo(const sw_problem& p) {
    const int N = p.mesh.N, M = p.mesh.M;
    SW_REQUIRE(N >= 4 && M >= 4, "N and M must be >= 4");
    SW_REQUIRE(N <= kMaxN, "N must be <= 1024");
    SW_REQUIRE((long long)N * M <= (1LL << 28), "mesh too large");
    const sw_domain& d = p.domain;
    SW_REQUIRE(std::isfinite(d.x1) && std::isfinite(d.xN) && d.x1 < d.xN, "need x1 < xN");
    SW_REQUIRE(std::isfinite(d.yM) && d.yM > 0.0, "need yM > 0");
    const sw_params& q = p.params;
    SW_REQUIRE(std::isfinite(q.F) && q.F > 0.0, "need F > 0");
    SW_REQUIRE(std::isfinite(q.eps) && q.eps >= 0.0, "need eps >= 0");
    SW_REQUIRE(std::isfinite(q.nu) && q.nu > 0.0, "need nu > 0");
    SW_REQUIRE(q.weights == SW_WEIGHTS_TRAPEZOID || q.weights == SW_WEIGHTS_SIMPSON,
               "weights must be 0 (trapezoid) or 1 (Simpson)");
    SW_REQUIRE(q.weights == SW_WEIGHTS_TRAPEZOID || (N % 2 == 1 && M % 2 == 1),
               "Simpson weights need odd N and M");
    SW_REQUIRE(q.spline_bc == SW_SPLINE_CLAMPED0 || q.spline_bc == SW_SPLINE_NOTAKNOT,
               "spline_bc must be 0 or 1");
    SW_REQUIRE(q.precision == SW_PREC_FP64 || q.precision == SW_PREC_FP32,
               "precision must be 0 (FP64) or 1 (FP32)");
    Geo g{};
    g.N = N;
    g.M = M;
    g.Nc = N - 1;
    g.NM = N * M;
    g.ncol = (N - 1) * M;
    g.weights = q.weights;
    g.bc = q.spline_bc;
    g.precision = q.precision;
    g.x1 = d.x1;
    g.xN = d.xN;
    g.yM = d.yM;
    g.dx = (d.xN - d.x1) / (N - 1);
    g.dy = d.yM / (M - 1);
    g.F = q.F;
    g.eps = q.eps;
    g.nu = q.nu;
    return g;
}

// ---- scratch ---------------------------------------------------------------------
void Scratch::ensure(size_t need) {
    if (need <= bytes) return;
    int cur = -1;
    SW_HIP(hipGetDevice(&cur));
    if (base) {
        SW_HIP(hipStreamSynchronize(stream));
        SW_HIP(hipFree(base));
        base = nullptr;
        bytes = 0;
    }
    size_t sz = (need + (1u << 20) - 1) & ~size_t((1u << 20) - 1);
    if (hipMalloc(&base, sz) != hipSuccess) {
        (void)hipGetLastError();
        base = nullptr;
        throw Error{SW_ENOMEM, "device allocation of scratch failed"};
    }
    bytes = sz;
    device = cur;
}

Scratch::~Scratch() {
    // Process exit: the runtime may already be gone; leave the memory to the driver.
}

Scratch& scratch_for(hipStream_t stream, int slot) {
    static std::mutex mu;
    static std::map<std::tuple<int, hipStream_t, int>, std::unique_ptr<Scratch>> reg;
    int dev = -1;
    SW_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    auto& p = reg[std::make_tuple(dev, stream, slot)];
    if (!p) {
        p.reset(new Scratch());
        p->stream = stream;
        p->device = dev;
    }
    return *p;
}

namespace {

__global__ void k_jvp_h(const double* norms_u, const double* norms_z, double sqrt_eps,
                        double* h) {
    // norms_*[1] = 2-norm; h[0] = step, h[1] = 1/step (0 if z == 0)
    const double nz = norms_z[1];
    if (nz > 0.0) {
        const double s = sqrt_eps * (1.0 + norms_u[1]) / nz;
        h[0] = s;
        h[1] = 1.0 / s;
    } else {
        h[0] = 0.0;
        h[1] = 0.0;
    }
}

__global__ void k_set_h(double h, double* out) {
    out[0] = h;
    out[1] = 1.0 / h;
}

__global__ void k_shift(int n, const double* __restrict__ u, const double* __restrict__ z,
                        const double* __restrict__ h, double* __restrict__ out) {
    const double s = h[0];
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x)
        out[t] = fma(s, z[t], u[t]);
}

__global__ void k_quot(int n, const double* __restrict__ Ep, const double* __restrict__ Eu,
                       const double* __restrict__ h, double* __restrict__ out) {
    const double r = h[1];
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x)
        out[t] = (Ep[t] - Eu[t]) * r;
}

}  // namespace

void residual_one(const Geo& g, const double* u, double* E, hipStream_t s) {
    const int G = choose_chunks(g);
    Scratch& sc = scratch_for(s, 0);
    sc.ensure(residual_scratch_bytes(g, G));
    Carve c(sc.base);
    ResidualBufs b = carve_residual(c, g, G);
    residual_enqueue(g, u, E, b, s);
}

void jvp_one(const Geo& g, const double* u, const double* Eu, const double* z, double h,
             double* Jz, hipStream_t s) {
    const int n = 2 * g.NM;
    Scratch& sc = scratch_for(s, 1);
    const size_t wd = reduce_work_doubles(n);
    sc.ensure(carve_size({(size_t)n * 8, (size_t)n * 8, 64, 64, 64, wd * 8}));
    Carve c(sc.base);
    double* up = c.take<double>(n);
    double* Ep = c.take<double>(n);
    double* hd = c.take<double>(2);
    double* nu_ = c.take<double>(2);
    double* nz_ = c.take<double>(2);
    double* work = c.take<double>(wd);
    if (h > 0.0) {
        k_set_h<<<1, 1, 0, s>>>(h, hd);
    } else {
        const double macheps = (g.precision == SW_PREC_FP32) ? 1.1920928955078125e-07
                                                              : 2.220446049250313e-16;
        norm_inf_2(n, u, nu_, work, s);
        norm_inf_2(n, z, nz_, work, s);
        k_jvp_h<<<1, 1, 0, s>>>(nu_, nz_, std::sqrt(macheps), hd);
    }
    k_shift<<<(n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096, 256, 0, s>>>(n, u, z, hd, up);
    residual_one(g, up, Ep, s);
    k_quot<<<(n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096, 256, 0, s>>>(n, Ep, Eu, hd, Jz);
    SW_HIP(hipGetLastError());
}

}  // namespace sw

using namespace sw;

extern "C" {

int32_t shipwave_abi_version(void) { return SHIPWAVE_ABI_VERSION; }

const char* shipwave_last_error(void) { return sw::g_last_error.c_str(); }

int32_t shipwave_residual(const sw_problem* prob, const double* u, double* E, hipStream_t stream) {
    return guard([&]() -> int32_t {
        SW_REQUIRE(prob && u && E, "null pointer");
        const Geo g = make_geo(*prob);
        SW_REQUIRE(u + 2 * (size_t)g.NM <= E || E + 2 * (size_t)g.NM <= u, "u and E overlap");
        residual_one(g, u, E, stream);
        return SW_OK;
    });
}

int32_t shipwave_jvp(const sw_problem* prob, const double* u, const double* Eu, const double* z,
                     double h, double* Jz, hipStream_t stream) {
    return guard([&]() -> int32_t {
        SW_REQUIRE(prob && u && Eu && z && Jz, "null pointer");
        SW_REQUIRE(std::isfinite(h), "h must be finite");
        const Geo g = make_geo(*prob);
        SW_REQUIRE(Jz != u && Jz != z, "Jz may not alias u or z");
        jvp_one(g, u, Eu, z, h, Jz, stream);
        return SW_OK;
    });
}

int32_t shipwave_zeta(const sw_problem* prob, const double* u, double* zeta, hipStream_t stream) {
    return guard([&]() -> int32_t {
        SW_REQUIRE(prob && u && zeta, "null pointer");
        const Geo g = make_geo(*prob);
        zeta_enqueue(g, u, zeta, stream);
        return SW_OK;
    });
}

}  // extern "C"
