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
    SW_REQUIRE(N <= kMaxGridN, "N must be <= 65536");
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

// ---- diagnostics: event timing of the all-pairs launches -------------------------
namespace {
std::mutex g_prof_mu;
bool g_prof_on = false;
struct ProfRec {
    hipEvent_t a, b;
    double pairs;
};
std::vector<ProfRec> g_prof;
std::vector<hipEvent_t> g_prof_pool;

hipEvent_t prof_event() {
    if (!g_prof_pool.empty()) {
        hipEvent_t e = g_prof_pool.back();
        g_prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    SW_HIP(hipEventCreate(&e));
    return e;
}
}  // namespace

ProfileMark profile_begin(hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    ProfileMark m;
    if (!g_prof_on) return m;
    m.a = prof_event();
    m.b = prof_event();
    SW_HIP(hipEventRecord(m.a, s));
    return m;
}

void profile_end(const ProfileMark& m, hipStream_t s, double pairs) {
    if (!m.a) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    SW_HIP(hipEventRecord(m.b, s));
    g_prof.push_back(ProfRec{m.a, m.b, pairs});
}

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
    const size_t wd = reduce_work_doubles(n, 2);
    sc.ensure(carve_size({(size_t)n * 8, (size_t)n * 8, 64, 64, 64, wd * 8}));
    Carve c(sc.base);
    double* up = c.take<double>(n);
    double* Ep = c.take<double>(n);
    double* hd = c.take<double>(2);
    double* nu_ = c.take<double>(2);
    double* nz_ = c.take<double>(2);
    double* work = c.take<double>(wd);
    if (h > 0.0) {
        set_step(h, hd, s);
    } else {
        const double macheps = (g.precision == SW_PREC_FP32) ? 1.1920928955078125e-07
                                                              : 2.220446049250313e-16;
        norm_inf_2(n, u, nu_, work, s);
        norm_inf_2(n, z, nz_, work, s);
        jvp_step(nu_, nz_, std::sqrt(macheps), std::sqrt((double)n), hd, s);
    }
    shift(n, u, z, hd, up, s);
    residual_one(g, up, Ep, s);
    quotient(n, Ep, Eu, hd, Jz, s);
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

int32_t shipwave_residual_batched(int32_t nb, const sw_problem* probs, const double* const* u,
                                  double* const* E, hipStream_t stream) {
    return guard([&]() -> int32_t {
        SW_REQUIRE(nb >= 0, "nb must be >= 0");
        if (nb == 0) return SW_OK;
        SW_REQUIRE(probs && u && E, "null pointer");
        std::vector<Geo> g(nb);
        for (int i = 0; i < nb; ++i) {
            g[i] = make_geo(probs[i]);
            SW_REQUIRE(u[i] && E[i], "null pointer");
        }
        residual_batched_enqueue(nb, g.data(), u, E, stream);
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

int32_t shipwave_profile_enable(int32_t on) {
    return guard([&]() -> int32_t {
        std::lock_guard<std::mutex> lk(sw::g_prof_mu);
        for (auto& r : sw::g_prof) {
            (void)hipEventSynchronize(r.b);
            sw::g_prof_pool.push_back(r.a);
            sw::g_prof_pool.push_back(r.b);
        }
        sw::g_prof.clear();
        sw::g_prof_on = (on != 0);
        return SW_OK;
    });
}

int32_t shipwave_profile_read(int64_t* launches, double* total_ms, double* pairs) {
    return guard([&]() -> int32_t {
        SW_REQUIRE(launches && total_ms && pairs, "null pointer");
        std::lock_guard<std::mutex> lk(sw::g_prof_mu);
        double ms = 0.0, pr = 0.0;
        for (auto& r : sw::g_prof) {
            SW_HIP(hipEventSynchronize(r.b));
            float t = 0.0f;
            SW_HIP(hipEventElapsedTime(&t, r.a, r.b));
            ms += t;
            pr += r.pairs;
        }
        *launches = (int64_t)sw::g_prof.size();
        *total_ms = ms;
        *pairs = pr;
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
