// E(u) for callers that cannot allocate device memory: the residual's intermediate arrays
// (grid fields, source and collocation records, per-chunk partial sums, spline sweep
// coefficients) live in one fixed array of the library, one copy per GPU.
#include <mutex>

#include "sw_internal.hpp"

namespace sw {
namespace {

constexpr size_t kFixedScratchBytes = (size_t)64 << 20;

// Host code never passes this name to a kernel: it stands for the array only in
// hipGetSymbolAddress, which gives each device's own address of it.
static __device__ __align__(256) unsigned char scratch[kFixedScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch`, looked up once per device.
void* fixed_scratch() {
    int dev = -1;
    SW_HIP(hipGetDevice(&dev));
    SW_REQUIRE(dev >= 0 && dev < kMaxDevices, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        SW_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        SW_REQUIRE(p != nullptr, "no device address for the fixed scratch array");
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace
}  // namespace sw

using namespace sw;

extern "C" {

int32_t shipwave_residual_noalloc(const sw_problem* prob, const double* u, double* E,
                                  hipStream_t stream) {
    return guard([&]() -> int32_t {
        SW_REQUIRE(prob && u && E, "null pointer");
        const Geo g = make_geo(*prob);
        SW_REQUIRE(u + 2 * (size_t)g.NM <= E || E + 2 * (size_t)g.NM <= u, "u and E overlap");
        const int G = choose_chunks(g);
        const size_t need = residual_scratch_bytes(g, G);
        if (need > kFixedScratchBytes)
            throw Error{SW_ENOMEM, "mesh needs " + std::to_string(need >> 20) +
                                       " MiB of scratch; the fixed array holds 64 MiB"};
        Carve c(fixed_scratch());
        const ResidualBufs b = carve_residual(c, g, G);
        residual_enqueue_fixed(g, u, E, b, stream);
        return SW_OK;
    });
}

}  // extern "C"
