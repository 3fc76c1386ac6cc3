// Allocation-free half-sweep (half_sweep_noalloc in include/coreals.h).
//
// A half-sweep needs per-call scratch beside its inputs and outputs: event
// counters, the row-queue counters of the persistent launches, the heavy rows'
// partial systems and their refinement residuals.  half_sweep_users/items take
// it from the context's workspace; this entry point takes it from `scratch`, a
// fixed array of this library in device memory, so that it can run where the
// caller may not allocate (and with a context whose workspace was sized for a
// small heavy_pair_cap).
//
// The array exists once per GPU and keeps the last call's contents.  Every
// call clears the counters it uses (by a kernel) and overwrites every partial
// system before reading it.  Calls on one GPU share the array, so calls that
// overlap in time on one GPU (two streams, two host threads) race.
#include <mutex>

#include "internal.hpp"

namespace coreals {

namespace {

// Most partial systems one batch of the heavy-row plan may hold here.
constexpr int64_t NA_PAIR_CAP = 1024;

constexpr size_t a256(size_t x) { return (x + 255) & ~size_t(255); }
constexpr size_t NA_STATS_OFF = 0;
constexpr size_t NA_QUEUES_OFF = a256(NA_STATS_OFF + sizeof(unsigned long long) * NSTATS);
constexpr size_t NA_PARTIALS_OFF = a256(NA_QUEUES_OFF + sizeof(unsigned int) * 2 * 16);
constexpr size_t NA_RESID_OFF = a256(NA_PARTIALS_OFF + sizeof(float) * (size_t)NA_PAIR_CAP * (NF + 1) * 64);
constexpr size_t NA_BYTES = a256(NA_RESID_OFF + sizeof(double) * (size_t)NA_PAIR_CAP * 128);  // 17.7 MB

// The scratch array.  Host code never uses this name as an address: it uses
// the device address hipGetSymbolAddress returns for the current GPU.
__device__ __align__(256) unsigned char scratch[NA_BYTES];

constexpr int NA_MAX_DEVICES = 64;
std::mutex g_mu;
unsigned char *g_ptr[NA_MAX_DEVICES] = {};

// Device address of `scratch` on the current GPU (looked up once per device).
hipError_t scratch_ptr(unsigned char **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= NA_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ptr[dev] = static_cast<unsigned char *>(p);
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

}  // namespace

}  // namespace coreals

using namespace coreals;

extern "C" {

size_t half_sweep_noalloc_scratch_bytes(void) { return NA_BYTES; }

int64_t half_sweep_noalloc_pair_cap(void) { return NA_PAIR_CAP; }

als_status half_sweep_noalloc(als_ctx *c, int side, const float *other, float *out, als_sweep_stats *st) {
    if (!c) return ALS_E_STATE;
    if (side != 0 && side != 1) return set_error(c, ALS_E_ARG, "side must be 0 or 1");
    if (c->fast || c->unif || c->implicit)
        return set_error(c, ALS_E_ARG,
                         "half_sweep_noalloc: the fast variant, UNIF and implicit feedback keep their state "
                         "(selection, Gram) in the workspace; use half_sweep_users / half_sweep_items");
    // partial systems of 65 x 64 floats (ranks up to 64) or 129 x 128 (above)
    const int64_t slot = c->wide ? (int64_t)(NFW + 1) * NFW : (int64_t)(NF + 1) * 64;
    if (c->pair_cap * slot > NA_PAIR_CAP * (NF + 1) * 64 || c->pair_cap * 2 * (c->wide ? NFW : 64) > NA_PAIR_CAP * 128)
        return set_error(c, ALS_E_ARG,
                         "half_sweep_noalloc: the context's heavy_pair_cap exceeds the partial systems of the "
                         "library's scratch array; create the context with heavy_pair_cap <= 1024 (n_f <= 64) "
                         "or <= 258 (n_f > 64)");
    unsigned char *base = nullptr;
    const hipError_t e = scratch_ptr(&base);
    if (e != hipSuccess) return set_error(c, ALS_E_DEVICE, hipGetErrorString(e));
    SweepScratch sc;
    sc.stats = reinterpret_cast<unsigned long long *>(base + NA_STATS_OFF);
    sc.queues = reinterpret_cast<unsigned int *>(base + NA_QUEUES_OFF);
    sc.partials = reinterpret_cast<float *>(base + NA_PARTIALS_OFF);
    sc.resid = reinterpret_cast<double *>(base + NA_RESID_OFF);
    const als_status rs = enqueue_half_sweep_scratch(c, side, other, out, sc);
    if (rs != ALS_OK) return rs;
    if (st) return fill_stats(c, side, sc.stats, st);
    return ALS_OK;
}

}  // extern "C"
