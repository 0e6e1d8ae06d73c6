// wd_apply_noalloc: the operator application of wd_apply for callers that
// cannot allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid allocation).  The two internal-layout fields
// that wd_apply allocates stream-ordered live instead in a file-scope device
// array of fixed size, one copy per GPU, held until the process ends.
//
// In host code `scratch` names a host-side stand-in, not device memory: its
// device address on each GPU comes from hipGetSymbolAddress, taken once per
// device with that device current, and only that address is ever passed to
// kernels.
#include <mutex>

#include "runtime.hpp"

namespace wd {

// largest scratch: two fields of nrhs spinors (e.g. float64 with V * nrhs up
// to 349,525 sites, float32 24^3 x 48 with one rhs)
constexpr size_t kNoallocScratchBytes = (size_t)128 << 20;

static __device__ __align__(256) char scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices] = {};

// device address of this device's scratch (nullptr and the error set on
// failure); the caller's device must be current
static void *scratch_on_device(int *err) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        *err = fail(WD_ERR_HIP, "no current device for the scratch buffer");
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            *err = fail(WD_ERR_HIP, "hipGetSymbolAddress of the scratch buffer failed: %s",
                        hipGetErrorString(e));
            return nullptr;
        }
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace wd

using namespace wd;

extern "C" int wd_apply_noalloc(wd_lattice *lat, double kappa, int prec, int dagger, int nrhs,
                                const double *in, double *out, void *stream) {
    if (!lat || !in || !out) return fail(WD_ERR_ARG, "null argument");
    if (!valid_prec(prec)) return fail(WD_ERR_ARG, "unknown precision %d", prec);
    if (nrhs < 1 || nrhs > 12) return fail(WD_ERR_ARG, "nrhs = %d outside 1..12", nrhs);
    if (!std::isfinite(kappa)) return fail(WD_ERR_ARG, "kappa not finite");
    if (dagger != 0 && dagger != 1) return fail(WD_ERR_ARG, "dagger must be 0 or 1");
    if (in == out) return fail(WD_ERR_ARG, "in and out must not overlap");
    const int V = lat->g.V;
    const size_t one = (field_data_bytes(prec, V, nrhs) + 255) & ~(size_t)255;
    if (2 * one > kNoallocScratchBytes)
        return fail(WD_ERR_ARG,
                    "wd_apply_noalloc needs %zu bytes of scratch for %d rhs on %d sites, more "
                    "than its fixed %zu (use wd_apply)",
                    2 * one, nrhs, V, kNoallocScratchBytes);
    // the link form must be resident already: building it would allocate
    const void *gauge = nullptr;
    {
        std::lock_guard<std::mutex> lk(lat->mu);
        if (!lat->has_gauge) return fail(WD_ERR_NOGAUGE, "gauge field not set");
        gauge = lat->gauge[prec];
    }
    if (!gauge)
        return fail(WD_ERR_STATE,
                    "the %s link form is not built yet (any wd_apply or solve in that precision "
                    "builds it once)",
                    prec == WD_F32 ? "float32" : "binary16");
    int err = WD_OK;
    char *base = (char *)scratch_on_device(&err);
    if (!base) return err;
    hipStream_t s = (hipStream_t)stream;
    char *cur = base;
    FieldRef a = carve(cur, prec, nrhs, V);
    cur = base + one;
    FieldRef b = carve(cur, prec, nrhs, V);
    // the kernels compute in - kappa' * (hops): the +kappa sign is kappa' = -kappa
    const double k = -lat->hop_sign * kappa;
    const void *g12 = prec == WD_F64 ? lat->gauge12 : nullptr;
    launch_import(in, a, lat->g, s);
    launch_dslash(lat->g, gauge, k, dagger, a, b, nullptr, Gate{nullptr, nullptr, GATE_ACTIVE}, s,
                  g12);
    launch_export(b, out, lat->g, s);
    WD_LAUNCH_CHECK();
    return WD_OK;
}
