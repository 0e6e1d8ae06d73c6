// wd_stream_probe: plain streaming kernels with the access pattern of the
// solver's vector kernels: one pass, no grid-stride loop, each lane issuing
// all its 16-byte non-temporal loads (eight per source, consecutive lanes on
// consecutive elements) before it stores.  dst = the element-wise sum of nsrc
// source arrays (as float64 pairs): nsrc reads per write, so the probe
// reproduces a kernel's read/write mix (1: a copy; 3: the stencil's 576 read
// / 192 written bytes per site; 4: the r-updating stencil's 768 / 192).  Its
// rate is the device's practical streaming ceiling for that mix, the
// reference for the stencils' rates beside the HBM peak.
#include "runtime.hpp"

namespace wd {

typedef double d2v __attribute__((ext_vector_type(2)));

constexpr int kProbeMaxSrc = 4;
constexpr int kProbeUnroll = 8;   // elements per lane and source
constexpr int kProbeBlock = 256;

struct ProbeSrc {
    const d2v *p[kProbeMaxSrc];
};

template <int NS>
__global__ void __launch_bounds__(kProbeBlock) k_stream_probe(ProbeSrc src, d2v *__restrict__ dst,
                                                              size_t n) {
    const size_t i0 = (size_t)blockIdx.x * (kProbeBlock * kProbeUnroll) + threadIdx.x;
    d2v a[NS][kProbeUnroll];
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) {
            const size_t i = i0 + (size_t)u * kProbeBlock;
            a[s][u] = i < n ? __builtin_nontemporal_load(src.p[s] + i) : d2v{0.0, 0.0};
        }
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) {
        d2v v = a[0][u];
#pragma unroll
        for (int s = 1; s < NS; ++s) v += a[s][u];
        const size_t i = i0 + (size_t)u * kProbeBlock;
        if (i < n) __builtin_nontemporal_store(v, dst + i);
    }
}

}  // namespace wd

using namespace wd;

extern "C" int wd_stream_probe(const void *const *src, int nsrc, void *dst, size_t bytes,
                               void *stream) {
    if (!src || !dst) return fail(WD_ERR_ARG, "null argument");
    if (nsrc < 1 || nsrc > kProbeMaxSrc) return fail(WD_ERR_ARG, "nsrc = %d outside 1..4", nsrc);
    if (bytes % 16 || (uintptr_t)dst % 16)
        return fail(WD_ERR_ARG, "bytes and every pointer must be multiples of 16");
    ProbeSrc ps{};
    const char *d = (const char *)dst;
    for (int k = 0; k < nsrc; ++k) {
        const char *s = (const char *)src[k];
        if (!s || (uintptr_t)s % 16)
            return fail(WD_ERR_ARG, "bytes and every pointer must be multiples of 16");
        if (s < d + bytes && d < s + bytes) return fail(WD_ERR_ARG, "a source overlaps dst");
        ps.p[k] = (const d2v *)s;
    }
    const size_t n = bytes / 16;
    if (!n) return WD_OK;
    const dim3 grid((unsigned)((n + kProbeBlock * kProbeUnroll - 1) / (kProbeBlock * kProbeUnroll))),
        bs(kProbeBlock);
    hipStream_t st = (hipStream_t)stream;
    switch (nsrc) {
        case 1: hipLaunchKernelGGL(k_stream_probe<1>, grid, bs, 0, st, ps, (d2v *)dst, n); break;
        case 2: hipLaunchKernelGGL(k_stream_probe<2>, grid, bs, 0, st, ps, (d2v *)dst, n); break;
        case 3: hipLaunchKernelGGL(k_stream_probe<3>, grid, bs, 0, st, ps, (d2v *)dst, n); break;
        default: hipLaunchKernelGGL(k_stream_probe<4>, grid, bs, 0, st, ps, (d2v *)dst, n); break;
    }
    WD_LAUNCH_CHECK();
    return WD_OK;
}
