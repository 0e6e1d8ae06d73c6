// wd_stream_copy: a plain streaming copy with the access pattern of the
// solver's vector kernels (16-byte non-temporal loads and stores, every
// lane moving four 16-byte elements per step of a grid-stride loop).  It
// measures the device's practical streaming rate for one read and one write
// per byte, the ceiling against which the stencils' rates are compared.
#include "runtime.hpp"

namespace wd {

typedef float f4v __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_stream_copy(const f4v *__restrict__ src,
                                                     f4v *__restrict__ dst, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const f4v a = __builtin_nontemporal_load(src + i);
        const f4v b = __builtin_nontemporal_load(src + i + stride);
        const f4v c = __builtin_nontemporal_load(src + i + 2 * stride);
        const f4v d = __builtin_nontemporal_load(src + i + 3 * stride);
        __builtin_nontemporal_store(a, dst + i);
        __builtin_nontemporal_store(b, dst + i + stride);
        __builtin_nontemporal_store(c, dst + i + 2 * stride);
        __builtin_nontemporal_store(d, dst + i + 3 * stride);
    }
    for (; i < n; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

}  // namespace wd

using namespace wd;

extern "C" int wd_stream_copy(const void *src, void *dst, size_t bytes, void *stream) {
    if (!src || !dst) return fail(WD_ERR_ARG, "null argument");
    if (bytes % 16 || ((uintptr_t)src | (uintptr_t)dst) % 16)
        return fail(WD_ERR_ARG, "bytes and both pointers must be multiples of 16");
    const char *s = (const char *)src;
    char *d = (char *)dst;
    if (s < d + bytes && d < s + bytes) return fail(WD_ERR_ARG, "src and dst overlap");
    const size_t n = bytes / 16;
    if (!n) return WD_OK;
    // 16 workgroups of 256 lanes per compute unit (256 CUs)
    const int blocks = 4096;
    hipLaunchKernelGGL(k_stream_copy, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                       (const f4v *)src, (f4v *)dst, n);
    WD_LAUNCH_CHECK();
    return WD_OK;
}
