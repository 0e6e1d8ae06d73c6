// Field kernels of the CG solve (Sec. 2.2): gauge and spinor packing between
// the canonical interleaved layout and the internal planes, precision
// conversion, the fused vector updates x += alpha p / r -= alpha Ap with the
// |r|^2 reduction, p = r + beta p, the float64 true residual, and norms.
// All of them stream their operands once; the reductions are the
// deterministic block reduction of device.hpp.
#include "device.hpp"

namespace wd {

static constexpr int kBS = 256;

// ------------------------------------------------------------------ reduction phase 2

// One block: fixed-order sum of nb partials per rhs, then the finaliser.
// gated: skip when no rhs is iterating (the producing kernel returned early
// and wrote no partials).
constexpr int kFinalizeThreads = 256;

__global__ void __launch_bounds__(kFinalizeThreads) k_finalize(RedArgs red, int nb, int gated) {
    if (gated && red.batch->n_active == 0) return;
    __shared__ double sm[kFinalizeThreads];
    const int nrhs = red.ctl.nrhs;
    const int tid = threadIdx.x;
    int S = kFinalizeThreads;
    while (S * nrhs > kFinalizeThreads) S >>= 1;
    const int slot = tid / nrhs;
    const int r = tid - slot * nrhs;
    double acc = 0.0;
    if (slot < S)
        for (int b = slot; b < nb; b += S) acc += red.partials[(size_t)b * nrhs + r];
    sm[tid] = acc;
    __syncthreads();
    for (int stride = S >> 1; stride > 0; stride >>= 1) {
        if (tid < stride * nrhs) sm[tid] += sm[tid + stride * nrhs];
        __syncthreads();
    }
    if (tid < nrhs && red.mode != RED_NONE) finalize_rhs(red, tid, sm[tid]);
    __syncthreads();
    if (tid == 0 && red.mode != RED_NONE) recount_batch(red);
}

void launch_finalize(const RedArgs &red, int nb, bool gated, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinalizeThreads), 0, s, red, nb, gated ? 1 : 0);
}

// ------------------------------------------------------------------ gauge

// canonical [s][mu][a][b][re,im] (lexicographic s) -> F64-18 tiles in brick order
__global__ void k_pack_gauge_f64(const double2 *__restrict__ canon, void *__restrict__ g, Geom geo) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= geo.V) return;
    int x, y, z, t;
    coords_of(geo, i, x, y, z, t);
    const double2 *src = canon + (size_t)lex_of(geo, x, y, z, t) * 36;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        cx<double> u[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            double2 d = src[mu * 9 + k];
            u[k] = {d.x, d.y};
        }
        Link<WD_F64>::store(g, mu, i, u);
    }
}

// F64-18 -> 12-real forms (rows 0 and 1), rounded to nearest even
template <int PREC>
__global__ void k_gauge_lo(const void *__restrict__ g, void *__restrict__ o, int V) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= V) return;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        cx<double> u[9];
        Link<WD_F64>::load(g, mu, i, u);
        Link<PREC>::store(o, mu, i, u);
    }
}

void launch_pack_gauge_f64(const double *canon, void *g64, const Geom &geo, hipStream_t s) {
    hipLaunchKernelGGL(k_pack_gauge_f64, dim3(blocks_for(geo.V, kBS)), dim3(kBS), 0, s,
                       (const double2 *)canon, g64, geo);
}

void launch_gauge_lo(const void *g64, void *glo, int prec, int V, hipStream_t s) {
    if (prec == WD_F32)
        hipLaunchKernelGGL(k_gauge_lo<WD_F32>, dim3(blocks_for(V, kBS)), dim3(kBS), 0, s, g64, glo, V);
    else
        hipLaunchKernelGGL(k_gauge_lo<WD_F16>, dim3(blocks_for(V, kBS)), dim3(kBS), 0, s, g64, glo, V);
}

// ------------------------------------------------------------------ spinors

template <int PREC>
__device__ __forceinline__ void load_as_double(const FieldRef &f, int i, cx<double> v[12]) {
    cx<typename Spinor<PREC>::R> t[12];
    Spinor<PREC>::load(f, i, t);
#pragma unroll
    for (int k = 0; k < 12; ++k) v[k] = {(double)t[k].re, (double)t[k].im};
}

template <int PREC>
__device__ __forceinline__ void store_from_double(const FieldRef &f, int i, const cx<double> v[12]) {
    using R = typename Spinor<PREC>::R;
    cx<R> t[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) t[k] = {(R)v[k].re, (R)v[k].im};
    Spinor<PREC>::store(f, i, t);
}

// canonical [rhs][s][12][re,im] (lexicographic s) -> field entry i*nrhs + rhs
template <int PREC>
__global__ void k_import(const double2 *__restrict__ canon, FieldRef f, Geom geo) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= f.n) return;
    const int i = e / f.nrhs, r = e - i * f.nrhs;
    int x, y, z, t;
    coords_of(geo, i, x, y, z, t);
    const double2 *src = canon + ((size_t)r * geo.V + lex_of(geo, x, y, z, t)) * 12;
    cx<double> v[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        double2 d = src[k];
        v[k] = {d.x, d.y};
    }
    store_from_double<PREC>(f, e, v);
}

template <int PREC>
__global__ void k_export(FieldRef f, double2 *__restrict__ canon, Geom geo) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= f.n) return;
    const int i = e / f.nrhs, r = e - i * f.nrhs;
    int x, y, z, t;
    coords_of(geo, i, x, y, z, t);
    cx<double> v[12];
    load_as_double<PREC>(f, e, v);
    double2 *dst = canon + ((size_t)r * geo.V + lex_of(geo, x, y, z, t)) * 12;
#pragma unroll
    for (int k = 0; k < 12; ++k) dst[k] = make_double2(v[k].re, v[k].im);
}

template <int SRC, int DST>
__global__ void k_convert(FieldRef a, FieldRef b, Gate gate) {
    if (gate.batch && gate.batch->n_active == 0) return;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= a.n) return;
    if (gate.st && !gate.st[e % a.nrhs].active) return;
    cx<double> v[12];
    load_as_double<SRC>(a, e, v);
    store_from_double<DST>(b, e, v);
}

template <int PREC>
__global__ void k_zero(FieldRef f) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= f.n) return;
    cx<double> v[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) v[k] = {0.0, 0.0};
    store_from_double<PREC>(f, e, v);
}

// x64 += xlo ; xlo = 0 for rhs not yet converged
template <int PL>
__global__ void k_accum_zero(FieldRef x, FieldRef xl, const RhsState *st) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= x.n) return;
    if (st[e % x.nrhs].converged) return;
    cx<double> a[12], b[12], z[12];
    load_as_double<WD_F64>(x, e, a);
    load_as_double<PL>(xl, e, b);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        a[k] = a[k] + b[k];
        z[k] = {0.0, 0.0};
    }
    store_from_double<WD_F64>(x, e, a);
    store_from_double<PL>(xl, e, z);
}

#define WD_DISPATCH_PREC(P, ...)                   \
    switch (P) {                                   \
        case WD_F64: { constexpr int PP = WD_F64; __VA_ARGS__; } break; \
        case WD_F32: { constexpr int PP = WD_F32; __VA_ARGS__; } break; \
        default: { constexpr int PP = WD_F16; __VA_ARGS__; } break;     \
    }

void launch_import(const double *canon, FieldRef f, const Geom &geo, hipStream_t s) {
    WD_DISPATCH_PREC(f.prec, hipLaunchKernelGGL(k_import<PP>, dim3(blocks_for(f.n, kBS)),
                                                dim3(kBS), 0, s, (const double2 *)canon, f, geo));
}

void launch_export(FieldRef f, double *canon, const Geom &geo, hipStream_t s) {
    WD_DISPATCH_PREC(f.prec, hipLaunchKernelGGL(k_export<PP>, dim3(blocks_for(f.n, kBS)),
                                                dim3(kBS), 0, s, f, (double2 *)canon, geo));
}

template <int SRC>
static void convert_to(FieldRef a, FieldRef b, Gate gate, hipStream_t s) {
    const int nb = blocks_for(a.n, kBS);
    switch (b.prec) {
        case WD_F64: hipLaunchKernelGGL((k_convert<SRC, WD_F64>), dim3(nb), dim3(kBS), 0, s, a, b, gate); break;
        case WD_F32: hipLaunchKernelGGL((k_convert<SRC, WD_F32>), dim3(nb), dim3(kBS), 0, s, a, b, gate); break;
        default: hipLaunchKernelGGL((k_convert<SRC, WD_F16>), dim3(nb), dim3(kBS), 0, s, a, b, gate); break;
    }
}

void launch_convert(FieldRef a, FieldRef b, Gate gate, hipStream_t s) {
    WD_DISPATCH_PREC(a.prec, convert_to<PP>(a, b, gate, s));
}

void launch_zero(FieldRef f, hipStream_t s) {
    WD_DISPATCH_PREC(f.prec,
                     hipLaunchKernelGGL(k_zero<PP>, dim3(blocks_for(f.n, kBS)), dim3(kBS), 0, s, f));
}

void launch_accum_zero(FieldRef x, FieldRef xl, const RhsState *st, hipStream_t s) {
    WD_DISPATCH_PREC(xl.prec, hipLaunchKernelGGL(k_accum_zero<PP>, dim3(blocks_for(x.n, kBS)),
                                                 dim3(kBS), 0, s, x, xl, st));
}

// ------------------------------------------------------------------ CG updates

// x += alpha p ; r -= alpha Ap ; |r|^2.  x, r in precision PX (F64 or F32);
// p, Ap in PP (same as PX, or F16 with PX = F32).  Arithmetic in the compute
// type of PX, the norm in float64.
template <int PX, int PPP>
__global__ void k_update_xr(FieldRef x, FieldRef r, FieldRef p, FieldRef Ap, RedArgs red,
                            Gate gate) {
    if (gate.batch->n_active == 0) return;
    using R = typename Spinor<PX>::R;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int nrhs = x.nrhs;
    const int rhs = e % nrhs;
    double nrm = 0.0;
    if (e < x.n && gate.st[rhs].active) {
        const R alpha = (R)gate.st[rhs].alpha;
        cx<R> xv[12], rv[12], pv[12], av[12];
        Spinor<PX>::load(x, e, xv);
        Spinor<PX>::load(r, e, rv);
        Spinor<PPP>::load(p, e, pv);
        Spinor<PPP>::load(Ap, e, av);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            xv[k] = {xv[k].re + alpha * pv[k].re, xv[k].im + alpha * pv[k].im};
            rv[k] = {rv[k].re - alpha * av[k].re, rv[k].im - alpha * av[k].im};
            nrm += (double)rv[k].re * (double)rv[k].re + (double)rv[k].im * (double)rv[k].im;
        }
        Spinor<PX>::store(x, e, xv);
        Spinor<PX>::store(r, e, rv);
    }
    reduce_block(nrm, red.partials, nrhs);
}

// p = r + beta p (RESTART: at the first reliable update p = r)
template <int PX, int PPP, bool RESTART>
__global__ void k_update_p(FieldRef p, FieldRef r, Gate gate) {
    if (gate.batch->n_active == 0) return;
    using R = typename Spinor<PX>::R;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= p.n) return;
    const RhsState &st = gate.st[e % p.nrhs];
    if (!st.active) return;
    cx<R> rv[12], pv[12];
    Spinor<PX>::load(r, e, rv);
    if (RESTART && st.updates == 1) {
#pragma unroll
        for (int k = 0; k < 12; ++k) pv[k] = rv[k];
    } else {
        const R beta = (R)st.beta;
        cx<typename Spinor<PPP>::R> q[12];
        Spinor<PPP>::load(p, e, q);
#pragma unroll
        for (int k = 0; k < 12; ++k)
            pv[k] = {rv[k].re + beta * (R)q[k].re, rv[k].im + beta * (R)q[k].im};
    }
    cx<typename Spinor<PPP>::R> o[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) o[k] = {(typename Spinor<PPP>::R)pv[k].re, (typename Spinor<PPP>::R)pv[k].im};
    Spinor<PPP>::store(p, e, o);
}

void launch_update_xr(FieldRef x, FieldRef r, FieldRef p, FieldRef Ap, const RedArgs &red,
                      Gate gate, hipStream_t s) {
    const int bs = block_for_nrhs(x.nrhs);
    const int nb = blocks_for(x.n, bs);
    if (x.prec == WD_F64)
        hipLaunchKernelGGL((k_update_xr<WD_F64, WD_F64>), dim3(nb), dim3(bs), 0, s, x, r, p, Ap, red, gate);
    else if (p.prec == WD_F32)
        hipLaunchKernelGGL((k_update_xr<WD_F32, WD_F32>), dim3(nb), dim3(bs), 0, s, x, r, p, Ap, red, gate);
    else
        hipLaunchKernelGGL((k_update_xr<WD_F32, WD_F16>), dim3(nb), dim3(bs), 0, s, x, r, p, Ap, red, gate);
    launch_finalize(red, nb, true, s);
}

template <bool RESTART>
static void update_p_impl(FieldRef p, FieldRef r, Gate gate, hipStream_t s) {
    const int nb = blocks_for(p.n, kBS);
    if (r.prec == WD_F64)
        hipLaunchKernelGGL((k_update_p<WD_F64, WD_F64, RESTART>), dim3(nb), dim3(kBS), 0, s, p, r, gate);
    else if (p.prec == WD_F32)
        hipLaunchKernelGGL((k_update_p<WD_F32, WD_F32, RESTART>), dim3(nb), dim3(kBS), 0, s, p, r, gate);
    else
        hipLaunchKernelGGL((k_update_p<WD_F32, WD_F16, RESTART>), dim3(nb), dim3(kBS), 0, s, p, r, gate);
}

void launch_update_p(FieldRef p, FieldRef r, Gate gate, hipStream_t s) {
    update_p_impl<false>(p, r, gate, s);
}

void launch_restart_p(FieldRef p, FieldRef r, Gate gate, hipStream_t s) {
    update_p_impl<true>(p, r, gate, s);
}

// ------------------------------------------------------------------ residual / norms

// r = b - Ax (Ax absent: r = b), float64; reduce |r|^2
__global__ void k_residual(FieldRef r, FieldRef b, FieldRef Ax, RedArgs red) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int nrhs = r.nrhs;
    double nrm = 0.0;
    if (e < r.n) {
        cx<double> bv[12];
        Spinor<WD_F64>::load(b, e, bv);
        if (Ax.data) {
            cx<double> av[12];
            Spinor<WD_F64>::load(Ax, e, av);
#pragma unroll
            for (int k = 0; k < 12; ++k) bv[k] = bv[k] - av[k];
        }
#pragma unroll
        for (int k = 0; k < 12; ++k) nrm += bv[k].re * bv[k].re + bv[k].im * bv[k].im;
        Spinor<WD_F64>::store(r, e, bv);
    }
    reduce_block(nrm, red.partials, nrhs);
}

template <int PREC>
__global__ void k_norm(FieldRef f, RedArgs red) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    double nrm = 0.0;
    if (e < f.n) {
        cx<double> v[12];
        load_as_double<PREC>(f, e, v);
#pragma unroll
        for (int k = 0; k < 12; ++k) nrm += v[k].re * v[k].re + v[k].im * v[k].im;
    }
    reduce_block(nrm, red.partials, f.nrhs);
}

void launch_residual(FieldRef r, FieldRef b, FieldRef Ax, const RedArgs &red, hipStream_t s) {
    const int bs = block_for_nrhs(r.nrhs);
    const int nb = blocks_for(r.n, bs);
    hipLaunchKernelGGL(k_residual, dim3(nb), dim3(bs), 0, s, r, b, Ax, red);
    launch_finalize(red, nb, false, s);
}

void launch_norm(FieldRef f, const RedArgs &red, hipStream_t s) {
    const int bs = block_for_nrhs(f.nrhs);
    const int nb = blocks_for(f.n, bs);
    WD_DISPATCH_PREC(f.prec, hipLaunchKernelGGL(k_norm<PP>, dim3(nb), dim3(bs), 0, s, f, red));
    launch_finalize(red, nb, false, s);
}

__global__ void k_init_state(RhsState *st, BatchState *batch, int nrhs) {
    const int r = threadIdx.x;
    if (r < nrhs) {
        RhsState z{};
        st[r] = z;
    }
    if (r == 0) {
        batch->n_active = 0;
        batch->n_trigger = 0;
        batch->n_done = 0;
        batch->pad = 0;
    }
}

void launch_init_state(RhsState *st, BatchState *batch, int nrhs, hipStream_t s) {
    hipLaunchKernelGGL(k_init_state, dim3(1), dim3(64), 0, s, st, batch, nrhs);
}

}  // namespace wd
