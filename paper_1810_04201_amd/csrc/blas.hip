// Field kernels of the CG solve (Sec. 2.2): gauge and spinor packing between
// the canonical interleaved layout and the internal planes, precision
// conversion, the vector updates of the CG iteration (x += alpha p with
// p = r + beta p in one pass; the unfused x/r update with the |r|^2
// reduction and p update), the float64 true residual, and norms.
// All of them stream their operands once; the reductions are the
// deterministic block reduction of device.hpp.
#include "device.hpp"

namespace wd {

static constexpr int kBS = 256;  // gauge kernels (one lane per site)

// ------------------------------------------------------------------ reduction phase 2

// One block: fixed-order sum of nb partials per rhs, then the finaliser.
// The order for an rhs does not depend on nrhs (thread t sums partials
// t + 4jT, t + (4j+1)T, t + (4j+2)T, t + (4j+3)T into four running sums,
// T = 1024; a butterfly inside each wave; the 16 waves in order), so a
// batched solve reproduces the single-rhs solves bit for bit.
// gate_mode >= 0: skipped when the producing kernel's batch gate was off
// (it returned early and wrote no partials).
constexpr int kFinalizeThreads = 1024;

__global__ void __launch_bounds__(kFinalizeThreads) k_finalize(RedArgs red, int nb, int gate_mode) {
    if (gate_mode >= 0 && gate_off(Gate{nullptr, red.batch, gate_mode})) return;
    constexpr int T = kFinalizeThreads, NW = T / 64;
    __shared__ double sm[NW * 12];
    const int nrhs = red.ctl.nrhs;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const double *P = red.partials;
    for (int r = 0; r < nrhs; ++r) {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int b = tid;
        for (; b + 3 * T < nb; b += 4 * T) {
            a0 += P[(size_t)b * nrhs + r];
            a1 += P[(size_t)(b + T) * nrhs + r];
            a2 += P[(size_t)(b + 2 * T) * nrhs + r];
            a3 += P[(size_t)(b + 3 * T) * nrhs + r];
        }
        for (; b < nb; b += T) a0 += P[(size_t)b * nrhs + r];
        double v = (a0 + a1) + (a2 + a3);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) sm[w * 12 + r] = v;
    }
    __syncthreads();
    if (tid < nrhs && red.mode != RED_NONE) {
        double t = 0.0;
        for (int k = 0; k < NW; ++k) t += sm[k * 12 + tid];
        finalize_rhs(red, tid, t);
    }
    __syncthreads();
    if (tid == 0 && red.mode != RED_NONE) recount_batch(red);
}

void launch_finalize(const RedArgs &red, int nb, int gate_mode, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinalizeThreads), 0, s, red, nb, gate_mode);
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

// F64-18 -> the compressed forms: 12 reals (rows 0 and 1, rounded to nearest
// even), or the 8-real binary16 form
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

void launch_gauge_lo(const void *g64, void *glo, int form, int V, hipStream_t s) {
    const dim3 gr(blocks_for(V, kBS)), bs(kBS);
    if (form == WD_F32)
        hipLaunchKernelGGL(k_gauge_lo<WD_F32>, gr, bs, 0, s, g64, glo, V);
    else if (form == WD_F16)
        hipLaunchKernelGGL(k_gauge_lo<WD_F16>, gr, bs, 0, s, g64, glo, V);
    else if (form == kLinkF16R8)
        hipLaunchKernelGGL(k_gauge_lo<kLinkF16R8>, gr, bs, 0, s, g64, glo, V);
    else
        hipLaunchKernelGGL(k_gauge_lo<kLinkF64R12>, gr, bs, 0, s, g64, glo, V);
}

// Largest deviation of a stored row 2 from conj(row 0 x row 1): per block in
// LDS, then one atomic maximum on the bit pattern (non-negative doubles
// order like their patterns)
__global__ void __launch_bounds__(256) k_su3_check(const void *__restrict__ g, int V,
                                                   unsigned long long *maxbits) {
    __shared__ double wmax[256 / 64];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double e = 0.0;
    if (i < V) {
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            cx<double> u[9], r[9];
            Link<WD_F64>::load(g, mu, i, u);
#pragma unroll
            for (int k = 0; k < 6; ++k) r[k] = u[k];
            reconstruct_row2(r);
#pragma unroll
            for (int j = 6; j < 9; ++j) {
                const double dr = u[j].re - r[j].re, di = u[j].im - r[j].im;
                const double d = sqrt(dr * dr + di * di);
                if (!(d <= e)) e = d == d ? d : INFINITY;
            }
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) e = fmax(e, __shfl_xor(e, off, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = e;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = wmax[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, wmax[w]);
        atomicMax(maxbits, (unsigned long long)__double_as_longlong(m));
    }
}

void launch_su3_check(const void *g64, int V, unsigned long long *maxbits, hipStream_t s) {
    hipLaunchKernelGGL(k_su3_check, dim3(blocks_for(V, 256)), dim3(256), 0, s, g64, V, maxbits);
}

// even-odd: links of the parity-p sites in the half layout and format PREC
template <int PREC>
__global__ void k_gauge_split(const void *__restrict__ g, void *__restrict__ o, int p, Geom geo) {
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= geo.V / 2) return;
    const int i = site_of_half(geo, h, p);
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        cx<double> u[9];
        Link<WD_F64>::load(g, mu, i, u);
        Link<PREC>::store(o, mu, h, u);
    }
}

void launch_gauge_split(const void *g64, void *half, int form, int p, const Geom &geo,
                        hipStream_t s) {
    const dim3 gr(blocks_for(geo.V / 2, kBS)), bs(kBS);
    const int prec = form;
    if (form == kLinkF64R12)
        hipLaunchKernelGGL(k_gauge_split<kLinkF64R12>, gr, bs, 0, s, g64, half, p, geo);
    else if (prec == WD_F64)
        hipLaunchKernelGGL(k_gauge_split<WD_F64>, gr, bs, 0, s, g64, half, p, geo);
    else if (prec == WD_F32)
        hipLaunchKernelGGL(k_gauge_split<WD_F32>, gr, bs, 0, s, g64, half, p, geo);
    else if (form == kLinkF16R8)
        hipLaunchKernelGGL(k_gauge_split<kLinkF16R8>, gr, bs, 0, s, g64, half, p, geo);
    else
        hipLaunchKernelGGL(k_gauge_split<WD_F16>, gr, bs, 0, s, g64, half, p, geo);
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

// Every field kernel below runs a grid of site_blocks(V) x nrhs workgroups:
// lane = site of the rhs blockIdx.y, so gating by the solver state is
// uniform over a workgroup.
static dim3 field_grid(const FieldRef &f) { return dim3(site_blocks(f.V), f.nrhs); }

// canonical [rhs][s][12][re,im] (lexicographic s) -> internal site i of rhs
template <int PREC>
__global__ void k_import(const double2 *__restrict__ canon, FieldRef f, Geom geo) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= geo.V) return;
    const int r = blockIdx.y;
    int x, y, z, t;
    coords_of(geo, i, x, y, z, t);
    const double2 *src = canon + ((size_t)r * geo.V + lex_of(geo, x, y, z, t)) * 12;
    cx<double> v[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        double2 d = src[k];
        v[k] = {d.x, d.y};
    }
    store_from_double<PREC>(rhs_view(f, r), i, v);
}

template <int PREC>
__global__ void k_export(FieldRef f, double2 *__restrict__ canon, Geom geo) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= geo.V) return;
    const int r = blockIdx.y;
    int x, y, z, t;
    coords_of(geo, i, x, y, z, t);
    cx<double> v[12];
    load_as_double<PREC>(rhs_view(f, r), i, v);
    double2 *dst = canon + ((size_t)r * geo.V + lex_of(geo, x, y, z, t)) * 12;
#pragma unroll
    for (int k = 0; k < 12; ++k) dst[k] = make_double2(v[k].re, v[k].im);
}

// canonical [rhs][s][12] <-> half field of parity p (entry h: site
// site_of_half(h, p)); f.V = V / 2
template <int PREC>
__global__ void k_import_half(const double2 *__restrict__ canon, FieldRef f, int p, Geom geo) {
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= f.V) return;
    const int r = blockIdx.y;
    int x, y, z, t;
    coords_of(geo, site_of_half(geo, h, p), x, y, z, t);
    const double2 *src = canon + ((size_t)r * geo.V + lex_of(geo, x, y, z, t)) * 12;
    cx<double> v[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        double2 d = src[k];
        v[k] = {d.x, d.y};
    }
    store_from_double<PREC>(rhs_view(f, r), h, v);
}

template <int PREC>
__global__ void k_export_half(FieldRef f, double2 *__restrict__ canon, int p, Geom geo) {
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= f.V) return;
    const int r = blockIdx.y;
    int x, y, z, t;
    coords_of(geo, site_of_half(geo, h, p), x, y, z, t);
    cx<double> v[12];
    load_as_double<PREC>(rhs_view(f, r), h, v);
    double2 *dst = canon + ((size_t)r * geo.V + lex_of(geo, x, y, z, t)) * 12;
#pragma unroll
    for (int k = 0; k < 12; ++k) dst[k] = make_double2(v[k].re, v[k].im);
}

template <int SRC, int DST>
__global__ void k_convert(FieldRef a, FieldRef b, Gate gate) {
    if (gate_off(gate)) return;
    const int r = blockIdx.y;
    if (!gate_rhs(gate, r)) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.V) return;
    cx<double> v[12];
    load_as_double<SRC>(rhs_view(a, r), i, v);
    store_from_double<DST>(rhs_view(b, r), i, v);
}

template <int PREC>
__global__ void k_zero(FieldRef f) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= f.V) return;
    cx<double> v[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) v[k] = {0.0, 0.0};
    store_from_double<PREC>(rhs_view(f, blockIdx.y), i, v);
}

// x64 += xlo ; xlo = 0 for the rhs a reliable update takes (GATE_TRIGGER),
// else for every rhs not yet converged.  An rhs whose last alpha p is still
// pending (it froze between the r update and the lagged x update) adds it:
// x64 += xlo + alpha p, in float64.
template <int PL, int PP>
__global__ void __launch_bounds__(kSiteBlock) k_accum_zero(FieldRef x, FieldRef xl, FieldRef p,
                                                         Gate gate) {
    const int r = blockIdx.y;
    if (gate.mode == GATE_TRIGGER) {
        if (gate_off(gate) || !gate_rhs(gate, r)) return;
    } else if (gate.st[r].converged) {
        return;
    }
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= x.V) return;
    const FieldRef xv = rhs_view(x, r), lv = rhs_view(xl, r);
    cx<double> b[12];
    load_as_double<PL>(lv, i, b);
    if (gate.st[r].pend) {
        const double alpha = gate.st[r].alpha;
        cx<double> q[12];
        load_as_double<PP>(rhs_view(p, r), i, q);
#pragma unroll
        for (int k = 0; k < 12; ++k) b[k] = {b[k].re + alpha * q[k].re, b[k].im + alpha * q[k].im};
    }
    {
        cx<double> a[12];
        load_as_double<WD_F64>(xv, i, a);
#pragma unroll
        for (int k = 0; k < 12; ++k) b[k] = a[k] + b[k];
    }
    store_from_double<WD_F64>(xv, i, b);
#pragma unroll
    for (int k = 0; k < 12; ++k) b[k] = {0.0, 0.0};
    store_from_double<PL>(lv, i, b);
}

#define WD_DISPATCH_PREC(P, ...)                   \
    switch (P) {                                   \
        case WD_F64: { constexpr int PP = WD_F64; __VA_ARGS__; } break; \
        case WD_F32: { constexpr int PP = WD_F32; __VA_ARGS__; } break; \
        default: { constexpr int PP = WD_F16; __VA_ARGS__; } break;     \
    }

void launch_import(const double *canon, FieldRef f, const Geom &geo, hipStream_t s) {
    WD_DISPATCH_PREC(f.prec, hipLaunchKernelGGL(k_import<PP>, field_grid(f), dim3(kSiteBlock), 0,
                                                s, (const double2 *)canon, f, geo));
}

void launch_export(FieldRef f, double *canon, const Geom &geo, hipStream_t s) {
    WD_DISPATCH_PREC(f.prec, hipLaunchKernelGGL(k_export<PP>, field_grid(f), dim3(kSiteBlock), 0,
                                                s, f, (double2 *)canon, geo));
}

void launch_import_half(const double *canon, FieldRef f, int p, const Geom &geo, hipStream_t s) {
    WD_DISPATCH_PREC(f.prec, hipLaunchKernelGGL(k_import_half<PP>, field_grid(f), dim3(kSiteBlock),
                                                0, s, (const double2 *)canon, f, p, geo));
}

void launch_export_half(FieldRef f, double *canon, int p, const Geom &geo, hipStream_t s) {
    WD_DISPATCH_PREC(f.prec, hipLaunchKernelGGL(k_export_half<PP>, field_grid(f), dim3(kSiteBlock),
                                                0, s, f, (double2 *)canon, p, geo));
}

template <int SRC>
static void convert_to(FieldRef a, FieldRef b, Gate gate, hipStream_t s) {
    const dim3 gr = field_grid(a), bs(kSiteBlock);
    switch (b.prec) {
        case WD_F64: hipLaunchKernelGGL((k_convert<SRC, WD_F64>), gr, bs, 0, s, a, b, gate); break;
        case WD_F32: hipLaunchKernelGGL((k_convert<SRC, WD_F32>), gr, bs, 0, s, a, b, gate); break;
        default: hipLaunchKernelGGL((k_convert<SRC, WD_F16>), gr, bs, 0, s, a, b, gate); break;
    }
}

void launch_convert(FieldRef a, FieldRef b, Gate gate, hipStream_t s) {
    WD_DISPATCH_PREC(a.prec, convert_to<PP>(a, b, gate, s));
}

void launch_zero(FieldRef f, hipStream_t s) {
    WD_DISPATCH_PREC(f.prec,
                     hipLaunchKernelGGL(k_zero<PP>, field_grid(f), dim3(kSiteBlock), 0, s, f));
}

void launch_accum_zero(FieldRef x, FieldRef xl, FieldRef p, Gate gate, hipStream_t s) {
    const dim3 gr = field_grid(x), bs(kSiteBlock);
    if (xl.prec == WD_F64)
        hipLaunchKernelGGL((k_accum_zero<WD_F64, WD_F64>), gr, bs, 0, s, x, xl, p, gate);
    else if (p.prec == WD_F32)
        hipLaunchKernelGGL((k_accum_zero<WD_F32, WD_F32>), gr, bs, 0, s, x, xl, p, gate);
    else
        hipLaunchKernelGGL((k_accum_zero<kF16XrPrec, WD_F16>), gr, bs, 0, s, x, xl, p, gate);
}

// ------------------------------------------------------------------ CG updates

// x += alpha p ; r -= alpha Ap ; |r|^2.  x, r in precision PX (F64 or F32);
// p, Ap in PP (same as PX, or F16 with PX = F32).  Arithmetic in the compute
// type of PX, the norm in float64.  A frozen rhs's workgroups return at once
// (the finaliser ignores its partials).
template <int PX, int PPP>
__global__ void __launch_bounds__(kSiteBlock) k_update_xr(FieldRef x, FieldRef r, FieldRef p,
                                                        FieldRef Ap, RedArgs red, Gate gate) {
    if (gate_off(gate)) return;
    const int rhs = blockIdx.y;
    if (!gate_rhs(gate, rhs)) return;
    using R = typename Spinor<PX>::R;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double nrm = 0.0;
    if (i < x.V) {
        const FieldRef xf = rhs_view(x, rhs), rf = rhs_view(r, rhs);
        const R alpha = (R)gate.st[rhs].alpha;
        cx<R> xv[12], rv[12], pv[12], av[12];
        Spinor<PX>::load(xf, i, xv);
        Spinor<PX>::load(rf, i, rv);
        Spinor<PPP>::load(rhs_view(p, rhs), i, pv);
        Spinor<PPP>::load(rhs_view(Ap, rhs), i, av);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            xv[k] = {xv[k].re + alpha * pv[k].re, xv[k].im + alpha * pv[k].im};
            rv[k] = {rv[k].re - alpha * av[k].re, rv[k].im - alpha * av[k].im};
            nrm += (double)rv[k].re * (double)rv[k].re + (double)rv[k].im * (double)rv[k].im;
        }
        Spinor<PX>::store(xf, i, xv);
        Spinor<PX>::store(rf, i, rv);
    }
    reduce_block(nrm, red.partials, (size_t)blockIdx.x * x.nrhs + rhs);
}

// p = r + beta p (RESTART: at the first reliable update p = r)
template <int PX, int PPP, bool RESTART>
__global__ void k_update_p(FieldRef p, FieldRef r, Gate gate) {
    if (gate_off(gate)) return;
    const int rhs = blockIdx.y;
    if (!gate_rhs(gate, rhs)) return;
    const RhsState &st = gate.st[rhs];
    using R = typename Spinor<PX>::R;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.V) return;
    const FieldRef pf = rhs_view(p, rhs);
    cx<R> rv[12], pv[12];
    Spinor<PX>::load(rhs_view(r, rhs), i, rv);
    if (RESTART && st.updates == 1) {
#pragma unroll
        for (int k = 0; k < 12; ++k) pv[k] = rv[k];
    } else {
        const R beta = (R)st.beta;
        cx<typename Spinor<PPP>::R> q[12];
        Spinor<PPP>::load(pf, i, q);
#pragma unroll
        for (int k = 0; k < 12; ++k)
            pv[k] = {rv[k].re + beta * (R)q[k].re, rv[k].im + beta * (R)q[k].im};
    }
    cx<typename Spinor<PPP>::R> o[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) o[k] = {(typename Spinor<PPP>::R)pv[k].re, (typename Spinor<PPP>::R)pv[k].im};
    Spinor<PPP>::store(pf, i, o);
}

// non-temporal loads and stores in k_update_xp: each field streams through
// once per iteration (48^3 x 96: -5% float64, -8% in the binary16 mode)
#ifndef WD_NT_XP
#define WD_NT_XP 1
#endif

// x += alpha p ; p = r + beta p: the x update of the iteration whose r
// update a stencil did, merged with the p update (p read once).  Same
// arithmetic as k_update_xr's x update and k_update_p.
template <int PX, int PPP>
__global__ void k_update_xp(FieldRef x, FieldRef p, FieldRef r, Gate gate) {
    if (gate_off(gate)) return;
    const int rhs = blockIdx.y;
    if (!gate_rhs(gate, rhs)) return;
    const RhsState &st = gate.st[rhs];
    using R = typename Spinor<PX>::R;
    using RP = typename Spinor<PPP>::R;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.V) return;
    const FieldRef xf = rhs_view(x, rhs), pf = rhs_view(p, rhs);
    const R alpha = (R)st.alpha, beta = (R)st.beta;
    cx<RP> q[12];
    cx<R> v[12];
    Spinor<PPP>::template load<WD_NT_XP>(pf, i, q);
    Spinor<PX>::template load<WD_NT_XP>(xf, i, v);
#pragma unroll
    for (int k = 0; k < 12; ++k)
        v[k] = {v[k].re + alpha * (R)q[k].re, v[k].im + alpha * (R)q[k].im};
    Spinor<PX>::template store<WD_NT_XP>(xf, i, v);
    Spinor<PX>::template load<WD_NT_XP>(rhs_view(r, rhs), i, v);
    cx<RP> o[12];
#pragma unroll
    for (int k = 0; k < 12; ++k)
        o[k] = {(RP)(v[k].re + beta * (R)q[k].re), (RP)(v[k].im + beta * (R)q[k].im)};
    Spinor<PPP>::template store<WD_NT_XP>(pf, i, o);
}

void launch_update_xp(FieldRef x, FieldRef p, FieldRef r, Gate gate, hipStream_t s) {
    const dim3 gr = field_grid(p), bs(kSiteBlock);
    if (x.prec == WD_F64)
        hipLaunchKernelGGL((k_update_xp<WD_F64, WD_F64>), gr, bs, 0, s, x, p, r, gate);
    else if (p.prec == WD_F32)
        hipLaunchKernelGGL((k_update_xp<WD_F32, WD_F32>), gr, bs, 0, s, x, p, r, gate);
    else
        hipLaunchKernelGGL((k_update_xp<kF16XrPrec, WD_F16>), gr, bs, 0, s, x, p, r, gate);
}

void launch_update_xr(FieldRef x, FieldRef r, FieldRef p, FieldRef Ap, const RedArgs &red,
                      Gate gate, hipStream_t s) {
    const dim3 gr = field_grid(x), bs(kSiteBlock);
    if (x.prec == WD_F64)
        hipLaunchKernelGGL((k_update_xr<WD_F64, WD_F64>), gr, bs, 0, s, x, r, p, Ap, red, gate);
    else if (p.prec == WD_F32)
        hipLaunchKernelGGL((k_update_xr<WD_F32, WD_F32>), gr, bs, 0, s, x, r, p, Ap, red, gate);
    else
        hipLaunchKernelGGL((k_update_xr<kF16XrPrec, WD_F16>), gr, bs, 0, s, x, r, p, Ap, red, gate);
    launch_finalize(red, gr.x, GATE_ACTIVE, s);
}

template <bool RESTART>
static void update_p_impl(FieldRef p, FieldRef r, Gate gate, hipStream_t s) {
    const dim3 gr = field_grid(p), bs(kSiteBlock);
    if (r.prec == WD_F64)
        hipLaunchKernelGGL((k_update_p<WD_F64, WD_F64, RESTART>), gr, bs, 0, s, p, r, gate);
    else if (p.prec == WD_F32)
        hipLaunchKernelGGL((k_update_p<WD_F32, WD_F32, RESTART>), gr, bs, 0, s, p, r, gate);
    else
        hipLaunchKernelGGL((k_update_p<kF16XrPrec, WD_F16, RESTART>), gr, bs, 0, s, p, r, gate);
}

void launch_update_p(FieldRef p, FieldRef r, Gate gate, hipStream_t s) {
    update_p_impl<false>(p, r, gate, s);
}

void launch_restart_p(FieldRef p, FieldRef r, Gate gate, hipStream_t s) {
    update_p_impl<true>(p, r, gate, s);
}

// ------------------------------------------------------------------ residual / norms

// r = b - Ax (Ax absent: r = b), float64; reduce |r|^2.  A gated-off rhs
// writes no partial (the finaliser ignores it).
__global__ void k_residual(FieldRef r, FieldRef b, FieldRef Ax, RedArgs red, Gate gate) {
    if (gate_off(gate)) return;
    const int rhs = blockIdx.y;
    if (!gate_rhs(gate, rhs)) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double nrm = 0.0;
    if (i < r.V) {
        cx<double> bv[12];
        Spinor<WD_F64>::load(rhs_view(b, rhs), i, bv);
        if (Ax.data) {
            cx<double> av[12];
            Spinor<WD_F64>::load(rhs_view(Ax, rhs), i, av);
#pragma unroll
            for (int k = 0; k < 12; ++k) bv[k] = bv[k] - av[k];
        }
#pragma unroll
        for (int k = 0; k < 12; ++k) nrm += bv[k].re * bv[k].re + bv[k].im * bv[k].im;
        Spinor<WD_F64>::store(rhs_view(r, rhs), i, bv);
    }
    reduce_block(nrm, red.partials, (size_t)blockIdx.x * r.nrhs + rhs);
}

template <int PREC>
__global__ void k_norm(FieldRef f, RedArgs red) {
    const int rhs = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double nrm = 0.0;
    if (i < f.V) {
        cx<double> v[12];
        load_as_double<PREC>(rhs_view(f, rhs), i, v);
#pragma unroll
        for (int k = 0; k < 12; ++k) nrm += v[k].re * v[k].re + v[k].im * v[k].im;
    }
    reduce_block(nrm, red.partials, (size_t)blockIdx.x * f.nrhs + rhs);
}

void launch_residual(FieldRef r, FieldRef b, FieldRef Ax, const RedArgs &red, Gate gate,
                     hipStream_t s) {
    const dim3 gr = field_grid(r);
    hipLaunchKernelGGL(k_residual, gr, dim3(kSiteBlock), 0, s, r, b, Ax, red, gate);
    launch_finalize(red, gr.x, gate.batch ? gate.mode : -1, s);
}

void launch_norm(FieldRef f, const RedArgs &red, hipStream_t s) {
    const dim3 gr = field_grid(f);
    WD_DISPATCH_PREC(f.prec, hipLaunchKernelGGL(k_norm<PP>, gr, dim3(kSiteBlock), 0, s, f, red));
    launch_finalize(red, gr.x, -1, s);
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
