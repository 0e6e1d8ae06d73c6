// Wilson-Dirac stencil (Eq. (1) of Sec. 2.1 with the minus sign) on gfx950.
//
// One lane per site of one right-hand side.  Each of the eight hops projects the
// neighbour spinor to a half-spinor with 1 -+ gamma_mu (two spin components
// of three colours; the projectors have rank 2, Sec. 2.1), multiplies the two
// colour vectors by U_mu(x) (forward) or U_mu(x-mu)^dag (backward), and
// rebuilds the lower two spin components from the upper two by a sign or a
// factor +-i.  The result is out(x) = in(x) - kappa * sum of the hops.
// D^dag uses the same kernel with the projector signs exchanged.
//
// Half-spinor table for (1 + s gamma_mu) psi with the Appendix A basis:
//   mu=0: h0 = psi0 + s i psi3, h1 = psi1 + s i psi2;  lower: -s i h1, -s i h0
//   mu=1: h0 = psi0 - s psi3,   h1 = psi1 + s psi2;    lower:  s h1,   -s h0
//   mu=2: h0 = psi0 + s i psi2, h1 = psi1 - s i psi3;  lower: -s i h0,  s i h1
//   mu=3: h0 = psi0 + s psi2,   h1 = psi1 + s psi3;    lower:  s h0,    s h1
// D uses s = -1 forward and s = +1 backward; D^dag the opposite.
//
// Bandwidth bound: 1320 flop per site against 960 bytes (FP64, 18-real
// links), so there is no matrix-core work here; the kernel is written for
// coalesced 16-byte loads from the structure-of-arrays planes.
#include <cstdlib>

#include "device.hpp"

#ifndef WD_XCD_REMAP
#define WD_XCD_REMAP 1
#endif
// hops per scheduling group (see k_dslash): with two marching workgroups
// per CU, float64 groups of 3 measured 1-2% faster than 1 (2 and 6 within
// 0.3% of 3)
#ifndef WD_GROUP_F64
#define WD_GROUP_F64 3
#endif
#ifndef WD_GROUP_LO
#define WD_GROUP_LO 2
#endif
// non-temporal forward links / outputs in the marching stencil (measured:
// streaming the outputs past the caches keeps more of the slices the
// neighbouring columns read; the links are re-read by the backward hops)
#ifndef WD_NT_LINK
#define WD_NT_LINK 0
#endif
// non-temporal forward t links: each is read once (the next slice's
// backward hop reuses it from registers), so streaming it past L2 leaves
// room for the faces neighbouring columns read (-1% time)
#ifndef WD_NT_LINK_T
#define WD_NT_LINK_T 1
#endif
#ifndef WD_NT_OUT
#define WD_NT_OUT 1
#endif
// binary16 hops (12-real links) with their link products on packed halves
// (v_dot2_f32_f16) instead of float32 operands: 48^3 x 96 binary16 stencil
// 0.63 -> 0.56 ms, its r-updating form 0.82 -> 0.79 ms
#ifndef WD_F16_DOT2
#define WD_F16_DOT2 1
#endif
// the marching stencil's fused r update: load r at the start of the step
// (its latency hidden behind the hops) instead of after them; per
// precision bit: 1 float64, 2 float32, 4 binary16
#ifndef WD_XR_PREFETCH
#define WD_XR_PREFETCH 1
#endif
// the prefetched r loaded non-temporally: read once per iteration (-1%)
#ifndef WD_NT_RLOAD
#define WD_NT_RLOAD 1
#endif


namespace wd {

template <int MU, int S, typename R>
__device__ __forceinline__ void project(const cx<R> p[12], cx<R> h0[3], cx<R> h1[3]) {
    // p[3*spin + colour]
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const cx<R> a0 = p[c], a1 = p[3 + c], a2 = p[6 + c], a3 = p[9 + c];
        if (MU == 0) {
            h0[c] = S > 0 ? a0 + times_i(a3) : a0 - times_i(a3);
            h1[c] = S > 0 ? a1 + times_i(a2) : a1 - times_i(a2);
        } else if (MU == 1) {
            h0[c] = S > 0 ? a0 - a3 : a0 + a3;
            h1[c] = S > 0 ? a1 + a2 : a1 - a2;
        } else if (MU == 2) {
            h0[c] = S > 0 ? a0 + times_i(a2) : a0 - times_i(a2);
            h1[c] = S > 0 ? a1 - times_i(a3) : a1 + times_i(a3);
        } else {
            h0[c] = S > 0 ? a0 + a2 : a0 - a2;
            h1[c] = S > 0 ? a1 + a3 : a1 - a3;
        }
    }
}

template <int MU, int S, typename R>
__device__ __forceinline__ void accumulate(const cx<R> w0[3], const cx<R> w1[3], cx<R> acc[12]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        acc[c] = acc[c] + w0[c];
        acc[3 + c] = acc[3 + c] + w1[c];
        if (MU == 0) {
            // lower: -s i w1, -s i w0
            acc[6 + c] = S > 0 ? acc[6 + c] - times_i(w1[c]) : acc[6 + c] + times_i(w1[c]);
            acc[9 + c] = S > 0 ? acc[9 + c] - times_i(w0[c]) : acc[9 + c] + times_i(w0[c]);
        } else if (MU == 1) {
            // lower: s w1, -s w0
            acc[6 + c] = S > 0 ? acc[6 + c] + w1[c] : acc[6 + c] - w1[c];
            acc[9 + c] = S > 0 ? acc[9 + c] - w0[c] : acc[9 + c] + w0[c];
        } else if (MU == 2) {
            // lower: -s i w0, s i w1
            acc[6 + c] = S > 0 ? acc[6 + c] - times_i(w0[c]) : acc[6 + c] + times_i(w0[c]);
            acc[9 + c] = S > 0 ? acc[9 + c] + times_i(w1[c]) : acc[9 + c] - times_i(w1[c]);
        } else {
            // lower: s w0, s w1
            acc[6 + c] = S > 0 ? acc[6 + c] + w0[c] : acc[6 + c] - w0[c];
            acc[9 + c] = S > 0 ? acc[9 + c] + w1[c] : acc[9 + c] - w1[c];
        }
    }
}

// w = U h  or  w = U^dag h
template <bool ADJ, typename R>
__device__ __forceinline__ void su3_mul(const cx<R> u[9], const cx<R> h[3], cx<R> w[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cx<R> s = {R(0), R(0)};
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            if (ADJ)
                s = cfmac(u[3 * b + a], h[b], s);  // conj(U[b][a]) h[b]
            else
                s = cfma(u[3 * a + b], h[b], s);   // U[a][b] h[b]
        }
        w[a] = s;
    }
}

// one hop: project the neighbour spinor, multiply by the link, rebuild, add
template <int MU, int S, bool BWD, int PREC, int LF = PREC>
__device__ __forceinline__ void hop(const void *gauge, const FieldRef &in, int nbr_entry,
                                    int link_site, bool negate,
                                    cx<typename Spinor<PREC>::R> acc[12]) {
    using R = typename Spinor<PREC>::R;
    if constexpr (PREC == WD_F16 && LF == WD_F16 && WD_F16_DOT2) {
        h2_t q[12];
        float sc;
        Spinor<WD_F16>::load_raw(in, nbr_entry, q, sc);
        h2_t h0[3], h1[3];
        project_h2<MU, S>(q, h0, h1);
        h2_t u[9];
        Link<WD_F16>::load_h2<false>(gauge, MU, link_site, u);
        cx<float> w0[3], w1[3];
        su3_mul_h2<BWD>(u, h0, w0);
        su3_mul_h2<BWD>(u, h1, w1);
        // the antiperiodic boundary sign rides on the site scale
        accumulate_s<MU, S>(MU == 3 && negate ? -sc : sc, w0, w1, acc);
        return;
    }
    cx<R> p[12];
    Spinor<PREC>::load(in, nbr_entry, p);
    cx<R> h0[3], h1[3];
    project<MU, S>(p, h0, h1);
    if (MU == 3) {
        // antiperiodic boundary: a select, not a branch, so that the
        // compiler keeps each hop's arithmetic next to its loads
        const R sg = negate ? R(-1) : R(1);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            h0[c] = scale(sg, h0[c]);
            h1[c] = scale(sg, h1[c]);
        }
    }
    cx<R> u[9];
    Link<LF>::load(gauge, MU, link_site, u);
    cx<R> w0[3], w1[3];
    su3_mul<BWD>(u, h0, w0);
    su3_mul<BWD>(u, h1, w1);
    accumulate<MU, S>(w0, w1, acc);
}

// Workgroups are dealt round-robin to the 8 XCDs (each with its own L2).
// With WD_XCD_REMAP each XCD instead walks one contiguous run of logical
// blocks, so that neighbours within a few thousand sites share an L2.
__device__ __forceinline__ int logical_block() {
#if WD_XCD_REMAP
    const int nb = gridDim.x, b = blockIdx.x;
    const int x = b & 7, i = b >> 3;
    const int q = nb >> 3, r = nb & 7;
    return x * q + (x < r ? x : r) + i;
#else
    return blockIdx.x;
#endif
}

// one hop with the neighbour spinor and the link already in registers
template <int MU, int S, bool BWD, typename R>
__device__ __forceinline__ void hop_p(const cx<R> p[12], const cx<R> u[9], bool negate,
                                      cx<R> acc[12]) {
    cx<R> h0[3], h1[3];
    project<MU, S>(p, h0, h1);
    const R sg = negate ? R(-1) : R(1);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        h0[c] = scale(sg, h0[c]);
        h1[c] = scale(sg, h1[c]);
    }
    cx<R> w0[3], w1[3];
    su3_mul<BWD>(u, h0, w0);
    su3_mul<BWD>(u, h1, w1);
    accumulate<MU, S>(w0, w1, acc);
}

// LDS image of a workgroup's part of a brick slice: its tiles copied
// verbatim (a part is a multiple of 64 sites and starts at a multiple of
// 64), so the field accessors read it with the field's own tile arithmetic.
template <int PREC>
__host__ __device__ inline size_t slice_bytes(int sites) {
    return (size_t)(sites >> 6) * Spinor<PREC>::kTileBytes;
}

// field view of an LDS slice image
__device__ __forceinline__ FieldRef lds_view(const FieldRef &f, const char *img) {
    FieldRef v = f;
    v.data = (void *)img;
    return v;
}

typedef __attribute__((address_space(3))) void lds_void;

// Asynchronous copy of the slice whose first tile is tile0 into the LDS image
// img: wave w copies tile w, plane by plane, each lane 16 bytes (4 for the
// binary16 scales) straight from memory into LDS (the wave's LDS target is
// uniform, lane k lands at k * size past it).  Completion is tracked by the
// vector memory counter.
template <int PREC>
__device__ __forceinline__ void slice_copy(const FieldRef &f, int tile0, char *img) {
    constexpr size_t TB = Spinor<PREC>::kTileBytes;
    constexpr int NP = PREC == WD_F64 ? 12 : (PREC == WD_F32 ? 6 : 3);
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = (int)(threadIdx.x & 63);
    const char *src = (const char *)f.data + (size_t)(tile0 + w) * TB;
    char *dst = img + (size_t)w * TB;
#pragma unroll
    for (int k = 0; k < NP; ++k)
        __builtin_amdgcn_global_load_lds((const void *)(src + k * 1024 + lane * 16),
                                         (lds_void *)(dst + k * 1024), 16, 0, 0);
    if (PREC == WD_F16)
        __builtin_amdgcn_global_load_lds((const void *)(src + NP * 1024 + lane * 4),
                                         (lds_void *)(dst + NP * 1024), 4, 0, 0);
}

// one spatial hop of the marching stencil: the neighbour comes from the LDS
// image when it lies in this workgroup's part of the slice (wvol sites from
// sbase), else (a brick face, or another part of the slice) from memory
template <int MU, int S, bool BWD, int PREC, int LF = PREC>
__device__ __forceinline__ void hop_s(const void *gauge, const FieldRef &in, const FieldRef &cur,
                                      int sbase, int wvol, int nbr, int link_site,
                                      cx<typename Spinor<PREC>::R> acc[12]) {
    using R = typename Spinor<PREC>::R;
    const int d = nbr - sbase;
    if constexpr (PREC == WD_F16 && LF == WD_F16 && WD_F16_DOT2) {
        h2_t q[12];
        float sc;
        if ((unsigned)d < (unsigned)wvol)
            Spinor<WD_F16>::load_raw(cur, d, q, sc);
        else
            Spinor<WD_F16>::load_raw(in, nbr, q, sc);
        h2_t h0[3], h1[3];
        project_h2<MU, S>(q, h0, h1);
        h2_t u[9];
        Link<WD_F16>::load_h2<WD_NT_LINK && !BWD>(gauge, MU, link_site, u);
        cx<float> w0[3], w1[3];
        su3_mul_h2<BWD>(u, h0, w0);
        su3_mul_h2<BWD>(u, h1, w1);
        accumulate_s<MU, S>(sc, w0, w1, acc);
        return;
    }
    cx<R> p[12];
    // the compiler merges the two loads into one flat load on the selected
    // pointer (LDS or memory); separate LDS-typed and global loads measured
    // four times slower in float64 (both paths' registers live at once)
    if ((unsigned)d < (unsigned)wvol)
        Spinor<PREC>::load(cur, d, p);
    else
        Spinor<PREC>::load(in, nbr, p);
    cx<R> h0[3], h1[3];
    project<MU, S>(p, h0, h1);
    cx<R> u[9];
    Link<LF>::template load<WD_NT_LINK && !BWD>(gauge, MU, link_site, u);
    cx<R> w0[3], w1[3];
    su3_mul<BWD>(u, h0, w0);
    su3_mul<BWD>(u, h1, w1);
    accumulate<MU, S>(w0, w1, acc);
}

template <int PREC, bool DAG, bool RED, int GROUP, int LF = PREC>
__global__ void __launch_bounds__(256) k_dslash(Geom g, const void *__restrict__ gauge, FieldRef in,
                                                FieldRef out, double kappa_d, RedArgs red,
                                                Gate gate) {
    using R = typename Spinor<PREC>::R;
    if (gate_off(gate)) return;  // grid-uniform
    // logical block = site block * nrhs + rhs: the workgroups of all rhs on
    // the same sites are neighbours in the XCD's run and share its L2 links
    const int nrhs = in.nrhs;
    const int lb = logical_block();
    const int sb = lb / nrhs;
    const int rhs = lb - sb * nrhs;
    // a gated-off rhs: the finaliser ignores its partials
    if (!gate_rhs(gate, rhs)) return;  // workgroup-uniform
    const FieldRef fin = rhs_view(in, rhs);
    const int site = sb * blockDim.x + threadIdx.x;
    double nrm = 0.0;
    if (site < g.V) {
        const Nbrs nb = neighbours(g, site);
        const int xp = nb.xp, xm = nb.xm, yp = nb.yp, ym = nb.ym;
        const int zp = nb.zp, zm = nb.zm, tp = nb.tp, tm = nb.tm;
        const bool neg_tp = g.antiperiodic && nb.cross_tp;
        const bool neg_tm = g.antiperiodic && nb.cross_tm;

        cx<R> acc[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = {R(0), R(0)};
        // forward projector sign: D -> s = -1, D^dag -> s = +1; backward opposite
        constexpr int SF = DAG ? +1 : -1;
        constexpr int SB = -SF;
        // A scheduling barrier after every GROUP hops bounds how many hops'
        // operands the compiler keeps in flight (registers versus
        // memory-level parallelism).
#define WD_HOP_FENCE(k) \
    if ((k) % GROUP == 0) __builtin_amdgcn_sched_barrier(0)
        hop<0, SF, false, PREC, LF>(gauge, fin, xp, site, false, acc);
        WD_HOP_FENCE(1);
        hop<0, SB, true, PREC, LF>(gauge, fin, xm, xm, false, acc);
        WD_HOP_FENCE(2);
        hop<1, SF, false, PREC, LF>(gauge, fin, yp, site, false, acc);
        WD_HOP_FENCE(3);
        hop<1, SB, true, PREC, LF>(gauge, fin, ym, ym, false, acc);
        WD_HOP_FENCE(4);
        hop<2, SF, false, PREC, LF>(gauge, fin, zp, site, false, acc);
        WD_HOP_FENCE(5);
        hop<2, SB, true, PREC, LF>(gauge, fin, zm, zm, false, acc);
        WD_HOP_FENCE(6);
        hop<3, SF, false, PREC, LF>(gauge, fin, tp, site, neg_tp, acc);
        WD_HOP_FENCE(7);
        hop<3, SB, true, PREC, LF>(gauge, fin, tm, tm, neg_tm, acc);
        WD_HOP_FENCE(8);
#undef WD_HOP_FENCE

        cx<R> c[12];
        Spinor<PREC>::load(fin, site, c);
        const R kappa = (R)kappa_d;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            c[k] = c[k] - scale(kappa, acc[k]);
            if (RED) nrm += (double)c[k].re * (double)c[k].re + (double)c[k].im * (double)c[k].im;
        }
        Spinor<PREC>::store(rhs_view(out, rhs), site, c);
    }
    if (RED) reduce_block(nrm, red.partials, (size_t)sb * nrhs + rhs);
}

// r -= alpha q at site i of one rhs (r in F64, or F32 beside an F32/F16
// stencil), in the compute type of the stencil; returns |r|^2 in float64.
// The same arithmetic as the stand-alone update of the solver, on the
// stencil's unrounded q.  xr_site_r: with r already loaded into v.
template <int PREC>
__device__ __forceinline__ double xr_site_r(const XrArgs &a, int rhs, int i,
                                            typename Spinor<PREC>::R alpha,
                                            const cx<typename Spinor<PREC>::R> q[12],
                                            cx<typename Spinor<PREC>::R> v[12]) {
    constexpr int PX = xr_prec_of(PREC);
    double nrm = 0.0;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        v[k] = {v[k].re - alpha * q[k].re, v[k].im - alpha * q[k].im};
        nrm += (double)v[k].re * (double)v[k].re + (double)v[k].im * (double)v[k].im;
    }
    Spinor<PX>::template store<WD_NT_OUT>(rhs_view(a.r, rhs), i, v);
    return nrm;
}

template <int PREC>
__device__ __forceinline__ double xr_site(const XrArgs &a, int rhs, int i,
                                          typename Spinor<PREC>::R alpha,
                                          const cx<typename Spinor<PREC>::R> q[12]) {
    constexpr int PX = xr_prec_of(PREC);
    using R = typename Spinor<PREC>::R;
    cx<R> v[12];
    Spinor<PX>::load(rhs_view(a.r, rhs), i, v);
    return xr_site_r<PREC>(a, rhs, i, alpha, q, v);
}

// Time-marching stencil.  One workgroup per brick column, chunk of time
// slices, part of the brick slice (all of it, or one of several contiguous
// runs of whole tiles) and rhs, one lane per site.  The workgroup steps through its
// slices together with two LDS images of its part:
//  - at the start of step t the next slice t+1 is copied from memory into
//    the spare image, while the x/y/z hops of slice t read their neighbours
//    from the current image (inside the part) or from memory (across a
//    brick face or into another part);
//  - the forward t hop reads psi(t+1) from the new image, which is the
//    current one of the next step, so every site of the column is read from
//    memory once;
//  - the backward t hop U_t(x, t-1)^dag (1 -+ gamma_t) psi(x, t-1) is carried
//    from the previous step in registers.
// The hops are summed in the order of the one-lane-per-site kernel.
// Logical blocks are ordered chunk, column, part, rhs (rhs fastest), so each
// XCD's contiguous run covers one band of time slices of many neighbouring
// columns, and the workgroups of all rhs of a column part run side by side
// and read its links from L2 after the first.
// The fused reduction writes one partial per (column, slice, part, rhs), so
// its summation order does not depend on the chunk length or on nrhs.
// HALO: the lattice is one t-slab of a larger one; the t hops across its
// ends read staged faces (see Halo) in place of the wrapped slices: only the
// sources of the prologue's spinor and link, of the last step's slice copy,
// and the boundary sign change.
// XR: the CG update that consumes q = A p is done where q is formed, so q is
// never stored: r -= alpha q, and the reduction is |r|^2 (see XrArgs).  out
// is unused.
// LF: the link form (PREC's own, or F64-12 for float64).
template <int PREC, bool DAG, bool RED, int GROUP, bool HALO = false, bool XR = false,
          int LF = PREC>
__global__ void __launch_bounds__(kTmMaxBlock) k_dslash_tm(Geom g, const void *__restrict__ gauge,
                                                   FieldRef in, FieldRef out, double kappa_d,
                                                   RedArgs red, Gate gate, int tchunk,
                                                   int ncols, Halo halo, XrArgs xr) {
    using R = typename Spinor<PREC>::R;
    extern __shared__ __align__(16) char lds[];
    __shared__ double wsum[kTmMaxBlock / 64];
    if (gate_off(gate)) return;  // grid-uniform
    const int nrhs = in.nrhs;
    const int wvol = (int)blockDim.x;  // sites of this workgroup's part of a slice
    const int nsub = g.bvol / wvol;
    const int lb = logical_block();
    const int cb = lb / nrhs;
    const int rhs = lb - cb * nrhs;
    // a gated-off rhs: the finaliser ignores its partials
    if (!gate_rhs(gate, rhs)) return;  // workgroup-uniform
    const FieldRef fin = rhs_view(in, rhs), fout = rhs_view(out, rhs);
    const int cc = cb / nsub;
    const int h = cb - cc * nsub;
    const int lchunk = cc / ncols;
    const int col = cc - lchunk * ncols;
    const int chunk = HALO ? halo.cfirst + lchunk * halo.cstep : lchunk;
    const int Lt = g.L[3], bvol = g.bvol;
    const int l = (int)threadIdx.x;
    const int t0 = chunk * tchunk;
    const int t1 = t0 + tchunk < Lt ? t0 + tchunk : Lt;
    // first site of this workgroup's part of slice t: cbase + t * bvol
    const int cbase = col * Lt * bvol + h * wvol;
    char *img0 = lds;
    char *img1 = lds + slice_bytes<PREC>(wvol);
    constexpr int SF = DAG ? +1 : -1;
    constexpr int SB = -SF;
    const R kappa = (R)kappa_d;

    // halo: this workgroup's part of a face (first face site, staged views)
    const int fbase = col * bvol + h * wvol;
    FieldRef hprev = fin, hnext = fin;
    if (HALO) {
        hprev.data = (void *)halo.prev;
        hnext.data = (void *)halo.next;
        const int vf = g.V / Lt;
        hprev.V = hnext.V = vf;
        hprev.stride = hnext.stride = rhs_stride(vf);
        hprev = rhs_view(hprev, rhs);
        hnext = rhs_view(hnext, rhs);
    }
    const bool prev_from_halo = HALO && t0 == 0;

    // prologue: slice t0 into image 0, and the backward t hop from t0 - 1
    slice_copy<PREC>(fin, (cbase + t0 * bvol) >> 6, img0);
    cx<R> cw0[3], cw1[3];
    {
        const int tprev = t0 == 0 ? Lt - 1 : t0 - 1;
        const int ip = cbase + tprev * bvol + l;
        cx<R> p[12];
        Spinor<PREC>::load(prev_from_halo ? hprev : fin, prev_from_halo ? fbase + l : ip, p);
        cx<R> h0[3], h1[3];
        project<3, SB>(p, h0, h1);
        const R sg = (g.antiperiodic && t0 == 0 && (!HALO || halo.first)) ? R(-1) : R(1);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            h0[c] = scale(sg, h0[c]);
            h1[c] = scale(sg, h1[c]);
        }
        cx<R> u[9];
        if constexpr (HALO && LF == PREC) {
            Link<PREC>::load(prev_from_halo ? halo.links : gauge, 3,
                             prev_from_halo ? fbase + l : ip, u);
        } else if constexpr (HALO) {
            // the entering links are float64 with 18 reals
            if (prev_from_halo)
                Link<PREC>::load(halo.links, 3, fbase + l, u);
            else
                Link<LF>::load(gauge, 3, ip, u);
        } else {
            Link<LF>::load(gauge, 3, ip, u);
        }
        su3_mul<true>(u, h0, cw0);
        su3_mul<true>(u, h1, cw1);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int t = t0; t < t1; ++t) {
        const bool odd = (t - t0) & 1;
        const FieldRef cur = lds_view(fin, odd ? img1 : img0);
        const FieldRef nxt = lds_view(fin, odd ? img0 : img1);
        const int tn = t + 1 < Lt ? t + 1 : 0;
        // the slice after the slab's last one is the staged next face
        const bool next_from_halo = HALO && t + 1 == Lt;
        slice_copy<PREC>(next_from_halo ? hnext : fin,
                         next_from_halo ? fbase >> 6 : (cbase + tn * bvol) >> 6, (char *)nxt.data);
        const int sbase = cbase + t * bvol;
        const int i = sbase + l;
        constexpr bool XPRE = XR && ((WD_XR_PREFETCH >> PREC) & 1);
        cx<R> rpre[XPRE ? 12 : 1];
        if constexpr (XPRE)
            Spinor<xr_prec_of(PREC)>::template load<WD_NT_RLOAD>(
                rhs_view(xr.r, rhs), i, rpre);
        const Nbrs nb = neighbours(g, i);
        cx<R> acc[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = {R(0), R(0)};
#define WD_HOP_FENCE(k) \
    if ((k) % GROUP == 0) __builtin_amdgcn_sched_barrier(0)
        hop_s<0, SF, false, PREC, LF>(gauge, fin, cur, sbase, wvol, nb.xp, i, acc);
        WD_HOP_FENCE(1);
        hop_s<0, SB, true, PREC, LF>(gauge, fin, cur, sbase, wvol, nb.xm, nb.xm, acc);
        WD_HOP_FENCE(2);
        hop_s<1, SF, false, PREC, LF>(gauge, fin, cur, sbase, wvol, nb.yp, i, acc);
        WD_HOP_FENCE(3);
        hop_s<1, SB, true, PREC, LF>(gauge, fin, cur, sbase, wvol, nb.ym, nb.ym, acc);
        WD_HOP_FENCE(4);
        hop_s<2, SF, false, PREC, LF>(gauge, fin, cur, sbase, wvol, nb.zp, i, acc);
        WD_HOP_FENCE(5);
        hop_s<2, SB, true, PREC, LF>(gauge, fin, cur, sbase, wvol, nb.zm, nb.zm, acc);
        WD_HOP_FENCE(6);
#undef WD_HOP_FENCE
        // binary16 with 12-real links: the t hops on packed halves too
        constexpr bool H2 = PREC == WD_F16 && LF == WD_F16 && WD_F16_DOT2;
        cx<R> ut[H2 ? 1 : 9];
        h2_t ut2[H2 ? 9 : 1];
        if constexpr (H2)
            Link<WD_F16>::template load_h2<WD_NT_LINK || WD_NT_LINK_T>(gauge, 3, i, ut2);
        else
            Link<LF>::template load<WD_NT_LINK || WD_NT_LINK_T>(gauge, 3, i, ut);
        // the next slice has landed in LDS (every wave's copy)
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        const bool neg_tp = g.antiperiodic && t == Lt - 1 && (!HALO || halo.last);
        cx<R> c[12];
        if constexpr (H2) {
            {
                h2_t q[12];
                float sc;
                Spinor<WD_F16>::load_raw(nxt, l, q, sc);
                h2_t h0[3], h1[3];
                project_h2<3, SF>(q, h0, h1);
                cx<float> w0[3], w1[3];
                su3_mul_h2<false>(ut2, h0, w0);
                su3_mul_h2<false>(ut2, h1, w1);
                accumulate_s<3, SF>(neg_tp ? -sc : sc, w0, w1, acc);
            }
            accumulate<3, SB>(cw0, cw1, acc);
            h2_t q[12];
            float sc;
            Spinor<WD_F16>::load_raw(cur, l, q, sc);
#pragma unroll
            for (int k = 0; k < 12; ++k) c[k] = {sc * (float)q[k].x, sc * (float)q[k].y};
            // carry for slice t + 1, scaled here as the float carry is
            h2_t h0[3], h1[3];
            project_h2<3, SB>(q, h0, h1);
            su3_mul_h2<true>(ut2, h0, cw0);
            su3_mul_h2<true>(ut2, h1, cw1);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                cw0[k] = scale(sc, cw0[k]);
                cw1[k] = scale(sc, cw1[k]);
            }
        } else {
            {
                cx<R> nx[12];
                Spinor<PREC>::load(nxt, l, nx);
                hop_p<3, SF, false>(nx, ut, neg_tp, acc);
            }
            accumulate<3, SB>(cw0, cw1, acc);
            Spinor<PREC>::load(cur, l, c);
            // carry for slice t + 1 (never crosses the boundary inside a chunk)
            cx<R> h0[3], h1[3];
            project<3, SB>(c, h0, h1);
            su3_mul<true>(ut, h0, cw0);
            su3_mul<true>(ut, h1, cw1);
        }
        double nrm = 0.0;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            c[k] = c[k] - scale(kappa, acc[k]);
            if (RED && !XR)
                nrm += (double)c[k].re * (double)c[k].re + (double)c[k].im * (double)c[k].im;
        }
        if constexpr (XPRE)
            nrm = xr_site_r<PREC>(xr, rhs, i, (R)gate.st[rhs].alpha, c, rpre);
        else if constexpr (XR)
            nrm = xr_site<PREC>(xr, rhs, i, (R)gate.st[rhs].alpha, c);
        else
            Spinor<PREC>::template store<WD_NT_OUT>(fout, i, c);
        if (RED) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) nrm += __shfl_xor(nrm, off, 64);
            if ((l & 63) == 0) wsum[l >> 6] = nrm;
        }
        __syncthreads();  // the current image is free for the next copy
        if (RED && l == 0) {
            double s = 0.0;
            for (int w = 0; w < (wvol >> 6); ++w) s += wsum[w];
            red.partials[(((size_t)col * Lt + t) * nsub + h) * nrhs + rhs] = s;
        }
    }
}

// WD_TCHUNK overrides the marching stencil's chunk length (tuning)
static int tm_chunk(const Geom &g, int nrhs) {
    static const int env = [] {
        const char *e = getenv("WD_TCHUNK");
        return e ? atoi(e) : 0;
    }();
    return tm_chunk_len(g, nrhs, env);
}

// WD_SITE_KERNEL=1 forces the one-lane-per-site stencil everywhere (tuning)
static const bool g_force_site_kernel = [] {
    const char *e = getenv("WD_SITE_KERNEL");
    return e && atoi(e) != 0;
}();

// hops per scheduling group (see k_dslash)
template <int PREC>
struct HopGroup {
    static constexpr int value = PREC == WD_F64 ? WD_GROUP_F64 : WD_GROUP_LO;
};

// LDS a workgroup may use on the current device
static size_t max_lds_per_block() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return 65536;
    return (size_t)v;
}

// dynamic LDS above 64 KiB must be allowed per kernel once
template <typename K>
static void allow_lds(K kernel, size_t bytes) {
    if (bytes > 65536)
        (void)hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)bytes);
}

template <int PREC>
static bool tm_fits(const Geom &g) {
    static const size_t cap = max_lds_per_block();
    return 2 * slice_bytes<PREC>(tm_wvol(g, PREC)) + 64 <= cap;
}

template <int PREC, bool DAG, bool RED, int LF = PREC>
static void launch_tm_k(dim3 grid, dim3 bs, size_t lds, hipStream_t s, const Geom &g,
                        const void *gauge, FieldRef in, FieldRef out, double kappa,
                        const RedArgs &r, Gate gate, int tch, int ncols) {
    constexpr int G = HopGroup<PREC>::value;
    auto k = k_dslash_tm<PREC, DAG, RED, G, false, false, LF>;
    allow_lds(k, lds);
    hipLaunchKernelGGL(k, grid, bs, lds, s, g, gauge, in, out, kappa, r, gate, tch, ncols,
                       Halo{nullptr, nullptr, nullptr, 0, 0, 0, 0, 1}, XrArgs{});
}

template <int PREC, int LF = PREC>
static void launch_tm(const Geom &g, const void *gauge, double kappa, int dagger, FieldRef in,
                      FieldRef out, const RedArgs *red, Gate gate, hipStream_t s) {
    const int wvol = tm_wvol(g, PREC);
    const int nsub = g.bvol / wvol;
    const int tch = tm_chunk(g, in.nrhs * nsub);
    const int ncols = g.V / (g.L[3] * g.bvol);
    const dim3 grid(tm_blocks(g, tch) * nsub * in.nrhs), bs(wvol);
    const size_t lds = 2 * slice_bytes<PREC>(wvol);
    RedArgs r{};
    if (red) r = *red;
    if (dagger) {
        if (red)
            launch_tm_k<PREC, true, true, LF>(grid, bs, lds, s, g, gauge, in, out, kappa, r, gate, tch, ncols);
        else
            launch_tm_k<PREC, true, false, LF>(grid, bs, lds, s, g, gauge, in, out, kappa, r, gate, tch, ncols);
    } else {
        if (red)
            launch_tm_k<PREC, false, true, LF>(grid, bs, lds, s, g, gauge, in, out, kappa, r, gate, tch, ncols);
        else
            launch_tm_k<PREC, false, false, LF>(grid, bs, lds, s, g, gauge, in, out, kappa, r, gate, tch, ncols);
    }
    // one partial per part of a brick slice: V / wvol of them per rhs
    if (red) launch_finalize(r, g.V / wvol, gate.batch ? gate.mode : -1, s);
}

template <int PREC, int LF = PREC>
static void launch_prec(const Geom &g, const void *gauge, double kappa, int dagger, FieldRef in,
                        FieldRef out, const RedArgs *red, Gate gate, hipStream_t s,
                        const void *g12) {
    // the marching stencil writes one partial per workgroup: use it only
    // when the caller's partial buffer holds them (it always does when sized
    // by reduce_partials_cap)
    if (tm_eligible(g) && tm_fits<PREC>(g) && !g_force_site_kernel &&
        (!red || (int64_t)(g.V / tm_wvol(g, PREC)) * in.nrhs <= red->partials_cap)) {
        if (PREC == WD_F64 && g12)
            launch_tm<WD_F64, kLinkF64R12>(g, g12, kappa, dagger, in, out, red, gate, s);
        else
            launch_tm<PREC, LF>(g, gauge, kappa, dagger, in, out, red, gate, s);
        return;
    }
    const int nb = site_blocks(g.V);
    const dim3 grid(nb * in.nrhs), bs(kSiteBlock);
    RedArgs r{};
    if (red) r = *red;
    constexpr int G = HopGroup<PREC>::value;
    if (dagger) {
        if (red)
            hipLaunchKernelGGL((k_dslash<PREC, true, true, G, LF>), grid, bs, 0, s, g, gauge, in, out, kappa, r, gate);
        else
            hipLaunchKernelGGL((k_dslash<PREC, true, false, G, LF>), grid, bs, 0, s, g, gauge, in, out, kappa, r, gate);
    } else {
        if (red)
            hipLaunchKernelGGL((k_dslash<PREC, false, true, G, LF>), grid, bs, 0, s, g, gauge, in, out, kappa, r, gate);
        else
            hipLaunchKernelGGL((k_dslash<PREC, false, false, G, LF>), grid, bs, 0, s, g, gauge, in, out, kappa, r, gate);
    }
    if (red) launch_finalize(r, nb, gate.batch ? gate.mode : -1, s);
}

void launch_dslash(const Geom &g, const void *gauge, double kappa, int dagger, FieldRef in,
                   FieldRef out, const RedArgs *red, Gate gate, hipStream_t s, const void *g12) {
    switch (in.prec) {
        case WD_F64: launch_prec<WD_F64>(g, gauge, kappa, dagger, in, out, red, gate, s, g12); break;
        case WD_F32: launch_prec<WD_F32>(g, gauge, kappa, dagger, in, out, red, gate, s, nullptr); break;
        default:
            if (g.f16_links8)
                launch_prec<WD_F16, kLinkF16R8>(g, gauge, kappa, dagger, in, out, red, gate, s,
                                                nullptr);
            else
                launch_prec<WD_F16>(g, gauge, kappa, dagger, in, out, red, gate, s, nullptr);
            break;
    }
}

template <int PREC>
static bool xr_ok(const Geom &g, int nrhs, int partials_cap) {
    return tm_eligible(g) && tm_fits<PREC>(g) && !g_force_site_kernel &&
           (int64_t)(g.V / tm_wvol(g, PREC)) * nrhs <= partials_cap;
}

bool dslash_xr_supported(const Geom &g, int prec, int nrhs, int partials_cap) {
    switch (prec) {
        case WD_F64: return xr_ok<WD_F64>(g, nrhs, partials_cap);
        case WD_F32: return xr_ok<WD_F32>(g, nrhs, partials_cap);
        default: return xr_ok<WD_F16>(g, nrhs, partials_cap);
    }
}

template <int PREC, int LF = PREC>
static bool xr_prec(const Geom &g, const void *gauge, double kappa, int dagger, FieldRef in,
                    const XrArgs &xr, const RedArgs &red, Gate gate, hipStream_t s) {
    if (!xr_ok<PREC>(g, in.nrhs, red.partials_cap)) return false;
    const int wvol = tm_wvol(g, PREC);
    const int nsub = g.bvol / wvol;
    const int tch = tm_chunk(g, in.nrhs * nsub);
    const int ncols = g.V / (g.L[3] * g.bvol);
    const dim3 grid(tm_blocks(g, tch) * nsub * in.nrhs), bs(wvol);
    const size_t lds = 2 * slice_bytes<PREC>(wvol);
    constexpr int G = HopGroup<PREC>::value;
    const Halo nh{nullptr, nullptr, nullptr, 0, 0, 0, 0, 1};
    if (dagger) {
        auto k = k_dslash_tm<PREC, true, true, G, false, true, LF>;
        allow_lds(k, lds);
        hipLaunchKernelGGL(k, grid, bs, lds, s, g, gauge, in, FieldRef{}, kappa, red, gate, tch,
                           ncols, nh, xr);
    } else {
        auto k = k_dslash_tm<PREC, false, true, G, false, true, LF>;
        allow_lds(k, lds);
        hipLaunchKernelGGL(k, grid, bs, lds, s, g, gauge, in, FieldRef{}, kappa, red, gate, tch,
                           ncols, nh, xr);
    }
    launch_finalize(red, g.V / wvol, gate.batch ? gate.mode : -1, s);
    return true;
}

bool launch_dslash_xr(const Geom &g, const void *gauge, double kappa, int dagger, FieldRef in,
                      const XrArgs &xr, const RedArgs &red, Gate gate, hipStream_t s,
                      const void *g12) {
    switch (in.prec) {
        case WD_F64:
            if (g12)
                return xr_prec<WD_F64, kLinkF64R12>(g, g12, kappa, dagger, in, xr, red, gate, s);
            return xr_prec<WD_F64>(g, gauge, kappa, dagger, in, xr, red, gate, s);
        case WD_F32: return xr_prec<WD_F32>(g, gauge, kappa, dagger, in, xr, red, gate, s);
        default:
            if (g.f16_links8)
                return xr_prec<WD_F16, kLinkF16R8>(g, gauge, kappa, dagger, in, xr, red, gate, s);
            return xr_prec<WD_F16>(g, gauge, kappa, dagger, in, xr, red, gate, s);
    }
}

// Even-odd hopping term on half fields (one lane per site of one rhs):
//   out_p = cs * c_p - k * H_{p,1-p} in_{1-p}
// with H the hop sum of Eq. (1) (projectors exchanged for DAG).  Entry h of a
// half field is site site_of_half(h, p); the neighbours, of the other
// parity, sit at their internal index >> 1.  Forward links come from the
// parity-p half array gp, backward links U_mu(x - mu) from gq.  The hops are
// summed in the order of the full stencil.
// XR: the CG update r -= alpha out_p in place of storing out (the reduction
// is then |r|^2; with HASC and RED).  LF: the link form.
template <int PREC, bool DAG, bool RED, bool HASC, int GROUP, bool XR = false, int LF = PREC>
__global__ void __launch_bounds__(256) k_hop_half(Geom g, const void *__restrict__ gp,
                                                  const void *__restrict__ gq, int p, FieldRef in,
                                                  FieldRef c, FieldRef out, double k_d,
                                                  double cs_d, RedArgs red, Gate gate,
                                                  XrArgs xr) {
    using R = typename Spinor<PREC>::R;
    if (gate_off(gate)) return;  // grid-uniform
    const int nrhs = in.nrhs;
    const int lb = logical_block();
    const int sb = lb / nrhs;
    const int rhs = lb - sb * nrhs;
    if (!gate_rhs(gate, rhs)) return;  // workgroup-uniform
    const FieldRef fin = rhs_view(in, rhs);
    const int h = sb * blockDim.x + threadIdx.x;
    double nrm = 0.0;
    if (h < out.V) {
        const int i = site_of_half(g, h, p);
        const Nbrs nb = neighbours(g, i);
        const bool neg_tp = g.antiperiodic && nb.cross_tp;
        const bool neg_tm = g.antiperiodic && nb.cross_tm;
        cx<R> acc[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = {R(0), R(0)};
        constexpr int SF = DAG ? +1 : -1;
        constexpr int SB = -SF;
#define WD_HOP_FENCE(k) \
    if ((k) % GROUP == 0) __builtin_amdgcn_sched_barrier(0)
        hop<0, SF, false, PREC, LF>(gp, fin, nb.xp >> 1, h, false, acc);
        WD_HOP_FENCE(1);
        hop<0, SB, true, PREC, LF>(gq, fin, nb.xm >> 1, nb.xm >> 1, false, acc);
        WD_HOP_FENCE(2);
        hop<1, SF, false, PREC, LF>(gp, fin, nb.yp >> 1, h, false, acc);
        WD_HOP_FENCE(3);
        hop<1, SB, true, PREC, LF>(gq, fin, nb.ym >> 1, nb.ym >> 1, false, acc);
        WD_HOP_FENCE(4);
        hop<2, SF, false, PREC, LF>(gp, fin, nb.zp >> 1, h, false, acc);
        WD_HOP_FENCE(5);
        hop<2, SB, true, PREC, LF>(gq, fin, nb.zm >> 1, nb.zm >> 1, false, acc);
        WD_HOP_FENCE(6);
        hop<3, SF, false, PREC, LF>(gp, fin, nb.tp >> 1, h, neg_tp, acc);
        WD_HOP_FENCE(7);
        hop<3, SB, true, PREC, LF>(gq, fin, nb.tm >> 1, nb.tm >> 1, neg_tm, acc);
        WD_HOP_FENCE(8);
#undef WD_HOP_FENCE
        cx<R> o[12];
        if constexpr (HASC) {
            Spinor<PREC>::load(rhs_view(c, rhs), h, o);
            const R cs = (R)cs_d;
#pragma unroll
            for (int k = 0; k < 12; ++k) o[k] = scale(cs, o[k]);
        } else {
#pragma unroll
            for (int k = 0; k < 12; ++k) o[k] = {R(0), R(0)};
        }
        const R kk = (R)k_d;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            o[k] = o[k] - scale(kk, acc[k]);
            if (RED && !XR)
                nrm += (double)o[k].re * (double)o[k].re + (double)o[k].im * (double)o[k].im;
        }
        if constexpr (XR)
            nrm = xr_site<PREC>(xr, rhs, h, (R)gate.st[rhs].alpha, o);
        else
            Spinor<PREC>::store(rhs_view(out, rhs), h, o);
    }
    if (RED) reduce_block(nrm, red.partials, (size_t)sb * nrhs + rhs);
}

// The half-field stencil in the time-marching form (lattices whose brick
// slices hold a multiple of 64 sites of each parity).  The parity-p half of
// a brick slice is bvol / 2 consecutive entries of a half field, and so is
// the parity-(1-p) half, pair by pair: output entry hs + l and input entry
// hs + l sit on the same site pair.  One workgroup per (chunk, column, part,
// rhs) marches t as the full stencil does, with two LDS images of its part
// of the input half slice:
//  - x/y/z neighbours (input entries nbr >> 1) from the current image when
//    they fall in the part, else from memory;
//  - the forward t neighbour of output lane l is input entry l of the next
//    half slice (same x, y, z; the other parity), from the new image;
//  - the backward t hop of slice t+1 is input entry l of slice t with its own
//    U_t (parity 1 - p links), carried in registers.
// Hops are summed in the order of k_hop_half.  Forward links come from gp at
// the output entry, backward ones from gq at the neighbour's entry.
template <int PREC, bool DAG, bool RED, bool HASC, int GROUP, bool XR, int LF>
__global__ void __launch_bounds__(kTmMaxBlock) k_hop_half_tm(Geom g, const void *__restrict__ gp,
                                                     const void *__restrict__ gq, int p,
                                                     FieldRef in, FieldRef c, FieldRef out,
                                                     double k_d, double cs_d, RedArgs red,
                                                     Gate gate, int tchunk, int ncols,
                                                     XrArgs xr) {
    using R = typename Spinor<PREC>::R;
    extern __shared__ __align__(16) char lds[];
    __shared__ double wsum[kTmMaxBlock / 64];
    if (gate_off(gate)) return;  // grid-uniform
    const int nrhs = in.nrhs;
    const int wvol = (int)blockDim.x;  // entries of this workgroup's part
    const int hvol = g.bvol >> 1;      // entries of one parity per brick slice
    const int nsub = hvol / wvol;
    const int lb = logical_block();
    const int cb = lb / nrhs;
    const int rhs = lb - cb * nrhs;
    if (!gate_rhs(gate, rhs)) return;  // workgroup-uniform
    const FieldRef fin = rhs_view(in, rhs);
    const int cc = cb / nsub;
    const int hp = cb - cc * nsub;
    const int chunk = cc / ncols;
    const int col = cc - chunk * ncols;
    const int Lt = g.L[3];
    const int l = (int)threadIdx.x;
    const int t0 = chunk * tchunk;
    const int t1 = t0 + tchunk < Lt ? t0 + tchunk : Lt;
    // first entry of this workgroup's part of half slice t: hbase + t * hvol
    const int hbase = col * Lt * hvol + hp * wvol;
    char *img0 = lds;
    char *img1 = lds + slice_bytes<PREC>(wvol);
    constexpr int SF = DAG ? +1 : -1;
    constexpr int SB = -SF;
    const R kappa = (R)k_d;

    // prologue: input half slice t0 into image 0, and the backward t hop of
    // slice t0 from input entry l of slice t0 - 1
    slice_copy<PREC>(fin, (hbase + t0 * hvol) >> 6, img0);
    cx<R> cw0[3], cw1[3];
    {
        const int ip = hbase + (t0 == 0 ? Lt - 1 : t0 - 1) * hvol + l;
        cx<R> v[12];
        Spinor<PREC>::load(fin, ip, v);
        cx<R> h0[3], h1[3];
        project<3, SB>(v, h0, h1);
        const R sg = (g.antiperiodic && t0 == 0) ? R(-1) : R(1);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            h0[k] = scale(sg, h0[k]);
            h1[k] = scale(sg, h1[k]);
        }
        cx<R> u[9];
        Link<LF>::load(gq, 3, ip, u);
        su3_mul<true>(u, h0, cw0);
        su3_mul<true>(u, h1, cw1);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int t = t0; t < t1; ++t) {
        const bool odd = (t - t0) & 1;
        const FieldRef cur = lds_view(fin, odd ? img1 : img0);
        const FieldRef nxt = lds_view(fin, odd ? img0 : img1);
        const int tn = t + 1 < Lt ? t + 1 : 0;
        slice_copy<PREC>(fin, (hbase + tn * hvol) >> 6, (char *)nxt.data);
        const int hs = hbase + t * hvol;
        const int H = hs + l;  // output entry
        // (not with 18-real float64 links: registers would spill)
        constexpr bool XPRE = XR && ((WD_XR_PREFETCH >> PREC) & 1) && LF != WD_F64;
        cx<R> rpre[XPRE ? 12 : 1];
        if constexpr (XPRE)
            Spinor<xr_prec_of(PREC)>::template load<WD_NT_RLOAD>(
                rhs_view(xr.r, rhs), H, rpre);
        const Nbrs nb = neighbours(g, site_of_half(g, H, p));
        cx<R> acc[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = {R(0), R(0)};
#define WD_HOP_FENCE(k) \
    if ((k) % GROUP == 0) __builtin_amdgcn_sched_barrier(0)
        hop_s<0, SF, false, PREC, LF>(gp, fin, cur, hs, wvol, nb.xp >> 1, H, acc);
        WD_HOP_FENCE(1);
        hop_s<0, SB, true, PREC, LF>(gq, fin, cur, hs, wvol, nb.xm >> 1, nb.xm >> 1, acc);
        WD_HOP_FENCE(2);
        hop_s<1, SF, false, PREC, LF>(gp, fin, cur, hs, wvol, nb.yp >> 1, H, acc);
        WD_HOP_FENCE(3);
        hop_s<1, SB, true, PREC, LF>(gq, fin, cur, hs, wvol, nb.ym >> 1, nb.ym >> 1, acc);
        WD_HOP_FENCE(4);
        hop_s<2, SF, false, PREC, LF>(gp, fin, cur, hs, wvol, nb.zp >> 1, H, acc);
        WD_HOP_FENCE(5);
        hop_s<2, SB, true, PREC, LF>(gq, fin, cur, hs, wvol, nb.zm >> 1, nb.zm >> 1, acc);
        WD_HOP_FENCE(6);
#undef WD_HOP_FENCE
        cx<R> ut[9], ub[9];
        Link<LF>::template load<WD_NT_LINK || WD_NT_LINK_T>(gp, 3, H, ut);
        Link<LF>::template load<WD_NT_LINK || WD_NT_LINK_T>(gq, 3, H, ub);
        // the next half slice has landed in LDS (every wave's copy)
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        {
            cx<R> nx[12];
            Spinor<PREC>::load(nxt, l, nx);
            hop_p<3, SF, false>(nx, ut, g.antiperiodic && t == Lt - 1, acc);
        }
        accumulate<3, SB>(cw0, cw1, acc);
        // carry for slice t + 1: input entry l of this slice with its U_t
        {
            cx<R> v[12];
            Spinor<PREC>::load(cur, l, v);
            cx<R> h0[3], h1[3];
            project<3, SB>(v, h0, h1);
            su3_mul<true>(ub, h0, cw0);
            su3_mul<true>(ub, h1, cw1);
        }
        cx<R> o[12];
        if constexpr (HASC) {
            Spinor<PREC>::load(rhs_view(c, rhs), H, o);
            const R cs = (R)cs_d;
#pragma unroll
            for (int k = 0; k < 12; ++k) o[k] = scale(cs, o[k]);
        } else {
#pragma unroll
            for (int k = 0; k < 12; ++k) o[k] = {R(0), R(0)};
        }
        double nrm = 0.0;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            o[k] = o[k] - scale(kappa, acc[k]);
            if (RED && !XR)
                nrm += (double)o[k].re * (double)o[k].re + (double)o[k].im * (double)o[k].im;
        }
        if constexpr (XPRE)
            nrm = xr_site_r<PREC>(xr, rhs, H, (R)gate.st[rhs].alpha, o, rpre);
        else if constexpr (XR)
            nrm = xr_site<PREC>(xr, rhs, H, (R)gate.st[rhs].alpha, o);
        else
            Spinor<PREC>::template store<WD_NT_OUT>(rhs_view(out, rhs), H, o);
        if (RED) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) nrm += __shfl_xor(nrm, off, 64);
            if ((l & 63) == 0) wsum[l >> 6] = nrm;
        }
        __syncthreads();  // the current image is free for the next copy
        if (RED && l == 0) {
            double sum = 0.0;
            for (int w = 0; w < (wvol >> 6); ++w) sum += wsum[w];
            red.partials[(((size_t)col * Lt + t) * nsub + hp) * nrhs + rhs] = sum;
        }
    }
}

// WD_EO_SITE=1 keeps the half-field stencil one lane per site (tuning and
// tests; read at every launch)
static bool eo_site_forced() {
    const char *e = getenv("WD_EO_SITE");
    return e && atoi(e) != 0;
}

// The marching form pays where link and spinor bytes bound the launch: at
// 48^3 x 96 float64 half launches take 1.29-1.49 ms against 1.65-1.77 one
// lane per site, float32 -2%, while binary16 (bound by its arithmetic) is
// 3-8% slower marching and stays one lane per site.
template <int PREC>
static bool eo_tm_ok(const Geom &g, int nrhs, bool red, int64_t partials_cap) {
    static const size_t cap = max_lds_per_block();
    const int w = eo_wvol(g, PREC);
    return PREC != WD_F16 && w > 0 && !eo_site_forced() && !g_force_site_kernel &&
           2 * slice_bytes<PREC>(w) + 64 <= cap &&
           (!red || (int64_t)(g.V / 2 / w) * nrhs <= partials_cap);
}

// one half-field launch, marching where the geometry allows, with its
// finaliser
template <int PREC, bool DAG, bool RED, bool HASC, bool XR, int LF>
static void launch_eo(const Geom &g, const void *gp, const void *gq, int p, FieldRef in,
                      FieldRef c, FieldRef out, double k, double cs, const RedArgs &r,
                      Gate gate, const XrArgs &xr, hipStream_t s) {
    constexpr int G = HopGroup<PREC>::value;
    int nb;
    if (eo_tm_ok<PREC>(g, in.nrhs, RED, r.partials_cap)) {
        const int w = eo_wvol(g, PREC);
        const int nsub = g.bvol / 2 / w;
        const int tch = tm_chunk(g, in.nrhs * nsub);
        const int ncols = g.V / (g.L[3] * g.bvol);
        const dim3 grid(tm_blocks(g, tch) * nsub * in.nrhs), bs(w);
        const size_t lds = 2 * slice_bytes<PREC>(w);
        auto kern = k_hop_half_tm<PREC, DAG, RED, HASC, G, XR, LF>;
        allow_lds(kern, lds);
        hipLaunchKernelGGL(kern, grid, bs, lds, s, g, gp, gq, p, in, c, out, k, cs, r, gate, tch,
                           ncols, xr);
        nb = g.V / 2 / w;
    } else {
        nb = site_blocks(out.V);
        hipLaunchKernelGGL((k_hop_half<PREC, DAG, RED, HASC, G, XR, LF>), dim3(nb * in.nrhs),
                           dim3(kSiteBlock), 0, s, g, gp, gq, p, in, c, out, k, cs, r, gate, xr);
    }
    if (RED) launch_finalize(r, nb, gate.batch ? gate.mode : -1, s);
}

template <int PREC, int LF = PREC>
static void launch_hop_half_prec(const Geom &g, const void *gp, const void *gq, int p, double k,
                                 double cs, int dagger, FieldRef in, FieldRef c, FieldRef out,
                                 const RedArgs *red, Gate gate, hipStream_t s) {
    RedArgs r{};
    if (red) r = *red;
    const XrArgs nx{};
    const bool hc = c.data != nullptr;
    const int sel = (dagger ? 4 : 0) | (red ? 2 : 0) | (hc ? 1 : 0);
    switch (sel) {
        case 0: launch_eo<PREC, false, false, false, false, LF>(g, gp, gq, p, in, c, out, k, cs, r, gate, nx, s); break;
        case 1: launch_eo<PREC, false, false, true, false, LF>(g, gp, gq, p, in, c, out, k, cs, r, gate, nx, s); break;
        case 2: launch_eo<PREC, false, true, false, false, LF>(g, gp, gq, p, in, c, out, k, cs, r, gate, nx, s); break;
        case 3: launch_eo<PREC, false, true, true, false, LF>(g, gp, gq, p, in, c, out, k, cs, r, gate, nx, s); break;
        case 4: launch_eo<PREC, true, false, false, false, LF>(g, gp, gq, p, in, c, out, k, cs, r, gate, nx, s); break;
        case 5: launch_eo<PREC, true, false, true, false, LF>(g, gp, gq, p, in, c, out, k, cs, r, gate, nx, s); break;
        case 6: launch_eo<PREC, true, true, false, false, LF>(g, gp, gq, p, in, c, out, k, cs, r, gate, nx, s); break;
        default: launch_eo<PREC, true, true, true, false, LF>(g, gp, gq, p, in, c, out, k, cs, r, gate, nx, s); break;
    }
}

template <int PREC, int LF = PREC>
static void launch_hop_half_xr_prec(const Geom &g, const void *gp, const void *gq, int p,
                                    double k, double cs, int dagger, FieldRef in, FieldRef c,
                                    const XrArgs &xr, const RedArgs &red, Gate gate,
                                    hipStream_t s) {
    // out only sizes the launch (xr.r is a half field like it)
    if (dagger)
        launch_eo<PREC, true, true, true, true, LF>(g, gp, gq, p, in, c, xr.r, k, cs, red, gate, xr, s);
    else
        launch_eo<PREC, false, true, true, true, LF>(g, gp, gq, p, in, c, xr.r, k, cs, red, gate, xr, s);
}

void launch_hop_half_xr(const Geom &g, const void *gp, const void *gq, int p, double k, double cs,
                        int dagger, FieldRef in, FieldRef c, const XrArgs &xr,
                        const RedArgs &red, Gate gate, hipStream_t s, bool r12) {
    switch (in.prec) {
        case WD_F64:
            if (r12)
                launch_hop_half_xr_prec<WD_F64, kLinkF64R12>(g, gp, gq, p, k, cs, dagger, in, c,
                                                              xr, red, gate, s);
            else
                launch_hop_half_xr_prec<WD_F64>(g, gp, gq, p, k, cs, dagger, in, c, xr, red, gate,
                                                s);
            break;
        case WD_F32:
            launch_hop_half_xr_prec<WD_F32>(g, gp, gq, p, k, cs, dagger, in, c, xr, red, gate, s);
            break;
        default:
            if (g.f16_links8)
                launch_hop_half_xr_prec<WD_F16, kLinkF16R8>(g, gp, gq, p, k, cs, dagger, in, c,
                                                             xr, red, gate, s);
            else
                launch_hop_half_xr_prec<WD_F16>(g, gp, gq, p, k, cs, dagger, in, c, xr, red, gate,
                                                s);
            break;
    }
}

void launch_hop_half(const Geom &g, const void *gp, const void *gq, int p, double k, double cs,
                     int dagger, FieldRef in, FieldRef c, FieldRef out, const RedArgs *red,
                     Gate gate, hipStream_t s, bool r12) {
    switch (in.prec) {
        case WD_F64:
            if (r12)
                launch_hop_half_prec<WD_F64, kLinkF64R12>(g, gp, gq, p, k, cs, dagger, in, c, out,
                                                          red, gate, s);
            else
                launch_hop_half_prec<WD_F64>(g, gp, gq, p, k, cs, dagger, in, c, out, red, gate, s);
            break;
        case WD_F32: launch_hop_half_prec<WD_F32>(g, gp, gq, p, k, cs, dagger, in, c, out, red, gate, s); break;
        default:
            if (g.f16_links8)
                launch_hop_half_prec<WD_F16, kLinkF16R8>(g, gp, gq, p, k, cs, dagger, in, c, out,
                                                         red, gate, s);
            else
                launch_hop_half_prec<WD_F16>(g, gp, gq, p, k, cs, dagger, in, c, out, red, gate,
                                             s);
            break;
    }
}

// ------------------------------------------------------------------ halo exchange

// Faces of a t-slab for its neighbours (float64, wire format): one lane per
// face site and rhs.  to_prev: (1 + SF gamma_t) psi(x, 0), the projection
// the previous slab's forward t hop applies; to_next: (1 + SB gamma_t)
// psi(x, Lt-1) for the next slab's backward t hop (which multiplies it by
// U_t(x, Lt-1)^dag, a link the next slab holds as its entering links).
template <bool DAG>
__global__ void __launch_bounds__(256) k_halo_pack(Geom g, FieldRef in, double2 *__restrict__ to_prev,
                                                   double2 *__restrict__ to_next) {
    constexpr int SF = DAG ? +1 : -1;
    constexpr int SB = -SF;
    const int Lt = g.L[3];
    const int vf = g.V / Lt;
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= vf) return;
    const int rhs = blockIdx.y;
    const FieldRef fin = rhs_view(in, rhs);
    const int col = f / g.bvol, loc = f - col * g.bvol;
    const int i0 = col * Lt * g.bvol + loc;  // slice 0
    const int il = i0 + (Lt - 1) * g.bvol;   // slice Lt - 1
    const size_t fofs = (size_t)rhs * 6 * vf;
    cx<double> p[12], h0[3], h1[3];
    Spinor<WD_F64>::load(fin, i0, p);
    project<3, SF>(p, h0, h1);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        to_prev[fofs + (size_t)c * vf + f] = make_double2(h0[c].re, h0[c].im);
        to_prev[fofs + (size_t)(3 + c) * vf + f] = make_double2(h1[c].re, h1[c].im);
    }
    Spinor<WD_F64>::load(fin, il, p);
    project<3, SB>(p, h0, h1);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        to_next[fofs + (size_t)c * vf + f] = make_double2(h0[c].re, h0[c].im);
        to_next[fofs + (size_t)(3 + c) * vf + f] = make_double2(h1[c].re, h1[c].im);
    }
}

void launch_halo_pack(const Geom &g, int dagger, FieldRef in, double *to_prev, double *to_next,
                      hipStream_t s) {
    const dim3 grid(blocks_for(g.V / g.L[3], 256), in.nrhs), bs(256);
    if (dagger)
        hipLaunchKernelGGL(k_halo_pack<true>, grid, bs, 0, s, g, in, (double2 *)to_prev,
                           (double2 *)to_next);
    else
        hipLaunchKernelGGL(k_halo_pack<false>, grid, bs, 0, s, g, in, (double2 *)to_prev,
                           (double2 *)to_next);
}

// wire-format face -> spinor tiles: spins 0, 1 = the half-spinor, spins 2, 3
// zero (the t projectors then return the half-spinor exactly)
__global__ void __launch_bounds__(256) k_halo_stage(const double2 *__restrict__ wire, FieldRef st,
                                                    int vf) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= vf) return;
    const int rhs = blockIdx.y;
    const size_t fofs = (size_t)rhs * 6 * vf;
    cx<double> v[12];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const double2 d = wire[fofs + (size_t)k * vf + f];
        v[k] = {d.x, d.y};
        v[6 + k] = {0.0, 0.0};
    }
    Spinor<WD_F64>::store(rhs_view(st, rhs), f, v);
}

void launch_halo_stage(const Geom &g, const double *wire, FieldRef staged, hipStream_t s) {
    const int vf = g.V / g.L[3];
    hipLaunchKernelGGL(k_halo_stage, dim3(blocks_for(vf, 256), staged.nrhs), dim3(256), 0, s,
                       (const double2 *)wire, staged, vf);
}

// canonical U_t(x, -1) over the (x, y, z) of a face -> gauge tiles over face
// sites (mu = 3 planes; the others are not read)
__global__ void __launch_bounds__(256) k_halo_links(Geom g, const double2 *__restrict__ canon,
                                                    void *__restrict__ links) {
    const int vf = g.V / g.L[3];
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= vf) return;
    const int col = f / g.bvol, loc = f - col * g.bvol;
    int x, y, z, t;
    coords_of(g, col * g.L[3] * g.bvol + loc, x, y, z, t);
    const double2 *src = canon + (size_t)(x + g.L[0] * (y + g.L[1] * z)) * 9;
    cx<double> u[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) u[k] = {src[k].x, src[k].y};
    Link<WD_F64>::store(links, 3, f, u);
}

void launch_halo_links(const Geom &g, const double *canon, void *links, hipStream_t s) {
    const int vf = g.V / g.L[3];
    hipLaunchKernelGGL(k_halo_links, dim3(blocks_for(vf, 256)), dim3(256), 0, s, g,
                       (const double2 *)canon, links);
}

bool halo_supported(const Geom &g) { return tm_eligible(g) && tm_fits<WD_F64>(g); }

template <int LF>
static void launch_halo_lf(const Geom &g, const void *gauge, double kappa, int dagger,
                           FieldRef in, FieldRef out, const Halo &region, hipStream_t s) {
    const int wvol = tm_wvol(g, WD_F64);
    const int nsub = g.bvol / wvol;
    const int tch = tm_chunk(g, in.nrhs * nsub);
    const int ncols = g.V / (g.L[3] * g.bvol);
    // chunks of this launch: all; the interior ones (neither slice 0 nor
    // Lt - 1: no staged face is read); or the one or two holding the ends
    const int nch = (g.L[3] + tch - 1) / tch;
    Halo halo = region;
    int count = nch;
    halo.cfirst = 0;
    halo.cstep = 1;
    if (region.region == 1) {
        count = nch - 2;
        halo.cfirst = 1;
    } else if (region.region == 2) {
        count = nch < 2 ? nch : 2;
        halo.cstep = nch - 1 > 0 ? nch - 1 : 1;
    }
    if (count <= 0) return;
    const dim3 grid(ncols * count * nsub * in.nrhs), bs(wvol);
    const size_t lds = 2 * slice_bytes<WD_F64>(wvol);
    constexpr int G = HopGroup<WD_F64>::value;
    const Gate none{nullptr, nullptr, GATE_ACTIVE};
    if (dagger) {
        auto k = k_dslash_tm<WD_F64, true, false, G, true, false, LF>;
        allow_lds(k, lds);
        hipLaunchKernelGGL(k, grid, bs, lds, s, g, gauge, in, out, kappa, RedArgs{}, none, tch,
                           ncols, halo, XrArgs{});
    } else {
        auto k = k_dslash_tm<WD_F64, false, false, G, true, false, LF>;
        allow_lds(k, lds);
        hipLaunchKernelGGL(k, grid, bs, lds, s, g, gauge, in, out, kappa, RedArgs{}, none, tch,
                           ncols, halo, XrArgs{});
    }
}

void launch_dslash_halo(const Geom &g, const void *gauge, double kappa, int dagger, FieldRef in,
                        FieldRef out, const Halo &halo, hipStream_t s, const void *g12) {
    if (g12)
        launch_halo_lf<kLinkF64R12>(g, g12, kappa, dagger, in, out, halo, s);
    else
        launch_halo_lf<WD_F64>(g, gauge, kappa, dagger, in, out, halo, s);
}

}  // namespace wd
