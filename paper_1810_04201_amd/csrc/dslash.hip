// Wilson-Dirac stencil (Eq. (1) of Sec. 2.1 with the minus sign) on gfx950.
//
// One lane per (site, rhs) entry.  Each of the eight hops projects the
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
#ifndef WD_GROUP_F64
#define WD_GROUP_F64 1
#endif
#ifndef WD_GROUP_LO
#define WD_GROUP_LO 2
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
template <int MU, int S, bool BWD, int PREC>
__device__ __forceinline__ void hop(const void *gauge, const FieldRef &in, int nbr_entry,
                                    int link_site, bool negate,
                                    cx<typename Spinor<PREC>::R> acc[12]) {
    using R = typename Spinor<PREC>::R;
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
    Link<PREC>::load(gauge, MU, link_site, u);
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

// one hop with the link already in registers
template <int MU, int S, bool BWD, int PREC>
__device__ __forceinline__ void hop_u(const cx<typename Spinor<PREC>::R> u[9], const FieldRef &in,
                                      int nbr_entry, bool negate,
                                      cx<typename Spinor<PREC>::R> acc[12]) {
    using R = typename Spinor<PREC>::R;
    cx<R> p[12];
    Spinor<PREC>::load(in, nbr_entry, p);
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

template <int PREC, bool DAG, bool RED, int GROUP>
__global__ void __launch_bounds__(256) k_dslash(Geom g, const void *__restrict__ gauge, FieldRef in,
                                                FieldRef out, double kappa_d, RedArgs red,
                                                Gate gate) {
    using R = typename Spinor<PREC>::R;
    if (gate.batch && gate.batch->n_active == 0) return;  // grid-uniform
    const int nrhs = in.nrhs;
    const int e = logical_block() * blockDim.x + threadIdx.x;
    bool live = e < in.n;
    const int site = e / nrhs;
    const int rhs = e - site * nrhs;
    if (live && gate.st && !gate.st[rhs].active) live = false;
    double nrm = 0.0;
    if (live) {
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
        hop<0, SF, false, PREC>(gauge, in, xp * nrhs + rhs, site, false, acc);
        WD_HOP_FENCE(1);
        hop<0, SB, true, PREC>(gauge, in, xm * nrhs + rhs, xm, false, acc);
        WD_HOP_FENCE(2);
        hop<1, SF, false, PREC>(gauge, in, yp * nrhs + rhs, site, false, acc);
        WD_HOP_FENCE(3);
        hop<1, SB, true, PREC>(gauge, in, ym * nrhs + rhs, ym, false, acc);
        WD_HOP_FENCE(4);
        hop<2, SF, false, PREC>(gauge, in, zp * nrhs + rhs, site, false, acc);
        WD_HOP_FENCE(5);
        hop<2, SB, true, PREC>(gauge, in, zm * nrhs + rhs, zm, false, acc);
        WD_HOP_FENCE(6);
        hop<3, SF, false, PREC>(gauge, in, tp * nrhs + rhs, site, neg_tp, acc);
        WD_HOP_FENCE(7);
        hop<3, SB, true, PREC>(gauge, in, tm * nrhs + rhs, tm, neg_tm, acc);
        WD_HOP_FENCE(8);
#undef WD_HOP_FENCE

        cx<R> c[12];
        Spinor<PREC>::load(in, e, c);
        const R kappa = (R)kappa_d;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            c[k] = c[k] - scale(kappa, acc[k]);
            if (RED) nrm += (double)c[k].re * (double)c[k].re + (double)c[k].im * (double)c[k].im;
        }
        Spinor<PREC>::store(out, e, c);
    }
    if (RED) reduce_block(nrm, red.partials, nrhs);
}


// Time-marching stencil (nrhs == 1).  One workgroup per brick column and
// chunk of time slices, one lane per brick site.  The workgroup steps
// through its time slices together, so the x/y/z neighbours a lane reads
// were fetched by its neighbour lanes moments earlier, and the backward t
// hop U_t(x, t-1)^dag (1 -+ gamma_t) psi(x, t-1) is carried from the previous
// slice in registers instead of being reloaded.  Blocks are ordered chunk
// major, so each XCD's contiguous block run covers one band of time slices
// of many neighbouring columns (their shared brick faces stay in its L2).
template <int PREC, bool DAG, bool RED, int GROUP>
__global__ void __launch_bounds__(256) k_dslash_tm(Geom g, const void *__restrict__ gauge,
                                                   FieldRef in, FieldRef out, double kappa_d,
                                                   RedArgs red, Gate gate, int tchunk,
                                                   int ncols) {
    using R = typename Spinor<PREC>::R;
    if (gate.batch && gate.batch->n_active == 0) return;  // grid-uniform
    const int b = logical_block();
    const int chunk = b / ncols;
    const int col = b - chunk * ncols;
    const int Lt = g.L[3];
    const int t0 = chunk * tchunk;
    const int t1 = t0 + tchunk < Lt ? t0 + tchunk : Lt;
    const bool live = !gate.st || gate.st[0].active;  // uniform (one rhs)
    constexpr int SF = DAG ? +1 : -1;
    constexpr int SB = -SF;
    const R kappa = (R)kappa_d;
    double nrm = 0.0;
    if (live) {
        const int base = col * Lt * g.bvol + (int)threadIdx.x;
        // carried backward t hop for the first slice: from t0 - 1
        cx<R> cw0[3], cw1[3];
        {
            const int tprev = t0 == 0 ? Lt - 1 : t0 - 1;
            const int ip = base + tprev * g.bvol;
            cx<R> p[12];
            Spinor<PREC>::load(in, ip, p);
            cx<R> h0[3], h1[3];
            project<3, SB>(p, h0, h1);
            const R sg = (g.antiperiodic && t0 == 0) ? R(-1) : R(1);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                h0[c] = scale(sg, h0[c]);
                h1[c] = scale(sg, h1[c]);
            }
            cx<R> u[9];
            Link<PREC>::load(gauge, 3, ip, u);
            su3_mul<true>(u, h0, cw0);
            su3_mul<true>(u, h1, cw1);
        }
        for (int t = t0; t < t1; ++t) {
            const int i = base + t * g.bvol;
            const Nbrs nb = neighbours(g, i);
            cx<R> acc[12];
#pragma unroll
            for (int k = 0; k < 12; ++k) acc[k] = {R(0), R(0)};
#define WD_HOP_FENCE(k) \
    if ((k) % GROUP == 0) __builtin_amdgcn_sched_barrier(0)
            hop<0, SF, false, PREC>(gauge, in, nb.xp, i, false, acc);
            WD_HOP_FENCE(1);
            hop<0, SB, true, PREC>(gauge, in, nb.xm, nb.xm, false, acc);
            WD_HOP_FENCE(2);
            hop<1, SF, false, PREC>(gauge, in, nb.yp, i, false, acc);
            WD_HOP_FENCE(3);
            hop<1, SB, true, PREC>(gauge, in, nb.ym, nb.ym, false, acc);
            WD_HOP_FENCE(4);
            hop<2, SF, false, PREC>(gauge, in, nb.zp, i, false, acc);
            WD_HOP_FENCE(5);
            hop<2, SB, true, PREC>(gauge, in, nb.zm, nb.zm, false, acc);
            WD_HOP_FENCE(6);
            cx<R> ut[9];
            Link<PREC>::load(gauge, 3, i, ut);
            hop_u<3, SF, false, PREC>(ut, in, nb.tp, g.antiperiodic && nb.cross_tp, acc);
            WD_HOP_FENCE(7);
#undef WD_HOP_FENCE
            accumulate<3, SB>(cw0, cw1, acc);
            cx<R> c[12];
            Spinor<PREC>::load(in, i, c);
            // carry for slice t + 1 (never crosses the boundary inside a chunk)
            {
                cx<R> h0[3], h1[3];
                project<3, SB>(c, h0, h1);
                su3_mul<true>(ut, h0, cw0);
                su3_mul<true>(ut, h1, cw1);
            }
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                c[k] = c[k] - scale(kappa, acc[k]);
                if (RED) nrm += (double)c[k].re * (double)c[k].re + (double)c[k].im * (double)c[k].im;
            }
            Spinor<PREC>::store(out, i, c);
            __syncthreads();  // keep the brick in step
        }
    }
    if (RED) reduce_block(nrm, red.partials, 1);
}

// WD_TCHUNK overrides the marching stencil's chunk length (tuning)
static int tm_chunk(const Geom &g) {
    static const int env = [] {
        const char *e = getenv("WD_TCHUNK");
        return e ? atoi(e) : 0;
    }();
    return tm_chunk_len(g, env);
}

// WD_SITE_KERNEL=1 forces the one-lane-per-entry stencil everywhere (tuning)
static const bool g_force_site_kernel = [] {
    const char *e = getenv("WD_SITE_KERNEL");
    return e && atoi(e) != 0;
}();

// hops per scheduling group (see k_dslash)
template <int PREC>
struct HopGroup {
    static constexpr int value = PREC == WD_F64 ? WD_GROUP_F64 : WD_GROUP_LO;
};

template <int PREC>
static void launch_tm(const Geom &g, const void *gauge, double kappa, int dagger, FieldRef in,
                      FieldRef out, const RedArgs *red, Gate gate, hipStream_t s) {
    const int tch = tm_chunk(g);
    const int ncols = g.V / (g.L[3] * g.bvol);
    const int nb = tm_blocks(g, tch);
    const int bs = g.bvol;
    constexpr int G = HopGroup<PREC>::value;
    RedArgs r{};
    if (red) r = *red;
    if (dagger) {
        if (red)
            hipLaunchKernelGGL((k_dslash_tm<PREC, true, true, G>), dim3(nb), dim3(bs), 0, s, g, gauge, in, out, kappa, r, gate, tch, ncols);
        else
            hipLaunchKernelGGL((k_dslash_tm<PREC, true, false, G>), dim3(nb), dim3(bs), 0, s, g, gauge, in, out, kappa, r, gate, tch, ncols);
    } else {
        if (red)
            hipLaunchKernelGGL((k_dslash_tm<PREC, false, true, G>), dim3(nb), dim3(bs), 0, s, g, gauge, in, out, kappa, r, gate, tch, ncols);
        else
            hipLaunchKernelGGL((k_dslash_tm<PREC, false, false, G>), dim3(nb), dim3(bs), 0, s, g, gauge, in, out, kappa, r, gate, tch, ncols);
    }
    if (red) launch_finalize(r, nb, gate.batch != nullptr, s);
}

template <int PREC>
static void launch_prec(const Geom &g, const void *gauge, double kappa, int dagger, FieldRef in,
                        FieldRef out, const RedArgs *red, Gate gate, hipStream_t s) {
    // the marching stencil needs one partial per workgroup: use it only when
    // the caller's partial buffer holds them (it always does when sized by
    // reduce_partials_cap)
    if (tm_eligible(g, in.nrhs) && !g_force_site_kernel &&
        (!red || tm_blocks(g, tm_chunk(g)) <= red->partials_cap)) {
        launch_tm<PREC>(g, gauge, kappa, dagger, in, out, red, gate, s);
        return;
    }
    const int bs = block_for_nrhs(in.nrhs);
    const int nb = blocks_for(in.n, bs);
    RedArgs r{};
    if (red) r = *red;
    if (dagger) {
        if (red)
            hipLaunchKernelGGL((k_dslash<PREC, true, true, HopGroup<PREC>::value>), dim3(nb), dim3(bs), 0, s, g, gauge, in,
                               out, kappa, r, gate);
        else
            hipLaunchKernelGGL((k_dslash<PREC, true, false, HopGroup<PREC>::value>), dim3(nb), dim3(bs), 0, s, g, gauge,
                               in, out, kappa, r, gate);
    } else {
        if (red)
            hipLaunchKernelGGL((k_dslash<PREC, false, true, HopGroup<PREC>::value>), dim3(nb), dim3(bs), 0, s, g, gauge,
                               in, out, kappa, r, gate);
        else
            hipLaunchKernelGGL((k_dslash<PREC, false, false, HopGroup<PREC>::value>), dim3(nb), dim3(bs), 0, s, g, gauge,
                               in, out, kappa, r, gate);
    }
    if (red) launch_finalize(r, nb, gate.batch != nullptr, s);
}

void launch_dslash(const Geom &g, const void *gauge, double kappa, int dagger, FieldRef in,
                   FieldRef out, const RedArgs *red, Gate gate, hipStream_t s) {
    switch (in.prec) {
        case WD_F64: launch_prec<WD_F64>(g, gauge, kappa, dagger, in, out, red, gate, s); break;
        case WD_F32: launch_prec<WD_F32>(g, gauge, kappa, dagger, in, out, red, gate, s); break;
        default: launch_prec<WD_F16>(g, gauge, kappa, dagger, in, out, red, gate, s); break;
    }
}

}  // namespace wd
