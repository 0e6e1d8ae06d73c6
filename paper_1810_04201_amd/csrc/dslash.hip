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
__device__ __forceinline__ void hop(const void *gauge, int V, const FieldRef &in, int nbr_entry,
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
    Link<PREC>::load(gauge, V, MU, link_site, u);
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
        const int Lx = g.L[0], Ly = g.L[1], Lz = g.L[2], Lt = g.L[3];
        const int x = site % Lx;
        int q = site / Lx;
        const int y = q % Ly;
        q /= Ly;
        const int z = q % Lz;
        const int t = q / Lz;
        const int sx = 1, sy = Lx, sz = Lx * Ly, st = Lx * Ly * Lz;
        const int xp = x == Lx - 1 ? site - (Lx - 1) * sx : site + sx;
        const int xm = x == 0 ? site + (Lx - 1) * sx : site - sx;
        const int yp = y == Ly - 1 ? site - (Ly - 1) * sy : site + sy;
        const int ym = y == 0 ? site + (Ly - 1) * sy : site - sy;
        const int zp = z == Lz - 1 ? site - (Lz - 1) * sz : site + sz;
        const int zm = z == 0 ? site + (Lz - 1) * sz : site - sz;
        const int tp = t == Lt - 1 ? site - (Lt - 1) * st : site + st;
        const int tm = t == 0 ? site + (Lt - 1) * st : site - st;
        const bool neg_tp = g.antiperiodic && t == Lt - 1;
        const bool neg_tm = g.antiperiodic && t == 0;
        const int V = g.V;

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
        hop<0, SF, false, PREC>(gauge, V, in, xp * nrhs + rhs, site, false, acc);
        WD_HOP_FENCE(1);
        hop<0, SB, true, PREC>(gauge, V, in, xm * nrhs + rhs, xm, false, acc);
        WD_HOP_FENCE(2);
        hop<1, SF, false, PREC>(gauge, V, in, yp * nrhs + rhs, site, false, acc);
        WD_HOP_FENCE(3);
        hop<1, SB, true, PREC>(gauge, V, in, ym * nrhs + rhs, ym, false, acc);
        WD_HOP_FENCE(4);
        hop<2, SF, false, PREC>(gauge, V, in, zp * nrhs + rhs, site, false, acc);
        WD_HOP_FENCE(5);
        hop<2, SB, true, PREC>(gauge, V, in, zm * nrhs + rhs, zm, false, acc);
        WD_HOP_FENCE(6);
        hop<3, SF, false, PREC>(gauge, V, in, tp * nrhs + rhs, site, neg_tp, acc);
        WD_HOP_FENCE(7);
        hop<3, SB, true, PREC>(gauge, V, in, tm * nrhs + rhs, tm, neg_tm, acc);
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

// hops per scheduling group (see k_dslash)
template <int PREC>
struct HopGroup {
    static constexpr int value = PREC == WD_F64 ? WD_GROUP_F64 : WD_GROUP_LO;
};

template <int PREC>
static void launch_prec(const Geom &g, const void *gauge, double kappa, int dagger, FieldRef in,
                        FieldRef out, const RedArgs *red, Gate gate, hipStream_t s) {
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
