// Device-side building blocks: complex arithmetic, field and link accessors
// for the three storage formats, and the deterministic block reduction with
// its solver-state finaliser.
#pragma once

#include "wd_internal.hpp"

namespace wd {

template <typename R>
struct cx {
    R re, im;
};

template <typename R>
__device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> operator-(cx<R> a) { return {-a.re, -a.im}; }
template <typename R>
__device__ __forceinline__ cx<R> scale(R s, cx<R> a) { return {s * a.re, s * a.im}; }
// i * a
template <typename R>
__device__ __forceinline__ cx<R> times_i(cx<R> a) { return {-a.im, a.re}; }
// a * b
template <typename R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// acc + a * b
template <typename R>
__device__ __forceinline__ cx<R> cfma(cx<R> a, cx<R> b, cx<R> acc) {
    return {acc.re + a.re * b.re - a.im * b.im, acc.im + a.re * b.im + a.im * b.re};
}
// acc + conj(a) * b
template <typename R>
__device__ __forceinline__ cx<R> cfmac(cx<R> a, cx<R> b, cx<R> acc) {
    return {acc.re + a.re * b.re + a.im * b.im, acc.im + a.re * b.im - a.im * b.re};
}
template <typename R>
__device__ __forceinline__ cx<R> conj(cx<R> a) { return {a.re, -a.im}; }
template <typename R>
__device__ __forceinline__ R norm2(cx<R> a) { return a.re * a.re + a.im * a.im; }

typedef _Float16 h2_t __attribute__((ext_vector_type(2)));
typedef _Float16 h4_t __attribute__((ext_vector_type(4)));
typedef _Float16 h8_t __attribute__((ext_vector_type(8)));
typedef double d2_t __attribute__((ext_vector_type(2)));
typedef float f4_t __attribute__((ext_vector_type(4)));

// vector load / store; NT: non-temporal (streamed data that should not
// displace reused data in the caches)
template <bool NT, typename T>
__device__ __forceinline__ T ldv(const T *p) {
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}
template <bool NT, typename T>
__device__ __forceinline__ void stv(T *p, T v) {
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// ------------------------------------------------------------------ tiles

// address of the 16-byte element of plane k for entry i in a field whose
// tiles are `tile_bytes` long
__device__ __forceinline__ const char *tile_elem(const void *base, size_t tile_bytes, int i, int k) {
    return (const char *)base + (size_t)(i >> 6) * tile_bytes + k * 1024 + (i & 63) * 16;
}

// ------------------------------------------------------------------ spinors

// the field of one right-hand side: entries are then site indices
__device__ __forceinline__ FieldRef rhs_view(FieldRef f, int rhs) {
    f.data = (char *)f.data + (size_t)rhs * (size_t)(f.stride >> 6) * spinor_tile_bytes(f.prec);
    f.nrhs = 1;
    return f;
}

template <int PREC>
struct Spinor;

template <>
struct Spinor<WD_F64> {
    using R = double;
    static constexpr size_t kTileBytes = 12 * 1024;
    template <bool NT = false>
    static __device__ __forceinline__ void load(const FieldRef &f, int i, cx<R> v[12]) {
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const d2_t d = ldv<NT>((const d2_t *)tile_elem(f.data, kTileBytes, i, k));
            v[k] = {d.x, d.y};
        }
    }
    template <bool NT = false>
    static __device__ __forceinline__ void store(const FieldRef &f, int i, const cx<R> v[12]) {
#pragma unroll
        for (int k = 0; k < 12; ++k)
            stv<NT>((d2_t *)tile_elem(f.data, kTileBytes, i, k), d2_t{v[k].re, v[k].im});
    }
};

template <>
struct Spinor<WD_F32> {
    using R = float;
    static constexpr size_t kTileBytes = 6 * 1024;
    template <bool NT = false>
    static __device__ __forceinline__ void load(const FieldRef &f, int i, cx<R> v[12]) {
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            const f4_t q = ldv<NT>((const f4_t *)tile_elem(f.data, kTileBytes, i, j));
            v[2 * j] = {q.x, q.y};
            v[2 * j + 1] = {q.z, q.w};
        }
    }
    template <bool NT = false>
    static __device__ __forceinline__ void store(const FieldRef &f, int i, const cx<R> v[12]) {
#pragma unroll
        for (int j = 0; j < 6; ++j)
            stv<NT>((f4_t *)tile_elem(f.data, kTileBytes, i, j),
                    f4_t{v[2 * j].re, v[2 * j].im, v[2 * j + 1].re, v[2 * j + 1].im});
    }
};

template <>
struct Spinor<WD_F16> {
    using R = float;
    static constexpr size_t kTileBytes = 3 * 1024 + 256;
    static __device__ __forceinline__ const float *scale_ptr(const FieldRef &f, int i) {
        return (const float *)((const char *)f.data + (size_t)(i >> 6) * kTileBytes + 3 * 1024 +
                               (i & 63) * 4);
    }
    template <bool NT = false>
    static __device__ __forceinline__ void load(const FieldRef &f, int i, cx<R> v[12]) {
        const float s = ldv<NT>(scale_ptr(f, i));
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const h8_t q = ldv<NT>((const h8_t *)tile_elem(f.data, kTileBytes, i, j));
#pragma unroll
            for (int m = 0; m < 4; ++m)
                v[4 * j + m] = {s * (float)q[2 * m], s * (float)q[2 * m + 1]};
        }
    }
    template <bool NT = false>
    static __device__ __forceinline__ void store(const FieldRef &f, int i, const cx<R> v[12]) {
        float mx = 0.f;
#pragma unroll
        for (int k = 0; k < 12; ++k) mx = fmaxf(mx, fmaxf(fabsf(v[k].re), fabsf(v[k].im)));
        const float inv = mx > 0.f ? 1.0f / mx : 0.f;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            h8_t q;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                q[2 * m] = (_Float16)(v[4 * j + m].re * inv);
                q[2 * m + 1] = (_Float16)(v[4 * j + m].im * inv);
            }
            stv<NT>((h8_t *)tile_elem(f.data, kTileBytes, i, j), q);
        }
        stv<NT>((float *)scale_ptr(f, i), mx);
    }
};

// ------------------------------------------------------------------ links

// row 2 of a special unitary matrix from rows 0 and 1: conj(row0 x row1)
template <typename R>
__device__ __forceinline__ void reconstruct_row2(cx<R> u[9]) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int j1 = (j + 1) % 3, j2 = (j + 2) % 3;
        cx<R> c = cmul(u[j1], u[3 + j2]) - cmul(u[j2], u[3 + j1]);
        u[6 + j] = conj(c);
    }
}

template <int PREC>
struct Link;

template <>
struct Link<WD_F64> {
    using R = double;
    static constexpr size_t kTileBytes = 36 * 1024;
    template <bool NT = false>
    static __device__ __forceinline__ void load(const void *g, int mu, int s, cx<R> u[9]) {
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const d2_t d = ldv<NT>((const d2_t *)tile_elem(g, kTileBytes, s, mu * 9 + k));
            u[k] = {d.x, d.y};
        }
    }
    static __device__ __forceinline__ void store(void *g, int mu, int s, const cx<R> u[9]) {
#pragma unroll
        for (int k = 0; k < 9; ++k)
            *(double2 *)tile_elem(g, kTileBytes, s, mu * 9 + k) = make_double2(u[k].re, u[k].im);
    }
};

template <>
struct Link<kLinkF64R12> {
    using R = double;
    static constexpr size_t kTileBytes = 24 * 1024;
    template <bool NT = false>
    static __device__ __forceinline__ void load(const void *g, int mu, int s, cx<R> u[9]) {
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const d2_t d = ldv<NT>((const d2_t *)tile_elem(g, kTileBytes, s, mu * 6 + k));
            u[k] = {d.x, d.y};
        }
        reconstruct_row2(u);
    }
    static __device__ __forceinline__ void store(void *g, int mu, int s, const cx<double> u[9]) {
#pragma unroll
        for (int k = 0; k < 6; ++k)
            *(double2 *)tile_elem(g, kTileBytes, s, mu * 6 + k) = make_double2(u[k].re, u[k].im);
    }
};

template <>
struct Link<WD_F32> {
    using R = float;
    static constexpr size_t kTileBytes = 12 * 1024;
    template <bool NT = false>
    static __device__ __forceinline__ void load(const void *g, int mu, int s, cx<R> u[9]) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const f4_t q = ldv<NT>((const f4_t *)tile_elem(g, kTileBytes, s, mu * 3 + j));
            u[2 * j] = {q.x, q.y};
            u[2 * j + 1] = {q.z, q.w};
        }
        reconstruct_row2(u);
    }
    static __device__ __forceinline__ void store(void *g, int mu, int s, const cx<double> u[9]) {
#pragma unroll
        for (int j = 0; j < 3; ++j)
            *(float4 *)tile_elem(g, kTileBytes, s, mu * 3 + j) =
                make_float4((float)u[2 * j].re, (float)u[2 * j].im, (float)u[2 * j + 1].re,
                            (float)u[2 * j + 1].im);
    }
};

template <>
struct Link<WD_F16> {
    using R = float;
    static constexpr size_t kTileBytes = 12 * 512;
    static __device__ __forceinline__ const char *elem(const void *g, int mu, int s, int j) {
        return (const char *)g + (size_t)(s >> 6) * kTileBytes + (mu * 3 + j) * 512 + (s & 63) * 8;
    }
    template <bool NT = false>
    static __device__ __forceinline__ void load(const void *g, int mu, int s, cx<R> u[9]) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const h4_t q = ldv<NT>((const h4_t *)elem(g, mu, s, j));
            u[2 * j] = {(float)q[0], (float)q[1]};
            u[2 * j + 1] = {(float)q[2], (float)q[3]};
        }
        reconstruct_row2(u);
    }
    static __device__ __forceinline__ void store(void *g, int mu, int s, const cx<double> u[9]) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            // double -> float -> half: the float step keeps 24 bits, the final
            // rounding to 11 bits dominates
            h4_t q;
            q[0] = (_Float16)(float)u[2 * j].re;
            q[1] = (_Float16)(float)u[2 * j].im;
            q[2] = (_Float16)(float)u[2 * j + 1].re;
            q[3] = (_Float16)(float)u[2 * j + 1].im;
            *(h4_t *)elem(g, mu, s, j) = q;
        }
    }
};

// ------------------------------------------------------------------ reduction
//
// Deterministic and split in two launches: every block of the producing
// kernel reduces its contribution (one rhs per block: a fixed butterfly
// inside each wave, then the waves in order) and writes one partial; a
// one-block finalize kernel then sums the partials of each rhs in a fixed
// order and updates the solver state.  The kernel boundary orders the
// two phases, so no device-scope fence (an L2 write-back on this chip) is
// issued per block.  Results are bitwise reproducible for a launch shape.

__device__ __forceinline__ bool finite(double x) { return __builtin_isfinite(x); }

// the launch is off for this gate (uniform over the grid)
__device__ __forceinline__ bool gate_off(const Gate &g) {
    if (!g.batch) return false;
    if (g.mode == GATE_TRIGGER) return !(g.batch->n_active == 0 && g.batch->n_trigger > 0);
    return g.batch->n_active == 0;
}

// the gate takes right-hand side r (uniform over a workgroup)
__device__ __forceinline__ bool gate_rhs(const Gate &g, int r) {
    if (!g.st) return true;
    const RhsState &s = g.st[r];
    if (g.mode == GATE_TRIGGER) return s.trigger && !s.converged;
    if (g.mode == GATE_RESTART) return s.restarted != 0;
    return s.active != 0;
}

__device__ inline void finalize_rhs(const RedArgs &red, int r, double total) {
    RhsState &st = red.st[r];
    const SolveCtl &c = red.ctl;
    switch (red.mode) {
        case RED_ALPHA:
            st.restarted = 0;
            if (st.active) {
                st.tt = total;
                if (!(total > 0.0) || !finite(total)) {
                    st.failed = WD_ERR_NUMERIC;
                    st.active = 0;
                    st.alpha = 0.0;
                } else {
                    st.alpha = st.rr / total;
                }
            }
            break;
        case RED_RR:
            if (st.active) {
                st.iters += 1;
                st.since += 1;
                st.rr_prev = st.rr;
                st.rr = total;
                if (!finite(total)) {
                    st.failed = WD_ERR_NUMERIC;
                    st.active = 0;
                    break;
                }
                st.beta = total / st.rr_prev;
                if (total > st.rr_max) st.rr_max = total;
                bool trig = total <= c.tol2 * st.rr0;
                if (c.mixed && total < c.delta2 * st.rr_max) trig = true;
                if (c.max_inner > 0 && st.since >= c.max_inner) trig = true;
                if (st.iters >= c.max_iter) {
                    st.failed = WD_ERR_NOCONV;
                    trig = true;
                }
                if (trig) {
                    st.active = 0;
                    st.trigger = 1;
                    st.pend = c.lag_x;  // its last alpha p is not in x_lo yet
                }
            }
            break;
        case RED_TRUE:
            if (!st.converged && st.trigger) {
                st.rr_true = total;
                st.updates += 1;
                st.trigger = 0;
                st.pend = 0;  // added to x by the update's accumulation
                if (!finite(total)) {
                    st.failed = WD_ERR_NUMERIC;
                    st.active = 0;
                } else if (total <= c.tol2 * st.rr0) {
                    st.converged = 1;
                    st.failed = 0;
                    st.active = 0;
                } else if (st.failed) {
                    st.active = 0;
                } else {
                    st.beta = (st.updates == 1) ? 0.0 : total / st.rr_prev;
                    st.rr = total;
                    st.rr_max = total;
                    st.since = 0;
                    st.active = 1;
                    st.restarted = 1;
                }
            }
            break;
        case RED_B0:
            st.rr0 = total;
            st.restarted = 0;
            st.pend = 0;
            st.active = 0;
            st.converged = 0;
            st.failed = 0;
            st.trigger = 0;
            if (!finite(total)) {
                st.failed = WD_ERR_NUMERIC;
            } else if (total == 0.0) {
                st.converged = 1;  // b' = 0: x = 0 is exact
            } else {
                st.trigger = 1;    // the first reliable update forms r and p
            }
            break;
        case RED_AUX: st.aux = total; break;
        case RED_AUX2: st.aux2 = total; break;
        case RED_AUX_ADD: st.aux += total; break;
        case RED_AUX2_ADD: st.aux2 += total; break;
        default: break;
    }
}

__device__ inline void recount_batch(const RedArgs &red) {
    int na = 0, nt = 0, nd = 0;
    for (int r = 0; r < red.ctl.nrhs; ++r) {
        const RhsState &st = red.st[r];
        na += st.active;
        nt += st.trigger;
        nd += (st.converged || (st.failed && !st.trigger)) ? 1 : 0;
    }
    red.batch->n_active = na;
    red.batch->n_trigger = nt;
    red.batch->n_done = nd;
}

// Phase 1.  v: this thread's contribution (0 for idle threads).  Must be
// reached by every thread of the block; blockDim.x is a multiple of 64.  A
// fixed butterfly inside each wave, then wave sums in order; writes
// partials[idx].
__device__ inline void reduce_block(double v, double *partials, size_t idx) {
    __shared__ double sm[16];
    const int tid = threadIdx.x;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((tid & 63) == 0) sm[tid >> 6] = v;
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sm[w];
        partials[idx] = s;
    }
}

// Phase 2 is k_finalize (blas.hip), launched by launch_finalize.

}  // namespace wd
