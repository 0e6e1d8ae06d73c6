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
    // the stored halves (v / s, one complex per half pair) and the scale s
    template <bool NT = false>
    static __device__ __forceinline__ void load_raw(const FieldRef &f, int i, h2_t q[12],
                                                    float &s) {
        s = ldv<NT>(scale_ptr(f, i));
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const h8_t v = ldv<NT>((const h8_t *)tile_elem(f.data, kTileBytes, i, j));
#pragma unroll
            for (int m = 0; m < 4; ++m) q[4 * j + m] = h2_t{v[2 * m], v[2 * m + 1]};
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
    // the link as packed halves (one complex per pair): rows 0 and 1 as
    // stored, row 2 = conj(row0 x row1) formed with float accumulation and
    // rounded to binary16
    template <bool NT = false>
    static __device__ __forceinline__ void load_h2(const void *g, int mu, int s, h2_t u[9]);
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

// ------------------------------------------------------------------ binary16 hops
//
// The binary16 stencil's link products on packed halves: a complex number is
// one pair (re, im) of halves, and each real or imaginary part of a product
// sum is a chain of two-term dot products of halves accumulated in float32
// (v_dot2_f32_f16: the products of halves are exact in float32).  The
// spin projection adds pairs of halves (the stored spinor is v / s with
// |v / s| <= 1, so the sums stay within binary16's range); the site scale s
// multiplies the hop's float result.

// Two-term dot products of halves accumulated in float32, with the sign
// modifiers of v_dot2_f32_f16 on the second operand's halves (the compiler
// does not fold a negated half into the instruction and would spend a
// separate instruction on it):
//   dot2_pp(a, b, c) = a.x b.x + a.y b.y + c     dot2_pm = a.x b.x - a.y b.y + c
//   dot2_mp          = -a.x b.x + a.y b.y + c    dot2_mm = -a.x b.x - a.y b.y + c
// The *0 forms start a chain at c = 0.  A dot product's result may be read
// by the next dot product of a chain as its accumulator at once, but by any
// other vector instruction only after three wait states; the compiler does
// not see inside the asm, so the *_e forms, which end a chain and whose
// results other instructions read, wait those states themselves.
#define WD_DOT2(NAME, MODS)                                                                 \
    __device__ __forceinline__ float NAME(h2_t a, h2_t b, float c) {                        \
        float d;                                                                            \
        asm("v_dot2_f32_f16 %0, %1, %2, %3" MODS : "=v"(d) : "v"(a), "v"(b), "v"(c));       \
        return d;                                                                           \
    }                                                                                       \
    __device__ __forceinline__ float NAME##0(h2_t a, h2_t b) {                              \
        float d;                                                                            \
        asm("v_dot2_f32_f16 %0, %1, %2, 0" MODS : "=v"(d) : "v"(a), "v"(b));                \
        return d;                                                                           \
    }                                                                                       \
    __device__ __forceinline__ float NAME##_e(h2_t a, h2_t b, float c) {                    \
        float d;                                                                            \
        asm("v_dot2_f32_f16 %0, %1, %2, %3" MODS "\n\ts_nop 2"                              \
            : "=v"(d)                                                                       \
            : "v"(a), "v"(b), "v"(c));                                                      \
        return d;                                                                           \
    }
WD_DOT2(dot2_pp, "")
WD_DOT2(dot2_pm, " neg_hi:[0,1,0]")
WD_DOT2(dot2_mp, " neg_lo:[0,1,0]")
WD_DOT2(dot2_mm, " neg_lo:[0,1,0] neg_hi:[0,1,0]")
#undef WD_DOT2

__device__ __forceinline__ h2_t h2_swap(h2_t b) { return __builtin_shufflevector(b, b, 1, 0); }

template <bool NT>
__device__ __forceinline__ void Link<WD_F16>::load_h2(const void *g, int mu, int s, h2_t u[9]) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const h4_t q = ldv<NT>((const h4_t *)elem(g, mu, s, j));
        u[2 * j] = h2_t{q[0], q[1]};
        u[2 * j + 1] = h2_t{q[2], q[3]};
    }
    // row 2 = conj(u0[j1] u1[j2] - u0[j2] u1[j1]): re(ab - cd) = a.b(-) - c.d(-),
    // im(ab - cd) = a.swap(b) - c.swap(d)
    h2_t s1[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) s1[j] = h2_swap(u[3 + j]);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int j1 = (j + 1) % 3, j2 = (j + 2) % 3;
        const float re = dot2_pm_e(u[j1], u[3 + j2], dot2_mp0(u[j2], u[3 + j1]));
        const float im = dot2_pp_e(u[j1], s1[j2], dot2_mm0(u[j2], s1[j1]));
        u[6 + j] = h2_t{(_Float16)re, (_Float16)(-im)};
    }
}

// (1 + S gamma_mu) psi on packed halves: the two upper spin components
template <int MU, int S>
__device__ __forceinline__ void project_h2(const h2_t p[12], h2_t h0[3], h2_t h1[3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const h2_t a0 = p[c], a1 = p[3 + c], a2 = p[6 + c], a3 = p[9 + c];
        if (MU == 0) {
            const h2_t i3{-a3.y, a3.x}, i2{-a2.y, a2.x};
            h0[c] = S > 0 ? a0 + i3 : a0 - i3;
            h1[c] = S > 0 ? a1 + i2 : a1 - i2;
        } else if (MU == 1) {
            h0[c] = S > 0 ? a0 - a3 : a0 + a3;
            h1[c] = S > 0 ? a1 + a2 : a1 - a2;
        } else if (MU == 2) {
            const h2_t i2{-a2.y, a2.x}, i3{-a3.y, a3.x};
            h0[c] = S > 0 ? a0 + i2 : a0 - i2;
            h1[c] = S > 0 ? a1 - i3 : a1 + i3;
        } else {
            h0[c] = S > 0 ? a0 + a2 : a0 - a2;
            h1[c] = S > 0 ? a1 + a3 : a1 - a3;
        }
    }
}

// w = U h (ADJ: U^dag h) in float32 from packed halves:
//   U h:     re = U.x h.x - U.y h.y,  im = U.x h.y + U.y h.x = U . swap(h)
//   U^dag h: re = U.x h.x + U.y h.y,  im = U.x h.y - U.y h.x = U . swap(h)(-)
template <bool ADJ>
__device__ __forceinline__ void su3_mul_h2(const h2_t u[9], const h2_t h[3], cx<float> w[3]) {
    h2_t hs[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) hs[b] = h2_swap(h[b]);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const h2_t m0 = ADJ ? u[a] : u[3 * a], m1 = ADJ ? u[3 + a] : u[3 * a + 1],
                   m2 = ADJ ? u[6 + a] : u[3 * a + 2];
        float re, im;
        // the chains without sign modifiers through the compiler's own dot
        // product, whose wait states it places (and fills) itself
        auto pp3 = [](h2_t x0, h2_t y0, h2_t x1, h2_t y1, h2_t x2, h2_t y2) {
            float c = __builtin_amdgcn_fdot2(x0, y0, 0.0f, false);
            c = __builtin_amdgcn_fdot2(x1, y1, c, false);
            return __builtin_amdgcn_fdot2(x2, y2, c, false);
        };
        if (ADJ) {
            re = pp3(m0, h[0], m1, h[1], m2, h[2]);
            im = dot2_pm_e(m2, hs[2], dot2_pm(m1, hs[1], dot2_pm0(m0, hs[0])));
        } else {
            re = dot2_pm_e(m2, h[2], dot2_pm(m1, h[1], dot2_pm0(m0, h[0])));
            im = pp3(m0, hs[0], m1, hs[1], m2, hs[2]);
        }
        w[a] = {re, im};
    }
}

// acc += s * (the hop result rebuilt to four spins), as accumulate(), with
// the site scale folded into fused multiply-adds
template <int MU, int S>
__device__ __forceinline__ void accumulate_s(float s, const cx<float> w0[3],
                                             const cx<float> w1[3], cx<float> acc[12]) {
    auto add = [](cx<float> &a, float f, cx<float> w) {  // a += f w
        a = {fmaf(f, w.re, a.re), fmaf(f, w.im, a.im)};
    };
    auto add_i = [](cx<float> &a, float f, cx<float> w) {  // a += f i w
        a = {fmaf(-f, w.im, a.re), fmaf(f, w.re, a.im)};
    };
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        add(acc[c], s, w0[c]);
        add(acc[3 + c], s, w1[c]);
        if (MU == 0) {  // lower: -S i w1, -S i w0
            add_i(acc[6 + c], S > 0 ? -s : s, w1[c]);
            add_i(acc[9 + c], S > 0 ? -s : s, w0[c]);
        } else if (MU == 1) {  // lower: S w1, -S w0
            add(acc[6 + c], S > 0 ? s : -s, w1[c]);
            add(acc[9 + c], S > 0 ? -s : s, w0[c]);
        } else if (MU == 2) {  // lower: -S i w0, S i w1
            add_i(acc[6 + c], S > 0 ? -s : s, w0[c]);
            add_i(acc[9 + c], S > 0 ? s : -s, w1[c]);
        } else {  // lower: S w0, S w1
            add(acc[6 + c], S > 0 ? s : -s, w0[c]);
            add(acc[9 + c], S > 0 ? s : -s, w1[c]);
        }
    }
}

// 8 reals per link in binary16 (16 bytes): a parametrisation of SU(3) in
// which no stored quantity is recovered from a difference of nearly equal
// numbers, so binary16 rounding is not amplified.  Columns are first
// relabelled cyclically by j (a cyclic relabelling keeps the matrix special
// unitary), so that entry a_j of row 0 with the largest modulus comes first:
// row 0 = (a_j, a_p, a_q), p = j+1, q = j+2 (mod 3).
//  - Row 0: a_p and a_q are stored (4 reals) and one component of a_j, the
//    other being +-sqrt(1 - |a_p|^2 - |a_q|^2 - comp^2), the larger of the two
//    (|a_j|^2 >= 1/3, so the root is taken of at least 1/6).
//  - A frame of the plane orthogonal to row 0: e1 = conj(row0 x e_k) / norm,
//    with e_k the unit vector at k = p or q, the smaller of the two entries
//    (the norm^2 = 1 - |a_k|^2 >= 2/3), and e2 = conj(row0 x e1); the rows
//    (row0, e1, e2) are special unitary.
//  - Row 1 = alpha e1 + beta e2 with |alpha|^2 + |beta|^2 = 1; the smaller of
//    alpha, beta is stored (2 reals) and one component of the larger, the
//    other derived as above.  Row 2 = conj(row0 x row1) = conj(alpha) e2 -
//    conj(beta) e1.
// The eight choices (j: 2 bits; which component of a_j and its sign; k; which
// of alpha, beta is stored; which component of the other and its sign) sit
// in the lowest significand bit of the eight halves: each value is rounded
// to the nearest binary16 number whose last bit is the choice bit (at most
// one unit in the last place off).
// Slots: 0,1 a_p; 2,3 a_q; 4 the stored component of a_j; 5,6 the stored one
// of alpha/beta; 7 the stored component of the other.  Bits (slot: meaning):
// 0,1 j; 2 a_j's derived component is Im; 3 it is negative; 4 k = q; 5 alpha
// is the stored one; 6 the other's derived component is Im; 7 it is negative.
typedef unsigned short u16x8_t __attribute__((ext_vector_type(8)));

// the binary16 number nearest to x whose last significand bit is `bit`
__device__ __forceinline__ unsigned short half_with_bit(double x, int bit) {
    const _Float16 h = (_Float16)(float)x;
    const unsigned short b = __builtin_bit_cast(unsigned short, h);
    if ((b & 1) == bit) return b;
    const unsigned short sgn = b & 0x8000, mag = b & 0x7fff;
    if (mag == 0) return (unsigned short)(sgn | 1);
    const unsigned short dn = (unsigned short)(sgn | (mag - 1));
    const unsigned short up = (unsigned short)(sgn | (mag + 1));
    const double vd = (double)__builtin_bit_cast(_Float16, dn);
    const double vu = (double)__builtin_bit_cast(_Float16, up);
    return fabs(vd - x) <= fabs(vu - x) ? dn : up;
}

template <typename R>
__device__ __forceinline__ cx<R> cross_entry(const cx<R> a[3], const cx<R> b[3], int i) {
    // (a x b)_i = a_{i+1} b_{i+2} - a_{i+2} b_{i+1}
    const int i1 = (i + 1) % 3, i2 = (i + 2) % 3;
    return cmul(a[i1], b[i2]) - cmul(a[i2], b[i1]);
}

// Rows 1 and 2 from row 0 (columns already relabelled), the pivot choice and
// the stored alpha/beta part; shared by the encoder's check and the decoder.
template <typename R>
__device__ __forceinline__ void r8_frame(const cx<R> r0[3], int kq, cx<R> e1[3], cx<R> e2[3]) {
    // c = row0 x e_k in the relabelled columns: k = p gives (-a_q, 0, a_j),
    // k = q gives (a_p, -a_j, 0)
    cx<R> c[3];
    R ak2;
    if (kq) {
        c[0] = r0[1];
        c[1] = -r0[0];
        c[2] = {R(0), R(0)};
        ak2 = norm2(r0[2]);
    } else {
        c[0] = -r0[2];
        c[1] = {R(0), R(0)};
        c[2] = r0[0];
        ak2 = norm2(r0[1]);
    }
    const R inv = R(1) / sqrt(R(1) - ak2);
#pragma unroll
    for (int i = 0; i < 3; ++i) e1[i] = scale(inv, conj(c[i]));
#pragma unroll
    for (int i = 0; i < 3; ++i) e2[i] = conj(cross_entry(r0, e1, i));
}

// the derived component: +-sqrt(1 - sum of squares of the stored ones)
template <typename R>
__device__ __forceinline__ cx<R> r8_derive(R s0, R s1, R s2, R s3, R comp, int im, int neg) {
    const R m = R(1) - (s0 * s0 + s1 * s1 + s2 * s2 + s3 * s3 + comp * comp);
    R d = sqrt(m > R(0) ? m : R(0));
    if (neg) d = -d;
    return im ? cx<R>{comp, d} : cx<R>{d, comp};
}

template <typename R>
__device__ __forceinline__ void r8_decode(const R f[8], const int b[8], cx<R> u[9]) {
    const int j = b[0] | (b[1] << 1);
    cx<R> r0[3];
    r0[1] = {f[0], f[1]};
    r0[2] = {f[2], f[3]};
    r0[0] = r8_derive(f[0], f[1], f[2], f[3], f[4], b[2], b[3]);
    cx<R> e1[3], e2[3];
    r8_frame(r0, b[4], e1, e2);
    const cx<R> g{f[5], f[6]};
    const cx<R> d = r8_derive(f[5], f[6], R(0), R(0), f[7], b[6], b[7]);
    const cx<R> al = b[5] ? g : d, be = b[5] ? d : g;
    cx<R> w[9];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        w[i] = r0[i];
        w[3 + i] = cmul(al, e1[i]) + cmul(be, e2[i]);
        w[6 + i] = cmul(conj(al), e2[i]) - cmul(conj(be), e1[i]);
    }
    // undo the column relabelling: column (j + c) mod 3 of U is column c
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const cx<R> x0 = w[3 * r], x1 = w[3 * r + 1], x2 = w[3 * r + 2];
        u[3 * r + 0] = j == 0 ? x0 : (j == 1 ? x2 : x1);
        u[3 * r + 1] = j == 0 ? x1 : (j == 1 ? x0 : x2);
        u[3 * r + 2] = j == 0 ? x2 : (j == 1 ? x1 : x0);
    }
}

template <>
struct Link<kLinkF16R8> {
    using R = float;
    static constexpr size_t kTileBytes = 4 * 1024;
    static __device__ __forceinline__ const char *elem(const void *g, int mu, int s) {
        return (const char *)g + (size_t)(s >> 6) * kTileBytes + mu * 1024 + (s & 63) * 16;
    }
    template <bool NT = false>
    static __device__ __forceinline__ void load(const void *g, int mu, int s, cx<R> u[9]) {
        const h8_t q = ldv<NT>((const h8_t *)elem(g, mu, s));
        const u16x8_t raw = __builtin_bit_cast(u16x8_t, q);
        R f[8];
        int b[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            f[i] = (R)q[i];
            b[i] = raw[i] & 1;
        }
        r8_decode(f, b, u);
    }
    static __device__ __forceinline__ void store(void *g, int mu, int s, const cx<double> u[9]) {
        // relabel columns so that the largest entry of row 0 comes first
        const double m0 = norm2(u[0]), m1 = norm2(u[1]), m2 = norm2(u[2]);
        const int j = (m0 >= m1 && m0 >= m2) ? 0 : (m1 >= m2 ? 1 : 2);
        cx<double> r0[3], r1[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            r0[c] = u[(j + c) % 3];
            r1[c] = u[3 + (j + c) % 3];
        }
        unsigned short h[8];
        int b[8];
        b[0] = j & 1;
        b[1] = j >> 1;
        b[2] = fabs(r0[0].im) > fabs(r0[0].re) ? 1 : 0;  // derive the larger component
        const double dv = b[2] ? r0[0].im : r0[0].re;
        b[3] = dv < 0 ? 1 : 0;
        h[0] = half_with_bit(r0[1].re, b[0]);
        h[1] = half_with_bit(r0[1].im, b[1]);
        h[2] = half_with_bit(r0[2].re, b[2]);
        h[3] = half_with_bit(r0[2].im, b[3]);
        double f[8];
#pragma unroll
        for (int i = 0; i < 4; ++i) f[i] = (double)__builtin_bit_cast(_Float16, h[i]);
        // the pivot of the frame: the smaller of the stored a_p, a_q as they
        // decode
        b[4] = f[2] * f[2] + f[3] * f[3] < f[0] * f[0] + f[1] * f[1] ? 1 : 0;
        h[4] = half_with_bit(b[2] ? r0[0].re : r0[0].im, b[4]);
        f[4] = (double)__builtin_bit_cast(_Float16, h[4]);
        // the frame as the decoder rebuilds it from the rounded row 0
        cx<double> d0[3], e1[3], e2[3];
        d0[1] = {f[0], f[1]};
        d0[2] = {f[2], f[3]};
        d0[0] = r8_derive(f[0], f[1], f[2], f[3], f[4], b[2], b[3]);
        r8_frame(d0, b[4], e1, e2);
        cx<double> al{0.0, 0.0}, be{0.0, 0.0};
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            al = cfmac(e1[i], r1[i], al);  // <e1, r1>
            be = cfmac(e2[i], r1[i], be);  // <e2, r1>
        }
        b[5] = norm2(al) < norm2(be) ? 1 : 0;  // store the smaller
        const cx<double> gs = b[5] ? al : be, dl = b[5] ? be : al;
        b[6] = fabs(dl.im) > fabs(dl.re) ? 1 : 0;
        b[7] = (b[6] ? dl.im : dl.re) < 0 ? 1 : 0;
        h[5] = half_with_bit(gs.re, b[5]);
        h[6] = half_with_bit(gs.im, b[6]);
        h[7] = half_with_bit(b[6] ? dl.re : dl.im, b[7]);
        u16x8_t raw;
#pragma unroll
        for (int i = 0; i < 8; ++i) raw[i] = h[i];
        *(h8_t *)elem(g, mu, s) = __builtin_bit_cast(h8_t, raw);
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
