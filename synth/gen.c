/*
 * Seeded synthetic inputs for the Wilson-Dirac solver: SU(3) gauge fields,
 * Gaussian spinor sources and random gauge transformations.
 *
 * This file holds none of the solver's arithmetic (no stencil, no Krylov
 * step): it only draws inputs.  Both the CPU oracle's tests and the GPU
 * path's tests and benchmark take their fields from here, so the two sides
 * see identical inputs.
 *
 * Random numbers: SplitMix64 (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014), used counter-style.  Every
 * object (a link U_mu(s), a site's spinor, a site's gauge rotation) has its
 * own 64-bit key, and its k-th draw (k = 1, 2, ...) is mix(key + k * GAMMA).
 * Output is therefore independent of thread count and of how the lattice is
 * split into chunks.  Uniforms take the top 53 bits; normals come from the
 * Box-Muller transform, both members of each pair used in order.
 *
 * Canonical layouts (all float64, interleaved re,im):
 *   gauge  [V][mu=0..3][a=0..2][b=0..2][2]   (18 reals per link)
 *   spinor [V][spin=0..3][colour=0..2][2]    (24 reals per site)
 *   site s = x + Lx*(y + Ly*(z + Lz*t)).
 *
 * Built with gcc; deterministic given -ffp-contract=off and no fast-math.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

typedef struct {
    uint64_t state;
    int have_spare;
    double spare;
} rng_t;

static inline void rng_init(rng_t *r, uint64_t key) {
    r->state = key;
    r->have_spare = 0;
    r->spare = 0.0;
}

/* next SplitMix64 output: state advances by GAMMA, then the finaliser */
static inline uint64_t rng_u64(rng_t *r) {
    r->state += GAMMA;
    return mix64(r->state);
}

/* uniform in [0, 1) from the top 53 bits */
static inline double rng_uniform(rng_t *r) {
    return (double)(rng_u64(r) >> 11) * 0x1.0p-53;
}

/* standard normal; Box-Muller pair (cos member first, then sin member) */
static inline double rng_normal(rng_t *r) {
    if (r->have_spare) {
        r->have_spare = 0;
        return r->spare;
    }
    double u1 = rng_uniform(r);
    double u2 = rng_uniform(r);
    double rad = sqrt(-2.0 * log(1.0 - u1)); /* 1-u1 in (0,1] */
    double th = 6.283185307179586476925286766559 * u2;
    r->spare = rad * sin(th);
    r->have_spare = 1;
    return rad * cos(th);
}

static inline uint64_t link_key(uint64_t seed, uint64_t site, int mu) {
    return (seed * GAMMA) ^ (4ULL * site + (uint64_t)mu);
}
static inline uint64_t site_key(uint64_t seed, uint64_t site) {
    return (seed * GAMMA) ^ site;
}

/* ---- 3x3 complex helpers, matrices as double[18] row-major (re,im) ---- */

static void cm_mul(const double *a, const double *b, double *c) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double re = 0.0, im = 0.0;
            for (int k = 0; k < 3; ++k) {
                double ar = a[2 * (3 * i + k)], ai = a[2 * (3 * i + k) + 1];
                double br = b[2 * (3 * k + j)], bi = b[2 * (3 * k + j) + 1];
                re += ar * br - ai * bi;
                im += ar * bi + ai * br;
            }
            c[2 * (3 * i + j)] = re;
            c[2 * (3 * i + j) + 1] = im;
        }
}

/* Gram-Schmidt on rows 0 and 1, then row 2 = conj(row0 x row1): the result
 * is special unitary (det = +1) and equals its own 12-real reconstruction. */
static void reunitarise_rows(double *m) {
    double n0 = 0.0;
    for (int k = 0; k < 6; ++k) n0 += m[k] * m[k];
    n0 = 1.0 / sqrt(n0);
    for (int k = 0; k < 6; ++k) m[k] *= n0;
    /* <row0, row1> = sum conj(r0) r1 */
    double pr = 0.0, pi = 0.0;
    for (int j = 0; j < 3; ++j) {
        double ar = m[2 * j], ai = m[2 * j + 1];
        double br = m[6 + 2 * j], bi = m[6 + 2 * j + 1];
        pr += ar * br + ai * bi;
        pi += ar * bi - ai * br;
    }
    for (int j = 0; j < 3; ++j) {
        double ar = m[2 * j], ai = m[2 * j + 1];
        m[6 + 2 * j] -= pr * ar - pi * ai;
        m[6 + 2 * j + 1] -= pr * ai + pi * ar;
    }
    double n1 = 0.0;
    for (int k = 6; k < 12; ++k) n1 += m[k] * m[k];
    n1 = 1.0 / sqrt(n1);
    for (int k = 6; k < 12; ++k) m[k] *= n1;
    /* row2_j = conj(row0_{j+1} row1_{j+2} - row0_{j+2} row1_{j+1}) */
    for (int j = 0; j < 3; ++j) {
        int j1 = (j + 1) % 3, j2 = (j + 2) % 3;
        double ar = m[2 * j1], ai = m[2 * j1 + 1];
        double br = m[6 + 2 * j2], bi = m[6 + 2 * j2 + 1];
        double cr = m[2 * j2], ci = m[2 * j2 + 1];
        double dr = m[6 + 2 * j1], di = m[6 + 2 * j1 + 1];
        double re = (ar * br - ai * bi) - (cr * dr - ci * di);
        double im = (ar * bi + ai * br) - (cr * di + ci * dr);
        m[12 + 2 * j] = re;
        m[12 + 2 * j + 1] = -im;
    }
}

/* Haar-distributed unitary via QR of a complex Ginibre matrix with the
 * diagonal of R made positive (Mezzadri 2007).  Gram-Schmidt on the columns
 * produces exactly that Q.  Then row 2 is multiplied by conj(det Q) so that
 * det = +1. */
static void draw_haar_su3(rng_t *r, double *m) {
    const double s = 0.70710678118654752440; /* 1/sqrt(2) */
    double z[18];
    for (int i = 0; i < 9; ++i) { /* entry-row-major, then re, then im */
        z[2 * i] = rng_normal(r) * s;
        z[2 * i + 1] = rng_normal(r) * s;
    }
    /* columns of z: col j entries z[2*(3*i+j)] */
    double q[18];
    for (int j = 0; j < 3; ++j) {
        double v[6];
        for (int i = 0; i < 3; ++i) {
            v[2 * i] = z[2 * (3 * i + j)];
            v[2 * i + 1] = z[2 * (3 * i + j) + 1];
        }
        for (int k = 0; k < j; ++k) {
            /* proj = <q_k, v> = sum conj(q_ik) v_i */
            double pr = 0.0, pi = 0.0;
            for (int i = 0; i < 3; ++i) {
                double qr = q[2 * (3 * i + k)], qi = q[2 * (3 * i + k) + 1];
                pr += qr * v[2 * i] + qi * v[2 * i + 1];
                pi += qr * v[2 * i + 1] - qi * v[2 * i];
            }
            for (int i = 0; i < 3; ++i) {
                double qr = q[2 * (3 * i + k)], qi = q[2 * (3 * i + k) + 1];
                v[2 * i] -= pr * qr - pi * qi;
                v[2 * i + 1] -= pr * qi + pi * qr;
            }
        }
        double n = 0.0;
        for (int i = 0; i < 6; ++i) n += v[i] * v[i];
        n = 1.0 / sqrt(n);
        for (int i = 0; i < 3; ++i) {
            q[2 * (3 * i + j)] = v[2 * i] * n;
            q[2 * (3 * i + j) + 1] = v[2 * i + 1] * n;
        }
    }
    /* det Q by cofactor expansion along row 0 */
    double dr = 0.0, di = 0.0;
    for (int j = 0; j < 3; ++j) {
        int j1 = (j + 1) % 3, j2 = (j + 2) % 3;
        double ar = q[6 + 2 * j1], ai = q[6 + 2 * j1 + 1];
        double br = q[12 + 2 * j2], bi = q[12 + 2 * j2 + 1];
        double cr = q[6 + 2 * j2], ci = q[6 + 2 * j2 + 1];
        double er = q[12 + 2 * j1], ei = q[12 + 2 * j1 + 1];
        double mr = (ar * br - ai * bi) - (cr * er - ci * ei);
        double mi = (ar * bi + ai * br) - (cr * ei + ci * er);
        double xr = q[2 * j], xi = q[2 * j + 1];
        dr += xr * mr - xi * mi;
        di += xr * mi + xi * mr;
    }
    double dn = sqrt(dr * dr + di * di);
    dr /= dn;
    di /= dn;
    for (int j = 0; j < 3; ++j) { /* row2 *= conj(det) */
        double xr = q[12 + 2 * j], xi = q[12 + 2 * j + 1];
        q[12 + 2 * j] = xr * dr + xi * di;
        q[12 + 2 * j + 1] = xi * dr - xr * di;
    }
    reunitarise_rows(q); /* row 2 = conj(row0 x row1) to the last bit */
    memcpy(m, q, sizeof(q));
}

/* U = exp(i eps H), H = sum_a w_a lambda_a / 2 (Gell-Mann basis, w_a ~ N(0,1)),
 * by scaling and squaring of a degree-16 Taylor polynomial, then rows
 * re-orthonormalised so that U is special unitary to rounding. */
static void draw_exp_su3(rng_t *r, double eps, double *m) {
    double w[8];
    for (int a = 0; a < 8; ++a) w[a] = rng_normal(r);
    const double is3 = 0.57735026918962576451; /* 1/sqrt(3) */
    double h[18] = {0};
    /* H = 1/2 * [[w3 + w8/sqrt3, w1 - i w2, w4 - i w5],
     *            [w1 + i w2, -w3 + w8/sqrt3, w6 - i w7],
     *            [w4 + i w5, w6 + i w7, -2 w8/sqrt3]]   (w indexed from 1) */
    h[0] = 0.5 * (w[2] + w[7] * is3);
    h[2] = 0.5 * w[0];  h[3] = -0.5 * w[1];
    h[4] = 0.5 * w[3];  h[5] = -0.5 * w[4];
    h[6] = 0.5 * w[0];  h[7] = 0.5 * w[1];
    h[8] = 0.5 * (-w[2] + w[7] * is3);
    h[10] = 0.5 * w[5]; h[11] = -0.5 * w[6];
    h[12] = 0.5 * w[3]; h[13] = 0.5 * w[4];
    h[14] = 0.5 * w[5]; h[15] = 0.5 * w[6];
    h[16] = -w[7] * is3;
    /* A = i eps H */
    double a[18];
    double fn = 0.0;
    for (int k = 0; k < 9; ++k) {
        a[2 * k] = -eps * h[2 * k + 1];
        a[2 * k + 1] = eps * h[2 * k];
        fn += a[2 * k] * a[2 * k] + a[2 * k + 1] * a[2 * k + 1];
    }
    fn = sqrt(fn);
    int sq = 0;
    while (fn > 0.25) {
        fn *= 0.5;
        ++sq;
    }
    double scale = ldexp(1.0, -sq);
    for (int k = 0; k < 18; ++k) a[k] *= scale;
    /* Horner: E = I + A(I + A/2(I + A/3(... (I + A/16)))) */
    double e[18] = {0}, t[18];
    e[0] = e[8] = e[16] = 1.0;
    for (int n = 16; n >= 1; --n) {
        cm_mul(a, e, t);
        double inv = 1.0 / (double)n;
        for (int k = 0; k < 18; ++k) e[k] = t[k] * inv;
        e[0] += 1.0;
        e[8] += 1.0;
        e[16] += 1.0;
    }
    for (int s = 0; s < sq; ++s) {
        cm_mul(e, e, t);
        memcpy(e, t, sizeof(t));
    }
    reunitarise_rows(e);
    memcpy(m, e, sizeof(e));
}

static inline int64_t nsites(const int32_t *d) {
    return (int64_t)d[0] * d[1] * d[2] * d[3];
}

/* Links for sites whose t lies in [t0, t1); out holds (t1-t0)*L^3 sites,
 * out[(s - t0*Lx*Ly*Lz)*72 + mu*18 + ...].  kind 0: Haar QR; kind 1: exp. */
int synth_gauge(const int32_t *dims, uint64_t seed, int kind, double eps, int32_t t0,
                int32_t t1, double *out) {
    if (kind != 0 && kind != 1) return -1;
    int64_t v3 = (int64_t)dims[0] * dims[1] * dims[2];
    int64_t s0 = (int64_t)t0 * v3, s1 = (int64_t)t1 * v3;
#pragma omp parallel for schedule(static)
    for (int64_t s = s0; s < s1; ++s) {
        for (int mu = 0; mu < 4; ++mu) {
            rng_t r;
            rng_init(&r, link_key(seed, (uint64_t)s, mu));
            double *m = out + (s - s0) * 72 + mu * 18;
            if (kind == 0)
                draw_haar_su3(&r, m);
            else
                draw_exp_su3(&r, eps, m);
        }
    }
    return 0;
}

/* Identity links (free field). */
int synth_gauge_unit(const int32_t *dims, double *out) {
    int64_t v = nsites(dims);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < v; ++s) {
        double *m = out + s * 72;
        memset(m, 0, 72 * sizeof(double));
        for (int mu = 0; mu < 4; ++mu) m[mu * 18 + 0] = m[mu * 18 + 8] = m[mu * 18 + 16] = 1.0;
    }
    return 0;
}

/* Gaussian spinor: every real and imaginary component N(0,1), drawn per site
 * in the order spin, colour, re, im.  Sites [s0, s1). */
int synth_gaussian_spinor(uint64_t seed, int64_t s0, int64_t s1, double *out) {
#pragma omp parallel for schedule(static)
    for (int64_t s = s0; s < s1; ++s) {
        rng_t r;
        rng_init(&r, site_key(seed, (uint64_t)s));
        double *p = out + (s - s0) * 24;
        for (int k = 0; k < 24; ++k) p[k] = rng_normal(&r);
    }
    return 0;
}

/* One Haar SU(3) matrix per site: a random gauge transformation G(x). */
int synth_gauge_rotation(uint64_t seed, int64_t nsite, double *out) {
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < nsite; ++s) {
        rng_t r;
        rng_init(&r, site_key(seed ^ 0x5851F42D4C957F2DULL, (uint64_t)s));
        draw_haar_su3(&r, out + s * 18);
    }
    return 0;
}

/* First n raw SplitMix64 outputs for a key (pins the generator itself). */
int synth_splitmix_stream(uint64_t key, int64_t n, uint64_t *out) {
    rng_t r;
    rng_init(&r, key);
    for (int64_t i = 0; i < n; ++i) out[i] = rng_u64(&r);
    return 0;
}
