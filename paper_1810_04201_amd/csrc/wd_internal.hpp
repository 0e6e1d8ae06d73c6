// Internal declarations shared by the kernels (.hip) and the host runtime
// (.cpp) of libwdirac.  Nothing here is exported; the ABI is include/wd.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <cstdlib>

#include "wd.h"

namespace wd {

// ------------------------------------------------------------------ layout
//
// Site order.  Internal fields do not use the canonical lexicographic order.
// The lattice is cut into bricks of tx * ty * tz sites (divisors of Lx, Ly,
// Lz); a brick column is the run of Lt bricks that share the same (x, y, z)
// ranges, one per time slice.  Internal site index
//     i = ((column * Lt + t) * bvol) + x % tx + tx * (y % ty + ty * (z % tz)),
//     column = x / tx + ncx * (y / ty + ncy * (z / tz)).
// A sweep in this order marches t inside each column, so a site's t-1
// neighbour was touched one brick (bvol sites) earlier; x, y and z
// neighbours are inside the brick except on its faces.
//
// Entries.  Spinor fields hold nrhs right-hand sides one after another, each
// padded to whole tiles: entry e = rhs * stride + i with stride = V rounded
// up to a multiple of 64.  Kernels take the right-hand side from the
// workgroup index, so one workgroup touches one rhs, a frozen rhs costs its
// workgroups nothing, and the workgroups of different rhs that share sites
// (and therefore links) can be scheduled side by side.
//
// Tiles.  Every field is an array of tiles of 64 consecutive entries (sites
// for links).  Inside a tile each component plane is one contiguous run of
// 64 elements of 16 bytes (8 for binary16 links), so a wave of 64 lanes moves
// one aligned 1 KiB block per load and the planes of neighbouring entries
// never alias in the caches:
//   spinor WD_F64: 12 planes of double2 (complex component k = 3 spin + colour)
//          WD_F32:  6 planes of float4  (components 2j, 2j+1 in plane j)
//          WD_F16:  3 planes of 4 x half2 (components 4j..4j+3) followed by
//                   64 float scales (the entry's max |real or imag part|)
//   links  F64-18: 36 planes of double2 (plane 9 mu + 3 a + b of U_mu)
//          F32-12: 12 planes of float4  (plane 3 mu + j: entries 2j, 2j+1 of
//                  rows 0 and 1)
//          F16-12: 12 planes of 2 x half2 (same entries, 8-byte elements)
//          F64-12: 24 planes of double2 (plane 6 mu + k: entry k of rows 0
//                  and 1); kept beside F64-18 when every link is special
//                  unitary to rounding
//          F16-8:  4 planes of 8 halves (plane mu; the 8-real form of
//                  Link<kLinkF16R8>), in place of F16-12 on lattices
//                  created with WD_F16_LINKS_8
// Row 2 of the 12-real forms is rebuilt as conj(row0 x row1), which is exact
// for special unitary links; the antiperiodic boundary sign is therefore
// never folded into stored links but applied to the hop result.

constexpr int kNComp = 12;  // 4 spins x 3 colours

// Precision of the inner solver's x and r beside binary16 p and t: float32,
// or (WD_F16_XR16=1) binary16 with a site scale like p.  Float64 and float32
// inner solves keep x and r in their own precision.
#ifndef WD_F16_XR16
#define WD_F16_XR16 0
#endif
constexpr int kF16XrPrec = WD_F16_XR16 ? WD_F16 : WD_F32;
__host__ __device__ constexpr int xr_prec_of(int prec) {
    return prec == WD_F16 ? kF16XrPrec : prec;
}
constexpr int kTile = 64;   // entries per tile

__host__ __device__ inline size_t tiles_of(int64_t n) { return (size_t)((n + kTile - 1) / kTile); }

__host__ __device__ inline size_t spinor_tile_bytes(int prec) {
    return prec == WD_F64 ? 12u * 1024u : (prec == WD_F32 ? 6u * 1024u : 3u * 1024u + 256u);
}

inline size_t spinor_bytes(int prec, int64_t n) { return tiles_of(n) * spinor_tile_bytes(prec); }

// link form of float64 links stored as 12 reals (the other forms are named
// by their precision)
constexpr int kLinkF64R12 = 3;
// link form of binary16 links stored as 8 reals (lattice flag
// WD_F16_LINKS_8), in place of the 12-real binary16 form
constexpr int kLinkF16R8 = 4;
// largest |row 2 - conj(row 0 x row 1)| of a link that may be stored as 12
// reals: a few hundred times the rounding of a special unitary matrix
constexpr double kSu3Tol = 1e-14;

inline size_t gauge_tile_bytes(int form) {
    switch (form) {
        case WD_F64: return 36u * 1024u;
        case WD_F32: return 12u * 1024u;
        case WD_F16: return 12u * 512u;
        case kLinkF16R8: return 4u * 1024u;
        default: return 24u * 1024u;  // kLinkF64R12
    }
}

inline size_t gauge_bytes(int prec, int64_t V) { return tiles_of(V) * gauge_tile_bytes(prec); }

struct Geom {
    int L[4];  // Lx, Ly, Lz, Lt
    int V;
    int antiperiodic;
    int f16_links8;     // binary16 links in the 8-real form (host-side choice)
    int tx, ty, tz;     // brick extents (divisors of Lx, Ly, Lz)
    int ncx, ncy, ncz;  // Lx / tx, Ly / ty, Lz / tz
    int bvol;           // tx * ty * tz
};

// storage form of a lattice's links for a precision (the float64 12-real
// form is chosen separately, where the links are special unitary)
inline int link_form(const Geom &g, int prec) {
    return prec == WD_F16 && g.f16_links8 ? kLinkF16R8 : prec;
}

// internal site index -> lattice coordinates
__host__ __device__ inline void coords_of(const Geom &g, int i, int &x, int &y, int &z, int &t) {
    const int local = i % g.bvol;
    const int ct = i / g.bvol;
    t = ct % g.L[3];
    int col = ct / g.L[3];
    const int bx = col % g.ncx;
    col /= g.ncx;
    const int by = col % g.ncy, bz = col / g.ncy;
    const int xl = local % g.tx;
    const int q = local / g.tx;
    x = bx * g.tx + xl;
    y = by * g.ty + q % g.ty;
    z = bz * g.tz + q / g.ty;
}

// lattice coordinates -> internal site index
__host__ __device__ inline int index_of(const Geom &g, int x, int y, int z, int t) {
    const int bx = x / g.tx, by = y / g.ty, bz = z / g.tz;
    const int col = bx + g.ncx * (by + g.ncy * bz);
    return (col * g.L[3] + t) * g.bvol + (x - bx * g.tx) +
           g.tx * ((y - by * g.ty) + g.ty * (z - bz * g.tz));
}

// canonical (lexicographic, x fastest) site of lattice coordinates
__host__ __device__ inline int lex_of(const Geom &g, int x, int y, int z, int t) {
    return x + g.L[0] * (y + g.L[1] * (z + g.L[2] * t));
}

// the eight neighbours of internal site i (x+, x-, y+, y-, z+, z-, t+, t-)
// and whether the t hops cross the time boundary
struct Nbrs {
    int xp, xm, yp, ym, zp, zm, tp, tm;
    bool cross_tp, cross_tm;
};

// one spatial direction: local offset inside the brick, or a step to the
// neighbouring column (periodic in the column index) on a brick face
__host__ __device__ inline void nbr_dir(int i, int l, int tl, int b, int nb, int lstride,
                                        int cstride, int &plus, int &minus) {
    plus = l < tl - 1 ? i + lstride
                      : i - (tl - 1) * lstride + (b == nb - 1 ? -(nb - 1) : 1) * cstride;
    minus = l > 0 ? i - lstride : i + (tl - 1) * lstride + (b == 0 ? (nb - 1) : -1) * cstride;
}

__host__ __device__ inline Nbrs neighbours(const Geom &g, int i) {
    const int Lt = g.L[3];
    const int local = i % g.bvol;
    const int ct = i / g.bvol;
    const int t = ct % Lt;
    int col = ct / Lt;
    const int bx = col % g.ncx;
    col /= g.ncx;
    const int by = col % g.ncy, bz = col / g.ncy;
    const int xl = local % g.tx;
    const int q = local / g.tx;
    const int yl = q % g.ty, zl = q / g.ty;
    const int cx = Lt * g.bvol;  // index stride of one column
    Nbrs n;
    nbr_dir(i, xl, g.tx, bx, g.ncx, 1, cx, n.xp, n.xm);
    nbr_dir(i, yl, g.ty, by, g.ncy, g.tx, g.ncx * cx, n.yp, n.ym);
    nbr_dir(i, zl, g.tz, bz, g.ncz, g.tx * g.ty, g.ncx * g.ncy * cx, n.zp, n.zm);
    n.tp = t == Lt - 1 ? i - (Lt - 1) * g.bvol : i + g.bvol;
    n.tm = t == 0 ? i + (Lt - 1) * g.bvol : i - g.bvol;
    n.cross_tp = t == Lt - 1;
    n.cross_tm = t == 0;
    return n;
}

// Even-odd halves.  With an even brick x extent the two sites 2h and 2h+1
// of the internal order differ only in x by one, so they have opposite
// parity (x+y+z+t) mod 2.  A half field of parity p stores at entry h the
// member of pair h with that parity; the half index of any site is its
// internal index >> 1, so neighbours in a half field are found from the
// full-lattice neighbour arithmetic.
__host__ __device__ inline int site_of_half(const Geom &g, int h, int p) {
    const int i0 = 2 * h;  // even x inside the brick (tx even), so x is even
    const int ct = i0 / g.bvol, local = i0 - ct * g.bvol;
    const int t = ct % g.L[3];
    int col = ct / g.L[3];
    col /= g.ncx;
    const int by = col % g.ncy, bz = col / g.ncy;
    const int q = local / g.tx;
    const int y = by * g.ty + q % g.ty, z = bz * g.tz + q / g.ty;
    return i0 + ((y + z + t + p) & 1);
}

inline bool eo_supported(const Geom &g) { return (g.tx & 1) == 0; }

struct FieldRef {
    int prec;
    int nrhs;
    int V;       // sites per rhs
    int stride;  // entries per rhs: V rounded up to a multiple of 64
    void *data;  // tiles
};

__host__ __device__ inline int rhs_stride(int V) { return (int)(tiles_of(V) * kTile); }

// bytes of a field of nrhs right-hand sides on V sites
inline size_t field_data_bytes(int prec, int V, int nrhs) {
    return tiles_of(V) * (size_t)nrhs * spinor_tile_bytes(prec);
}

// ------------------------------------------------------------------ solver state
//
// One RhsState per right-hand side lives in device memory.  The kernels read
// alpha/beta/active from it and the reduction finaliser (run by the last
// block of a reducing kernel) writes it, so a CG iteration needs no host
// round trip.  A frozen rhs (active == 0) is skipped by every kernel, which
// makes iterations enqueued after convergence exact no-ops.
struct RhsState {
    double rr;       // |r|^2 of the current (iterated) residual
    double rr0;      // |b'|^2, b' = D^dag b
    double rr_prev;  // |r|^2 before the last update (for beta at a reliable update)
    double rr_max;   // max |r|^2 since the last reliable update
    double alpha;
    double beta;
    double tt;       // |D p|^2
    double rr_true;  // last FP64 true residual |b' - D^dag D x|^2
    double aux;      // scratch sum (|b|^2, |b - D x|^2)
    double aux2;
    int active;      // iterating
    int converged;   // FP64 true residual met the tolerance
    int trigger;     // frozen, waiting for a reliable update
    int failed;      // WD_ERR_NUMERIC / WD_ERR_NOCONV or 0
    int iters;       // CG iterations done
    int since;       // iterations since the last reliable update
    int updates;     // reliable updates (true-residual recomputations)
    int restarted;   // the last reliable update restarted the recursion (until
                     // the next inner iteration): r_lo and p are to be reset
    int pend;        // x lags one step (see SolveCtl::lag_x) and this rhs froze
                     // with alpha p not yet in x_lo: the reliable update adds it
};

struct BatchState {
    int n_active;   // rhs still iterating (grid-uniform early-exit flag)
    int n_trigger;  // rhs frozen and waiting for a reliable update
    int n_done;     // rhs converged or failed
    int pad;
};

// Optional gating of a kernel on the solver state, uniform over the launch
// (batch) and over a workgroup (rhs):
//   GATE_ACTIVE   inner iterations: off when no rhs is iterating; rhs with
//                 active != 0.
//   GATE_TRIGGER  a reliable update: off unless every unfinished rhs is
//                 frozen and at least one waits for it; rhs with trigger set
//                 (not converged).
//   GATE_RESTART  the reset of r_lo and p after a reliable update: rhs the
//                 update restarted.
// batch == nullptr: no batch test; st == nullptr: every rhs.
enum GateMode { GATE_ACTIVE = 0, GATE_TRIGGER = 1, GATE_RESTART = 2 };

struct Gate {
    const RhsState *st;
    const BatchState *batch;
    int mode;
};

// Halo exchange for a lattice that is one t-slab of a larger one (one slab
// per GPU).  Face site f = column * bvol + local site of a brick slice
// (V / Lt of them, the same order on every slab of the same shape).  On the
// wire a face is the projected half-spinor (1 +- gamma_t) psi of a boundary
// slice: per rhs 6 planes of V / Lt double2, element ((rhs * 6 + k) * (V / Lt)
// + f).  The receiver expands it into spinor tiles whose spins 0 and 1 hold
// the half-spinor and spins 2 and 3 are zero, which the t projector maps
// back to the same half-spinor exactly, so the stencil's code reads a staged
// face like a slice:
//   prev / next: staged faces (float64 spinor tiles of V / Lt sites, nrhs)
//   links:       U_t(x, -1), the links entering from the previous slab
//                (float64 gauge tiles of V / Lt sites, mu = 3 planes)
//   first, last: this slab holds global t = 0 / t = T - 1 (antiperiodic sign)
// The CG residual update r -= alpha q done by the stencil that forms
// q = A p, so q is never stored (alpha from the rhs's state); x += alpha p
// then follows in the p update (launch_update_xp)
struct XrArgs {
    FieldRef r;
};

struct Halo {
    const void *prev;
    const void *next;
    const void *links;
    int first, last;
    // the chunks of t slices a launch covers: chunk cfirst + k * cstep for
    // the launch's k-th chunk (all chunks: 0, 1); region selects them in
    // launch_dslash_halo (0 all, 1 interior, 2 the two holding the slab ends)
    int region, cfirst, cstep;
};

struct SolveCtl {
    double tol2;      // tol^2: converged when rr <= tol2 * rr0
    double delta2;    // reliable trigger when rr < delta2 * rr_max
    int max_iter;
    int max_inner;    // reliable update at least every max_inner iterations (0: never)
    int nrhs;
    int mixed;        // 1: inner iterations in low precision
    int lag_x;        // 1: x += alpha p is done by the next p update (the
                      // stencil that forms A p only updates r)
};

enum RedMode {
    RED_NONE = 0,
    RED_ALPHA = 1,   // total = |D p|^2 -> alpha = rr / tt
    RED_RR = 2,      // total = |r_new|^2 -> beta, convergence / reliable triggers
    RED_TRUE = 3,    // total = |b' - A x|^2 -> converged, or restart with beta
    RED_B0 = 4,      // total = |b'|^2 -> rr0; start
    RED_AUX = 5,     // total -> aux
    RED_AUX2 = 6,    // total -> aux2
    RED_AUX_ADD = 7, // aux += total
    RED_AUX2_ADD = 8 // aux2 += total
};

struct RedArgs {
    double *partials;    // partials_cap doubles (one per block and rhs)
    int partials_cap;    // launchers never use more blocks * nrhs than this
    RhsState *st;        // nrhs entries
    BatchState *batch;
    SolveCtl ctl;
    int mode;
};

inline int blocks_for(int64_t n, int bs) { return (int)((n + bs - 1) / bs); }

// ------------------------------------------------------------------ launch shapes
//
// Field kernels run a grid of site_blocks(V) x nrhs workgroups of kSiteBlock
// lanes (one lane per site of one rhs) and a reducing one writes a partial
// per workgroup, at index site block * nrhs + rhs.  The time-marching stencil
// runs one workgroup of w = tm_wvol lanes per brick column, chunk of time
// slices, part h of the bvol / w parts of a brick slice, and rhs, and writes
// a partial per part of a brick slice, at index
// ((column * Lt + t) * (bvol / w) + h) * nrhs + rhs.  The solver sizes its
// partial buffer from these same functions.

constexpr int kSiteBlock = 256;

inline int site_blocks(int V) { return blocks_for(V, kSiteBlock); }

// largest workgroup (part of a brick slice) of the time-marching stencil
#ifndef WD_TM_MAXB
#define WD_TM_MAXB 512
#endif
constexpr int kTmMaxBlock = WD_TM_MAXB;

// any brick of whole tiles: a workgroup takes a part of at most kTmMaxBlock
// sites (tm_wvol)
inline bool tm_eligible(const Geom &g) { return g.bvol % 64 == 0; }

// sites per marching workgroup: a contiguous part of n sites of a brick
// slice (a multiple of 64 dividing n).  float64 takes parts of 192 where they
// divide n: two such workgroups, each with two 36 KiB LDS slice images, share
// a CU and fill each other's per-step barrier waits (measured at 48^3 x 96
// against whole 384-site slices, one workgroup per CU); else up to 384.  The
// float kernels run four waves per SIMD and do best with at most 256.
inline int part_sites(int n, int prec) {
    if (prec == WD_F64 && n % 192 == 0) return 192;
    // WD_PART_CAP overrides the float kernels' cap (tuning; at most the
    // marching stencil's largest workgroup)
    static const int lo_cap = [] {
        const char *e = getenv("WD_PART_CAP");
        const int v = e ? atoi(e) : 0;
        return v >= 64 && v <= kTmMaxBlock ? v : 256;
    }();
    const int cap = prec == WD_F64 ? 384 : lo_cap;
    if (n <= cap) return n;
    // the largest multiple of 64 within the cap that divides n
    for (int w = cap - cap % 64; w >= 64; w -= 64)
        if (n % w == 0) return w;
    return n;
}

inline int tm_wvol(const Geom &g, int prec) { return part_sites(g.bvol, prec); }

// entries per workgroup of the marching half-field stencil: the same rule
// on a half slice (bvol / 2 entries of one parity); 0 where a half slice is
// not whole tiles
inline int eo_wvol(const Geom &g, int prec) {
    const int hvol = g.bvol / 2;
    if (hvol % 64) return 0;
    return part_sites(hvol, prec);
}

// time slices per chunk: enough workgroups over all rhs to fill the chip (a
// multiple of 8 chunks where the extent allows); env_chunk > 0 overrides
// (tuning)
inline int tm_chunk_len(const Geom &g, int nrhs, int env_chunk) {
    const int Lt = g.L[3];
    if (env_chunk > 0) return env_chunk < Lt ? env_chunk : Lt;
    const int ncols = g.V / (Lt * g.bvol);
    int nch = 8;
    while (nch < Lt && ncols * nch * nrhs < 2048) nch += 8;
    if (nch > Lt) nch = Lt;
    return (Lt + nch - 1) / nch;
}

// column chunks of the time-marching stencil (each runs bvol / w
// workgroups per rhs)
inline int tm_blocks(const Geom &g, int chunk_len) {
    const int ncols = g.V / (g.L[3] * g.bvol);
    return ncols * ((g.L[3] + chunk_len - 1) / chunk_len);
}

// partial sums any reducing launch on this geometry may write (the time
// marching stencil writes V / w <= V / 64 per rhs)
inline int64_t reduce_partials_cap(const Geom &g, int nrhs) {
    int64_t nb = site_blocks(g.V);
    if (tm_eligible(g)) {
        const int64_t tmb = (int64_t)g.V / 64;
        if (tmb > nb) nb = tmb;
    }
    return (nb + 1) * nrhs;
}

// ------------------------------------------------------------------ brick choice

// Brick extents.  Preferred: whole x rows (the x neighbours and the
// backward x links stay inside the brick), then the largest volume that is a
// multiple of 64 (a brick slice is whole tiles): 768 sites where the lattice
// has at least 128 such brick columns to spread over the chip (48^3 x 96:
// float64 marches four 192-site parts of each slice, the float kernels three
// of 256; measured 2-4% faster than 384-site bricks), else at most 256; then
// the fewest neighbours per site outside the float64 workgroup's part of the
// slice (brick faces, and the boundaries between parts), then the thinner y
// extent.  Lattices too small for a 64-site brick take whole x rows with the
// largest y/z divisors up to 8 and 4.
// WD_BRICK="tx,ty,tz" overrides the choice (tuning).
inline int largest_divisor_le(int n, int cap) {
    for (int d = cap < n ? cap : n; d >= 1; --d)
        if (n % d == 0) return d;
    return 1;
}

// neighbours (x, y, z; both ways) that a brick slice of a x b x c sites in
// parts of w consecutive local sites reads from outside each site's own part,
// times 240 / (a b c): a direction the brick spans whole wraps inside it
inline int part_faces(const int L[4], int a, int b, int c, int w) {
    const int e[3] = {a, b, c};
    long long out = 0;
    for (int s = 0; s < a * b * c; ++s) {
        const int q[3] = {s % a, (s / a) % b, s / (a * b)};
        for (int d = 0; d < 3; ++d)
            for (int step = -1; step <= 1; step += 2) {
                int r[3] = {q[0], q[1], q[2]};
                r[d] += step;
                if (r[d] < 0 || r[d] >= e[d]) {
                    if (e[d] < L[d]) {
                        ++out;  // a brick face
                        continue;
                    }
                    r[d] = (r[d] + e[d]) % e[d];
                }
                if ((r[0] + a * (r[1] + b * r[2])) / w != s / w) ++out;
            }
    }
    return (int)(out * 240 / (a * b * c));
}

inline void choose_bricks(Geom &g) {
    int bx = 0, by = 0, bz = 0;
    long long best = 0;
    const bool big_ok = (long long)g.V / ((long long)g.L[3] * 768) >= 128;
    for (int a = 1; a <= g.L[0]; ++a) {
        if (g.L[0] % a) continue;
        for (int b = 1; b <= g.L[1]; ++b) {
            if (g.L[1] % b) continue;
            for (int c = 1; c <= g.L[2]; ++c) {
                if (g.L[2] % c) continue;
                const int v = a * b * c;
                if (v % 64 || (v > 256 && !(v == 768 && big_ok))) continue;
                if (a & 1) continue;  // even-odd halves pair x neighbours
                const int faces = part_faces(g.L, a, b, c, part_sites(v, WD_F64));
                const long long score = (a == g.L[0] ? (1LL << 40) : 0) + ((long long)v << 20) +
                                        (long long)(2048 - faces) * 128 + (127 - b);
                if (score > best) {
                    best = score;
                    bx = a;
                    by = b;
                    bz = c;
                }
            }
        }
    }
    if (!best) {
        bx = g.L[0];
        by = largest_divisor_le(g.L[1], 8);
        bz = largest_divisor_le(g.L[2], 4);
    }
    if (const char *e = getenv("WD_BRICK")) {
        int a = 0, b = 0, c = 0;
        if (sscanf(e, "%d,%d,%d", &a, &b, &c) == 3 && a >= 1 && b >= 1 && c >= 1 &&
            g.L[0] % a == 0 && g.L[1] % b == 0 && g.L[2] % c == 0) {
            bx = a;
            by = b;
            bz = c;
        }
    }
    g.tx = bx;
    g.ty = by;
    g.tz = bz;
    g.ncx = g.L[0] / bx;
    g.ncy = g.L[1] / by;
    g.ncz = g.L[2] / bz;
    g.bvol = bx * by * bz;
}

// ------------------------------------------------------------------ launchers
// (defined in the .hip files; all stream-ordered, no host synchronisation)

// canonical float64 links -> F64-18 tiles (brick order)
void launch_pack_gauge_f64(const double *canon, void *g64, const Geom &g, hipStream_t s);
// F64-18 tiles -> 12-real F32, F16 or F64 (form kLinkF64R12) tiles
void launch_gauge_lo(const void *g64, void *glo, int form, int V, hipStream_t s);
// *maxbits = max(*maxbits, largest |row 2 - conj(row 0 x row 1)| over the
// F64-18 links) as the bit pattern of a non-negative double (NaN counts as
// infinity); *maxbits must be set beforehand
void launch_su3_check(const void *g64, int V, unsigned long long *maxbits, hipStream_t s);

// canonical [rhs][V][12] float64 <-> field (format conversion + reorder)
void launch_import(const double *canon, FieldRef f, const Geom &g, hipStream_t s);
void launch_export(FieldRef f, double *canon, const Geom &g, hipStream_t s);
// dst = src with a format conversion (same nrhs); gated rhs only
void launch_convert(FieldRef src, FieldRef dst, Gate gate, hipStream_t s);
void launch_zero(FieldRef f, hipStream_t s);
// even-odd halves (V / 2 sites each, parity p): links of the parity-p sites
// from the F64-18 tiles, in the half layout and link form `form`
void launch_gauge_split(const void *g64, void *half, int form, int p, const Geom &g,
                        hipStream_t s);
// canonical [rhs][V][12] float64 <-> half field of parity p (sites of the
// other parity untouched on export)
void launch_import_half(const double *canon, FieldRef f, int p, const Geom &g, hipStream_t s);
void launch_export_half(FieldRef f, double *canon, int p, const Geom &g, hipStream_t s);
// out_p = cs * c_p - k * H_{p,1-p} in_{1-p} on half fields (H the hopping
// sum of Eq. (1), projectors exchanged for dagger; c.data == nullptr: no
// c term), links gp of parity p and gq of parity 1 - p; red fuses |out|^2;
// r12: float64 halves in the F64-12 form
void launch_hop_half(const Geom &g, const void *gp, const void *gq, int p, double k,
                     double cs, int dagger, FieldRef in, FieldRef c, FieldRef out,
                     const RedArgs *red, Gate gate, hipStream_t s, bool r12 = false);
// the same with c present and its output q consumed where it is formed:
// r -= alpha q (XrArgs on half fields), |r|^2 reduced with red.mode and
// finalised; q is not stored
void launch_hop_half_xr(const Geom &g, const void *gp, const void *gq, int p, double k,
                        double cs, int dagger, FieldRef in, FieldRef c, const XrArgs &xr,
                        const RedArgs &red, Gate gate, hipStream_t s, bool r12 = false);

// halo exchange (float64): the two faces of in for the neighbouring slabs
// (to_prev: (1 -+ gamma_t) psi(x, 0) for its forward hop; to_next: the
// backward projection of psi(x, Lt-1)), wire format
void launch_halo_pack(const Geom &g, int dagger, FieldRef in, double *to_prev, double *to_next,
                      hipStream_t s);
// wire-format face -> staged face (spinor tiles of V / Lt sites)
void launch_halo_stage(const Geom &g, const double *wire, FieldRef staged, hipStream_t s);
// canonical U_t(x, -1) [Lx*Ly*Lz][3][3][2] -> gauge tiles over face sites
void launch_halo_links(const Geom &g, const double *canon, void *links, hipStream_t s);
// the marching stencil with t hops across the slab ends from staged faces
bool halo_supported(const Geom &g);
void launch_dslash_halo(const Geom &g, const void *gauge, double kappa, int dagger, FieldRef in,
                        FieldRef out, const Halo &halo, hipStream_t s,
                        const void *g12 = nullptr);

// x64 += xlo ; xlo = 0: gate.mode GATE_TRIGGER for the rhs a reliable update
// takes (with its batch test), otherwise every rhs that has not converged
// A pending alpha p (RhsState::pend) is added too: x64 += xlo + alpha p.
void launch_accum_zero(FieldRef x64, FieldRef xlo, FieldRef p, Gate gate, hipStream_t s);

// out = D in (dagger 0) or D^dag in (dagger 1); red != nullptr fuses the
// reduction of |out|^2 with red->mode
// g12: the F64-12 form of the same float64 links, read instead of gauge by
// the marching stencil (nullptr: F64-18 only)
void launch_dslash(const Geom &g, const void *gauge, double kappa, int dagger, FieldRef in,
                   FieldRef out, const RedArgs *red, Gate gate, hipStream_t s,
                   const void *g12 = nullptr);
// q = D in (or D^dag in) consumed where it is formed: r -= alpha q, |r|^2
// reduced with red.mode (RED_RR) and finalised; q is not stored.  Only the marching stencil does this: returns false (nothing
// launched) where it does not run
bool launch_dslash_xr(const Geom &g, const void *gauge, double kappa, int dagger, FieldRef in,
                      const XrArgs &xr, const RedArgs &red, Gate gate, hipStream_t s,
                      const void *g12 = nullptr);
bool dslash_xr_supported(const Geom &g, int prec, int nrhs, int partials_cap);

// x += alpha p ; r -= alpha Ap ; reduce |r|^2 (red.mode = RED_RR); active rhs
void launch_update_xr(FieldRef x, FieldRef r, FieldRef p, FieldRef Ap, const RedArgs &red,
                      Gate gate, hipStream_t s);
// p = r + beta p for active rhs
void launch_update_p(FieldRef p, FieldRef r, Gate gate, hipStream_t s);
// x += alpha p ; p = r + beta p (active rhs): the x update lagged behind the
// r update of a stencil with XrArgs
void launch_update_xp(FieldRef x, FieldRef p, FieldRef r, Gate gate, hipStream_t s);
// r = b - Ax (Ax.data == nullptr: r = b) in float64, reduce |r|^2 with red.mode
void launch_residual(FieldRef r, FieldRef b, FieldRef Ax, const RedArgs &red, Gate gate,
                     hipStream_t s);
// reduce |f|^2 (any precision) with red.mode
void launch_norm(FieldRef f, const RedArgs &red, hipStream_t s);
// phase 2 of a reduction: one block sums the nb per-block partials in a fixed
// order and runs the finaliser; gate_mode >= 0: skipped when the producing
// kernel's batch gate (GateMode) was off, -1: always runs
void launch_finalize(const RedArgs &red, int nb, int gate_mode, hipStream_t s);
// zero the states and the batch counters
void launch_init_state(RhsState *st, BatchState *batch, int nrhs, hipStream_t s);
// after a reliable update, for the rhs it restarted (gate GATE_RESTART):
// p = r at the first update, p = r + beta p afterwards
void launch_restart_p(FieldRef p, FieldRef r, Gate gate, hipStream_t s);

}  // namespace wd
