// Internal declarations shared by the kernels (.hip) and the host runtime
// (.cpp) of libwdirac.  Nothing here is exported; the ABI is include/wd.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "wd.h"

namespace wd {

// ------------------------------------------------------------------ layout
//
// Spinor fields are site-major structure-of-arrays.  An entry index
// i = s * nrhs + rhs runs over sites and right-hand sides (rhs fastest), and
// the 12 complex components k = 3 * spin + colour are spread over planes of
// 16-byte vectors so that one lane moves 16 bytes per load:
//   WD_F64: 12 planes of double2 (one complex per plane)
//   WD_F32:  6 planes of float4  (components 2j, 2j+1 in plane j)
//   WD_F16:  3 planes of 4 x half2 (components 4j..4j+3 in plane j) plus one
//            float plane holding the site scale (max |real or imag part|)
// Plane p of a field with n entries starts at byte p * n * 16.
//
// Gauge links: for each direction mu a group of planes indexed by site:
//   F64-18: 9 planes of double2 (entry a*3+b of U_mu(s))
//   F32-12: 3 planes of float4  (rows 0 and 1: entries 0..5, two per plane)
//   F16-12: 3 planes of 2 x half2 (rows 0 and 1, two entries per plane)
// Row 2 of the 12-real forms is rebuilt as conj(row0 x row1), which is exact
// for special unitary links; the antiperiodic boundary sign is therefore
// never folded into stored links but applied to the hop result.

constexpr int kNComp = 12;  // 4 spins x 3 colours

inline int planes_for(int prec) { return prec == WD_F64 ? 12 : (prec == WD_F32 ? 6 : 3); }

inline size_t spinor_bytes(int prec, int64_t n) {
    size_t b = (size_t)planes_for(prec) * 16u * (size_t)n;
    if (prec == WD_F16) b += 4u * (size_t)n;
    return b;
}

inline size_t gauge_bytes(int prec, int64_t V) {
    size_t per_link = prec == WD_F64 ? 144u : (prec == WD_F32 ? 48u : 24u);
    return (size_t)4 * per_link * (size_t)V;
}

struct Geom {
    int L[4];
    int V;
    int antiperiodic;
};

struct FieldRef {
    int prec;
    int nrhs;
    int n;        // V * nrhs entries per plane
    void *data;   // planes
    float *scale; // WD_F16 only (n floats)
};

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
    int pad;
};

struct BatchState {
    int n_active;   // rhs still iterating (grid-uniform early-exit flag)
    int n_trigger;  // rhs frozen and waiting for a reliable update
    int n_done;     // rhs converged or failed
    int pad;
};

// Optional gating of a kernel on the solver state: a kernel returns at once
// when batch->n_active == 0 and skips rhs whose st[rhs].active == 0.
struct Gate {
    const RhsState *st;
    const BatchState *batch;
};

struct SolveCtl {
    double tol2;      // tol^2: converged when rr <= tol2 * rr0
    double delta2;    // reliable trigger when rr < delta2 * rr_max
    int max_iter;
    int max_inner;    // reliable update at least every max_inner iterations (0: never)
    int nrhs;
    int mixed;        // 1: inner iterations in low precision
};

enum RedMode {
    RED_NONE = 0,
    RED_ALPHA = 1,   // total = |D p|^2 -> alpha = rr / tt
    RED_RR = 2,      // total = |r_new|^2 -> beta, convergence / reliable triggers
    RED_TRUE = 3,    // total = |b' - A x|^2 -> converged, or restart with beta
    RED_B0 = 4,      // total = |b'|^2 -> rr0; start
    RED_AUX = 5,     // total -> aux
    RED_AUX2 = 6,    // total -> aux2
};

struct RedArgs {
    double *partials;    // >= nblocks * nrhs doubles (one per block and rhs)
    RhsState *st;        // nrhs entries
    BatchState *batch;
    SolveCtl ctl;
    int mode;
};

// block size for nrhs right-hand sides: nrhs * S threads with S a power of
// two and at most 256 threads, so every block holds all rhs of its sites and
// the per-rhs tree reduction runs over S site slots.  Whole 64-wide waves for
// nrhs in {1, 2, 3, 4, 6, 8, 12}; the last wave is partly idle otherwise.
inline int block_for_nrhs(int nrhs) {
    if (nrhs < 1 || nrhs > 12) return 0;
    int S = 256;
    while (S * nrhs > 256) S >>= 1;
    return S * nrhs;
}

inline int blocks_for(int64_t n, int bs) { return (int)((n + bs - 1) / bs); }

// ------------------------------------------------------------------ launchers
// (defined in the .hip files; all stream-ordered, no host synchronisation)

void launch_pack_gauge_f64(const double *canon, void *g64, int V, hipStream_t s);
void launch_gauge_lo(const void *g64, void *glo, int prec, int V, hipStream_t s);

void launch_import(const double *canon, FieldRef f, hipStream_t s);
void launch_export(FieldRef f, double *canon, hipStream_t s);
// dst = src with a format conversion (same nrhs); gated rhs only
void launch_convert(FieldRef src, FieldRef dst, Gate gate, hipStream_t s);
void launch_zero(FieldRef f, hipStream_t s);
// x64 += xlo ; xlo = 0 for every rhs that has not converged
void launch_accum_zero(FieldRef x64, FieldRef xlo, const RhsState *st, hipStream_t s);

// out = D in (dagger 0) or D^dag in (dagger 1); red != nullptr fuses the
// reduction of |out|^2 with red->mode
void launch_dslash(const Geom &g, const void *gauge, double kappa, int dagger, FieldRef in,
                   FieldRef out, const RedArgs *red, Gate gate, hipStream_t s);

// x += alpha p ; r -= alpha Ap ; reduce |r|^2 (red.mode = RED_RR); active rhs
void launch_update_xr(FieldRef x, FieldRef r, FieldRef p, FieldRef Ap, const RedArgs &red,
                      Gate gate, hipStream_t s);
// p = r + beta p for active rhs
void launch_update_p(FieldRef p, FieldRef r, Gate gate, hipStream_t s);
// r = b - Ax (Ax.data == nullptr: r = b) in float64, reduce |r|^2 with red.mode
void launch_residual(FieldRef r, FieldRef b, FieldRef Ax, const RedArgs &red, hipStream_t s);
// reduce |f|^2 (any precision) with red.mode
void launch_norm(FieldRef f, const RedArgs &red, hipStream_t s);
// phase 2 of a reduction: one block sums the nb per-block partials in a fixed
// order and runs the finaliser (gated: skip when no rhs is iterating)
void launch_finalize(const RedArgs &red, int nb, bool gated, hipStream_t s);
// zero the states and the batch counters
void launch_init_state(RhsState *st, BatchState *batch, int nrhs, hipStream_t s);
// after a reliable update, for the rhs it restarted (active): p = r at the
// first update, p = r + beta p afterwards
void launch_restart_p(FieldRef p, FieldRef r, Gate gate, hipStream_t s);

}  // namespace wd
