/*
 * wd.h -- C ABI of the MI355X Wilson-Dirac solver library (libwdirac.so).
 *
 * The library applies the Wilson-Dirac operator of the paper "Towards
 * Lattice Quantum Chromodynamics on FPGA devices" (Korcyl & Korcyl), Eq. (1)
 * of Sec. 2.1, with the hopping term taken with a minus sign,
 *
 *   (D psi)(x) = psi(x) - kappa * sum_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu)
 *                                        + (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu) ],
 *
 * gamma_mu as printed in the paper's Appendix A, and solves D x = b by
 * conjugate gradient (Sec. 2.2) on the normal equations D^dag D x = D^dag b.
 * Boundary conditions are periodic in x, y, z and (by default) antiperiodic
 * in t: a hop across the t boundary is multiplied by -1 (Sec. 2.3 allows
 * periodic or antiperiodic conditions).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Lattice extents dims[4] = {Lx, Ly, Lz, Lt}, each even and >= 2; V is
 *   their product, at most 2^28.
 * - Site index s = x + Lx*(y + Ly*(z + Lz*t)); direction mu = 0,1,2,3 =
 *   x,y,z,t (the link arrays U_x..U_t of Sec. 6.2).
 * - Canonical gauge field (caller-owned, DEVICE memory, float64):
 *   U[s][mu][a][b][re,im], 72 doubles per site, U_mu(s) row-major (the
 *   su3_matrix nesting of Sec. 6.1).  Links must be special unitary for the
 *   12-real compressed forms (row 3 is rebuilt as conj(row1 x row2),
 *   Sec. 6.1) to be exact.
 * - Canonical spinor (caller-owned, DEVICE memory, float64):
 *   psi[rhs][s][spin][colour][re,im], 24 doubles per site and right-hand
 *   side (the su3_spinor nesting of Sec. 6.1).
 * - Precision codes select the internal storage/compute format:
 *   WD_F64 (float64 fields and links), WD_F32 (float32 spinors, 12-real
 *   float32 links, float32 arithmetic), WD_F16 (binary16 spinors with a
 *   float32 scale per site, 12-real binary16 links, float32 arithmetic).
 *   Global sums are always accumulated in float64.
 * - `stream` is a hipStream_t (NULL = the null stream).  Unless stated,
 *   calls are stream-ordered and asynchronous with respect to the host.
 * - Every function returns WD_OK (0), WD_PENDING (1) or a negative error
 *   code; wd_last_error() returns a thread-local message for the last
 *   error on the calling thread.  Arguments are validated before any GPU
 *   work is issued; on error nothing is enqueued and outputs are untouched.
 * - Pointers passed in are never freed or retained by the library, except
 *   that b and x given to wd_submit must stay valid until wd_poll returns
 *   something other than WD_PENDING for that ticket.
 */
#ifndef WD_H
#define WD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wd_lattice wd_lattice; /* geometry + resident packed gauge forms */
typedef struct wd_field wd_field;     /* a spinor field in the internal layout */
typedef struct wd_server wd_server;   /* continuous-batching solve server */

enum {
    WD_OK = 0,
    WD_PENDING = 1,
    WD_ERR_ARG = -1,     /* invalid argument */
    WD_ERR_NOMEM = -2,   /* device allocation failed or request exceeds the budget */
    WD_ERR_HIP = -3,     /* a HIP runtime call failed */
    WD_ERR_NOCONV = -4,  /* max_iter reached before the tolerance */
    WD_ERR_NUMERIC = -5, /* NaN/Inf or a zero denominator inside the solve */
    WD_ERR_NOGAUGE = -6, /* operator used before wd_set_gauge */
    WD_ERR_NOTFOUND = -7,/* unknown ticket */
    WD_ERR_STATE = -8    /* call not valid in the object's current state */
};

enum { WD_F64 = 0, WD_F32 = 1, WD_F16 = 2 };

/* Lattice flags.  WD_SIGN_PLUS_KAPPA selects the hopping sign as printed in
 * Eq. (1), D = 1 + kappa * (hops); the default is D = 1 - kappa * (hops).
 * On even lattices the two are related by D_+ = eps D_- eps with
 * eps(x) = (-1)^(x+y+z+t): same spectrum, solutions differ by eps.
 * WD_F16_LINKS_8 stores this lattice's binary16 links (WD_F16 operators and
 * inner solves) as 8 reals per link, 16 bytes, instead of 12 (24 bytes):
 * the parametrisation of a link by 8 real numbers that Sec. 6.1 leaves for
 * later work, in a form whose rebuilt entries stay within a few binary16
 * rounding units (row 0 led by its largest entry, rows 1 and 2 in a pivoted
 * frame orthogonal to it).  Links must be special unitary. */
enum {
    WD_BC_ANTIPERIODIC_T = 1u << 0,
    WD_SIGN_PLUS_KAPPA = 1u << 1,
    WD_F16_LINKS_8 = 1u << 2
};

/* Normal-equation forms of the CG solve (Sec. 2.2), optionally on the
 * even-odd Schur complement: with WD_SOLVE_EVEN_ODD or'ed in, CG runs on
 * M = 1 - D_eo D_oe for the even sites (b^_e = b_e - D_eo b_o) and the odd
 * sites follow as x_o = b_o - D_oe x_e. */
enum {
    WD_FORM_CGNR = 0,          /* D^dag D x = D^dag b */
    WD_FORM_CGNE = 1,          /* the paper's listing: D D^dag y = b, x = D^dag y */
    WD_SOLVE_EVEN_ODD = 1 << 8 /* flag: the same forms with M in place of D */
};

/* ---------------------------------------------------------------- lattice */

/* Create a lattice of extents dims (each even, >= 2).  bc_flags:
 * WD_BC_ANTIPERIODIC_T for antiperiodic t (else periodic everywhere),
 * WD_SIGN_PLUS_KAPPA for the +kappa hopping sign on every operator of this
 * lattice, and WD_F16_LINKS_8 for 8-real binary16 links.
 * *out receives an opaque handle owned by the caller; free it with
 * wd_destroy_lattice.  Allocates no device memory yet. */
int wd_create_lattice(const int32_t dims[4], uint32_t bc_flags, wd_lattice **out);

/* Free the lattice and its packed gauge forms.  WD_ERR_STATE if a server
 * still holds requests on it. */
int wd_destroy_lattice(wd_lattice *lat);

/* Volume V of a lattice (host query). */
int wd_lattice_volume(const wd_lattice *lat, int64_t *volume);

/* Gauge ingest (Sec. 2.3: links are loaded once and stay resident).
 * U: canonical float64 device array (72 doubles per site).  Packs the
 * float64 18-real form now (the low-precision 12-real forms are derived
 * from it on first use).  It also measures how far each link is from
 * special unitary (the largest |row 2 - conj(row 0 x row 1)|, Sec. 6.1's
 * compressed form); if no link is further than 1e-14 (and the device has
 * room for it), the float64 links are kept as 12 reals too, and the float64
 * marching stencils read that form (384 instead of 576 link bytes per site;
 * the rebuilt row agrees to rounding).  Environment WD_LINKS64_12=0 skips
 * the check and the form.
 * The library keeps its own copy; U may be freed after the stream reaches
 * this point.  Synchronises `stream`. */
int wd_set_gauge(wd_lattice *lat, const double *U, void *stream);

/* Float64 link storage chosen by the last wd_set_gauge: *f64_link_reals =
 * 12 or 18 and *su3_deviation = the largest row-2 deviation it measured
 * (-1 if it did not check).  Either pointer may be NULL. */
int wd_lattice_links_info(const wd_lattice *lat, int *f64_link_reals, double *su3_deviation);

/* Bytes of device memory the lattice's packed gauge forms use now. */
int wd_lattice_gauge_bytes(const wd_lattice *lat, size_t *bytes);

/* ---------------------------------------------------------------- operator */

/* out = D in (Eq. (1), minus sign) for one right-hand side, in and out
 * canonical float64 device spinors of V*24 doubles (must not overlap).
 * prec chooses the internal format; for WD_F32/WD_F16 the input is rounded
 * to that format first and the result widened to float64. */
int wd_apply_D(wd_lattice *lat, double kappa, int prec, const double *in, double *out,
               void *stream);

/* out = D^dag in.  D^dag = gamma5 D gamma5 (Sec. 2.2): D with the two spin
 * projectors exchanged. */
int wd_apply_Ddag(wd_lattice *lat, double kappa, int prec, const double *in, double *out,
                  void *stream);

/* Even-odd (Schur complement) operator: out = M in (dagger = 0) or M^dag in
 * (dagger = 1) with M = 1 - D_eo D_oe on the even sites (parity
 * (x+y+z+t) mod 2 = 0), D_eo / D_oe the blocks of D between even and odd
 * sites.  Canonical float64 device spinors [nrhs][V][24]; odd sites of in
 * are ignored and odd sites of out are set to zero.  Needs bricks with an
 * even x extent (the default choice).  Stream-ordered; allocates its
 * workspace stream-ordered. */
int wd_apply_schur(wd_lattice *lat, double kappa, int prec, int dagger, int nrhs,
                   const double *in, double *out, void *stream);

/* Batched form: nrhs (1..12) canonical spinors stacked as [rhs][V][24].  The
 * workgroups of all right-hand sides on the same sites run side by side, so
 * a gauge link is read from HBM about once per site for all of them. */
int wd_apply(wd_lattice *lat, double kappa, int prec, int dagger, int nrhs, const double *in,
             double *out, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): wd_apply
 * with no allocation.  The two internal-layout fields wd_apply allocates
 * live instead in a fixed 128 MiB scratch array that the library holds on
 * each GPU it runs on until the process ends; the call makes no hipMalloc,
 * hipFree or allocating library call.  2 * (internal field bytes of nrhs
 * spinors on V sites) must fit the scratch (e.g. float64 with V * nrhs up to
 * 349,525 sites), else WD_ERR_ARG; the lattice's link form for `prec` must
 * already be resident (float64 always is; float32 and binary16 forms are
 * built by the first wd_apply or solve in that precision), else
 * WD_ERR_STATE.  Every call on one GPU shares that GPU's scratch: calls that
 * overlap on a GPU (different streams, or threads) race.  Stream-ordered;
 * same arguments and results as wd_apply. */
int wd_apply_noalloc(wd_lattice *lat, double kappa, int prec, int dagger, int nrhs,
                     const double *in, double *out, void *stream);

/* --------------------------------------------------- fields (internal layout)
 * A wd_field holds nrhs spinors in the layout the kernels use: sites in
 * brick-column order (bricks of the lattice, each column marching in t),
 * one right-hand side after another (each padded to whole tiles of 64
 * sites), and inside a tile one contiguous run per spin-colour component
 * (plus per-site float32 scales for WD_F16).  The layout is private; import/export convert from/to the
 * canonical order.  Fields time the stencil on resident data and chain
 * operators without the canonical round trip. */
int wd_field_create(wd_lattice *lat, int prec, int nrhs, wd_field **out);
int wd_field_destroy(wd_field *f);
/* canonical float64 [rhs][V][24] (device) -> field, rounding to its format */
int wd_field_import(wd_field *f, const double *canon, void *stream);
/* field -> canonical float64 [rhs][V][24] (device) */
int wd_field_export(const wd_field *f, double *canon, void *stream);
/* out = D in (dagger = 0) or D^dag in (dagger = 1) on fields of the same
 * lattice, precision and nrhs; in and out must be different fields. */
int wd_dslash(wd_lattice *lat, double kappa, int dagger, const wd_field *in, wd_field *out,
              void *stream);

/* ------------------------------------------------------- halo exchange
 * A lattice may be one t-slab of a larger lattice cut along t over several
 * GPUs (one process per GPU, slab r holding global t in [r Lt, (r+1) Lt)).
 * Its stencil then takes the t hops across the slab ends from faces that
 * the neighbouring slabs pack, instead of wrapping around:
 *   wd_set_halo_gauge  once per gauge field: U_t(x, -1), the t links that
 *                      enter this slab from the previous one (the previous
 *                      slab's U_t on its last slice), canonical float64
 *                      device array [Lx*Ly*Lz][3][3][2] (x fastest).
 *   wd_halo_pack       writes this slab's two faces: send_prev goes to the
 *                      previous slab, send_next to the next one.
 *   wd_dslash_halo     out = D in (dagger 0) or D^dag in (dagger 1) on the
 *                      slab, with recv_prev / recv_next the faces received
 *                      from the previous / next slab (packed with the same
 *                      dagger).  WD_HALO_FIRST / WD_HALO_LAST: this slab holds
 *                      global t = 0 / t = T-1, where the antiperiodic sign
 *                      applies.  A single slab with its own faces and
 *                      WD_HALO_FIRST | WD_HALO_LAST is the whole lattice.
 *                      WD_HALO_INTERIOR computes only the slab's interior
 *                      chunks of t slices (those holding neither its first
 *                      nor its last slice) and reads no face, so it may run
 *                      while the faces are in flight (recv_prev / recv_next
 *                      may be NULL); WD_HALO_ENDS then computes the rest.
 *                      The two together write what one call without either
 *                      flag writes, bit for bit.
 * Faces (device, caller-owned): per rhs 6 planes of V/Lt complex float64 (the
 * projected half-spinor of a boundary slice, 96 bytes per face site), sites
 * in the library's internal face order, the same on every slab of one shape.
 * Float64 fields; lattices whose bricks are whole multiples of 64 sites (the
 * marching stencil).  Stream-ordered; wd_dslash_halo allocates its staging
 * stream-ordered. */
enum {
    WD_HALO_FIRST = 1u << 0,
    WD_HALO_LAST = 1u << 1,
    WD_HALO_INTERIOR = 1u << 2,
    WD_HALO_ENDS = 1u << 3
};
int wd_set_halo_gauge(wd_lattice *lat, const double *U_prev, void *stream);
int wd_halo_pack(wd_lattice *lat, int dagger, const wd_field *in, double *send_prev,
                 double *send_next, void *stream);
int wd_dslash_halo(wd_lattice *lat, double kappa, int dagger, const wd_field *in, wd_field *out,
                   const double *recv_prev, const double *recv_next, uint32_t flags,
                   void *stream);

/* ---------------------------------------------------------------- solver */

typedef struct {
    double kappa;              /* hopping parameter */
    double tol;                /* stop when ||r|| <= tol * ||D^dag b|| (CGNR) or
                                  ||b - D x|| <= tol * ||b|| (CGNE) */
    int32_t max_iter;          /* cap on CG iterations (inner iterations for mixed) */
    int32_t prec_inner;        /* WD_F64: plain FP64 CG; WD_F32 / WD_F16: mixed precision */
    int32_t nrhs;              /* 1..12 independent right-hand sides */
    int32_t reliable_max_iter; /* mixed: FP64 reliable update at least this often (<= 0: 50) */
    double reliable_delta;     /* mixed: update when ||r_lo|| < delta * max||r_lo|| (<= 0: 0.1) */
    int32_t x0_given;          /* 1: x holds a starting guess on entry; 0: start from x = 0
                                  (CGNR only: CGNE always starts from y = 0) */
    int32_t form;              /* WD_FORM_CGNR (0) or WD_FORM_CGNE (1), optionally
                                  | WD_SOLVE_EVEN_ODD */
} wd_solve_params;

typedef struct {
    int32_t status;           /* WD_OK, WD_ERR_NOCONV or WD_ERR_NUMERIC for this rhs */
    int32_t iters;            /* CG iterations (inner iterations for mixed) */
    int32_t reliable_updates; /* FP64 true-residual recomputations (incl. the final check) */
    double true_rel_resid;    /* FP64: ||D^dag b - D^dag D x|| / ||D^dag b|| (CGNR),
                                 ||b - D D^dag y|| / ||b|| (CGNE); with
                                 WD_SOLVE_EVEN_ODD the same with M, b^_e, x_e */
    double rel_resid_D;       /* ||b - D x|| / ||b|| in FP64 */
    double seconds;           /* wall time of the solve (submit to completion when served) */
    double queued_seconds;    /* served: submission to admission; 0 for wd_cg_solve */
} wd_solve_info;

/* Solve D x = b by CG on the normal equations (Sec. 2.2) for nrhs
 * right-hand sides (blocking; returns when x is written): D^dag D x = D^dag b
 * (form WD_FORM_CGNR) or, as in the paper's listing, D D^dag y = b with
 * x = D^dag y (WD_FORM_CGNE).  b, x: canonical float64 device spinors
 * [nrhs][V][24].
 * info: host array of nrhs entries.  Returns WD_OK if every rhs converged,
 * else the first failing rhs's status; x always holds the last iterate.
 * Mixed precision (prec_inner = WD_F32/WD_F16) runs the inner CG in that
 * format on 12-real links and recomputes the residual in FP64 (reliable
 * updates); the stopping test is always the FP64 true residual. */
int wd_cg_solve(wd_lattice *lat, const wd_solve_params *p, const double *b, double *x,
                wd_solve_info *info, void *stream);

/* ---------------------------------------------------------------- serving
 * Sec. 2.3 poses the solver's workload as a stream of solves: the gauge
 * field stays resident while new sources eta arrive (and now and then a new
 * field with its own sources).  A server takes such a stream of CG requests
 * (lattices of different sizes, kappa, precisions, 1..12 sources each) and
 * solves them concurrently on one GPU (continuous batching): requests are
 * admitted in arrival order as slots and HBM free up, iterate side by side on
 * their own streams, and retire independently.  Each request's result is
 * bitwise the same as the same wd_cg_solve alone. */

typedef struct {
    size_t hbm_budget_bytes; /* cap on what the server's work holds in HBM:
                                workspaces of running requests, float64 links
                                of lattices with running requests, and every
                                derived gauge form (float32, binary16,
                                even-odd halves) resident on a lattice the
                                server has solved on */
    int32_t max_active;      /* requests iterating at once (<= 0: 8); with
                                caller streams it is n_streams */
    int32_t chunk_iters;     /* CG iterations enqueued per request per
                                scheduling turn (<= 0: chosen from the volume) */
    int32_t n_streams;       /* 0: the server creates one non-blocking stream
                                per slot; > 0 (at most 64): the slots run on
                                the caller's streams[0..n_streams-1] */
    void *const *streams;    /* hipStream_t values (e.g. torch streams), owned
                                by the caller, valid until wd_server_destroy
                                returns; never destroyed by the server */
} wd_server_config;

/* Start a server with its own scheduler thread and one HIP stream per active
 * slot.  Requests are admitted in arrival order while the HBM budget and the
 * slot count allow; admitted requests iterate concurrently on their streams
 * and retire independently (continuous batching).  When a request does not
 * fit the budget, the server first releases derived gauge forms of lattices
 * that have no running requests (they are rebuilt, bit for bit, on next
 * use; a caller using such a lattice directly while the server runs must
 * expect that).  WD_ERR_ARG for a zero budget or an invalid stream list. */
int wd_server_create(const wd_server_config *cfg, wd_server **out);

/* Queue a solve (non-blocking).  Same arguments as wd_cg_solve; the lattice
 * must have its gauge set and must outlive the request, and b must already
 * hold the source on the device (the server reads it from its own stream,
 * unordered with the caller's streams).  *ticket identifies the request.
 * WD_ERR_NOMEM if the request alone (its workspace, the lattice's float64
 * links and the forms it reads) exceeds the whole budget; WD_ERR_STATE once
 * the server is being destroyed. */
int wd_submit(wd_server *s, wd_lattice *lat, const wd_solve_params *p, const double *b,
              double *x, uint64_t *ticket);

/* WD_PENDING while queued or running; otherwise the solve's return code, with
 * info (host, nrhs entries) filled in.  The 4096 most recently finished
 * tickets may be polled again; older ones report WD_ERR_NOTFOUND (the
 * server's bookkeeping does not grow with the requests it has served). */
int wd_poll(wd_server *s, uint64_t ticket, wd_solve_info *info);

/* Completed solves per second since the server started, and the 50th/99th
 * percentile (nearest rank) of completion - submission latency, seconds. */
int wd_server_stats(wd_server *s, double *solves_per_s, double *p50_s, double *p99_s);

/* Peak bytes the server has charged against its budget at once. */
int wd_server_peak_bytes(wd_server *s, size_t *bytes);

/* Drain every queued and running request, then free the server. */
int wd_server_destroy(wd_server *s);

/* ---------------------------------------------------------------- misc */

/* Thread-local text of the last error on this thread (library-owned, valid
 * until the next call on this thread). */
const char *wd_last_error(void);

/* Streaming probe for measurement: dst = the element-wise sum (as float64)
 * of nsrc (1..4) device arrays of `bytes` bytes each (a multiple of 16; all
 * pointers 16-byte aligned; no source overlapping dst), moved with 16-byte
 * non-temporal loads and stores, the access pattern of the solver's vector
 * kernels.  nsrc reads per write reproduce a kernel's read/write mix (1 is a
 * copy; 3 matches the stencil, 4 the r-updating stencil), and the rate (bytes
 * read plus written over the kernel time) is the device's practical
 * streaming ceiling for that mix, beside the published HBM peak.
 * Stream-ordered. */
int wd_stream_probe(const void *const *src, int nsrc, void *dst, size_t bytes, void *stream);

/* Kernel timing with HIP events recorded on the launch stream around every
 * stencil launch.  wd_timing_read returns the summed milliseconds and launch
 * count for one kernel family since the last reset; it synchronises the
 * pending events.  Families: "dslash_f64", "dslash_f32", "dslash_f16" (the
 * stencil), "dslash_xr_<prec>" (a CG iteration's second stencil with the r
 * update fused), "eo_<prec>" and "eo_xr_<prec>" (half-field stencils of the
 * even-odd form, plain and r-updating), "halo_f64" (slab stencil).  Solver chunks are not captured into HIP graphs
 * while timing is on. */
int wd_timing_enable(int on);
int wd_timing_reset(void);
int wd_timing_read(const char *name, double *total_ms, int64_t *count);

#ifdef __cplusplus
}
#endif

#endif /* WD_H */
