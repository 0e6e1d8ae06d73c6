// Host-side runtime objects behind the C ABI: lattices with their resident
// gauge forms, spinor fields, the CG solve state machine and the server.
#pragma once

#include <atomic>
#include <cmath>
#include <cstdio>
#include <deque>
#include <mutex>
#include <string>
#include <vector>

#include "server_core.hpp"
#include "wd_internal.hpp"

struct wd_lattice {
    wd::Geom g{};
    void *gauge[3] = {nullptr, nullptr, nullptr};  // F64-18, F32-12, F16-12
    void *gauge12 = nullptr;  // F64-12 beside F64-18 when the links are special unitary
    double su3_dev = -1.0;    // largest row-2 deviation found by wd_set_gauge (-1: not checked)
    bool eo64_r12 = false;    // gauge_eo[WD_F64] holds the F64-12 form
    void *gauge_eo[3][2] = {};                     // even-odd halves [prec][parity]
    void *halo_links = nullptr;                    // U_t(x, -1) over face sites (t-slab)
    std::atomic<bool> has_gauge{false};  // read without the lock by validation
    double hop_sign = -1.0;  // D = 1 + hop_sign * kappa * (hops); kernels take 1 - kappa' H
    std::mutex mu;
    std::atomic<int> users{0};  // requests in flight on a server
};

struct wd_field {
    wd_lattice *lat = nullptr;
    int prec = WD_F64;
    int nrhs = 1;
    void *mem = nullptr;
    wd::FieldRef ref{};
};

namespace wd {

void set_error(const char *fmt, ...);
int fail(int code, const char *fmt, ...);
#define WD_HIP_CHECK(call)                                                               \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return ::wd::fail(WD_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// hipGetLastError reports the last status of any runtime call on this thread,
// including hipErrorNotReady from an event or stream query (ours or the
// caller's); that status is not a launch failure.
inline bool launch_failed() {
    const hipError_t e = hipGetLastError();
    return e != hipSuccess && e != hipErrorNotReady;
}
#define WD_LAUNCH_CHECK()                                                      \
    do {                                                                       \
        if (::wd::launch_failed()) return ::wd::fail(WD_ERR_HIP, "kernel launch failed"); \
    } while (0)

bool valid_prec(int p);
// packed gauge form for a precision, building the 12-real forms on first use
// (enqueued on stream s).  Returns nullptr and sets the error on failure.
void *gauge_for(wd_lattice *lat, int prec, hipStream_t s, int *err);

// even-odd half forms of a precision (both parities), built on first use
// from the F64-18 tiles; false and the error set on failure
bool gauge_eo_for(wd_lattice *lat, int prec, hipStream_t s, int *err, void *out[2]);

// Resident gauge forms, for a server's HBM ledger (under the lattice lock):
// *master = the float64 links (18 reals, plus 12 where kept), derived[f] the
// bytes of each derived form (DerivedForm) now resident, 0 where not built.
void lattice_forms(wd_lattice *lat, size_t *master, size_t derived[kNumDerived]);
// Release one derived form of the lattice (it is rebuilt, bit for bit, on
// next use).  The caller makes sure no queued work reads it.
void release_form(wd_lattice *lat, int form);
// Bytes of the derived forms a solve with parameters p reads (0 where it
// reads none of that form).
void solve_forms(const wd_lattice *lat, const wd_solve_params &p, size_t out[kNumDerived]);

// A lattice is being destroyed: every live server drops it from its ledger
// (server.cpp).
void servers_forget(wd_lattice *lat);

// out_p = cs * c_p + D_{p,1-p} in_{1-p} on half fields: the off-diagonal block
// of D (D^dag for dagger) from parity 1-p to p at hopping parameter kappa
// (the lattice's sign applied), plus an optional scaled c term
void hop_half(wd_lattice *lat, void *const gh[2], int p, double kappa, double cs, int dagger,
              const FieldRef &in, const FieldRef &c, const FieldRef &out, const RedArgs *red,
              Gate gate, hipStream_t s);

// hop_half with c present whose output q is consumed where it is formed
// (r -= alpha q; see launch_hop_half_xr)
void hop_half_xr(wd_lattice *lat, void *const gh[2], int p, double kappa, double cs, int dagger,
                 const FieldRef &in, const FieldRef &c, const XrArgs &xr, const RedArgs &red,
                 Gate gate, hipStream_t s);

// stencil launch with optional event timing
void dslash(wd_lattice *lat, const void *gauge, double kappa, int dagger, const FieldRef &in,
            const FieldRef &out, const RedArgs *red, Gate gate, hipStream_t s);

// stencil launch fused with the CG update that consumes its output (see
// launch_dslash_xr), with optional event timing; false if not supported
bool dslash_xr(wd_lattice *lat, const void *gauge, double kappa, int dagger, const FieldRef &in,
               const XrArgs &xr, const RedArgs &red, Gate gate, hipStream_t s);

FieldRef carve(char *&cursor, int prec, int nrhs, int V);

// ------------------------------------------------------------------ solve

// Pinned status buffers and events a solve polls through.  A server keeps
// one per slot so that admitting and retiring requests allocates no pinned
// memory; a blocking solve creates its own.
struct SlotRes {
    static constexpr int kSlots = 6;
    RhsState *h_st = nullptr;       // kSlots * 12 (one ring slot per status read)
    BatchState *h_batch = nullptr;  // kSlots
    hipEvent_t ev[kSlots] = {};
    hipEvent_t final_ev = nullptr;
    int create();
    void destroy();
};

class Solve {
  public:
    Solve(wd_lattice *lat, const wd_solve_params &p, const double *b, double *x);
    ~Solve();
    static int validate(wd_lattice *lat, const wd_solve_params *p);
    static size_t footprint(const wd_lattice *lat, const wd_solve_params &p);
    // allocate the workspace (stream-ordered) and bind a stream and status
    // buffers (res == nullptr: own ones); no work enqueued
    int setup(hipStream_t stream, SlotRes *res = nullptr);
    // enqueue the start sequence (source prep and first residual)
    int start();
    // advance the state machine; block: wait for device status.  Returns
    // 1 when the solve has finished (info valid), 0 if still running, <0 error
    int advance(bool block);
    void info(wd_solve_info *out) const;
    int result() const { return result_; }
    size_t bytes() const { return bytes_; }
    int nrhs() const { return p_.nrhs; }
    // iterations enqueued per status read (default chosen from the volume)
    void set_chunk(int c) { chunk_ = c < 1 ? 1 : c; }
    double seconds = 0.0;

  private:
    struct Pending {
        hipEvent_t ev;
        int slot;
    };
    void enqueue_inner(int iters);
    int enqueue_chunk();
    void enqueue_reliable();
    void op(bool first, const FieldRef &in, const FieldRef &out, const RedArgs *red, Gate gate,
            bool lo);
    bool op_xr(const FieldRef &in, const RedArgs &rr, Gate gate);
    void enqueue_finish();
    int push_status();
    RedArgs red(int mode) const;
    Gate gate() const { return Gate{st_, batch_, GATE_ACTIVE}; }

    wd_lattice *lat_;
    wd_solve_params p_;
    const double *b_;
    double *x_;
    hipStream_t s_ = nullptr;
    int prec_;
    int d1_ = 0, d2_ = 1;  // daggers of the two operators of the normal equations
    bool eo_ = false;      // on the even-odd Schur complement
    bool fuse_xr_ = false;  // the second operator application updates r (x lags)
    int chunk_ = 8;
    int rel_every_ = 1;  // inner iterations between gated reliable updates
    bool use_graph_ = false;
    hipGraph_t graph_ = nullptr;       // one captured chunk of inner iterations
    hipGraphExec_t gexec_ = nullptr;
    void *gauge64_ = nullptr, *gauge_lo_ = nullptr;
    void *gh64_[2] = {}, *ghlo_[2] = {};  // even-odd halves
    void *mem_ = nullptr;
    size_t bytes_ = 0;
    FieldRef b64_{}, bp_{}, x64_{}, r64_{}, t64_{}, ax64_{};
    FieldRef xl_{}, rl_{}, pl_{}, tl_{}, apl_{};
    FieldRef bo64_{}, tmp64_{}, tmpl_{};  // even-odd: b_o and odd temporaries
    RhsState *st_ = nullptr;
    BatchState *batch_ = nullptr;
    double *partials_ = nullptr;
    int partials_cap_ = 0;
    SolveCtl ctl_{};
    // pinned status ring
    static constexpr int kSlots = SlotRes::kSlots;
    SlotRes own_{};
    SlotRes *res_ = nullptr;
    RhsState *h_st_ = nullptr;       // res_->h_st
    BatchState *h_batch_ = nullptr;  // res_->h_batch
    std::deque<Pending> pending_;
    int next_slot_ = 0;
    int phase_ = 0;  // 0 running, 1 finishing, 2 done
    hipEvent_t final_ev_ = nullptr;
    int result_ = WD_OK;
};

double now_seconds();
bool timing_enabled();

}  // namespace wd
