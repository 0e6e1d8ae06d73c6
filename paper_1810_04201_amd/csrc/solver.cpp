// Conjugate gradient on the normal equations (Sec. 2.2) as a resumable,
// stream-ordered state machine.
//
// Per inner iteration three kernels run back to back on the solve's stream
// (CGNR; the CGNE form of the paper's listing exchanges D and D^dag, solves
// D D^dag y = b from b' = b and returns x = D^dag y):
//   t  = D p                        (stencil, fused |t|^2 -> alpha = |r|^2 / |t|^2)
//   r -= alpha D^dag t              (stencil forming D^dag t where r is updated,
//                                    fused |r|^2 -> beta, convergence, triggers)
//   x += alpha p, p = r + beta p    (one pass over p)
// (the unfused form stores Ap = D^dag t and runs the x/r and p updates as
// two kernels).  On the even-odd form each stencil is two half-field
// launches.
// All scalars stay on the device (RhsState); the host only reads a small
// status record every `chunk_` iterations and never stalls the stream on it:
// inner iterations enqueued after an rhs froze are exact no-ops, so results
// do not depend on host timing.
//
// A reliable update (Sleijpen and van der Vorst) recomputes the residual in
// float64: x64 += x_lo, r64 = D^dag b - D^dag D x64, and resumes the
// recursion from r64 with beta = |r64|^2 / |r_prev|^2.  It runs once at the
// start (forming r and p), whenever every unfinished rhs is frozen, and is
// the final stopping test: an rhs converges only when its float64 true
// residual meets the tolerance.  Plain FP64 CG triggers it only at the
// convergence estimate; mixed precision also every `reliable_max_iter`
// iterations and when |r_lo| drops below delta * max |r_lo|.
//
// The decision is taken on the device: every few inner iterations the
// stream carries a reliable update gated on the solver state (it runs only
// when every unfinished rhs is frozen and one waits for it), so the host only
// watches for the end of the solve and never sits between a trigger and its
// update.
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "runtime.hpp"

namespace wd {

Solve::Solve(wd_lattice *lat, const wd_solve_params &p, const double *b, double *x)
    : lat_(lat), p_(p), b_(b), x_(x), prec_(p.prec_inner) {
    // the normal operator as two applications: A^dag A (CGNR) or A A^dag
    // (CGNE), A = D, or the Schur complement M with WD_SOLVE_EVEN_ODD
    eo_ = (p.form & WD_SOLVE_EVEN_ODD) != 0;
    d1_ = (p.form & 0xff) == WD_FORM_CGNE ? 1 : 0;
    d2_ = 1 - d1_;
}

int SlotRes::create() {
    if (hipHostMalloc((void **)&h_st, sizeof(RhsState) * kSlots * 12) != hipSuccess ||
        hipHostMalloc((void **)&h_batch, sizeof(BatchState) * kSlots) != hipSuccess)
        return fail(WD_ERR_NOMEM, "pinned host allocation failed");
    for (int i = 0; i < kSlots; ++i)
        if (hipEventCreateWithFlags(&ev[i], hipEventDisableTiming) != hipSuccess)
            return fail(WD_ERR_HIP, "hipEventCreate failed");
    if (hipEventCreateWithFlags(&final_ev, hipEventDisableTiming) != hipSuccess)
        return fail(WD_ERR_HIP, "hipEventCreate failed");
    return WD_OK;
}

void SlotRes::destroy() {
    for (int i = 0; i < kSlots; ++i)
        if (ev[i]) (void)hipEventDestroy(ev[i]);
    if (final_ev) (void)hipEventDestroy(final_ev);
    if (h_st) (void)hipHostFree(h_st);
    if (h_batch) (void)hipHostFree(h_batch);
    *this = SlotRes{};
}

Solve::~Solve() {
    if (gexec_) {
        // the graph's last replay precedes the final status on the stream;
        // make sure it has retired before the executable goes
        (void)hipStreamSynchronize(s_);
        (void)hipGraphExecDestroy(gexec_);
    }
    if (graph_) (void)hipGraphDestroy(graph_);
    // stream-ordered release after the solve's last kernel
    if (mem_) (void)hipFreeAsync(mem_, s_);
    own_.destroy();
}

int Solve::validate(wd_lattice *lat, const wd_solve_params *p) {
    if (!lat || !p) return fail(WD_ERR_ARG, "null argument");
    if (!std::isfinite(p->kappa)) return fail(WD_ERR_ARG, "kappa not finite");
    if (!(p->tol > 0.0) || !std::isfinite(p->tol)) return fail(WD_ERR_ARG, "tol must be > 0");
    if (p->max_iter < 1) return fail(WD_ERR_ARG, "max_iter must be >= 1");
    if (!valid_prec(p->prec_inner)) return fail(WD_ERR_ARG, "unknown precision %d", p->prec_inner);
    if (p->nrhs < 1 || p->nrhs > 12) return fail(WD_ERR_ARG, "nrhs = %d outside 1..12", p->nrhs);
    if (p->x0_given != 0 && p->x0_given != 1) return fail(WD_ERR_ARG, "x0_given must be 0 or 1");
    const int base = p->form & ~WD_SOLVE_EVEN_ODD;
    if (base != WD_FORM_CGNR && base != WD_FORM_CGNE)
        return fail(WD_ERR_ARG, "unknown form %d", p->form);
    if (base == WD_FORM_CGNE && p->x0_given)
        return fail(WD_ERR_ARG, "a starting guess needs the CGNR form");
    if ((p->form & WD_SOLVE_EVEN_ODD) && !eo_supported(lat->g))
        return fail(WD_ERR_ARG, "even-odd needs bricks with an even x extent");
    if (!lat->has_gauge) return fail(WD_ERR_NOGAUGE, "gauge field not set");
    return WD_OK;
}

static size_t align256(size_t b) { return (b + 255u) & ~(size_t)255u; }

static size_t field_bytes(int prec, int V, int nrhs) {
    return align256(field_data_bytes(prec, V, nrhs)) + 256;
}

// A^dag (A p) formed where r is updated (q never stored), and x += alpha p
// moved into the p update (p read once for both): besides the stencils'
// inputs an iteration moves 7 fields instead of 10.  Done by the marching
// stencil on the full lattice and by the second half-field launch on the
// even-odd form; WD_FUSE_XR=0 turns it off.
static bool fused_iteration(const wd_lattice *lat, const wd_solve_params &p) {
    const char *fx = getenv("WD_FUSE_XR");
    if (fx && atoi(fx) == 0) return false;
    if (p.form & WD_SOLVE_EVEN_ODD) return true;
    return dslash_xr_supported(lat->g, p.prec_inner, p.nrhs,
                               (int)reduce_partials_cap(lat->g, p.nrhs));
}

size_t Solve::footprint(const wd_lattice *lat, const wd_solve_params &p) {
    const bool eo = (p.form & WD_SOLVE_EVEN_ODD) != 0;
    const int V = eo ? lat->g.V / 2 : lat->g.V, nr = p.nrhs;
    const int lo = p.prec_inner;
    const int lo_xr = xr_prec_of(lo);
    // float64: b, b', x, r, t, Ax (+ b_o and an odd temporary for even-odd)
    size_t b = (eo ? 8 : 6) * field_bytes(WD_F64, V, nr);
    // inner: x, r in lo_xr; p, t (+ Ap unless the iteration is fused, + an
    // odd temporary) in lo
    const int nlo = 2 + (fused_iteration(lat, p) ? 0 : 1) + (eo ? 1 : 0);
    b += 2 * field_bytes(lo_xr, V, nr) + nlo * field_bytes(lo, V, nr);
    b += align256((size_t)reduce_partials_cap(lat->g, p.nrhs) * sizeof(double));
    b += align256(sizeof(RhsState) * 12) + 256;
    return b;
}

int Solve::setup(hipStream_t stream, SlotRes *res) {
    s_ = stream;
    const int V = eo_ ? lat_->g.V / 2 : lat_->g.V;  // sites of the solved fields
    const int nrhs = p_.nrhs;
    const int64_t n = (int64_t)V * nrhs;
    int err = WD_OK;
    if (eo_) {
        if (!gauge_eo_for(lat_, WD_F64, s_, &err, gh64_)) return err;
        if (!gauge_eo_for(lat_, prec_, s_, &err, ghlo_)) return err;
    } else {
        gauge64_ = gauge_for(lat_, WD_F64, s_, &err);
        if (!gauge64_) return err;
        if (prec_ != WD_F64) {
            gauge_lo_ = gauge_for(lat_, prec_, s_, &err);
            if (!gauge_lo_) return err;
        } else {
            gauge_lo_ = gauge64_;
        }
    }
    bytes_ = footprint(lat_, p_);
    hipError_t he = hipMallocAsync(&mem_, bytes_, s_);
    if (he != hipSuccess) {
        mem_ = nullptr;
        return fail(WD_ERR_NOMEM, "allocation of %zu bytes of solver workspace failed: %s", bytes_,
                    hipGetErrorString(he));
    }
    char *base = (char *)mem_;
    char *cur = base;
    auto next = [&](int prec) {
        char *c = cur;
        FieldRef f = carve(c, prec, nrhs, V);
        cur += field_bytes(prec, V, nrhs);
        return f;
    };
    b64_ = next(WD_F64);
    bp_ = next(WD_F64);
    x64_ = next(WD_F64);
    r64_ = next(WD_F64);
    t64_ = next(WD_F64);
    ax64_ = next(WD_F64);
    if (eo_) {
        bo64_ = next(WD_F64);
        tmp64_ = next(WD_F64);
    }
    const int lo_xr = xr_prec_of(prec_);
    fuse_xr_ = fused_iteration(lat_, p_);
    xl_ = next(lo_xr);
    rl_ = next(lo_xr);
    pl_ = next(prec_);
    tl_ = next(prec_);
    if (!fuse_xr_) apl_ = next(prec_);
    if (eo_) tmpl_ = next(prec_);
    partials_ = (double *)cur;
    partials_cap_ = (int)reduce_partials_cap(lat_->g, nrhs);
    cur += align256((size_t)partials_cap_ * sizeof(double));
    st_ = (RhsState *)cur;
    cur += align256(sizeof(RhsState) * 12);
    batch_ = (BatchState *)cur;
    cur += 256;
    if ((size_t)(cur - base) > bytes_) return fail(WD_ERR_STATE, "workspace layout overflow");

    if (!res) {
        int rc = own_.create();
        if (rc) return rc;
        res = &own_;
    }
    res_ = res;
    h_st_ = res->h_st;
    h_batch_ = res->h_batch;
    final_ev_ = res->final_ev;

    ctl_.tol2 = p_.tol * p_.tol;
    const double delta = p_.reliable_delta > 0 ? p_.reliable_delta : 0.1;
    ctl_.delta2 = delta * delta;
    ctl_.max_iter = p_.max_iter;
    ctl_.nrhs = nrhs;
    ctl_.mixed = prec_ != WD_F64;
    ctl_.max_inner = ctl_.mixed ? (p_.reliable_max_iter > 0 ? p_.reliable_max_iter : 50) : 0;
    // iterations per status read: large lattices need few, small ones more,
    // up to 16 (a solve enqueues whole chunks, so the iterations after its
    // convergence, gated no-ops of a few microseconds each, grow with the
    // chunk: 4^4 FP64 CG 3.6 ms at 64, 2.1 ms at 16); WD_CHUNK_MAX overrides
    const double site_iters = 4.0e7 / (double)n;
    static const int chunk_max = [] {
        const char *e = getenv("WD_CHUNK_MAX");
        const int v = e ? atoi(e) : 16;
        return v < 4 ? 4 : v;
    }();
    chunk_ = site_iters < 4 ? 4 : (site_iters > chunk_max ? chunk_max : (int)site_iters);
    // a gated reliable update after every iteration on large lattices (its
    // launches cost nothing next to an iteration), every 4 on small ones
    rel_every_ = n >= (1 << 20) ? 1 : 4;
    // chunks replayed from a captured HIP graph: cuts the host's launch work,
    // which bounds a server driving many small solves from one thread
    // (measured 113 -> 182 solves/s on 8^4 / 12^4 requests).  Needs a stream
    // that can be captured (not the null stream); off while stencil launches
    // are being timed; WD_GRAPH=0 turns it off.
    const char *ge = getenv("WD_GRAPH");
    use_graph_ = s_ != nullptr && !timing_enabled() && !(ge && atoi(ge) == 0);
    ctl_.lag_x = fuse_xr_ ? 1 : 0;
    return WD_OK;
}

RedArgs Solve::red(int mode) const {
    RedArgs r{};
    r.partials = partials_;
    r.partials_cap = partials_cap_;
    r.st = st_;
    r.batch = batch_;
    r.ctl = ctl_;
    r.mode = mode;
    return r;
}

// One application of the operator A of the normal equations (first: the
// one applied to p, giving t; else the one applied to t): D or D^dag, or on
// the even sites M = 1 - D_eo D_oe or M^dag (two half-field stencils through
// an odd temporary); red fuses |out|^2 into the last launch.
void Solve::op(bool first, const FieldRef &in, const FieldRef &out, const RedArgs *red, Gate gate,
               bool lo) {
    const double k = p_.kappa;
    const int dag = first ? d1_ : d2_;
    if (!eo_) {
        dslash(lat_, lo ? gauge_lo_ : gauge64_, k, dag, in, out, red, gate, s_);
        return;
    }
    void *const *gh = lo ? ghlo_ : gh64_;
    const FieldRef &tmp = lo ? tmpl_ : tmp64_;
    hop_half(lat_, gh, 1, k, 0.0, dag, in, FieldRef{}, tmp, nullptr, gate, s_);  // D_oe in
    hop_half(lat_, gh, 0, -k, 1.0, dag, tmp, in, out, red, gate, s_);           // in - D_eo tmp
}

// The second operator application of an iteration on in = A p, with the
// r update fused into its last launch; false if nothing was launched
bool Solve::op_xr(const FieldRef &in, const RedArgs &rr, Gate gate) {
    const double k = p_.kappa;
    const XrArgs xr{rl_};
    if (!eo_) return dslash_xr(lat_, gauge_lo_, k, d2_, in, xr, rr, gate, s_);
    hop_half(lat_, ghlo_, 1, k, 0.0, d2_, in, FieldRef{}, tmpl_, nullptr, gate, s_);
    hop_half_xr(lat_, ghlo_, 0, -k, 1.0, d2_, tmpl_, in, xr, rr, gate, s_);
    return true;
}

int Solve::start() {
    const double k = p_.kappa;
    const Gate none{nullptr, nullptr, GATE_ACTIVE};
    launch_init_state(st_, batch_, p_.nrhs, s_);
    RedArgs rb = red(RED_B0);
    // b' = A^dag b^ (CGNR) or b^ (CGNE), |b'|^2; b^ = b, or b_e - D_eo b_o
    FieldRef bh = b64_;
    if (eo_) {
        launch_import_half(b_, b64_, 0, lat_->g, s_);
        launch_import_half(b_, bo64_, 1, lat_->g, s_);
        hop_half(lat_, gh64_, 0, -k, 1.0, 0, bo64_, b64_, t64_, nullptr, none, s_);
        bh = t64_;
    } else {
        launch_import(b_, b64_, lat_->g, s_);
    }
    if (d1_ == 1)
        launch_residual(bp_, bh, FieldRef{}, rb, none, s_);  // CGNE: b' = b^
    else
        op(false, bh, bp_, &rb, none, false);                 // CGNR: b' = A^dag b^
    if (p_.x0_given) {
        if (eo_)
            launch_import_half(x_, x64_, 0, lat_->g, s_);
        else
            launch_import(x_, x64_, lat_->g, s_);
    } else {
        launch_zero(x64_, s_);
    }
    launch_zero(xl_, s_);
    // the first reliable update forms r and p for every rhs with b' != 0
    if (p_.x0_given) {
        enqueue_reliable();
    } else {
        const Gate trig{st_, batch_, GATE_TRIGGER};
        const Gate rst{st_, batch_, GATE_RESTART};
        RedArgs rt = red(RED_TRUE);
        launch_residual(r64_, bp_, FieldRef{}, rt, trig, s_);  // x = 0: r = b'
        launch_convert(r64_, rl_, rst, s_);
        launch_restart_p(pl_, rl_, rst, s_);
    }
    if (launch_failed()) return fail(WD_ERR_HIP, "kernel launch failed");
    return push_status();
}

void Solve::enqueue_inner(int iters) {
    const Gate g = gate();
    RedArgs ra = red(RED_ALPHA);
    RedArgs rr = red(RED_RR);
    for (int i = 0; i < iters; ++i) {
        op(true, pl_, tl_, &ra, g, true);
        if (fuse_xr_) {
            // r updated where A p is formed; x += alpha p with the p update
            op_xr(tl_, rr, g);
            launch_update_xp(xl_, pl_, rl_, g, s_);
        } else {
            op(false, tl_, apl_, nullptr, g, true);
            launch_update_xr(xl_, rl_, pl_, apl_, rr, g, s_);
            launch_update_p(pl_, rl_, g, s_);
        }
        if ((i + 1) % rel_every_ == 0 || i + 1 == iters) enqueue_reliable();
    }
}

// One chunk of inner iterations: eager launches, or a replay of the chunk
// captured once into a HIP graph (kernel nodes only; every argument is fixed
// for the solve).  A capture that fails falls back to eager launches.
int Solve::enqueue_chunk() {
    if (use_graph_ && !gexec_) {
        hipGraph_t gr = nullptr;
        bool ok = hipStreamBeginCapture(s_, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
            enqueue_inner(chunk_);
            ok = hipStreamEndCapture(s_, &gr) == hipSuccess && gr != nullptr;
        }
        if (ok) ok = hipGraphInstantiate(&gexec_, gr, nullptr, nullptr, 0) == hipSuccess;
        if (ok) {
            graph_ = gr;
        } else {
            if (gr) (void)hipGraphDestroy(gr);
            gexec_ = nullptr;
            use_graph_ = false;
            (void)hipGetLastError();
        }
    }
    if (use_graph_) {
        if (hipGraphLaunch(gexec_, s_) != hipSuccess)
            return fail(WD_ERR_HIP, "graph launch failed");
        return WD_OK;
    }
    enqueue_inner(chunk_);
    return WD_OK;
}

// A reliable update gated on the device (GATE_TRIGGER): a no-op unless every
// unfinished rhs is frozen and at least one waits for it; then it takes the
// waiting rhs, and resets r_lo and p of those it restarts (GATE_RESTART).
void Solve::enqueue_reliable() {
    const Gate trig{st_, batch_, GATE_TRIGGER};
    const Gate rst{st_, batch_, GATE_RESTART};
    RedArgs rt = red(RED_TRUE);
    launch_accum_zero(x64_, xl_, pl_, trig, s_);
    op(true, x64_, t64_, nullptr, trig, false);
    op(false, t64_, ax64_, nullptr, trig, false);
    launch_residual(r64_, bp_, ax64_, rt, trig, s_);
    launch_convert(r64_, rl_, rst, s_);
    launch_restart_p(pl_, rl_, rst, s_);
}

void Solve::enqueue_finish() {
    const double k = p_.kappa;
    const Gate none{nullptr, nullptr, GATE_ACTIVE};
    launch_accum_zero(x64_, xl_, pl_, Gate{st_, nullptr, GATE_ACTIVE}, s_);  // unconverged rhs
    RedArgs ra = red(RED_AUX);
    RedArgs ra2 = red(RED_AUX_ADD);
    RedArgs rb = red(RED_AUX2);
    RedArgs rb2 = red(RED_AUX2_ADD);
    // the solution of A z = b^: z = x (CGNR) or A^dag y (CGNE)
    FieldRef z = x64_;
    if (d1_ == 1) {
        op(true, x64_, t64_, nullptr, none, false);
        z = t64_;
    }
    if (eo_) {
        // x_o = b_o - D_oe x_e, then |b - D x|^2 over both halves
        const FieldRef xo = r64_;
        hop_half(lat_, gh64_, 1, -k, 1.0, 0, z, bo64_, xo, nullptr, none, s_);
        hop_half(lat_, gh64_, 0, k, 1.0, 0, xo, z, ax64_, nullptr, none, s_);  // (D x)_e
        launch_residual(bp_, b64_, ax64_, ra, none, s_);
        hop_half(lat_, gh64_, 1, k, 1.0, 0, z, xo, ax64_, nullptr, none, s_);  // (D x)_o
        launch_residual(bp_, bo64_, ax64_, ra2, none, s_);
        launch_norm(b64_, rb, s_);
        launch_norm(bo64_, rb2, s_);
        launch_export_half(z, x_, 0, lat_->g, s_);
        launch_export_half(xo, x_, 1, lat_->g, s_);
    } else {
        const FieldRef dx = z.data == t64_.data ? r64_ : t64_;
        dslash(lat_, gauge64_, k, 0, z, dx, nullptr, none, s_);
        launch_residual(ax64_, b64_, dx, ra, none, s_);  // |b - D x|^2
        launch_norm(b64_, rb, s_);                        // |b|^2
        launch_export(z, x_, lat_->g, s_);
    }
    (void)hipMemcpyAsync(h_st_, st_, sizeof(RhsState) * p_.nrhs, hipMemcpyDeviceToHost, s_);
    (void)hipEventRecord(final_ev_, s_);
}

int Solve::push_status() {
    // reuse a slot only once its previous copy has been consumed
    const int slot = next_slot_;
    next_slot_ = (next_slot_ + 1) % kSlots;
    RhsState *hs = h_st_ + (size_t)slot * p_.nrhs;
    if (hipMemcpyAsync(hs, st_, sizeof(RhsState) * p_.nrhs, hipMemcpyDeviceToHost, s_) !=
            hipSuccess ||
        hipMemcpyAsync(h_batch_ + slot, batch_, sizeof(BatchState), hipMemcpyDeviceToHost, s_) !=
            hipSuccess ||
        hipEventRecord(res_->ev[slot], s_) != hipSuccess)
        return fail(WD_ERR_HIP, "status copy failed");
    pending_.push_back(Pending{res_->ev[slot], slot});
    return WD_OK;
}

int Solve::advance(bool block) {
    for (;;) {
        if (phase_ == 2) return 1;
        if (phase_ == 1) {
            hipError_t e = block ? hipEventSynchronize(final_ev_) : hipEventQuery(final_ev_);
            if (e == hipErrorNotReady) return 0;
            if (e != hipSuccess) return fail(WD_ERR_HIP, "solve failed on the device: %s",
                                             hipGetErrorString(e));
            result_ = WD_OK;
            for (int r = 0; r < p_.nrhs; ++r) {
                const RhsState &st = h_st_[r];
                if (!st.converged) {
                    result_ = st.failed ? st.failed : WD_ERR_NOCONV;
                    break;
                }
            }
            phase_ = 2;
            return 1;
        }
        // keep two status reads in flight so the device never idles on the host
        while (pending_.size() < 2) {
            int rc0 = enqueue_chunk();
            if (rc0) return rc0;
            if (launch_failed()) return fail(WD_ERR_HIP, "kernel launch failed");
            int rc = push_status();
            if (rc) return rc;
        }
        Pending f = pending_.front();
        hipError_t e = block ? hipEventSynchronize(f.ev) : hipEventQuery(f.ev);
        if (e == hipErrorNotReady) return 0;
        if (e != hipSuccess) return fail(WD_ERR_HIP, "solve failed on the device: %s",
                                         hipGetErrorString(e));
        pending_.pop_front();
        const BatchState &bs = h_batch_[f.slot];
        // still iterating, or frozen rhs that the next gated reliable update
        // (already in the stream) will take
        if (bs.n_active > 0 || bs.n_trigger > 0) continue;
        // every rhs converged or failed: pending inner chunks are no-ops
        enqueue_finish();
        if (launch_failed()) return fail(WD_ERR_HIP, "kernel launch failed");
        phase_ = 1;
    }
}

void Solve::info(wd_solve_info *out) const {
    for (int r = 0; r < p_.nrhs; ++r) {
        const RhsState &st = h_st_[r];
        wd_solve_info &o = out[r];
        o.status = st.converged ? WD_OK : (st.failed ? st.failed : WD_ERR_NOCONV);
        o.iters = st.iters;
        o.reliable_updates = st.updates;
        o.true_rel_resid = st.rr0 > 0 ? std::sqrt(st.rr_true / st.rr0) : 0.0;
        o.rel_resid_D = st.aux2 > 0 ? std::sqrt(st.aux / st.aux2) : 0.0;
        o.seconds = seconds;
        o.queued_seconds = 0.0;
    }
}

}  // namespace wd

using namespace wd;

extern "C" int wd_cg_solve(wd_lattice *lat, const wd_solve_params *p, const double *b,
                           double *x, wd_solve_info *info, void *stream) {
    int rc = Solve::validate(lat, p);
    if (rc) return rc;
    if (!b || !x || !info) return fail(WD_ERR_ARG, "null argument");
    if (b == x) return fail(WD_ERR_ARG, "b and x must not overlap");
    const double t0 = now_seconds();
    Solve s(lat, *p, b, x);
    rc = s.setup((hipStream_t)stream);
    if (rc) return rc;
    rc = s.start();
    if (rc) return rc;
    for (;;) {
        int a = s.advance(true);
        if (a < 0) return a;
        if (a == 1) break;
    }
    s.seconds = now_seconds() - t0;
    s.info(info);
    return s.result();
}
