// C ABI: lattices, gauge ingest, fields, operator application, errors and
// stencil timing.  The solver is in solver.cpp and the server in server.cpp.
#include "runtime.hpp"

#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>

namespace wd {

static thread_local std::string g_err;

void set_error(const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

double now_seconds() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

bool valid_prec(int p) { return p == WD_F64 || p == WD_F32 || p == WD_F16; }

FieldRef carve(char *&cursor, int prec, int nrhs, int V) {
    FieldRef f{};
    f.prec = prec;
    f.nrhs = nrhs;
    f.V = V;
    f.stride = rhs_stride(V);
    f.data = cursor;
    cursor += field_data_bytes(prec, V, nrhs);
    return f;
}

void *gauge_for(wd_lattice *lat, int prec, hipStream_t s, int *err) {
    std::lock_guard<std::mutex> lk(lat->mu);
    if (!lat->has_gauge) {
        *err = fail(WD_ERR_NOGAUGE, "gauge field not set (call wd_set_gauge first)");
        return nullptr;
    }
    if (lat->gauge[prec]) return lat->gauge[prec];
    void *p = nullptr;
    const int form = link_form(lat->g, prec);
    hipError_t he = hipMalloc(&p, gauge_bytes(form, lat->g.V));
    if (he != hipSuccess) {
        *err = fail(WD_ERR_NOMEM, "hipMalloc of the %s gauge form failed: %s",
                    prec == WD_F32 ? "F32-12" : (form == kLinkF16R8 ? "F16-8" : "F16-12"),
                    hipGetErrorString(he));
        return nullptr;
    }
    launch_gauge_lo(lat->gauge[WD_F64], p, form, lat->g.V, s);
    // other streams (server slots) may use the form next: finish building it
    if (hipStreamSynchronize(s) != hipSuccess) {
        (void)hipFree(p);
        *err = fail(WD_ERR_HIP, "building the low-precision gauge form failed");
        return nullptr;
    }
    lat->gauge[prec] = p;
    return p;
}

bool gauge_eo_for(wd_lattice *lat, int prec, hipStream_t s, int *err, void *out[2]) {
    std::lock_guard<std::mutex> lk(lat->mu);
    if (!lat->has_gauge) {
        *err = fail(WD_ERR_NOGAUGE, "gauge field not set (call wd_set_gauge first)");
        return false;
    }
    if (!eo_supported(lat->g)) {
        *err = fail(WD_ERR_ARG, "even-odd needs bricks with an even x extent (got %d)", lat->g.tx);
        return false;
    }
    if (!lat->gauge_eo[prec][0]) {
        void *h[2] = {nullptr, nullptr};
        // float64 halves as 12 reals when the full-lattice links have that form
        const int form = prec == WD_F64 && lat->gauge12 ? kLinkF64R12 : link_form(lat->g, prec);
        const size_t bytes = gauge_bytes(form, lat->g.V / 2);
        for (int p = 0; p < 2; ++p) {
            if (hipMalloc(&h[p], bytes) != hipSuccess) {
                if (h[0]) (void)hipFree(h[0]);
                *err = fail(WD_ERR_NOMEM, "hipMalloc of an even-odd gauge form failed");
                return false;
            }
        }
        for (int p = 0; p < 2; ++p) launch_gauge_split(lat->gauge[WD_F64], h[p], form, p, lat->g, s);
        // other streams (server slots) may use the form next: finish building it
        if (hipStreamSynchronize(s) != hipSuccess) {
            (void)hipFree(h[0]);
            (void)hipFree(h[1]);
            *err = fail(WD_ERR_HIP, "building an even-odd gauge form failed");
            return false;
        }
        lat->gauge_eo[prec][0] = h[0];
        lat->gauge_eo[prec][1] = h[1];
        if (prec == WD_F64) lat->eo64_r12 = form == kLinkF64R12;
    }
    out[0] = lat->gauge_eo[prec][0];
    out[1] = lat->gauge_eo[prec][1];
    return true;
}

static size_t eo_form_bytes(const wd_lattice *lat, int prec) {
    const int form = prec == WD_F64 && lat->gauge12 ? kLinkF64R12 : link_form(lat->g, prec);
    return 2 * gauge_bytes(form, lat->g.V / 2);
}

void lattice_forms(wd_lattice *lat, size_t *master, size_t derived[kNumDerived]) {
    std::lock_guard<std::mutex> lk(lat->mu);
    const int V = lat->g.V;
    *master = (lat->gauge[WD_F64] ? gauge_bytes(WD_F64, V) : 0) +
              (lat->gauge12 ? gauge_bytes(kLinkF64R12, V) : 0);
    derived[kFormF32] = lat->gauge[WD_F32] ? gauge_bytes(WD_F32, V) : 0;
    derived[kFormF16] = lat->gauge[WD_F16] ? gauge_bytes(link_form(lat->g, WD_F16), V) : 0;
    derived[kFormEo64] =
        lat->gauge_eo[WD_F64][0]
            ? 2 * gauge_bytes(lat->eo64_r12 ? kLinkF64R12 : WD_F64, V / 2)
            : 0;
    derived[kFormEo32] = lat->gauge_eo[WD_F32][0] ? eo_form_bytes(lat, WD_F32) : 0;
    derived[kFormEo16] = lat->gauge_eo[WD_F16][0] ? eo_form_bytes(lat, WD_F16) : 0;
}

void release_form(wd_lattice *lat, int form) {
    std::lock_guard<std::mutex> lk(lat->mu);
    auto drop = [](void *&p) {
        if (p) (void)hipFree(p);
        p = nullptr;
    };
    switch (form) {
        case kFormF32: drop(lat->gauge[WD_F32]); break;
        case kFormF16: drop(lat->gauge[WD_F16]); break;
        case kFormEo64: drop(lat->gauge_eo[WD_F64][0]); drop(lat->gauge_eo[WD_F64][1]); break;
        case kFormEo32: drop(lat->gauge_eo[WD_F32][0]); drop(lat->gauge_eo[WD_F32][1]); break;
        case kFormEo16: drop(lat->gauge_eo[WD_F16][0]); drop(lat->gauge_eo[WD_F16][1]); break;
        default: break;
    }
}

void solve_forms(const wd_lattice *lat, const wd_solve_params &p, size_t out[kNumDerived]) {
    for (int f = 0; f < kNumDerived; ++f) out[f] = 0;
    const int prec = p.prec_inner;
    if (p.form & WD_SOLVE_EVEN_ODD) {
        out[kFormEo64] = eo_form_bytes(lat, WD_F64);
        if (prec == WD_F32) out[kFormEo32] = eo_form_bytes(lat, WD_F32);
        if (prec == WD_F16) out[kFormEo16] = eo_form_bytes(lat, WD_F16);
    } else {
        if (prec == WD_F32) out[kFormF32] = gauge_bytes(WD_F32, lat->g.V);
        if (prec == WD_F16) out[kFormF16] = gauge_bytes(link_form(lat->g, WD_F16), lat->g.V);
    }
}

// ------------------------------------------------------------------ timing

struct TimingRec {
    double ms = 0.0;
    int64_t count = 0;
};
struct PendingTime {
    std::string name;
    hipEvent_t a, b;
};
static std::mutex g_tmu;
static std::atomic<int> g_timing{0};
static std::map<std::string, TimingRec> g_times;
static std::vector<PendingTime> g_pending;
static std::vector<hipEvent_t> g_evpool;

static hipEvent_t take_event() {
    if (!g_evpool.empty()) {
        hipEvent_t e = g_evpool.back();
        g_evpool.pop_back();
        return e;
    }
    // timing only: no system-scope release at the record, so the bracket
    // holds the kernel and not a cache write-back for host visibility
    hipEvent_t e = nullptr;
    (void)hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
    return e;
}

static void drain_pending_locked() {
    for (auto &p : g_pending) {
        (void)hipEventSynchronize(p.b);
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            auto &r = g_times[p.name];
            r.ms += ms;
            r.count += 1;
        }
        g_evpool.push_back(p.a);
        g_evpool.push_back(p.b);
    }
    g_pending.clear();
}

bool timing_enabled() { return g_timing.load(std::memory_order_relaxed) != 0; }

// a stencil launch, bracketed by events on its stream while timing is on
template <typename F>
static void timed(const char *name, hipStream_t s, F &&launch) {
    if (!g_timing.load(std::memory_order_relaxed)) {
        launch();
        return;
    }
    hipEvent_t a, b;
    {
        std::lock_guard<std::mutex> lk(g_tmu);
        if (g_pending.size() > 4096) drain_pending_locked();
        a = take_event();
        b = take_event();
    }
    (void)hipEventRecord(a, s);
    launch();
    (void)hipEventRecord(b, s);
    std::lock_guard<std::mutex> lk(g_tmu);
    g_pending.push_back({name, a, b});
}

void dslash(wd_lattice *lat, const void *gauge, double kappa, int dagger, const FieldRef &in,
            const FieldRef &out, const RedArgs *red, Gate gate, hipStream_t s) {
    // the kernels compute in - kappa' * (hops): the +kappa sign is kappa' = -kappa
    kappa = -lat->hop_sign * kappa;
    static const char *names[3] = {"dslash_f64", "dslash_f32", "dslash_f16"};
    // float64 on the lattice's own links: the 12-real form where it exists
    const void *g12 = in.prec == WD_F64 && gauge == lat->gauge[WD_F64] ? lat->gauge12 : nullptr;
    timed(names[in.prec], s,
          [&] { launch_dslash(lat->g, gauge, kappa, dagger, in, out, red, gate, s, g12); });
}

bool dslash_xr(wd_lattice *lat, const void *gauge, double kappa, int dagger, const FieldRef &in,
               const XrArgs &xr, const RedArgs &red, Gate gate, hipStream_t s) {
    if (!dslash_xr_supported(lat->g, in.prec, in.nrhs, red.partials_cap)) return false;
    kappa = -lat->hop_sign * kappa;
    static const char *names[3] = {"dslash_xr_f64", "dslash_xr_f32", "dslash_xr_f16"};
    const void *g12 = in.prec == WD_F64 && gauge == lat->gauge[WD_F64] ? lat->gauge12 : nullptr;
    bool ok = false;
    timed(names[in.prec], s, [&] {
        ok = launch_dslash_xr(lat->g, gauge, kappa, dagger, in, xr, red, gate, s, g12);
    });
    return ok;
}

void hop_half(wd_lattice *lat, void *const gh[2], int p, double kappa, double cs, int dagger,
              const FieldRef &in, const FieldRef &c, const FieldRef &out, const RedArgs *red,
              Gate gate, hipStream_t s) {
    // D_{p,1-p} = hop_sign * kappa * H_{p,1-p}; the kernel computes cs c - k H in
    const double k = -lat->hop_sign * kappa;
    static const char *names[3] = {"eo_f64", "eo_f32", "eo_f16"};
    const bool r12 = in.prec == WD_F64 && lat->eo64_r12 && gh[0] == lat->gauge_eo[WD_F64][0];
    timed(names[in.prec], s, [&] {
        launch_hop_half(lat->g, gh[p], gh[1 - p], p, k, cs, dagger, in, c, out, red, gate, s, r12);
    });
}

void hop_half_xr(wd_lattice *lat, void *const gh[2], int p, double kappa, double cs, int dagger,
                 const FieldRef &in, const FieldRef &c, const XrArgs &xr, const RedArgs &red,
                 Gate gate, hipStream_t s) {
    const double k = -lat->hop_sign * kappa;
    static const char *names[3] = {"eo_xr_f64", "eo_xr_f32", "eo_xr_f16"};
    const bool r12 = in.prec == WD_F64 && lat->eo64_r12 && gh[0] == lat->gauge_eo[WD_F64][0];
    timed(names[in.prec], s, [&] {
        launch_hop_half_xr(lat->g, gh[p], gh[1 - p], p, k, cs, dagger, in, c, xr, red, gate, s,
                           r12);
    });
}

}  // namespace wd

using namespace wd;

// ------------------------------------------------------------------ C ABI

extern "C" {

const char *wd_last_error(void) { return g_err.c_str(); }

int wd_create_lattice(const int32_t dims[4], uint32_t bc_flags, wd_lattice **out) {
    if (!dims || !out) return fail(WD_ERR_ARG, "null argument");
    int64_t V = 1;
    for (int m = 0; m < 4; ++m) {
        if (dims[m] < 2 || (dims[m] & 1))
            return fail(WD_ERR_ARG, "dims[%d] = %d: every extent must be even and >= 2", m,
                        (int)dims[m]);
        V *= dims[m];
    }
    // device index arithmetic is 32-bit over sites of one rhs (offsets up to
    // a few V); byte offsets are 64-bit
    if (V > ((int64_t)1 << 28))
        return fail(WD_ERR_ARG, "volume %lld too large (at most 2^28 sites)", (long long)V);
    if (bc_flags & ~(uint32_t)(WD_BC_ANTIPERIODIC_T | WD_SIGN_PLUS_KAPPA | WD_F16_LINKS_8))
        return fail(WD_ERR_ARG, "unknown lattice flags 0x%x", bc_flags);
    wd_lattice *lat = new (std::nothrow) wd_lattice();
    if (!lat) return fail(WD_ERR_NOMEM, "host allocation failed");
    for (int m = 0; m < 4; ++m) lat->g.L[m] = dims[m];
    lat->g.V = (int)V;
    lat->g.antiperiodic = (bc_flags & WD_BC_ANTIPERIODIC_T) ? 1 : 0;
    lat->g.f16_links8 = (bc_flags & WD_F16_LINKS_8) ? 1 : 0;
    lat->hop_sign = (bc_flags & WD_SIGN_PLUS_KAPPA) ? 1.0 : -1.0;
    choose_bricks(lat->g);
    *out = lat;
    return WD_OK;
}

int wd_destroy_lattice(wd_lattice *lat) {
    if (!lat) return fail(WD_ERR_ARG, "null lattice");
    if (lat->users.load() != 0)
        return fail(WD_ERR_STATE, "lattice still has %d requests on a server", lat->users.load());
    servers_forget(lat);
    for (int p = 0; p < 3; ++p) {
        if (lat->gauge[p]) (void)hipFree(lat->gauge[p]);
        for (int q = 0; q < 2; ++q)
            if (lat->gauge_eo[p][q]) (void)hipFree(lat->gauge_eo[p][q]);
    }
    if (lat->halo_links) (void)hipFree(lat->halo_links);
    if (lat->gauge12) (void)hipFree(lat->gauge12);
    delete lat;
    return WD_OK;
}

int wd_lattice_volume(const wd_lattice *lat, int64_t *volume) {
    if (!lat || !volume) return fail(WD_ERR_ARG, "null argument");
    *volume = lat->g.V;
    return WD_OK;
}

int wd_lattice_links_info(const wd_lattice *lat, int *f64_link_reals, double *su3_deviation) {
    if (!lat) return fail(WD_ERR_ARG, "null lattice");
    if (f64_link_reals) *f64_link_reals = lat->gauge12 ? 12 : 18;
    if (su3_deviation) *su3_deviation = lat->su3_dev;
    return WD_OK;
}

int wd_lattice_gauge_bytes(const wd_lattice *lat, size_t *bytes) {
    if (!lat || !bytes) return fail(WD_ERR_ARG, "null argument");
    size_t b = lat->gauge12 ? gauge_bytes(kLinkF64R12, lat->g.V) : 0;
    for (int p = 0; p < 3; ++p) {
        if (lat->gauge[p]) b += gauge_bytes(link_form(lat->g, p), lat->g.V);
        if (lat->gauge_eo[p][0])
            b += 2 * gauge_bytes(p == WD_F64 && lat->eo64_r12 ? kLinkF64R12 : link_form(lat->g, p),
                                 lat->g.V / 2);
    }
    if (lat->halo_links) b += gauge_bytes(WD_F64, lat->g.V / lat->g.L[3]);
    *bytes = b;
    return WD_OK;
}

int wd_set_gauge(wd_lattice *lat, const double *U, void *stream) {
    if (!lat || !U) return fail(WD_ERR_ARG, "null argument");
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lk(lat->mu);
    if (lat->users.load() != 0)
        return fail(WD_ERR_STATE, "gauge cannot change while requests are in flight");
    // every resident form is rebuilt below; until all of them hold the new
    // links (an early error return leaves them mixed) the lattice has none
    lat->has_gauge = false;
    if (!lat->gauge[WD_F64]) {
        void *p = nullptr;
        hipError_t he = hipMalloc(&p, gauge_bytes(WD_F64, lat->g.V));
        if (he != hipSuccess)
            return fail(WD_ERR_NOMEM, "hipMalloc of the F64 gauge form failed: %s",
                        hipGetErrorString(he));
        lat->gauge[WD_F64] = p;
    }
    launch_pack_gauge_f64(U, lat->gauge[WD_F64], lat->g, s);
    // float64 links also stored as 12 reals when every link is special
    // unitary to rounding (the marching stencil then reads 384 instead of
    // 576 link bytes per site); WD_LINKS64_12=0 keeps 18 reals only
    const char *e12 = getenv("WD_LINKS64_12");
    const bool want12 = !(e12 && atoi(e12) == 0);
    lat->su3_dev = -1.0;
    if (want12) {
        unsigned long long *dm = nullptr, hm = 0;
        WD_HIP_CHECK(hipMallocAsync((void **)&dm, sizeof(hm), s));
        (void)hipMemsetAsync(dm, 0, sizeof(hm), s);
        launch_su3_check(lat->gauge[WD_F64], lat->g.V, dm, s);
        (void)hipMemcpyAsync(&hm, dm, sizeof(hm), hipMemcpyDeviceToHost, s);
        (void)hipFreeAsync(dm, s);
        WD_LAUNCH_CHECK();
        WD_HIP_CHECK(hipStreamSynchronize(s));
        double dev;
        memcpy(&dev, &hm, sizeof(dev));
        lat->su3_dev = dev;
    }
    if (want12 && lat->su3_dev <= kSu3Tol && !lat->gauge12) {
        // without memory for it the lattice keeps 18 reals only
        void *p = nullptr;
        if (hipMalloc(&p, gauge_bytes(kLinkF64R12, lat->g.V)) == hipSuccess)
            lat->gauge12 = p;
        else
            (void)hipGetLastError();
    }
    if (want12 && lat->su3_dev <= kSu3Tol && lat->gauge12) {
        launch_gauge_lo(lat->gauge[WD_F64], lat->gauge12, kLinkF64R12, lat->g.V, s);
    } else if (lat->gauge12) {
        (void)hipFree(lat->gauge12);
        lat->gauge12 = nullptr;
    }
    for (int p = 1; p < 3; ++p)
        if (lat->gauge[p])
            launch_gauge_lo(lat->gauge[WD_F64], lat->gauge[p], link_form(lat->g, p), lat->g.V, s);
    // float64 halves whose form no longer matches are dropped (rebuilt on use)
    if (lat->gauge_eo[WD_F64][0] && lat->eo64_r12 != (lat->gauge12 != nullptr)) {
        for (int q = 0; q < 2; ++q) {
            (void)hipFree(lat->gauge_eo[WD_F64][q]);
            lat->gauge_eo[WD_F64][q] = nullptr;
        }
    }
    for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 2; ++q)
            if (lat->gauge_eo[p][q])
                launch_gauge_split(lat->gauge[WD_F64], lat->gauge_eo[p][q],
                                   p == WD_F64 && lat->eo64_r12 ? kLinkF64R12
                                                                : link_form(lat->g, p),
                                   q, lat->g, s);
    WD_LAUNCH_CHECK();
    WD_HIP_CHECK(hipStreamSynchronize(s));
    lat->has_gauge = true;
    return WD_OK;
}

int wd_field_create(wd_lattice *lat, int prec, int nrhs, wd_field **out) {
    if (!lat || !out) return fail(WD_ERR_ARG, "null argument");
    if (!valid_prec(prec)) return fail(WD_ERR_ARG, "unknown precision %d", prec);
    if (nrhs < 1 || nrhs > 12) return fail(WD_ERR_ARG, "nrhs = %d outside 1..12", nrhs);
    wd_field *f = new (std::nothrow) wd_field();
    if (!f) return fail(WD_ERR_NOMEM, "host allocation failed");
    size_t bytes = field_data_bytes(prec, lat->g.V, nrhs);
    hipError_t he = hipMalloc(&f->mem, bytes);
    if (he != hipSuccess) {
        delete f;
        return fail(WD_ERR_NOMEM, "hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(he));
    }
    char *cur = (char *)f->mem;
    f->ref = carve(cur, prec, nrhs, lat->g.V);
    f->lat = lat;
    f->prec = prec;
    f->nrhs = nrhs;
    *out = f;
    return WD_OK;
}

int wd_field_destroy(wd_field *f) {
    if (!f) return fail(WD_ERR_ARG, "null field");
    (void)hipFree(f->mem);
    delete f;
    return WD_OK;
}

int wd_field_import(wd_field *f, const double *canon, void *stream) {
    if (!f || !canon) return fail(WD_ERR_ARG, "null argument");
    launch_import(canon, f->ref, f->lat->g, (hipStream_t)stream);
    WD_LAUNCH_CHECK();
    return WD_OK;
}

int wd_field_export(const wd_field *f, double *canon, void *stream) {
    if (!f || !canon) return fail(WD_ERR_ARG, "null argument");
    launch_export(f->ref, canon, f->lat->g, (hipStream_t)stream);
    WD_LAUNCH_CHECK();
    return WD_OK;
}

int wd_dslash(wd_lattice *lat, double kappa, int dagger, const wd_field *in, wd_field *out,
              void *stream) {
    if (!lat || !in || !out) return fail(WD_ERR_ARG, "null argument");
    if (in == out) return fail(WD_ERR_ARG, "in and out must be different fields");
    if (in->lat != lat || out->lat != lat) return fail(WD_ERR_ARG, "fields of another lattice");
    if (in->prec != out->prec || in->nrhs != out->nrhs)
        return fail(WD_ERR_ARG, "in/out precision or nrhs differ");
    if (!std::isfinite(kappa)) return fail(WD_ERR_ARG, "kappa not finite");
    if (dagger != 0 && dagger != 1) return fail(WD_ERR_ARG, "dagger must be 0 or 1");
    int err = WD_OK;
    hipStream_t s = (hipStream_t)stream;
    void *g = gauge_for(lat, in->prec, s, &err);
    if (!g) return err;
    dslash(lat, g, kappa, dagger, in->ref, out->ref, nullptr, Gate{nullptr, nullptr, GATE_ACTIVE}, s);
    WD_LAUNCH_CHECK();
    return WD_OK;
}

int wd_apply(wd_lattice *lat, double kappa, int prec, int dagger, int nrhs, const double *in,
             double *out, void *stream) {
    if (!lat || !in || !out) return fail(WD_ERR_ARG, "null argument");
    if (!valid_prec(prec)) return fail(WD_ERR_ARG, "unknown precision %d", prec);
    if (nrhs < 1 || nrhs > 12) return fail(WD_ERR_ARG, "nrhs = %d outside 1..12", nrhs);
    if (!std::isfinite(kappa)) return fail(WD_ERR_ARG, "kappa not finite");
    if (dagger != 0 && dagger != 1) return fail(WD_ERR_ARG, "dagger must be 0 or 1");
    if (in == out) return fail(WD_ERR_ARG, "in and out must not overlap");
    hipStream_t s = (hipStream_t)stream;
    int err = WD_OK;
    void *g = gauge_for(lat, prec, s, &err);
    if (!g) return err;
    const int V = lat->g.V;
    size_t one = field_data_bytes(prec, V, nrhs) + 256;
    void *mem = nullptr;
    hipError_t he = hipMallocAsync(&mem, 2 * one, s);
    if (he != hipSuccess)
        return fail(WD_ERR_NOMEM, "workspace allocation of %zu bytes failed: %s", 2 * one,
                    hipGetErrorString(he));
    char *cur = (char *)mem;
    FieldRef a = carve(cur, prec, nrhs, V);
    cur = (char *)mem + one;
    FieldRef b = carve(cur, prec, nrhs, V);
    launch_import(in, a, lat->g, s);
    dslash(lat, g, kappa, dagger, a, b, nullptr, Gate{nullptr, nullptr, GATE_ACTIVE}, s);
    launch_export(b, out, lat->g, s);
    (void)hipFreeAsync(mem, s);
    WD_LAUNCH_CHECK();
    return WD_OK;
}

int wd_apply_D(wd_lattice *lat, double kappa, int prec, const double *in, double *out,
               void *stream) {
    return wd_apply(lat, kappa, prec, 0, 1, in, out, stream);
}

int wd_apply_Ddag(wd_lattice *lat, double kappa, int prec, const double *in, double *out,
                  void *stream) {
    return wd_apply(lat, kappa, prec, 1, 1, in, out, stream);
}

int wd_apply_schur(wd_lattice *lat, double kappa, int prec, int dagger, int nrhs,
                   const double *in, double *out, void *stream) {
    if (!lat || !in || !out) return fail(WD_ERR_ARG, "null argument");
    if (!valid_prec(prec)) return fail(WD_ERR_ARG, "unknown precision %d", prec);
    if (nrhs < 1 || nrhs > 12) return fail(WD_ERR_ARG, "nrhs = %d outside 1..12", nrhs);
    if (!std::isfinite(kappa)) return fail(WD_ERR_ARG, "kappa not finite");
    if (dagger != 0 && dagger != 1) return fail(WD_ERR_ARG, "dagger must be 0 or 1");
    if (in == out) return fail(WD_ERR_ARG, "in and out must not overlap");
    if (!eo_supported(lat->g))
        return fail(WD_ERR_ARG, "even-odd needs bricks with an even x extent");
    hipStream_t s = (hipStream_t)stream;
    int err = WD_OK;
    void *gh[2];
    if (!gauge_eo_for(lat, prec, s, &err, gh)) return err;
    const int Vh = lat->g.V / 2;
    const size_t one = field_data_bytes(prec, Vh, nrhs) + 256;
    void *mem = nullptr;
    hipError_t he = hipMallocAsync(&mem, 3 * one, s);
    if (he != hipSuccess)
        return fail(WD_ERR_NOMEM, "workspace allocation of %zu bytes failed: %s", 3 * one,
                    hipGetErrorString(he));
    char *cur = (char *)mem;
    FieldRef ve = carve(cur, prec, nrhs, Vh);
    cur = (char *)mem + one;
    FieldRef to = carve(cur, prec, nrhs, Vh);
    cur = (char *)mem + 2 * one;
    FieldRef oe = carve(cur, prec, nrhs, Vh);
    const Gate none{nullptr, nullptr, GATE_ACTIVE};
    launch_import_half(in, ve, 0, lat->g, s);
    // t_o = D_oe v_e ; out_e = v_e - D_eo t_o  (D^dag's blocks for dagger)
    hop_half(lat, gh, 1, kappa, 0.0, dagger, ve, FieldRef{}, to, nullptr, none, s);
    hop_half(lat, gh, 0, -kappa, 1.0, dagger, to, ve, oe, nullptr, none, s);
    launch_export_half(oe, out, 0, lat->g, s);
    launch_zero(to, s);
    launch_export_half(to, out, 1, lat->g, s);  // odd sites of out = 0
    (void)hipFreeAsync(mem, s);
    WD_LAUNCH_CHECK();
    return WD_OK;
}

int wd_set_halo_gauge(wd_lattice *lat, const double *U_prev, void *stream) {
    if (!lat || !U_prev) return fail(WD_ERR_ARG, "null argument");
    if (!halo_supported(lat->g))
        return fail(WD_ERR_ARG, "halo exchange needs the marching stencil (bricks of a multiple "
                                "of 64 sites)");
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lk(lat->mu);
    if (!lat->halo_links) {
        void *p = nullptr;
        if (hipMalloc(&p, gauge_bytes(WD_F64, lat->g.V / lat->g.L[3])) != hipSuccess)
            return fail(WD_ERR_NOMEM, "hipMalloc of the halo links failed");
        lat->halo_links = p;
    }
    launch_halo_links(lat->g, U_prev, lat->halo_links, s);
    WD_LAUNCH_CHECK();
    WD_HIP_CHECK(hipStreamSynchronize(s));
    return WD_OK;
}

int wd_halo_pack(wd_lattice *lat, int dagger, const wd_field *in, double *send_prev,
                 double *send_next, void *stream) {
    if (!lat || !in || !send_prev || !send_next) return fail(WD_ERR_ARG, "null argument");
    if (in->lat != lat) return fail(WD_ERR_ARG, "field of another lattice");
    if (in->prec != WD_F64) return fail(WD_ERR_ARG, "halo exchange is float64");
    if (dagger != 0 && dagger != 1) return fail(WD_ERR_ARG, "dagger must be 0 or 1");
    if (send_prev == send_next) return fail(WD_ERR_ARG, "the two faces must not overlap");
    launch_halo_pack(lat->g, dagger, in->ref, send_prev, send_next, (hipStream_t)stream);
    WD_LAUNCH_CHECK();
    return WD_OK;
}

int wd_dslash_halo(wd_lattice *lat, double kappa, int dagger, const wd_field *in, wd_field *out,
                   const double *recv_prev, const double *recv_next, uint32_t flags,
                   void *stream) {
    const bool interior = (flags & WD_HALO_INTERIOR) != 0;
    if (!lat || !in || !out || (!interior && (!recv_prev || !recv_next)))
        return fail(WD_ERR_ARG, "null argument");
    if (in == out) return fail(WD_ERR_ARG, "in and out must be different fields");
    if (in->lat != lat || out->lat != lat) return fail(WD_ERR_ARG, "fields of another lattice");
    if (in->prec != WD_F64 || out->prec != WD_F64)
        return fail(WD_ERR_ARG, "halo exchange is float64");
    if (in->nrhs != out->nrhs) return fail(WD_ERR_ARG, "in/out nrhs differ");
    if (!std::isfinite(kappa)) return fail(WD_ERR_ARG, "kappa not finite");
    if (dagger != 0 && dagger != 1) return fail(WD_ERR_ARG, "dagger must be 0 or 1");
    if (flags & ~(uint32_t)(WD_HALO_FIRST | WD_HALO_LAST | WD_HALO_INTERIOR | WD_HALO_ENDS))
        return fail(WD_ERR_ARG, "unknown halo flags 0x%x", flags);
    if (interior && (flags & WD_HALO_ENDS))
        return fail(WD_ERR_ARG, "WD_HALO_INTERIOR and WD_HALO_ENDS exclude each other");
    if (!halo_supported(lat->g))
        return fail(WD_ERR_ARG, "halo exchange needs the marching stencil (bricks of a multiple "
                                "of 64 sites)");
    if (!lat->has_gauge) return fail(WD_ERR_NOGAUGE, "gauge field not set");
    if (!lat->halo_links) return fail(WD_ERR_STATE, "halo links not set (wd_set_halo_gauge)");
    hipStream_t s = (hipStream_t)stream;
    const int region = interior ? 1 : ((flags & WD_HALO_ENDS) ? 2 : 0);
    const double k = -lat->hop_sign * kappa;
    if (interior) {
        // no staged face is read: the faces need not have arrived
        const Halo halo{nullptr, nullptr, lat->halo_links, (flags & WD_HALO_FIRST) ? 1 : 0,
                        (flags & WD_HALO_LAST) ? 1 : 0, region, 0, 1};
        timed("halo_f64", s, [&] {
            launch_dslash_halo(lat->g, lat->gauge[WD_F64], k, dagger, in->ref, out->ref, halo, s,
                               lat->gauge12);
        });
        WD_LAUNCH_CHECK();
        return WD_OK;
    }
    const int vf = lat->g.V / lat->g.L[3];
    const size_t one = field_data_bytes(WD_F64, vf, in->nrhs) + 256;
    void *mem = nullptr;
    hipError_t he = hipMallocAsync(&mem, 2 * one, s);
    if (he != hipSuccess)
        return fail(WD_ERR_NOMEM, "workspace allocation of %zu bytes failed: %s", 2 * one,
                    hipGetErrorString(he));
    char *cur = (char *)mem;
    FieldRef sp = carve(cur, WD_F64, in->nrhs, vf);
    cur = (char *)mem + one;
    FieldRef sn = carve(cur, WD_F64, in->nrhs, vf);
    launch_halo_stage(lat->g, recv_prev, sp, s);
    launch_halo_stage(lat->g, recv_next, sn, s);
    const Halo halo{sp.data, sn.data, lat->halo_links, (flags & WD_HALO_FIRST) ? 1 : 0,
                    (flags & WD_HALO_LAST) ? 1 : 0, region, 0, 1};
    timed("halo_f64", s, [&] {
        launch_dslash_halo(lat->g, lat->gauge[WD_F64], k, dagger, in->ref, out->ref, halo, s,
                           lat->gauge12);
    });
    (void)hipFreeAsync(mem, s);
    WD_LAUNCH_CHECK();
    return WD_OK;
}

int wd_timing_enable(int on) {
    std::lock_guard<std::mutex> lk(g_tmu);
    g_timing.store(on ? 1 : 0);
    return WD_OK;
}

int wd_timing_reset(void) {
    std::lock_guard<std::mutex> lk(g_tmu);
    drain_pending_locked();
    g_times.clear();
    return WD_OK;
}

int wd_timing_read(const char *name, double *total_ms, int64_t *count) {
    if (!name || !total_ms || !count) return fail(WD_ERR_ARG, "null argument");
    std::lock_guard<std::mutex> lk(g_tmu);
    drain_pending_locked();
    auto it = g_times.find(name);
    if (it == g_times.end()) {
        *total_ms = 0.0;
        *count = 0;
    } else {
        *total_ms = it->second.ms;
        *count = it->second.count;
    }
    return WD_OK;
}

}  // extern "C"
