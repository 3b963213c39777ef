// C ABI of the library (declared in include/nsf.h): argument validation,
// workspace layout, the per-algorithm kernel sequences of one residual
// evaluation and the low-storage RK time loop (paper Section 2, Figure 1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "nsf.h"
#include "nsf_internal.h"

namespace nsf {

// ------------------------------------------------------------ error text
namespace {
thread_local std::string g_err;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

}  // namespace

int set_error(int code, const char* msg) {
    g_err = msg ? msg : "";
    return code;
}

namespace {
int check_hip(const char* where) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(NSF_EHIP, "%s: %s", where, hipGetErrorString(e));
    return NSF_OK;
}
}  // namespace

// ------------------------------------------------------------ kernel timer
namespace {
struct Timer {
    std::mutex mu;
    std::string family;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    size_t used = 0;
};
Timer& timer() {
    static Timer* t = new Timer();  // intentionally never destroyed
    return *t;
}
}  // namespace

TimerScope::TimerScope(const char* family, hipStream_t s) : on(false), stream(s) {
    Timer& t = timer();
    std::lock_guard<std::mutex> lk(t.mu);
    if (t.family.empty() || t.family != family) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    if (t.used == t.ev.size()) {
        hipEvent_t a, b;
        if (hipEventCreate(&a) != hipSuccess) return;
        if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); return; }
        t.ev.emplace_back(a, b);
    }
    if (hipEventRecord(t.ev[t.used].first, s) != hipSuccess) return;
    on = true;
}

TimerScope::~TimerScope() {
    if (!on) return;
    Timer& t = timer();
    std::lock_guard<std::mutex> lk(t.mu);
    if (hipEventRecord(t.ev[t.used].second, stream) == hipSuccess) ++t.used;
}

// ------------------------------------------------------------ constants
template <typename T>
Coef<T> make_coef(const Dims& d, double Re, double Ma, double Pr, double gamma) {
    Coef<T> c;
    const int n[3] = {d.nx, d.ny, d.nz};
    for (int a = 0; a < 3; ++a) {
        const double h = 2.0 * M_PI / (double)n[a];
        c.a1[a] = (T)(8.0 / (12.0 * h));
        c.a2[a] = (T)(-1.0 / (12.0 * h));
        c.b0[a] = (T)(-30.0 / (12.0 * h * h));
        c.b1[a] = (T)(16.0 / (12.0 * h * h));
        c.b2[a] = (T)(-1.0 / (12.0 * h * h));
    }
    c.inv_Re = (T)(1.0 / Re);
    c.third = (T)(1.0 / 3.0);
    c.two_thirds = (T)(2.0 / 3.0);
    c.gm1 = (T)(gamma - 1.0);
    c.gM2 = (T)(gamma * Ma * Ma);
    c.kappa = (T)(1.0 / ((gamma - 1.0) * Ma * Ma * Pr * Re));
    c.b0s = c.b0[0] + c.b0[1] + c.b0[2];
    return c;
}
template Coef<float> make_coef<float>(const Dims&, double, double, double, double);
template Coef<double> make_coef<double>(const Dims&, double, double, double, double);

// ------------------------------------------------------------ layout
namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t prim = 0, deriv = 0, prod = 0, qb = 0, qc = 0, mon = 0, diag_partial = 0,
           diag_out = 0, total = 0;
    int nderiv = 0;
    bool fused = false;     // fused SN / RA stages
    bool ss_fused = false;  // fused SS stages
    bool pg_mon = false;    // SS / RS monitor folded into the first stage's gradient pass
    bool zs_mon = false;    // SN / RA (stored primitives) monitor folded into its residual pass
};

int zchunk_of(const Dims& d, const nsf_tuning* tune) {
    return tune && tune->zchunk > 0 ? tune->zchunk : default_zchunk(d);
}

int tile_y_of(const Dims& d, const nsf_tuning* tune, int es) {
    return tune && (tune->block_y == 8 || tune->block_y == 16) ? tune->block_y : default_tile_y(es, d);
}

// Store set of the stored-gradient algorithms (nsf_tuning.gstore): 9 = the
// nine velocity gradients (the paper's 3D set), 3 = the three diagonal ones,
// 4 = the four in-plane ones (single-plane grids only, the paper's 2D count);
// 0 = the algorithm's own, nine in 3D and four on a single plane. The
// untiled kernels store all nine.
int gmask_of(const Dims& d, int variant, const nsf_tuning* tune) {
    if (variant != NSF_SS && variant != NSF_RS) return 0;
    if (tune && tune->naive) return kGradAll;
    const int g = tune ? tune->gstore : 0;
    if (g == 3) return kGradDiag;
    if (g == 4 || (g == 0 && d.nz == 1)) return kGradPlane;
    return kGradAll;
}

int validate_tune(const Dims& d, int variant, const nsf_tuning* tune) {
    if (!tune || variant == NSF_AUTO) return NSF_OK;
    const int g = tune->gstore;
    if (g != 0 && g != 3 && g != 4 && g != 9)
        return fail(NSF_EINVAL, "tuning gstore %d: 0, 3, 4 or 9", g);
    if (g != 0 && variant != NSF_SS && variant != NSF_RS)
        return fail(NSF_EINVAL, "tuning gstore applies to SS and RS only");
    if (g == 4 && d.nz != 1)
        return fail(NSF_EINVAL, "the four in-plane gradients store set needs a single-plane grid");
    if ((g == 3 || g == 4) && tune->naive)
        return fail(NSF_EUNSUPPORTED, "the untiled kernels store all nine gradients");
    return NSF_OK;
}

bool wants_fused(int variant, const nsf_tuning* tune) {
    return (variant == NSF_RA || variant == NSF_SN) && tune && tune->fuse && !tune->naive;
}

// SS with the stage update applied in the residual kernel's epilogue
bool wants_ss_fused(int variant, const nsf_tuning* tune) {
    return variant == NSF_SS && tune && tune->fuse && !tune->naive;
}

// Double-precision tiled SS / RS: the monitored step takes the kinetic energy
// and enstrophy of its input from the first stage's primitive and gradient
// pass instead of a separate diagnostics pass.
bool pg_monitor(int variant, int precision, const nsf_tuning* tune) {
    return (variant == NSF_SS || variant == NSF_RS) && precision == NSF_F64 && !(tune && tune->naive);
}

// Double-precision tiled SN / RA with stored primitives: the same from the
// first stage's residual pass.
bool zs_monitor(int variant, int precision, const nsf_tuning* tune) {
    return (variant == NSF_SN || variant == NSF_RA) && precision == NSF_F64 &&
           !(tune && (tune->naive || tune->fuse));
}

bool is_variant(int v) { return v >= NSF_BL && v <= NSF_AUTO; }

// NSF_AUTO -> the recorded (or default) algorithm and tuning; `store`
// receives the tuning when it has to be substituted.
void resolve(const Dims& d, int precision, int* variant, const nsf_tuning** tune,
             nsf_tuning* store) {
    if (*variant != NSF_AUTO) return;
    int v = NSF_SN;
    std::memset(store, 0, sizeof *store);
    if (!tune_lookup(d, precision, &v, store)) {
        v = NSF_SN;
        store->fuse = 1;
    }
    *variant = v;
    *tune = store;
}
bool is_precision(int p) { return p == NSF_F64 || p == NSF_F32; }

int deriv_arrays(const Dims& d, int variant, const nsf_tuning* tune) {
    switch (variant) {
        case NSF_BL: return 60;
        case NSF_SS:
        case NSF_RS: return __builtin_popcount(gmask_of(d, variant, tune));
        default: return 0;
    }
}

Layout layout_for(const Dims& d, int variant, int precision, const nsf_tuning* tune) {
    const size_t es = precision == NSF_F32 ? 4 : 8;
    Layout L;
    L.fused = wants_fused(variant, tune);
    L.ss_fused = wants_ss_fused(variant, tune);
    size_t off = 0;
    L.prim = off;
    off = align_up(off + 5 * d.npts * es);
    L.nderiv = deriv_arrays(d, variant, tune);
    L.deriv = off;
    off = align_up(off + (size_t)L.nderiv * d.npts * es);
    L.prod = off;
    off = align_up(off + (variant == NSF_BL ? d.npts * es : 0));
    // fused SN / RA stages rotate the state through q -> qb -> qc -> q. qb
    // shares the primitive region: nsf_rhs uses the primitives and
    // nsf_rk_step the rotating state, never both in one call. Fused SS
    // stages read the primitives, and rotate through q -> r -> qc -> q.
    L.qb = L.fused ? L.prim : off;
    L.qc = off;
    off = align_up(off + (L.fused || L.ss_fused ? 5 * d.npts * es : 0));
    // per-tile (KE, enstrophy) sums of the monitored first stage: the fused
    // SN / RA stage's tiles, or the double-precision SS / RS primitive and
    // gradient kernel's
    L.pg_mon = pg_monitor(variant, precision, tune);
    L.zs_mon = zs_monitor(variant, precision, tune);
    L.mon = off;
    off = align_up(off + (L.fused || L.zs_mon ? 2 * sizeof(double) *
                                                  (size_t)sweep_tiles(d, zchunk_of(d, tune),
                                                                      tile_y_of(d, tune, (int)es))
                          : L.pg_mon ? 2 * sizeof(double) * (size_t)ss_prims_grad_tiles(d)
                                     : 0));
    L.diag_partial = off;
    off = align_up(off + diag_partial_count(d) * NSF_NDIAG * sizeof(double));
    L.diag_out = off;
    off = align_up(off + NSF_NDIAG * sizeof(double));
    L.total = off;
    return L;
}

int validate_grid(const nsf_grid* g, Dims* d) {
    if (!g) return fail(NSF_EINVAL, "grid is NULL");
    // radius-2 stencils need five distinct points per axis; nz = 1 is the
    // two-dimensional (z-independent) problem, where every z-difference is 0
    if (g->nx < 5 || g->ny < 5 || (g->nz < 5 && g->nz != 1))
        return fail(NSF_EINVAL, "grid %dx%dx%d: x and y need >= 5 points, z >= 5 or 1 (2D)",
                    g->nx, g->ny, g->nz);
    const size_t n = (size_t)g->nx * g->ny * g->nz;
    if (n > (size_t)1 << 31) return fail(NSF_EINVAL, "grid has %zu points, limit 2^31", n);
    // the fused stage addresses one z-plane of doubles with 32-bit byte offsets
    if ((size_t)g->nx * g->ny >= (size_t)1 << 28)
        return fail(NSF_EINVAL, "grid plane %dx%d has 2^28 or more points", g->nx, g->ny);
    d->nx = g->nx;
    d->ny = g->ny;
    d->nz = g->nz;
    d->npts = n;
    return NSF_OK;
}

int validate_phys(const nsf_phys* p) {
    if (!p) return fail(NSF_EINVAL, "phys is NULL");
    if (!(p->Re > 0) || !(p->Ma > 0) || !(p->Pr > 0) || !(p->gamma > 1) || !std::isfinite(p->Re) ||
        !std::isfinite(p->Ma) || !std::isfinite(p->Pr) || !std::isfinite(p->gamma))
        return fail(NSF_EINVAL, "phys: need finite Re, Ma, Pr > 0 and gamma > 1");
    return NSF_OK;
}

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
    const char* x = (const char*)a;
    const char* y = (const char*)b;
    return x < y + nb && y < x + na;
}

// One residual evaluation r = R(q) with algorithm `variant`.
template <typename T>
int rhs_impl(const Dims& d, const nsf_phys* ph, int variant, const nsf_tuning* tune, const T* q,
             T* r, char* work, const Layout& L, hipStream_t s, double* mpart = nullptr) {
    (void)tune;
    const Coef<T> c = make_coef<T>(d, ph->Re, ph->Ma, ph->Pr, ph->gamma);
    T* prim = (T*)(work + L.prim);
    const size_t n = d.npts;
    const T* rho = q;
    const T* m[3] = {q + n, q + 2 * n, q + 3 * n};
    const T* E = q + 4 * n;
    const T* vel[3] = {prim, prim + n, prim + 2 * n};
    const T* p = prim + 3 * n;
    const T* Tt = prim + 4 * n;
    switch (variant) {
        case NSF_BL: {
            // primitives in three loops, then one loop per derivative
            launch_prims_bl<T>(d, c, q, prim, s);
            T* dv = (T*)(work + L.deriv);
            T* prod = (T*)(work + L.prod);
            auto D = [&](int idx) { return dv + (size_t)idx * n; };
            for (int b = 0; b < 3; ++b) {
                launch_bl_deriv<T>(d, c, b, 1, rho, D(0 + b), s);
                launch_bl_deriv<T>(d, c, b, 1, E, D(12 + b), s);
                launch_bl_deriv<T>(d, c, b, 1, p, D(39 + b), s);
                launch_bl_deriv<T>(d, c, b, 2, Tt, D(57 + b), s);
                for (int a = 0; a < 3; ++a) {
                    launch_bl_deriv<T>(d, c, b, 1, m[a], D(3 + 3 * a + b), s);
                    launch_bl_deriv<T>(d, c, b, 1, vel[a], D(15 + 3 * a + b), s);
                    launch_bl_deriv<T>(d, c, b, 2, vel[a], D(42 + 3 * a + b), s);
                    launch_product<T>(d, m[a], vel[b], prod, s);
                    launch_bl_deriv<T>(d, c, b, 1, prod, D(24 + 3 * a + b), s);
                }
                launch_product<T>(d, E, vel[b], prod, s);
                launch_bl_deriv<T>(d, c, b, 1, prod, D(33 + b), s);
                launch_product<T>(d, p, vel[b], prod, s);
                launch_bl_deriv<T>(d, c, b, 1, prod, D(36 + b), s);
            }
            // cross derivatives D_a(G_kk) from the stored diagonal gradients
            const int pairs[6][2] = {{0, 1}, {0, 2}, {1, 0}, {1, 2}, {2, 0}, {2, 1}};
            for (int t = 0; t < 6; ++t) {
                const int a = pairs[t][0], kk = pairs[t][1];
                launch_bl_deriv<T>(d, c, a, 1, D(15 + 4 * kk), D(51 + t), s);
            }
            launch_bl_assemble<T>(d, c, q, prim, dv, r, s);
            break;
        }
        case NSF_RA:
        case NSF_SN:
            launch_prims<T>(d, c, q, prim, s);
            if (tune && tune->naive) launch_ra_naive<T>(d, c, q, prim, r, s);
            else launch_ra_zsweep<T>(d, c, q, prim, r, zchunk_of(d, tune), tile_y_of(d, tune, sizeof(T)), s,
                                     variant == NSF_RA, mpart);
            break;
        case NSF_SS:
        case NSF_RS: {
            T* grad = (T*)(work + L.deriv);
            if (tune && tune->naive) {
                launch_prims<T>(d, c, q, prim, s);
                launch_ss_grad_naive<T>(d, c, prim, grad, s);
                launch_ss_naive<T>(d, c, q, prim, grad, r, s);
            } else {
                // the primitive and gradient loops in one pass (same values)
                const int gm = gmask_of(d, variant, tune);
                launch_ss_prims_grad<T>(d, c, q, prim, grad, gm, s, mpart);
                launch_ss_zsweep<T>(d, c, q, prim, grad, r, zchunk_of(d, tune),
                                    tile_y_of(d, tune, sizeof(T)), s, variant == NSF_RS, gm);
            }
            break;
        }
        default:
            return fail(NSF_EUNSUPPORTED, "variant %d", variant);
    }
    return check_hip("rhs launch");
}

// monitor (device, 2 * nsteps doubles, or NULL): mean kinetic energy and
// enstrophy of the state at the start of every step.
template <typename T>
int rk_impl(const Dims& d, const nsf_phys* ph, int variant, const nsf_tuning* tune, double dt,
            int nsteps, T* q, double* qacc, T* r, char* work, const Layout& L, hipStream_t s,
            double* monitor = nullptr) {
    static const double A[2] = {2.0 / 3.0, 5.0 / 12.0};
    static const double B[3] = {1.0 / 4.0, 3.0 / 20.0, 3.0 / 5.0};
    const double inv_n = 1.0 / (double)d.npts;
    if (L.fused) {
        const Coef<T> c = make_coef<T>(d, ph->Re, ph->Ma, ph->Pr, ph->gamma);
        const int zc = zchunk_of(d, tune);
        const int ty = tile_y_of(d, tune, sizeof(T));
        T* qb = (T*)(work + L.qb);
        T* qc = (T*)(work + L.qc);
        T* in[3] = {q, qb, qc};
        T* out[3] = {qb, qc, q};
        double* mpart = (double*)(work + L.mon);
        for (int step = 0; step < nsteps; ++step)
            for (int st = 0; st < 3; ++st) {
                StageCoef sc;
                sc.a_dt = st < 2 ? A[st] * dt : 0.0;
                sc.b_dt = B[st] * dt;
                sc.last = st == 2;
                // double precision: the state and the accumulator are equal at
                // a step boundary, so the first substep reads the accumulator
                // from q and stores none (the second forms the first's
                // accumulator, q0 + B_1 dt R_1, as q0 + (B_1 / A_1)(q1 - q0)
                // from the step's initial state, still in q, and its own
                // input), and only the call's last step stores q_acc in its
                // third substep (the next step reads the state from q)
                if (sizeof(T) == 8) {
                    sc.acc_from_q = st == 0;
                    sc.store_acc = st == 1 || (st == 2 && step == nsteps - 1);
                    if (st == 1) {
                        sc.acc_src = q;
                        sc.acc_mix = B[0] / A[0];
                    }
                }
                const bool mon = monitor && st == 0;
                launch_ra_fused<T>(d, c, in[st], out[st], qacc, sc, zc, ty, s,
                                   mon ? mpart : nullptr, variant == NSF_RA);
                if (mon)
                    launch_monitor_final(mpart, sweep_tiles(d, zc, ty), inv_n, monitor + 2 * step, s);
            }
        return check_hip("rk_step launch");
    }
    const Coef<double> cd = make_coef<double>(d, ph->Re, ph->Ma, ph->Pr, ph->gamma);
    if (L.ss_fused) {
        const Coef<T> c = make_coef<T>(d, ph->Re, ph->Ma, ph->Pr, ph->gamma);
        T* prim = (T*)(work + L.prim);
        T* grad = (T*)(work + L.deriv);
        T* qc = (T*)(work + L.qc);
        T* in[3] = {q, r, qc};
        T* out[3] = {r, qc, q};
        const int gm = gmask_of(d, variant, tune);
        const int zc = zchunk_of(d, tune);
        const int ty = tile_y_of(d, tune, sizeof(T));
        double* mpart = (double*)(work + L.mon);
        for (int step = 0; step < nsteps; ++step) {
            if (monitor && !L.pg_mon) {
                double* dout = (double*)(work + L.diag_out);
                launch_diag<T>(d, cd, q, (double*)(work + L.diag_partial), dout, s);
                hipError_t e = hipMemcpyAsync(monitor + 2 * step, dout, 2 * sizeof(double),
                                              hipMemcpyDeviceToDevice, s);
                if (e != hipSuccess) return fail(NSF_EHIP, "monitor copy: %s", hipGetErrorString(e));
            }
            for (int st = 0; st < 3; ++st) {
                StageCoef sc;
                sc.a_dt = st < 2 ? A[st] * dt : 0.0;
                sc.b_dt = B[st] * dt;
                sc.last = st == 2;
                const bool mon = monitor && L.pg_mon && st == 0;
                launch_ss_prims_grad<T>(d, c, in[st], prim, grad, gm, s, mon ? mpart : nullptr);
                if (mon)
                    launch_monitor_final(mpart, ss_prims_grad_tiles(d), inv_n, monitor + 2 * step, s);
                launch_ss_fused<T>(d, c, in[st], prim, grad, out[st], qacc, sc, zc, ty, s, gm);
            }
        }
        return check_hip("rk_step launch");
    }
    double* mpart = (double*)(work + L.mon);
    const bool folded = L.pg_mon || L.zs_mon;
    const int mon_tiles = L.pg_mon ? ss_prims_grad_tiles(d)
                                   : sweep_tiles(d, zchunk_of(d, tune), tile_y_of(d, tune, sizeof(T)));
    for (int step = 0; step < nsteps; ++step) {
        if (monitor && !folded) {
            // the diagnostics pass writes NDIAG means; KE and enstrophy lead
            double* dout = (double*)(work + L.diag_out);
            launch_diag<T>(d, cd, q, (double*)(work + L.diag_partial), dout, s);
            hipError_t e = hipMemcpyAsync(monitor + 2 * step, dout, 2 * sizeof(double),
                                          hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) return fail(NSF_EHIP, "monitor copy: %s", hipGetErrorString(e));
        }
        for (int st = 0; st < 3; ++st) {
            // double precision, SS / RS and SN / RA with stored primitives:
            // the first stage's gradient or residual pass also sums the
            // monitor of its input state
            const bool mon = monitor && folded && st == 0;
            int rc = rhs_impl<T>(d, ph, variant, tune, q, r, work, L, s, mon ? mpart : nullptr);
            if (rc) return rc;
            if (mon) launch_monitor_final(mpart, mon_tiles, inv_n, monitor + 2 * step, s);
            StageCoef sc;
            sc.a_dt = st < 2 ? A[st] * dt : 0.0;
            sc.b_dt = B[st] * dt;
            sc.last = st == 2;
            launch_update<T>(d, sc, r, q, qacc, s);
        }
    }
    return check_hip("rk_step launch");
}

}  // namespace
}  // namespace nsf

using namespace nsf;

extern "C" {

const char* nsf_status_string(int status) {
    switch (status) {
        case NSF_OK: return "NSF_OK";
        case NSF_EINVAL: return "NSF_EINVAL: invalid argument";
        case NSF_EWORKSPACE: return "NSF_EWORKSPACE: work buffer too small";
        case NSF_EHIP: return "NSF_EHIP: HIP runtime error";
        case NSF_EUNSUPPORTED: return "NSF_EUNSUPPORTED: not supported";
        case NSF_ENONFINITE: return "NSF_ENONFINITE: non-finite values in state";
        default: return "unknown nsf status";
    }
}

const char* nsf_last_error(void) { return g_err.c_str(); }

int nsf_version(void) { return 100; }

int nsf_workspace_bytes(const nsf_grid* g, int variant, int precision, const nsf_tuning* tune,
                        size_t* bytes) {
    (void)tune;
    Dims d;
    int rc = validate_grid(g, &d);
    if (rc) return rc;
    if (!is_variant(variant)) return fail(NSF_EINVAL, "variant %d", variant);
    if (!is_precision(precision)) return fail(NSF_EINVAL, "precision %d", precision);
    if (!bytes) return fail(NSF_EINVAL, "bytes is NULL");
    if ((rc = validate_tune(d, variant, tune))) return rc;
    nsf_tuning store;
    resolve(d, precision, &variant, &tune, &store);
    *bytes = layout_for(d, variant, precision, tune).total;
    return NSF_OK;
}

int nsf_init_fields(const nsf_grid* g, const nsf_phys* phys, const nsf_tgv* tgv, int precision,
                    void* q, double* q_acc, void* stream) {
    Dims d;
    int rc = validate_grid(g, &d);
    if (rc) return rc;
    if ((rc = validate_phys(phys))) return rc;
    if (!tgv) return fail(NSF_EINVAL, "tgv is NULL");
    if (!is_precision(precision)) return fail(NSF_EINVAL, "precision %d", precision);
    if (!q) return fail(NSF_EINVAL, "q is NULL");
    if (tgv->pert_kind < 0 || tgv->pert_kind > 2) return fail(NSF_EINVAL, "pert_kind %d", tgv->pert_kind);
    if (!std::isfinite(tgv->V0) || !std::isfinite(tgv->pert_amp)) return fail(NSF_EINVAL, "tgv values not finite");
    InitParams p;
    p.gamma = phys->gamma;
    p.Ma = phys->Ma;
    p.V0 = tgv->V0;
    p.amp = tgv->pert_amp;
    p.seed = tgv->seed;
    p.kind = tgv->pert_kind;
    for (int a = 0; a < 3; ++a) p.phase[a] = tgv->phase[a];
    hipStream_t s = (hipStream_t)stream;
    if (precision == NSF_F64) launch_init<double>(d, p, (double*)q, q_acc, s);
    else launch_init<float>(d, p, (float*)q, q_acc, s);
    return check_hip("init launch");
}

int nsf_rhs(const nsf_grid* g, const nsf_phys* phys, int variant, int precision,
            const nsf_tuning* tune, const void* q, void* r, void* work, size_t work_bytes,
            void* stream) {
    Dims d;
    int rc = validate_grid(g, &d);
    if (rc) return rc;
    if ((rc = validate_phys(phys))) return rc;
    if (!is_variant(variant)) return fail(NSF_EINVAL, "variant %d", variant);
    if (!is_precision(precision)) return fail(NSF_EINVAL, "precision %d", precision);
    if (!q || !r || !work) return fail(NSF_EINVAL, "q, r and work must be non-NULL");
    if ((rc = validate_tune(d, variant, tune))) return rc;
    nsf_tuning store;
    resolve(d, precision, &variant, &tune, &store);
    const Layout L = layout_for(d, variant, precision, tune);
    if (work_bytes < L.total)
        return fail(NSF_EWORKSPACE, "work is %zu bytes, need %zu", work_bytes, L.total);
    const size_t fb = 5 * d.npts * (precision == NSF_F32 ? 4 : 8);
    if (overlap(q, fb, r, fb) || overlap(r, fb, work, L.total) || overlap(q, fb, work, L.total))
        return fail(NSF_EINVAL, "q, r and work must not overlap");
    hipStream_t s = (hipStream_t)stream;
    if (precision == NSF_F64)
        return rhs_impl<double>(d, phys, variant, tune, (const double*)q, (double*)r, (char*)work, L, s);
    return rhs_impl<float>(d, phys, variant, tune, (const float*)q, (float*)r, (char*)work, L, s);
}

namespace {
int rk_entry(const nsf_grid* g, const nsf_phys* phys, int variant, int precision,
             const nsf_tuning* tune, double dt, int32_t nsteps, void* q, double* q_acc, void* r,
             void* work, size_t work_bytes, double* monitor, void* stream) {
    Dims d;
    int rc = validate_grid(g, &d);
    if (rc) return rc;
    if ((rc = validate_phys(phys))) return rc;
    if (!is_variant(variant)) return fail(NSF_EINVAL, "variant %d", variant);
    if (!is_precision(precision)) return fail(NSF_EINVAL, "precision %d", precision);
    if (!q || !q_acc || !r || !work) return fail(NSF_EINVAL, "q, q_acc, r and work must be non-NULL");
    if (nsteps < 0) return fail(NSF_EINVAL, "nsteps %d", nsteps);
    if (!std::isfinite(dt)) return fail(NSF_EINVAL, "dt not finite");
    if ((rc = validate_tune(d, variant, tune))) return rc;
    nsf_tuning store;
    resolve(d, precision, &variant, &tune, &store);
    const Layout L = layout_for(d, variant, precision, tune);
    if (work_bytes < L.total)
        return fail(NSF_EWORKSPACE, "work is %zu bytes, need %zu", work_bytes, L.total);
    const size_t fb = 5 * d.npts * (precision == NSF_F32 ? 4 : 8);
    const size_t ab = 5 * d.npts * sizeof(double);
    if (overlap(q, fb, r, fb) || overlap(q, fb, q_acc, ab) || overlap(r, fb, q_acc, ab) ||
        overlap(q, fb, work, L.total) || overlap(r, fb, work, L.total) ||
        overlap(q_acc, ab, work, L.total))
        return fail(NSF_EINVAL, "q, q_acc, r and work must not overlap");
    const size_t mb = 2 * sizeof(double) * (size_t)nsteps;
    if (monitor && (overlap(monitor, mb, q, fb) || overlap(monitor, mb, q_acc, ab) ||
                    overlap(monitor, mb, r, fb) || overlap(monitor, mb, work, L.total)))
        return fail(NSF_EINVAL, "monitor must not overlap q, q_acc, r or work");
    hipStream_t s = (hipStream_t)stream;
    if (precision == NSF_F64)
        return rk_impl<double>(d, phys, variant, tune, dt, nsteps, (double*)q, q_acc, (double*)r,
                               (char*)work, L, s, monitor);
    return rk_impl<float>(d, phys, variant, tune, dt, nsteps, (float*)q, q_acc, (float*)r,
                          (char*)work, L, s, monitor);
}
}  // namespace

int nsf_rk_step(const nsf_grid* g, const nsf_phys* phys, int variant, int precision,
                const nsf_tuning* tune, double dt, int32_t nsteps, void* q, double* q_acc,
                void* r, void* work, size_t work_bytes, void* stream) {
    return rk_entry(g, phys, variant, precision, tune, dt, nsteps, q, q_acc, r, work, work_bytes,
                    nullptr, stream);
}

int nsf_rk_step_monitored(const nsf_grid* g, const nsf_phys* phys, int variant, int precision,
                          const nsf_tuning* tune, double dt, int32_t nsteps, void* q,
                          double* q_acc, void* r, void* work, size_t work_bytes, double* monitor,
                          void* stream) {
    if (!monitor) return fail(NSF_EINVAL, "monitor is NULL");
    if ((uintptr_t)monitor % sizeof(double)) return fail(NSF_EINVAL, "monitor is not 8-byte aligned");
    return rk_entry(g, phys, variant, precision, tune, dt, nsteps, q, q_acc, r, work, work_bytes,
                    monitor, stream);
}

int nsf_diagnostics(const nsf_grid* g, const nsf_phys* phys, int precision, const void* q,
                    void* work, size_t work_bytes, double* out, void* stream) {
    Dims d;
    int rc = validate_grid(g, &d);
    if (rc) return rc;
    if ((rc = validate_phys(phys))) return rc;
    if (!is_precision(precision)) return fail(NSF_EINVAL, "precision %d", precision);
    if (!q || !work || !out) return fail(NSF_EINVAL, "q, work and out must be non-NULL");
    // the diagnostics region is the tail of every layout; RA's is the smallest
    const Layout L = layout_for(d, NSF_RA, precision, nullptr);
    if (work_bytes < L.total)
        return fail(NSF_EWORKSPACE, "work is %zu bytes, need %zu", work_bytes, L.total);
    hipStream_t s = (hipStream_t)stream;
    char* w = (char*)work;
    const Coef<double> c = make_coef<double>(d, phys->Re, phys->Ma, phys->Pr, phys->gamma);
    double* partial = (double*)(w + L.diag_partial);
    double* dout = (double*)(w + L.diag_out);
    if (precision == NSF_F64) launch_diag<double>(d, c, (const double*)q, partial, dout, s);
    else launch_diag<float>(d, c, (const float*)q, partial, dout, s);
    if ((rc = check_hip("diagnostics launch"))) return rc;
    hipError_t e = hipMemcpyAsync(out, dout, NSF_NDIAG * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(NSF_EHIP, "diagnostics copy: %s", hipGetErrorString(e));
    if (out[14] > 0) return fail(NSF_ENONFINITE, "%.0f non-finite values in q", out[14]);
    return NSF_OK;
}

int nsf_diagnostics_noalloc(const nsf_grid* g, const nsf_phys* phys, int precision, const void* q,
                            double* out, void* stream) {
    Dims d;
    int rc = validate_grid(g, &d);
    if (rc) return rc;
    if ((rc = validate_phys(phys))) return rc;
    if (!is_precision(precision)) return fail(NSF_EINVAL, "precision %d", precision);
    if (!q || !out) return fail(NSF_EINVAL, "q and out must be non-NULL");
    if (diag_partial_count(d) > diag_noalloc_max_tiles())
        return fail(NSF_EINVAL, "grid %dx%dx%d needs %zu diagnostics tiles; the allocation-free "
                    "form holds at most %zu", d.nx, d.ny, d.nz, diag_partial_count(d),
                    diag_noalloc_max_tiles());
    const Coef<double> c = make_coef<double>(d, phys->Re, phys->Ma, phys->Pr, phys->gamma);
    if ((rc = diag_noalloc(d, c, precision, q, out, (hipStream_t)stream))) return rc;
    if (out[14] > 0) return fail(NSF_ENONFINITE, "%.0f non-finite values in q", out[14]);
    return NSF_OK;
}

int nsf_device_copy(const void* src, void* dst, size_t bytes, void* stream) {
    if (!src || !dst) return fail(NSF_EINVAL, "src and dst must be non-NULL");
    if (overlap(src, bytes, dst, bytes)) return fail(NSF_EINVAL, "src and dst overlap");
    if ((uintptr_t)src % 16 || (uintptr_t)dst % 16)
        return fail(NSF_EINVAL, "src and dst must be 16-byte aligned");
    launch_copy(src, dst, bytes, (hipStream_t)stream);
    return check_hip("copy launch");
}

static const char* kTimerNames =
    "init,prims,update,bl_product,bl_deriv,bl_assemble,ra_naive,ra_zsweep,ra_fused,ra_fused_mon,"
    "ra_fused_first,ra_fused_last,sn_zsweep,sn_fused,sn_fused_mon,sn_fused_first,sn_fused_last,"
    "ss_grad_naive,ss_naive,ss_prims_grad,ss_zsweep,ss_fused,rs_zsweep,diag,copy,ra_batch,"
    "batch_step";

const char* nsf_timer_names(void) { return kTimerNames; }

int nsf_timer_enable(const char* name) {
    Timer& t = timer();
    std::lock_guard<std::mutex> lk(t.mu);
    t.family = name ? name : "";
    t.used = 0;
    return NSF_OK;
}

int nsf_timer_read(int64_t* count, double* total_ms) {
    if (!count || !total_ms) return fail(NSF_EINVAL, "count and total_ms must be non-NULL");
    Timer& t = timer();
    std::lock_guard<std::mutex> lk(t.mu);
    double ms = 0.0;
    for (size_t i = 0; i < t.used; ++i) {
        hipError_t e = hipEventSynchronize(t.ev[i].second);
        float x = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&x, t.ev[i].first, t.ev[i].second);
        if (e != hipSuccess) return fail(NSF_EHIP, "timer read: %s", hipGetErrorString(e));
        ms += x;
    }
    *count = (int64_t)t.used;
    *total_ms = ms;
    return NSF_OK;
}

}  // extern "C"
