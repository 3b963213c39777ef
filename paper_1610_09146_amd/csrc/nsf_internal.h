// Host-side launch interface between the C ABI (nsf_api.cpp) and the kernel
// translation units. Not exported from the shared library.
#pragma once

#include <hip/hip_runtime.h>

#include "nsf.h"
#include "nsf_device.h"

namespace nsf {

// Store sets of the stored-gradient algorithms (bit 3a + b: G_ab = D_b u_a
// stored in a work array, the stored ones in order of 3a + b): all nine (the
// paper's SS and RS in 3D), the three diagonal ones, or the four in-plane
// ones of a two-dimensional grid (the paper's 2D count; the z gradients
// vanish there and D_x w, D_y w are formed in the tile).
constexpr int kGradAll = 0x1FF, kGradDiag = 0x111, kGradPlane = 0x01B;

struct InitParams {
    double gamma, Ma, V0, amp;
    uint64_t seed;
    int kind;
    double phase[3];
};

// Low-storage RK3 substep coefficients (see nsf_rk_step).
struct StageCoef {
    double a_dt;  // A_s dt (unused on the last substep)
    double b_dt;  // B_s dt
    int last;     // 1 on the third substep: q = q_acc after the update
    // Double-precision fused stages only: the first substep reads the
    // accumulator from the state q (equal to q_acc at a step boundary) and
    // leaves q_acc unwritten; the second forms the accumulator of the first,
    // q0 + B_1 dt R_1 = q0 + (B_1 / A_1)(q1 - q0), from the step's initial
    // state q0 (read from acc_src) and its own input q1 (acc_mix = B_1 / A_1);
    // a third substep other than the call's last leaves q_acc unwritten (its
    // value is the state the next step's first substep reads from q).
    int acc_from_q = 0;
    int store_acc = 1;
    const void* acc_src = nullptr;
    double acc_mix = 0.0;
};

// Record an error message for nsf_last_error() and return `code`.
int set_error(int code, const char* msg);

// Autotuner table (nsf_tune.cpp): the recorded algorithm and tuning.
bool tune_lookup(const Dims& d, int precision, int* variant, nsf_tuning* tune);

// Launch-time kernel timer (nsf_timer_*): brackets launches of the enabled
// kernel family with HIP events on the launch stream.
struct TimerScope {
    TimerScope(const char* family, hipStream_t s);
    ~TimerScope();
    bool on;
    hipStream_t stream;
};

template <typename T>
Coef<T> make_coef(const Dims& d, double Re, double Ma, double Pr, double gamma);

// pointwise kernels (nsf_pointwise.hip)
template <typename T>
void launch_init(const Dims& d, const InitParams& p, T* q, double* qacc, hipStream_t s);
template <typename T>
void launch_prims(const Dims& d, const Coef<T>& c, const T* q, T* prim, hipStream_t s);
template <typename T>
void launch_prims_bl(const Dims& d, const Coef<T>& c, const T* q, T* prim, hipStream_t s);
template <typename T>
void launch_update(const Dims& d, const StageCoef& sc, const T* r, T* q, double* qacc,
                   hipStream_t s);
template <typename T>
void launch_product(const Dims& d, const T* f, const T* g, T* out, hipStream_t s);
void launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s);

// BL derivative kernels and assembly (nsf_bl.hip)
template <typename T>
void launch_bl_deriv(const Dims& d, const Coef<T>& c, int axis, int order, const T* f, T* out,
                     hipStream_t s);
template <typename T>
void launch_bl_assemble(const Dims& d, const Coef<T>& c, const T* q, const T* prim,
                        const T* deriv, T* r, hipStream_t s);

// untiled per-point residual kernels (nsf_naive.hip)
template <typename T>
void launch_ra_naive(const Dims& d, const Coef<T>& c, const T* q, const T* prim, T* r,
                     hipStream_t s);
template <typename T>
void launch_ss_grad_naive(const Dims& d, const Coef<T>& c, const T* prim, T* grad, hipStream_t s);
template <typename T>
void launch_ss_naive(const Dims& d, const Coef<T>& c, const T* q, const T* prim, const T* grad,
                     T* r, hipStream_t s);

// Arguments of one tile sweep (nsf_zsweep.hip): residual to r, or (fused)
// the stage update qout / qacc from the state q.
template <typename T>
struct ZArgs {
    Dims d;
    Coef<T> k;
    const T* q;
    const T* prim;
    const T* grad;  // stored velocity gradients (SS), G_ab at field 3a + b
    T* r;
    T* qout;
    double* qacc;
    const double* qacc_in;  // where the fused stage reads the accumulator (qacc, or q)
    int acc_store;          // fused stage: 0 leaves q_acc unwritten
    // fused stage: the accumulator used is acc + acc_mix * (q_own - acc),
    // q_own the stage input at the point (0 = acc itself)
    double acc_mix;
    double a_dt, b_dt;
    int last;
    int zchunk, tiles_x, tiles_y;
    // fused form, monitored launch: each tile also reduces the kinetic
    // energy and enstrophy sums of its input state into mpart[2 * tile]
    double* mpart;
};

// One instance of a batch: its grid, constants, the three state buffers of
// the fused stage rotation (q -> qb -> qc -> q), the accumulator and dt.
template <typename T>
struct BatchDesc {
    Dims d;
    Coef<T> k;
    T* q;
    T* qb;
    T* qc;
    double* qacc;
    double dt;
    int zchunk, tiles_x, tiles_y, tiles;
};

// z-marching tiled residual kernels (nsf_zsweep.hip)
// Tiles are 32 x tile_y (tile_y = 8 or 16) columns; zchunk planes deep.
constexpr int kXCD = 8;  // gfx950: 8 XCDs, workgroups dispatched round-robin
int default_zchunk(const Dims& d);
int default_tile_y(int precision_bytes, const Dims& d);
void tile_counts(const Dims& d, int zchunk, int tile_y, int* tx, int* ty, int* tz, int* zc);
// Persistent batched fused stage (recompute: RA, else SN): items[i] =
// (instance, tile index), band by band; band x (items boff[x] ..
// boff[x + 1] - 1) is taken in order by the workgroups of XCD x through the
// counter ctr[stage * 8 + x], and then by any workgroup whose own band is
// used up. ctr holds 3 * 8 ints, zero before a batch's first stage; each
// stage launch zeroes the next stage's counters.
// store_acc = 0 lets the double-precision 16-row form leave q_acc unwritten
// in the third substep (every step but a call's last).
template <typename T>
void launch_ra_batch(const BatchDesc<T>* desc, const int2* items, const int* boff, int* ctr,
                     int stage, int nblocks, int tile_y, hipStream_t s, bool recompute,
                     int store_acc);
template <typename T>
int batch_blocks_per_cu(int tile_y, bool recompute);
// Residual from stored primitives, no derivative arrays: recompute = true is
// the recompute-all algorithm RA (every derivative formed where a term uses
// it, equation by equation), false the store-none algorithm SN (every
// derivative formed once per point into thread-local values). With mpart
// (double precision only) each tile also writes the kinetic-energy and
// enstrophy sums of its points to mpart[2 * tile] (sweep_tiles tiles).
template <typename T>
void launch_ra_zsweep(const Dims& d, const Coef<T>& c, const T* q, const T* prim, T* r,
                      int zchunk, int tile_y, hipStream_t s, bool recompute,
                      double* mpart = nullptr);
// Residual with the velocity gradients and D_a(G_cc) read from the nine
// stored gradient arrays: recompute = true is the recompute-some algorithm
// RS (the other derivatives formed where used, equation by equation), false
// the store-some algorithm SS (thread-local values).
template <typename T>
void launch_ss_zsweep(const Dims& d, const Coef<T>& c, const T* q, const T* prim, const T* grad,
                      T* r, int zchunk, int tile_y, hipStream_t s, bool recompute,
                      int gmask = kGradAll);
// Fused SS stage: the stored-gradient residual of q (stored primitives and
// gradients as launch_ss_zsweep) with the stage update applied in its
// epilogue, qout = q_acc + a dt R (b dt in the last stage), q_acc += b dt R;
// qout must not overlap q.
template <typename T>
void launch_ss_fused(const Dims& d, const Coef<T>& c, const T* q, const T* prim, const T* grad,
                     T* qout, double* qacc, const StageCoef& sc, int zchunk, int tile_y,
                     hipStream_t s, int gmask);
// SS / RS primitive and gradient loops in one pass (z-marching tiles): prim =
// u, v, w, p, T of q (eqs (9)-(10)) and the store set's G_ab = D_b u_a. With
// mpart (double precision only) each tile also writes its kinetic-energy and
// enstrophy sums to mpart[2 * tile] (ss_prims_grad_tiles(d) tiles), for
// launch_monitor_final.
template <typename T>
void launch_ss_prims_grad(const Dims& d, const Coef<T>& c, const T* q, T* prim, T* grad,
                          int gmask, hipStream_t s, double* mpart = nullptr);
int ss_prims_grad_tiles(const Dims& d);
// Fused stage with no derivative arrays (RA with recompute = true, SN
// otherwise): primitives recomputed in-tile, residual, and the RK stage
// update: qout = q_acc + A dt R (or q_acc_new on the last substep),
// q_acc += B dt R. qout must not alias q.
template <typename T>
void launch_ra_fused(const Dims& d, const Coef<T>& c, const T* q, T* qout, double* qacc,
                     const StageCoef& sc, int zchunk, int tile_y, hipStream_t s, double* mpart,
                     bool recompute);

// Fold per-tile (KE, enstrophy) sums in tile order into out2[0..1] as means.
void launch_monitor_final(const double* mpart, int ntiles, double inv_n, double* out2,
                          hipStream_t s);
// Tiles of the z-sweep for this grid and tuning.
int sweep_tiles(const Dims& d, int zchunk, int tile_y);

// diagnostics (nsf_diag.hip); partial holds diag_partial_count(d) * NDIAG doubles
size_t diag_partial_count(const Dims& d);
template <typename T>
void launch_diag(const Dims& d, const Coef<double>& c, const T* q, double* partial, double* out_dev,
                 hipStream_t s);
// Diagnostics with the partials in the library's fixed per-GPU scratch
// (nsf_diagnostics_noalloc): NSF_EINVAL when the grid has more tiles than
// diag_noalloc_max_tiles(). Waits for the stream and writes out_host.
size_t diag_noalloc_max_tiles();
int diag_noalloc(const Dims& d, const Coef<double>& c, int precision, const void* q,
                 double* out_host, hipStream_t s);

}  // namespace nsf
