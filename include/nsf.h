/*
 * nsf.h -- C ABI of the MI355X (gfx950) library for the explicit
 * finite-difference compressible Navier-Stokes hot path of Jammy, Jacobs &
 * Sandham, "Performance evaluation of explicit finite difference algorithms
 * with varying amounts of computational and memory intensity"
 * (arXiv 1610.09146).
 *
 * What the library computes (paper Section 2):
 *   - the residual R(q) of the 3D compressible Navier-Stokes equations with
 *     constant viscosity, eqs (1)-(3), stress eq (4), heat flux eq (5),
 *     pressure and temperature eqs (6)-(7), or (9)-(10) from the
 *     conservative variables; convective terms in the skew-symmetric
 *     form eq (8); viscous terms expanded to second
 *     derivatives; fourth-order central differences on a periodic grid;
 *   - the three-stage low-storage Runge-Kutta time advance (Figure 1);
 *   - in the paper's derivative-storage algorithms BL, RA, SN, RS, SS
 *     (Section 2, one paragraph each);
 *   - the Taylor-Green initial state and the kinetic-energy and enstrophy
 *     integrals of Section 3.
 *
 * Conventions shared by every entry point
 *   - Layout: a field is nz*ny*nx contiguous elements, x fastest
 *     (index (k*ny + j)*nx + i, point x_i = 2*pi*i/nx, same for y and z).
 *     A state q is five consecutive fields rho, rho*u, rho*v, rho*w, rho*E.
 *   - Precision: NSF_F64 -> q, r are double; NSF_F32 -> q, r are float
 *     (fields and stencil arithmetic in single precision). The Runge-Kutta
 *     accumulator q_acc and all reductions are always double.
 *   - Memory: every pointer argument named q, q_acc, r, work, workspace
 *     is device memory owned by the caller; the library only borrows it for
 *     the call and allocates no device memory outside the nsf_batch_create
 *     family (its descriptor tables, freed by nsf_batch_destroy).
 *   - Streams: `stream` is a hipStream_t passed as void* (NULL = default
 *     stream). Calls enqueue work and return without waiting, except where
 *     stated (diagnostics, autotune, batch diagnostics).
 *   - Errors: every call returns an nsf_status. Arguments are validated
 *     before anything is enqueued; on a non-zero return nothing was
 *     enqueued unless the code is NSF_EHIP. nsf_last_error() gives text.
 *   - Thread safety: calls are reentrant; the kernel timer
 *     (nsf_timer_*) is process-global.
 */
#ifndef NSF_H
#define NSF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NSF_OK = 0,
    NSF_EINVAL = -1,       /* bad argument, size or pointer            */
    NSF_EWORKSPACE = -2,   /* work buffer smaller than required        */
    NSF_EHIP = -3,         /* HIP runtime or launch error              */
    NSF_EUNSUPPORTED = -4, /* combination the library does not provide */
    NSF_ENONFINITE = -5    /* diagnostics found NaN/Inf in the state   */
} nsf_status;

/* The paper's algorithms (Section 2), each a kernel sequence of its own:
 *   NSF_BL  baseline: every first/second derivative is a grid-sized work
 *           array; products staged in one reused work array; primitives in
 *           three separate loops (u_i, then p by eq (6), then T by eq (7)).
 *   NSF_RA  recompute all: no derivative arrays; the five equations are
 *           evaluated one after another and each forms every derivative it
 *           uses from the staged grid values, nothing being carried from one
 *           equation to the next (cross derivatives as nested stencils);
 *           p, T by eqs (9)-(10).
 *   NSF_SN  store none: no derivative arrays; each derivative is formed once
 *           per point into a thread-local value and reused wherever it
 *           occurs (the velocity gradients, for instance, in all five
 *           equations).
 *   NSF_RS  recompute some: the nine velocity gradients du_i/dx_j stored in
 *           work arrays by their own kernel and read wherever they occur;
 *           the other derivatives formed where used, equation by equation.
 *   NSF_SS  store some: the nine velocity gradients stored as in RS, the
 *           other derivatives formed once into thread-local values.
 * In every algorithm the primitive variables are a stored array and the RK
 * update its own kernel (the paper's structure); RA, SN and SS also have a
 * fused form (nsf_tuning.fuse). */
typedef enum { NSF_BL = 0, NSF_RA = 1, NSF_SS = 2, NSF_SN = 3, NSF_RS = 4, NSF_AUTO = 5 } nsf_variant;
/* NSF_AUTO: the algorithm and tuning that nsf_autotune (or nsf_tune_load)
 * recorded for this grid and precision in this process; SN with the fused
 * stage kernel if nothing was recorded. The tuning argument is ignored. */
typedef enum { NSF_F64 = 0, NSF_F32 = 1 } nsf_precision;

#define NSF_NDIAG 16

/* Grid: points per axis on the periodic cube [0, 2*pi)^3 (Section 3).
 * nx and ny must be >= 5 (distinct radius-2 wrap neighbours); nz >= 5, or
 * nz = 1 for a two-dimensional problem (the z-independent flow: every
 * z-difference vanishes, and w stays 0 when it starts at 0; the Taylor-Green
 * initial state is then its z = 0 plane). nx*ny*nz <= 2^31 and
 * nx*ny < 2^28 (one z-plane of doubles is addressed with 32-bit byte
 * offsets). The batched form takes cubes only. */
typedef struct { int32_t nx, ny, nz; } nsf_grid;

/* Non-dimensional parameters of eqs (4)-(7): Reynolds, Mach, Prandtl
 * numbers and ratio of specific heats. Re, Ma, Pr > 0, gamma > 1. */
typedef struct { double Re, Ma, Pr, gamma; } nsf_phys;

/* Taylor-Green initial state (Section 3, after DeBonis 2013):
 *   u = V0 sin x cos y cos z, v = -V0 cos x sin y cos z, w = 0,
 *   p = 1/(gamma Ma^2) + V0^2 (cos 2x + cos 2y)(cos 2z + 2)/16, T = 1.
 * pert_kind 0: none.
 * pert_kind 1: u_a *= 1 + pert_amp*(2U - 1), U uniform in [0,1) from the
 *              SplitMix64 stream of `seed` at counter a*npts + point index
 *              (output number counter + 1).
 * pert_kind 2: velocity += pert_amp * (sin(x+f0)cos(y+f1)cos(z+f2),
 *              -cos(x+f0)sin(y+f1)cos(z+f2), 0) with f = phase[]. */
typedef struct {
    double V0;
    double pert_amp;
    uint64_t seed;
    int32_t pert_kind;
    int32_t reserved;
    double phase[3];
} nsf_tgv;

/* Implementation knobs (not part of the method). Pass NULL for defaults.
 *   block_x, block_y: x-y tile of the z-sweeping kernels: block_x is 32,
 *         block_y 8 or 16 (0 = default);
 *   zchunk: planes marched per workgroup by the z-sweeping kernels (0 = default);
 *   fuse: RA/SN/SS (ignored elsewhere). 0 = primitives stored by their
 *         own kernel and the RK update a separate kernel, as in the paper;
 *         1 = the RK update applied in the residual kernel's epilogue, and
 *         in RA and SN the primitives recomputed inside the residual tile
 *         (SS keeps its stored primitives and gradients). nsf_rk_step then
 *         rotates the state through a copy of q in `work` (and, in SS,
 *         through r); nsf_rhs is unchanged.
 *   naive: 1 = use the untiled per-point kernels (reference GPU path): one
 *         kernel per store set, so RA and SN run the same untiled kernel,
 *         and so do RS and SS;
 *   gstore: SS/RS only, which velocity gradients G_ab = du_a/dx_b are
 *         stored in work arrays (the others are formed in the residual
 *         kernel: thread-local in SS, at each use in RS). 0 = the
 *         algorithm's own set (the nine gradients; on a single-plane grid
 *         the four in-plane ones, the paper's 2D count); 9 = all nine;
 *         3 = the three diagonal ones; 4 = the four in-plane ones
 *         (single-plane grids only). The untiled kernels need 0 or 9.
 *         NSF_EINVAL for other values or other algorithms. */
typedef struct {
    int32_t block_x, block_y, zchunk, fuse, naive, gstore;
    int32_t reserved[2];
} nsf_tuning;

const char *nsf_status_string(int status);
const char *nsf_last_error(void);
/* Library version as major*10000 + minor*100 + patch. */
int nsf_version(void);

/* Bytes of `work` needed by nsf_rhs / nsf_rk_step / nsf_diagnostics for this
 * grid, algorithm, precision and tuning (tuning may be NULL): primitive
 * fields, stored derivative arrays of the algorithm, the ping-pong state of
 * the fused form, the monitor's per-tile sums and reduction scratch.
 * Written to *bytes. */
int nsf_workspace_bytes(const nsf_grid *g, int variant, int precision,
                        const nsf_tuning *tune, size_t *bytes);

/* Write the Taylor-Green state (Section 3) to q (precision dtype, 5 fields)
 * and, if q_acc != NULL, its double-precision value to q_acc (5 fields).
 * Asynchronous on `stream`. */
int nsf_init_fields(const nsf_grid *g, const nsf_phys *phys, const nsf_tgv *tgv,
                    int precision, void *q, double *q_acc, void *stream);

/* r = R(q): the residual of eqs (1)-(3) (Section 2) evaluated with
 * algorithm `variant`. q is read-only; r (5 fields, same dtype as q) must
 * not overlap q or work. Asynchronous. */
int nsf_rhs(const nsf_grid *g, const nsf_phys *phys, int variant, int precision,
            const nsf_tuning *tune, const void *q, void *r, void *work,
            size_t work_bytes, void *stream);

/* Advance nsteps steps of the three-stage low-storage Runge-Kutta scheme
 * (Section 2, Figure 1) with time step dt: for substep s = 1..3,
 *   r = R(q); q = q_acc + A_s dt r (s < 3); q_acc = q_acc + B_s dt r;
 * then q = q_acc; A = (2/3, 5/12), B = (1/4, 3/20, 3/5).
 * On entry q_acc must hold the state (double) and q its value in the
 * precision dtype; on return both hold the new state. (In double precision
 * the two are then equal, and the fused SN and RA stages with 16-row tiles
 * use that, with results equal up to one rounding of the accumulator: the
 * first substep reads the accumulator from q and writes none, the second
 * forms the first's accumulator as q0 + (B_1 / A_1)(q1 - q0) from the
 * step's initial state q0 and its own input q1, and the third writes q_acc
 * only in the call's last step.) r is a 5-field scratch in the precision
 * dtype.
 * Asynchronous. */
int nsf_rk_step(const nsf_grid *g, const nsf_phys *phys, int variant, int precision,
                const nsf_tuning *tune, double dt, int32_t nsteps, void *q,
                double *q_acc, void *r, void *work, size_t work_bytes, void *stream);

/* nsf_rk_step that also records the kinetic-energy and enstrophy integrals
 * of Section 3 (after DeBonis 2013) on the device, for monitoring a run
 * without a host round trip. monitor: device memory, 8-byte aligned,
 * 2 * nsteps doubles, not overlapping the other buffers; entries 2s and
 * 2s+1 receive the grid means of rho|u|^2/2 and rho|omega|^2/2 (omega =
 * curl u by the fourth-order first difference) of the state at the start of
 * step s, the quantities of out[0] and out[1] of nsf_diagnostics. The sums
 * are formed inside the first stage's kernels from the values they already
 * hold in the fused SN and RA forms, and in double precision also for SS
 * and RS (their primitive and gradient pass) and for SN and RA with stored
 * primitives (their residual pass); otherwise (BL, the untiled kernels, the
 * other single-precision forms) a diagnostics pass runs before every step.
 * NSF_EINVAL for a NULL or misaligned monitor.
 * Asynchronous. */
int nsf_rk_step_monitored(const nsf_grid *g, const nsf_phys *phys, int variant, int precision,
                          const nsf_tuning *tune, double dt, int32_t nsteps, void *q,
                          double *q_acc, void *r, void *work, size_t work_bytes,
                          double *monitor, void *stream);

/* Diagnostics of q (Section 3: kinetic-energy and enstrophy integrals),
 * reduced in double in a fixed order (bitwise reproducible). Waits for the
 * stream, then fills out[NSF_NDIAG] (host memory):
 *   0 KE = <rho|u|^2/2>   1 enstrophy = <rho|curl u|^2/2> (curl by the
 *   fourth-order first derivative)   2..6 <q_f>   7..11 max|q_f|
 *   12 min rho   13 min p   14 number of non-finite values in q   15 <p>
 * where <.> is the mean over grid points (volume integral / (2 pi)^3).
 * Returns NSF_ENONFINITE (after filling out) if out[14] > 0. */
int nsf_diagnostics(const nsf_grid *g, const nsf_phys *phys, int precision,
                    const void *q, void *work, size_t work_bytes, double *out,
                    void *stream);

/* nsf_diagnostics for callers that cannot allocate device memory (no
 * hipMalloc and no work buffer: serving loops and harnesses that forbid
 * allocation). Same kernels, same outputs, same synchronisation and the same
 * NSF_ENONFINITE rule as nsf_diagnostics, but the per-tile partial sums and
 * the result live in a fixed array of the library (8 MiB of device memory on
 * each GPU it runs on, held until the process ends) instead of `work`; no
 * memory is allocated by this call. The grid may have at most 65536
 * diagnostics tiles of 32 x 8 columns x 64 planes (ceil(nx/32) *
 * ceil(ny/8) * ceil(nz/64); a 1024^3 grid has exactly 65536); larger grids
 * return NSF_EINVAL before anything is enqueued. The stream must belong to
 * the current device (NSF_EINVAL otherwise). Every call on one GPU shares
 * that array, so calls that overlap in time on one GPU (other host threads,
 * other streams) race and must be serialised by the caller. */
int nsf_diagnostics_noalloc(const nsf_grid *g, const nsf_phys *phys, int precision,
                            const void *q, double *out, void *stream);

/* ---------------------------------------------------------------- autotuner
 * Searches the paper's store-versus-recompute trade-off (Section 2: which
 * derivatives to store in work arrays, which to recompute; the
 * conclusion's point that the best algorithm depends on the machine) made
 * searchable: the store set (no derivative arrays: SN, RA; the velocity
 * gradients: SS, RS with all nine or the three diagonal ones, or on a
 * single-plane grid the four in-plane ones or all nine), whether the
 * derivatives not stored are thread-local values (SN, SS) or formed at each
 * use (RA, RS), the primitives stored or recomputed in the tile with the RK
 * update fused (SN, RA), the RK update fused into the stored-gradient
 * residual (SS), and BL, crossed with the tile height and z-chunk of
 * the z-sweeping kernels. Every candidate is first checked, per field,
 * against a reference residual on a seeded perturbed Taylor-Green state of
 * the same grid: in double precision the untiled kernels', at 1e-10
 * relative max-norm difference; in single precision the double-precision
 * untiled residual of the same single-precision state, within 4 times the
 * change that rounding the state to single precision makes to that
 * residual. The residual checked is the one nsf_rhs forms, which for the
 * fused forms is their algorithm's separate-update kernel; a fused
 * candidate must also reproduce one RK step of that path from the same
 * state (step: half the acoustic CFL limit of the finest axis), per field
 * relative to the step's increment, at the residual bar (twice it in single
 * precision) or 64 units in the last place of the state, whichever is
 * larger. Only passing candidates are timed (`steps` RK steps each, from
 * the same initial state and accumulator). Candidates within 2% of the
 * fastest count as ties, resolved toward the default tuning and then the
 * larger z-chunk. The winner is recorded for NSF_AUTO and, if cache_path
 * is not NULL, appended as one JSON line to that file. Synchronous.
 * workspace: caller-owned device memory of at least
 * nsf_autotune_workspace_bytes bytes (seven to nine states and the largest
 * candidate's work), used for the duration of the call; NSF_EWORKSPACE if
 * smaller. The library allocates no device memory here. */
#define NSF_TUNE_QUICK 1 /* skip BL and the untiled kernels */
typedef struct {
    int32_t variant;
    nsf_tuning tune;
    double pt_rhs_per_s;   /* measured grid-point residual evaluations/s */
    double parity_rel_err; /* worst per-field relative residual difference */
} nsf_tune_result;

/* Bytes of the workspace nsf_autotune needs for this grid, precision and
 * flags, written to *bytes. */
int nsf_autotune_workspace_bytes(const nsf_grid *g, int precision, int flags, size_t *bytes);
int nsf_autotune(const nsf_grid *g, const nsf_phys *phys, int precision, int flags, int32_t steps,
                 const char *cache_path, void *workspace, size_t workspace_bytes,
                 nsf_tune_result *best, void *stream);
/* Load gfx950 entries of a cache file written by nsf_autotune (later lines
 * override earlier ones). A line that names no configuration the library
 * runs on its grid (algorithm, tile height, z-chunk, flags, store set) is
 * skipped. Returns the number of entries loaded, or an error status. */
int nsf_tune_load(const char *cache_path);
/* The recorded choice for a grid and precision (NSF_EUNSUPPORTED if none). */
int nsf_tune_get(const nsf_grid *g, int precision, nsf_tune_result *out);

/* ---------------------------------------------------------------- batched form
 * Many independent Taylor-Green-type instances (own grid, parameters, dt)
 * advance together with a fused stage kernel (SN or RA): one persistent
 * launch per RK stage in which the workgroups take (instance, tile) items
 * from a list built once on the host (one band of neighbouring tiles of
 * equal cost per XCD, longest first) through a device counter per band,
 * and the three stage launches of a step are captured once in a hipGraph.
 * Each instance's q (precision dtype) and q_acc (double) are caller-owned
 * device buffers with the single-grid contract of nsf_rk_step; `work`
 * (nsf_batch_workspace_bytes) holds the other two stage states and the
 * diagnostics scratch of every instance and must stay allocated until
 * nsf_batch_destroy. The handle owns only the graph, a private capture
 * stream and the small device work list, band table and counters it
 * allocates. Steps of one handle must not run concurrently (they share the
 * counters, as they share the states). */
typedef struct nsf_batch nsf_batch;

int nsf_batch_workspace_bytes(int32_t count, const nsf_grid *grids, int precision, size_t *bytes);

/* Build the work list and capture one step. grids, phys, dt, q, q_acc are
 * host arrays of `count` entries. Synchronous (allocates and uploads). */
int nsf_batch_create(int32_t count, const nsf_grid *grids, const nsf_phys *phys, const double *dt,
                     int precision, void *const *q, double *const *q_acc, void *work,
                     size_t work_bytes, void *stream, nsf_batch **out);

/* As nsf_batch_create with implementation knobs: block_y selects the tile
 * height 8 or 16 of the stage kernel (0: 16 in double, 8 in single
 * precision), zchunk the planes per tile for every instance (clamped to its
 * grid; 0: 48, or 64 from 256 planes up, or the whole grid below 64);
 * other fields are ignored. NSF_EINVAL for other values. */
int nsf_batch_create_tuned(int32_t count, const nsf_grid *grids, const nsf_phys *phys,
                           const double *dt, int precision, const nsf_tuning *tune, void *const *q,
                           double *const *q_acc, void *work, size_t work_bytes, void *stream,
                           nsf_batch **out);

/* As nsf_batch_create_tuned with the algorithm of the fused stage kernel:
 * NSF_SN (the other entry points) or NSF_RA (derivatives formed where each
 * equation uses them); NSF_EUNSUPPORTED for others. */
int nsf_batch_create_variant(int32_t count, const nsf_grid *grids, const nsf_phys *phys,
                             const double *dt, int precision, int variant, const nsf_tuning *tune,
                             void *const *q, double *const *q_acc, void *work, size_t work_bytes,
                             void *stream, nsf_batch **out);

/* Autotuner of the batched form (the paper's store-versus-recompute choice
 * and the tile knobs, searched on the batch itself): for the ensemble of
 * `count` instances (grids, phys, dt as for nsf_batch_create) it times
 * `steps` graph replays of every candidate -- stage algorithm SN or RA,
 * tile height 16 or 8, z-chunks of the default rule or 16, 32, 64 planes --
 * on its own seeded Taylor-Green states, after checking each candidate's
 * first step against the first candidate's (SN, 16 rows, default chunks)
 * per instance and field (1e-10 relative in double, 1e-5 in single
 * precision). Candidates within 2% of the fastest count as ties, resolved
 * toward SN, 16 rows and the default chunks. Writes the winner to
 * *best_variant and *best_tune (for nsf_batch_create_variant) and its rate
 * in grid-point RHS evaluations per second to *best_pt_rhs_per_s (may be
 * NULL). Synchronous. workspace: caller-owned device memory of at least
 * nsf_batch_autotune_workspace_bytes bytes (five ensemble states and a batch
 * work area); NSF_EWORKSPACE if smaller. Device memory is allocated only by
 * the nsf_batch_create_variant calls it makes (their descriptor tables,
 * freed before it returns). */
int nsf_batch_autotune_workspace_bytes(int32_t count, const nsf_grid *grids, int precision,
                                       size_t *bytes);
int nsf_batch_autotune(int32_t count, const nsf_grid *grids, const nsf_phys *phys,
                       const double *dt, int precision, int32_t steps, void *workspace,
                       size_t workspace_bytes, int32_t *best_variant, nsf_tuning *best_tune,
                       double *best_pt_rhs_per_s, void *stream);

/* Advance every instance nsteps steps by replaying the captured graph on
 * `stream`; on completion q and q_acc hold the new states (in double
 * precision with 16-row tiles, the steps before the last replay a second
 * graph whose third substep leaves q_acc unwritten, as nsf_rk_step does).
 * Asynchronous. */
int nsf_batch_step(nsf_batch *b, int32_t nsteps, void *stream);

/* The same stage launches issued directly (no graph); same results. */
int nsf_batch_step_eager(nsf_batch *b, int32_t nsteps, void *stream);

/* Diagnostics (as nsf_diagnostics) of every instance into out[count][NSF_NDIAG]
 * (host memory). Waits for the stream. */
int nsf_batch_diagnostics(nsf_batch *b, double *out, void *stream);

/* Work-list size and persistent grid size of the stage launches. */
int nsf_batch_info(const nsf_batch *b, int32_t *nitems, int32_t *nblocks);

/* The batch's stage algorithm (NSF_SN or NSF_RA), tile height and each
 * instance's z-chunk (zchunk: host array of `count` entries). */
int nsf_batch_config(const nsf_batch *b, int32_t *variant, int32_t *tile_y, int32_t *zchunk);

int nsf_batch_destroy(nsf_batch *b);

/* Device-to-device copy of `bytes` with a plain streaming kernel (one
 * 16-byte element per lane, non-temporal), the reference for achievable HBM
 * bandwidth and for the memory-counter calibration. src and dst: device
 * memory, 16-byte aligned (NSF_EINVAL otherwise), not overlapping.
 * Asynchronous. */
int nsf_device_copy(const void *src, void *dst, size_t bytes, void *stream);

/* Kernel timer for roofline reporting. nsf_timer_enable(name) records a
 * HIP event pair around every launch of the kernel family `name` (see
 * nsf_timer_names), on the stream it is launched on; NULL disables it and
 * discards the records. nsf_timer_read waits for the recorded events and
 * returns the launch count and the summed duration in milliseconds. */
int nsf_timer_enable(const char *name);
int nsf_timer_read(int64_t *count, double *total_ms);
/* Comma-separated list of kernel family names known to the timer. */
const char *nsf_timer_names(void);

#ifdef __cplusplus
}
#endif

#endif /* NSF_H */
