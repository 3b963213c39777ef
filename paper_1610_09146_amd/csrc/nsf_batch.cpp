// Batched form: many independent Taylor-Green-type instances of uneven grid
// sizes and parameters advance together, one persistent launch per RK stage
// over a work list of (instance, tile) items, the three stage launches of a
// step captured once in a hipGraph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <queue>
#include <vector>

#include "nsf.h"
#include "nsf_internal.h"

using namespace nsf;

struct nsf_batch {
    int count = 0;
    int precision = NSF_F64;
    int nitems = 0;
    int nblocks = 0;
    int tile_y = 8;
    int recompute = 0;        // stage kernel: 1 = RA, 0 = SN
    std::vector<int> zchunk;  // per instance
    std::vector<Dims> dims;
    std::vector<nsf_phys> phys;
    std::vector<void*> q;
    std::vector<double*> diag_partial;
    double* diag_out = nullptr;  // count * NSF_NDIAG doubles inside `work`
    void* desc_dev = nullptr;
    int2* items_dev = nullptr;  // items, band by band (one band per XCD), longest first
    int* boff_dev = nullptr;    // band x holds items [boff[x], boff[x+1])
    int* ctr_dev = nullptr;     // per stage and band: the next item to take
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;      // one step, storing q_acc in its third substep
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph_ns = nullptr;   // double-precision 16-row tiles: the same step
    hipGraphExec_t exec_ns = nullptr;  // without that store (every step of a call but the last)
};

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int bfail(int code, const char* msg) { return set_error(code, msg); }

// Per-instance work: the two extra stage states (qb, qc) and the
// diagnostics partials; then count * NDIAG doubles of reduced output.
size_t instance_bytes(const Dims& d, int precision) {
    const size_t es = precision == NSF_F32 ? 4 : 8;
    return 2 * align_up(5 * d.npts * es) + align_up(diag_partial_count(d) * NSF_NDIAG * sizeof(double));
}

int check_grids(int32_t count, const nsf_grid* grids, std::vector<Dims>& dims) {
    if (count < 1 || !grids) return bfail(NSF_EINVAL, "batch: count < 1 or grids NULL");
    dims.resize(count);
    for (int i = 0; i < count; ++i) {
        const nsf_grid& g = grids[i];
        if (g.nx < 5 || g.ny < 5 || g.nz < 5) return bfail(NSF_EINVAL, "batch: every axis needs >= 5 points");
        const size_t n = (size_t)g.nx * g.ny * g.nz;
        if (n > (size_t)1 << 31 || (size_t)g.nx * g.ny >= (size_t)1 << 28)
            return bfail(NSF_EINVAL, "batch: instance too large");
        dims[i] = Dims{g.nx, g.ny, g.nz, n};
    }
    return NSF_OK;
}

// z-chunk of a batched instance: 48 planes from 64-point grids up (against
// the single-grid 32 below 256 points: fewer chunk preambles, and on the
// 64-instance mix of sizes 32 to 128 the batched step ran 1-2% faster than
// with 32 or 64 planes).
int batch_zchunk(const Dims& d) { return d.nz >= 256 ? 64 : (d.nz >= 64 ? 48 : d.nz); }

// The pre-loop loads of a z-chunk (four planes of fields and halos) cost
// about three planes of the loop.
constexpr int kWarmPlanes = 3;

// Schedule of the persistent stage launch. The item list (instances in
// order, each one's tiles in launch order) is cut into one contiguous band of
// equal cost per XCD, so the tiles that share halos run under one L2; each
// band is sorted longest item first (a stable sort: equal items stay in tile
// order, so neighbouring tiles still run together). At run time the
// workgroups of an XCD take their band's items in that order from a counter,
// and a workgroup whose band is used up takes items from the next band:
// longest-first dealing to whichever workgroup is free, which ends a stage
// within about one short item of the mean load, where the static deal it
// replaces left the busiest workgroup 6% above the mean on the 64-instance
// mix (its 51-plane items outnumber what the short ones can even out within
// a band).
void schedule_items(const std::vector<int2>& items, const std::vector<int>& cost,
                    std::vector<int2>& order, std::vector<int>& boff) {
    long long total = 0;
    for (int c : cost) total += c;
    order.clear();
    boff.assign(kXCD + 1, 0);
    size_t first = 0;
    long long run = 0;
    for (int x = 0; x < kXCD; ++x) {
        // band x: items up to the cumulative cost total * (x + 1) / 8
        size_t last = first;
        const long long cut = total * (x + 1) / kXCD;
        while (last < items.size() && (x == kXCD - 1 || run + cost[last] <= cut || last == first)) {
            run += cost[last];
            ++last;
        }
        std::vector<size_t> band;
        for (size_t i = first; i < last; ++i) band.push_back(i);
        std::stable_sort(band.begin(), band.end(), [&](size_t a, size_t c) { return cost[a] > cost[c]; });
        for (size_t i : band) order.push_back(items[i]);
        boff[x + 1] = (int)order.size();
        first = last;
    }
}

template <typename T>
int build_tables(nsf_batch* b, const std::vector<Dims>& dims, const nsf_phys* phys,
                 const double* dt, void* const* q, double* const* qacc, char* work) {
    std::vector<BatchDesc<T>> desc(b->count);
    std::vector<int2> items;
    std::vector<int> cost;
    size_t off = 0;
    const size_t es = sizeof(T);
    for (int i = 0; i < b->count; ++i) {
        const Dims& d = dims[i];
        BatchDesc<T>& bd = desc[i];
        bd.d = d;
        bd.k = make_coef<T>(d, phys[i].Re, phys[i].Ma, phys[i].Pr, phys[i].gamma);
        bd.q = (T*)q[i];
        bd.qb = (T*)(work + off);
        off += align_up(5 * d.npts * es);
        bd.qc = (T*)(work + off);
        off += align_up(5 * d.npts * es);
        b->diag_partial[i] = (double*)(work + off);
        off += align_up(diag_partial_count(d) * NSF_NDIAG * sizeof(double));
        bd.qacc = qacc[i];
        bd.dt = dt[i];
        int tx, ty, tz, zc;
        tile_counts(d, b->zchunk[i], b->tile_y, &tx, &ty, &tz, &zc);
        bd.zchunk = zc;
        bd.tiles_x = tx;
        bd.tiles_y = ty;
        bd.tiles = tx * ty * tz;
        for (int t = 0; t < bd.tiles; ++t) {
            items.push_back(int2{i, t});
            const int z0 = (t / (tx * ty)) * zc;
            cost.push_back(std::min(zc, d.nz - z0) + kWarmPlanes);
        }
    }
    b->diag_out = (double*)(work + off);
    b->nitems = (int)items.size();
    std::vector<int2> order;
    std::vector<int> boff;
    schedule_items(items, cost, order, boff);
    hipError_t e = hipMalloc(&b->desc_dev, desc.size() * sizeof(BatchDesc<T>));
    if (e == hipSuccess) e = hipMalloc((void**)&b->items_dev, order.size() * sizeof(int2));
    if (e == hipSuccess) e = hipMalloc((void**)&b->boff_dev, boff.size() * sizeof(int));
    if (e == hipSuccess) e = hipMalloc((void**)&b->ctr_dev, 3 * kXCD * sizeof(int));
    if (e == hipSuccess)
        e = hipMemcpy(b->desc_dev, desc.data(), desc.size() * sizeof(BatchDesc<T>), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b->items_dev, order.data(), order.size() * sizeof(int2), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b->boff_dev, boff.data(), boff.size() * sizeof(int), hipMemcpyHostToDevice);
    // the stage counters start at zero; each stage launch then zeroes the
    // next stage's (outside any graph: a synchronous set at creation)
    if (e == hipSuccess) e = hipMemset(b->ctr_dev, 0, 3 * kXCD * sizeof(int));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return bfail(NSF_EHIP, hipGetErrorString(e));
    return NSF_OK;
}

template <typename T>
void enqueue_step(nsf_batch* b, hipStream_t s, int store_acc) {
    for (int st = 0; st < 3; ++st)
        launch_ra_batch<T>((const BatchDesc<T>*)b->desc_dev, b->items_dev, b->boff_dev, b->ctr_dev,
                           st, b->nblocks, b->tile_y, s, b->recompute != 0, store_acc);
}

// whether the stage kernel can leave q_acc unwritten (see launch_ra_batch)
bool saves_acc(const nsf_batch* b) { return b->precision == NSF_F64 && b->tile_y == 16; }

void release(nsf_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->exec_ns) (void)hipGraphExecDestroy(b->exec_ns);
    if (b->graph_ns) (void)hipGraphDestroy(b->graph_ns);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->desc_dev) (void)hipFree(b->desc_dev);
    if (b->items_dev) (void)hipFree(b->items_dev);
    if (b->boff_dev) (void)hipFree(b->boff_dev);
    if (b->ctr_dev) (void)hipFree(b->ctr_dev);
    delete b;
}

}  // namespace

extern "C" {

int nsf_batch_workspace_bytes(int32_t count, const nsf_grid* grids, int precision, size_t* bytes) {
    std::vector<Dims> dims;
    int rc = check_grids(count, grids, dims);
    if (rc) return rc;
    if (precision != NSF_F64 && precision != NSF_F32) return bfail(NSF_EINVAL, "batch: precision");
    if (!bytes) return bfail(NSF_EINVAL, "batch: bytes NULL");
    size_t total = 0;
    for (const Dims& d : dims) total += instance_bytes(d, precision);
    *bytes = total + align_up((size_t)count * NSF_NDIAG * sizeof(double));
    return NSF_OK;
}

int nsf_batch_create(int32_t count, const nsf_grid* grids, const nsf_phys* phys, const double* dt,
                     int precision, void* const* q, double* const* q_acc, void* work,
                     size_t work_bytes, void* stream, nsf_batch** out) {
    return nsf_batch_create_variant(count, grids, phys, dt, precision, NSF_SN, nullptr, q, q_acc,
                                    work, work_bytes, stream, out);
}

int nsf_batch_create_tuned(int32_t count, const nsf_grid* grids, const nsf_phys* phys,
                           const double* dt, int precision, const nsf_tuning* tune, void* const* q,
                           double* const* q_acc, void* work, size_t work_bytes, void* stream,
                           nsf_batch** out) {
    return nsf_batch_create_variant(count, grids, phys, dt, precision, NSF_SN, tune, q, q_acc, work,
                                    work_bytes, stream, out);
}

int nsf_batch_create_variant(int32_t count, const nsf_grid* grids, const nsf_phys* phys,
                             const double* dt, int precision, int variant, const nsf_tuning* tune,
                             void* const* q, double* const* q_acc, void* work, size_t work_bytes,
                             void* stream, nsf_batch** out) {
    (void)stream;
    if (!out) return bfail(NSF_EINVAL, "batch: out NULL");
    *out = nullptr;
    std::vector<Dims> dims;
    int rc = check_grids(count, grids, dims);
    if (rc) return rc;
    if (!phys || !dt || !q || !q_acc || !work) return bfail(NSF_EINVAL, "batch: NULL argument");
    if (precision != NSF_F64 && precision != NSF_F32) return bfail(NSF_EINVAL, "batch: precision");
    if (variant != NSF_SN && variant != NSF_RA)
        return bfail(NSF_EUNSUPPORTED, "batch: the batched stage is SN or RA");
    if (tune && ((tune->block_y != 0 && tune->block_y != 8 && tune->block_y != 16) || tune->zchunk < 0))
        return bfail(NSF_EINVAL, "batch: block_y 0, 8 or 16 and zchunk >= 0");
    for (int i = 0; i < count; ++i) {
        const nsf_phys& p = phys[i];
        if (!(p.Re > 0) || !(p.Ma > 0) || !(p.Pr > 0) || !(p.gamma > 1) || !std::isfinite(dt[i]))
            return bfail(NSF_EINVAL, "batch: bad phys or dt");
        if (!q[i] || !q_acc[i]) return bfail(NSF_EINVAL, "batch: NULL state pointer");
    }
    size_t need = 0;
    if ((rc = nsf_batch_workspace_bytes(count, grids, precision, &need))) return rc;
    if (work_bytes < need) return bfail(NSF_EWORKSPACE, "batch: work buffer too small");

    nsf_batch* b = new nsf_batch();
    b->count = count;
    b->precision = precision;
    b->dims = dims;
    b->phys.assign(phys, phys + count);
    b->q.assign(q, q + count);
    b->diag_partial.resize(count);
    b->recompute = variant == NSF_RA;
    b->tile_y = tune && tune->block_y ? tune->block_y : (precision == NSF_F64 ? 16 : 8);
    b->zchunk.resize(count);
    for (int i = 0; i < count; ++i)
        b->zchunk[i] = tune && tune->zchunk > 0 ? std::min(tune->zchunk, dims[i].nz)
                                                : batch_zchunk(dims[i]);
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int per_cu = precision == NSF_F64 ? batch_blocks_per_cu<double>(b->tile_y, b->recompute)
                                            : batch_blocks_per_cu<float>(b->tile_y, b->recompute);
    if (e != hipSuccess || cus < 1 || per_cu < 1) { release(b); return bfail(NSF_EHIP, "batch: occupancy query failed"); }
    b->nblocks = (cus * per_cu) / 8 * 8;  // a multiple of the XCD count
    if (b->nblocks < 8) b->nblocks = 8;
    rc = precision == NSF_F64
             ? build_tables<double>(b, dims, phys, dt, q, q_acc, (char*)work)
             : build_tables<float>(b, dims, phys, dt, q, q_acc, (char*)work);
    if (rc) { release(b); return rc; }

    // capture one step (three stage launches) into a graph on a private
    // stream; where the third substep can skip the q_acc store, also the
    // step without it
    e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    for (int k = 0; k < (saves_acc(b) ? 2 : 1) && e == hipSuccess; ++k) {
        hipGraph_t* g = k == 0 ? &b->graph : &b->graph_ns;
        hipGraphExec_t* x = k == 0 ? &b->exec : &b->exec_ns;
        e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            if (precision == NSF_F64) enqueue_step<double>(b, b->cap, k == 0);
            else enqueue_step<float>(b, b->cap, k == 0);
            e = hipStreamEndCapture(b->cap, g);
        }
        if (e == hipSuccess) e = hipGraphInstantiate(x, *g, nullptr, nullptr, 0);
    }
    if (e != hipSuccess) { release(b); return bfail(NSF_EHIP, hipGetErrorString(e)); }
    *out = b;
    return NSF_OK;
}

int nsf_batch_step(nsf_batch* b, int32_t nsteps, void* stream) {
    if (!b || nsteps < 0) return bfail(NSF_EINVAL, "batch_step: bad handle or nsteps");
    hipStream_t s = (hipStream_t)stream;
    for (int i = 0; i < nsteps; ++i) {
        TimerScope ts("batch_step", s);  // one record per replayed step
        hipError_t e = hipGraphLaunch(i + 1 < nsteps && b->exec_ns ? b->exec_ns : b->exec, s);
        if (e != hipSuccess) return bfail(NSF_EHIP, hipGetErrorString(e));
    }
    return NSF_OK;
}

int nsf_batch_step_eager(nsf_batch* b, int32_t nsteps, void* stream) {
    if (!b || nsteps < 0) return bfail(NSF_EINVAL, "batch_step_eager: bad handle or nsteps");
    hipStream_t s = (hipStream_t)stream;
    for (int i = 0; i < nsteps; ++i) {
        TimerScope ts("batch_step", s);
        const int store = i + 1 == nsteps || !saves_acc(b);
        if (b->precision == NSF_F64) enqueue_step<double>(b, s, store);
        else enqueue_step<float>(b, s, store);
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? NSF_OK : bfail(NSF_EHIP, hipGetErrorString(e));
}

int nsf_batch_diagnostics(nsf_batch* b, double* out, void* stream) {
    if (!b || !out) return bfail(NSF_EINVAL, "batch_diagnostics: NULL argument");
    hipStream_t s = (hipStream_t)stream;
    for (int i = 0; i < b->count; ++i) {
        const Dims& d = b->dims[i];
        const nsf_phys& p = b->phys[i];
        const Coef<double> c = make_coef<double>(d, p.Re, p.Ma, p.Pr, p.gamma);
        double* o = b->diag_out + (size_t)i * NSF_NDIAG;
        if (b->precision == NSF_F64) launch_diag<double>(d, c, (const double*)b->q[i], b->diag_partial[i], o, s);
        else launch_diag<float>(d, c, (const float*)b->q[i], b->diag_partial[i], o, s);
    }
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipMemcpyAsync(out, b->diag_out, (size_t)b->count * NSF_NDIAG * sizeof(double),
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return bfail(NSF_EHIP, hipGetErrorString(e));
    for (int i = 0; i < b->count; ++i)
        if (out[(size_t)i * NSF_NDIAG + 14] > 0) return bfail(NSF_ENONFINITE, "batch: non-finite values");
    return NSF_OK;
}

int nsf_batch_info(const nsf_batch* b, int32_t* nitems, int32_t* nblocks) {
    if (!b || !nitems || !nblocks) return bfail(NSF_EINVAL, "batch_info: NULL argument");
    *nitems = b->nitems;
    *nblocks = b->nblocks;
    return NSF_OK;
}

int nsf_batch_config(const nsf_batch* b, int32_t* variant, int32_t* tile_y, int32_t* zchunk) {
    if (!b || !variant || !tile_y || !zchunk) return bfail(NSF_EINVAL, "batch_config: NULL argument");
    *variant = b->recompute ? NSF_RA : NSF_SN;
    *tile_y = b->tile_y;
    for (int i = 0; i < b->count; ++i) zchunk[i] = b->zchunk[i];
    return NSF_OK;
}

int nsf_batch_destroy(nsf_batch* b) {
    if (!b) return NSF_OK;
    release(b);
    return NSF_OK;
}

}  // extern "C"
