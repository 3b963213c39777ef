// Diagnostics of paper Section 3 (kinetic-energy and enstrophy integrals,
// after DeBonis 2013) plus conservation sums, extrema and a non-finite
// count, all in double precision.
//
// Pass 1 is a z-marching tile kernel: a workgroup owns a 32 x 8 column tile
// and a chunk of planes; the velocity of every plane it touches is computed
// once from q and kept, with a two-point x-y halo, in a five-plane LDS ring,
// from which the fourth-order first derivatives (hence the vorticity) of
// the centre plane are formed. Pointwise quantities are accumulated as each
// plane enters the ring. Reductions run in a fixed order -- per-thread
// plane order, wave shuffles, LDS across waves, then a one-block pass over
// the per-tile partials in tile order -- with no atomics, so results are
// bitwise reproducible for a given grid.
#include <math.h>

#include <mutex>

#include "nsf_internal.h"

namespace nsf {

namespace {

constexpr int kTX = 32, kTY = 8, kNT = kTX * kTY;
constexpr int kLX = kTX + 4, kLY = kTY + 4, kNPL = kLX * kLY, kNHALO = kNPL - kNT;
constexpr int kRing = 5;
constexpr int kND = 16;
constexpr int kXCD = 8;

__device__ __forceinline__ int pmodi(int a, int n) {
    int r = a % n;
    return r < 0 ? r + n : r;
}

__device__ __forceinline__ int xcd_tile(int bid, int nb) {
    const int per = nb / kXCD, extra = nb % kXCD;
    const int x = bid % kXCD, k = bid / kXCD;
    return x * per + (x < extra ? x : extra) + k;
}

// slot kinds: sums 0..6, 15; maxima 7..11; minima 12, 13; count 14 (a sum)
__device__ __forceinline__ bool is_max(int s) { return s >= 7 && s <= 11; }
__device__ __forceinline__ bool is_min(int s) { return s == 12 || s == 13; }

__device__ __forceinline__ double combine(int s, double a, double b) {
    if (is_max(s)) return fmax(a, b);
    if (is_min(s)) return fmin(a, b);
    return a + b;
}

__device__ __forceinline__ double identity(int s) {
    if (is_min(s)) return INFINITY;
    return 0.0;
}

// Reduce acc[kND] over the block in a fixed order; thread 0 gets the result.
template <int NTHREADS>
__device__ void block_reduce(double acc[kND], double* sh /* [NTHREADS/64][kND] */) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int s = 0; s < kND; ++s) {
        double v = acc[s];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v = combine(s, v, __shfl_down(v, off, 64));
        acc[s] = v;
    }
    if (lane == 0)
#pragma unroll
        for (int s = 0; s < kND; ++s) sh[wave * kND + s] = acc[s];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int s = 0; s < kND; ++s) {
            double v = sh[s];
            for (int w = 1; w < NTHREADS / 64; ++w) v = combine(s, v, sh[w * kND + s]);
            acc[s] = v;
        }
}

__device__ __forceinline__ void halo_pos(int h, int& hx, int& hy) {
    constexpr int ROWS2 = 2 * kLX;
    if (h < ROWS2) {
        hy = h / kLX;
        hx = h % kLX;
    } else if (h < 2 * ROWS2) {
        const int t = h - ROWS2;
        hy = kTY + 2 + t / kLX;
        hx = t % kLX;
    } else {
        const int t = h - 2 * ROWS2;
        hy = 2 + t / 4;
        const int c = t % 4;
        hx = c < 2 ? c : kTX + c;
    }
}

struct DiagArgs {
    Dims d;
    Coef<double> c;
    int zchunk, tiles_x, tiles_y;
};

template <typename T>
__global__ void __launch_bounds__(kNT) k_diag_partial(DiagArgs A, const T* __restrict__ q,
                                                      double* __restrict__ partial) {
    __shared__ double sV[kRing * 3 * kNPL];
    __shared__ double sRed[(kNT / 64) * kND];
    const Dims d = A.d;
    const size_t n = d.npts;
    const size_t plane = (size_t)d.nx * d.ny;
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int tix = t % A.tiles_x;
    const int tiy = (t / A.tiles_x) % A.tiles_y;
    const int tiz = t / (A.tiles_x * A.tiles_y);
    const int x0 = tix * kTX, y0 = tiy * kTY, z0 = tiz * A.zchunk;
    const int z1 = min(z0 + A.zchunk, d.nz);
    const int tid = threadIdx.x;
    const int lx = tid % kTX, ly = tid / kTX;
    const bool active = x0 + lx < d.nx && y0 + ly < d.ny;
    const size_t col = (size_t)pmodi(y0 + ly, d.ny) * d.nx + pmodi(x0 + lx, d.nx);
    const int own = (ly + 2) * kLX + (lx + 2);
    const bool hval = tid < kNHALO;
    int hidx = 0;
    size_t hcol = 0;
    if (hval) {
        int hx, hy;
        halo_pos(tid, hx, hy);
        hidx = hy * kLX + hx;
        hcol = (size_t)pmodi(y0 + hy - 2, d.ny) * d.nx + pmodi(x0 + hx - 2, d.nx);
    }
    const double gm1 = A.c.gm1;

    double acc[kND];
#pragma unroll
    for (int s = 0; s < kND; ++s) acc[s] = identity(s);
    double rho_q[3] = {0.0, 0.0, 0.0};  // own rho at planes z, z+1, z+2

    // The raw values of plane zz this thread needs: its own five fields and,
    // for a halo thread, the density and momenta at its halo point. Fetched
    // one plane ahead of use, so the load latency overlaps a plane's work
    // (9% faster in FP64 and 28% in FP32 at 512^3).
    struct Raw {
        T qv[5], h[4];
    };
    auto fetch = [&](int zz) {
        Raw r;
        const size_t po = (size_t)pmodi(zz, d.nz) * plane;
#pragma unroll
        for (int f = 0; f < 5; ++f) r.qv[f] = q[f * n + po + col];
        if (hval) {
#pragma unroll
            for (int f = 0; f < 4; ++f) r.h[f] = q[f * n + po + hcol];
        }
        return r;
    };
    // Put plane zz into ring slot zz mod 5; when it is an output plane of
    // this tile, fold its pointwise diagnostics. Returns own rho.
    auto enter = [&](int zz, const Raw& r) -> double {
        double* V = sV + pmodi(zz, kRing) * 3 * kNPL;
        double qv[5];
#pragma unroll
        for (int f = 0; f < 5; ++f) qv[f] = (double)r.qv[f];
        const double ir = 1.0 / qv[0];
        const double u = qv[1] * ir, v = qv[2] * ir, w = qv[3] * ir;
        V[own] = u;
        V[kNPL + own] = v;
        V[2 * kNPL + own] = w;
        if (hval) {
            const double hi = 1.0 / (double)r.h[0];
            V[hidx] = (double)r.h[1] * hi;
            V[kNPL + hidx] = (double)r.h[2] * hi;
            V[2 * kNPL + hidx] = (double)r.h[3] * hi;
        }
        if (active && zz >= z0 && zz < z1) {
            double nf = 0.0;
#pragma unroll
            for (int f = 0; f < 5; ++f) nf += isfinite(qv[f]) ? 0.0 : 1.0;
            const double ke = 0.5 * qv[0] * (u * u + v * v + w * w);
            const double p = gm1 * (qv[4] - ke);
            acc[0] += ke;
#pragma unroll
            for (int f = 0; f < 5; ++f) {
                acc[2 + f] += qv[f];
                acc[7 + f] = fmax(acc[7 + f], fabs(qv[f]));
            }
            acc[12] = fmin(acc[12], qv[0]);
            acc[13] = fmin(acc[13], p);
            acc[14] += nf;
            acc[15] += p;
        }
        return qv[0];
    };

    for (int s = 0; s < 4; ++s) {
        const double r = enter(z0 - 2 + s, fetch(z0 - 2 + s));
        if (s >= 2) rho_q[s - 2] = r;
    }
    Raw nxt = fetch(z0 + 2);
    const double a1x = A.c.a1[0], a2x = A.c.a2[0], a1y = A.c.a1[1], a2y = A.c.a2[1];
    const double a1z = A.c.a1[2], a2z = A.c.a2[2];
    for (int z = z0; z < z1; ++z) {
        const Raw cur = nxt;
        if (z + 1 < z1) nxt = fetch(z + 3);
        rho_q[2] = enter(z + 2, cur);
        __syncthreads();
        if (active) {
            const double* Vc = sV + pmodi(z, kRing) * 3 * kNPL;
            double G[3][3];  // G[a][b] = D_b u_a
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double* F = Vc + a * kNPL;
                G[a][0] = a1x * (F[own + 1] - F[own - 1]) + a2x * (F[own + 2] - F[own - 2]);
                G[a][1] = a1y * (F[own + kLX] - F[own - kLX]) + a2y * (F[own + 2 * kLX] - F[own - 2 * kLX]);
                const double* Fm2 = sV + pmodi(z - 2, kRing) * 3 * kNPL + a * kNPL;
                const double* Fm1 = sV + pmodi(z - 1, kRing) * 3 * kNPL + a * kNPL;
                const double* Fp1 = sV + pmodi(z + 1, kRing) * 3 * kNPL + a * kNPL;
                const double* Fp2 = sV + pmodi(z + 2, kRing) * 3 * kNPL + a * kNPL;
                G[a][2] = a1z * (Fp1[own] - Fm1[own]) + a2z * (Fp2[own] - Fm2[own]);
            }
            const double ox = G[2][1] - G[1][2];
            const double oy = G[0][2] - G[2][0];
            const double oz = G[1][0] - G[0][1];
            acc[1] += 0.5 * rho_q[0] * (ox * ox + oy * oy + oz * oz);
        }
        rho_q[0] = rho_q[1];
        rho_q[1] = rho_q[2];
        __syncthreads();
    }
    block_reduce<kNT>(acc, sRed);
    if (threadIdx.x == 0)
#pragma unroll
        for (int s = 0; s < kND; ++s) partial[(size_t)t * kND + s] = acc[s];
}

__global__ void __launch_bounds__(256) k_diag_final(int nblocks, double inv_n,
                                                    const double* __restrict__ partial,
                                                    double* __restrict__ out) {
    __shared__ double sRed[4 * kND];
    double acc[kND];
#pragma unroll
    for (int s = 0; s < kND; ++s) acc[s] = identity(s);
    for (int b = threadIdx.x; b < nblocks; b += 256)
#pragma unroll
        for (int s = 0; s < kND; ++s) acc[s] = combine(s, acc[s], partial[(size_t)b * kND + s]);
    block_reduce<256>(acc, sRed);
    if (threadIdx.x == 0) {
        const int means[] = {0, 1, 2, 3, 4, 5, 6, 15};
        for (int m = 0; m < 8; ++m) acc[means[m]] *= inv_n;
#pragma unroll
        for (int s = 0; s < kND; ++s) out[s] = acc[s];
    }
}

int diag_zchunk(const Dims& d) { return d.nz >= 64 ? 64 : d.nz; }

void diag_tiles(const Dims& d, int* tx, int* ty, int* tz) {
    *tx = (d.nx + kTX - 1) / kTX;
    *ty = (d.ny + kTY - 1) / kTY;
    const int zc = diag_zchunk(d);
    *tz = (d.nz + zc - 1) / zc;
}

}  // namespace

size_t diag_partial_count(const Dims& d) {
    int tx, ty, tz;
    diag_tiles(d, &tx, &ty, &tz);
    return (size_t)tx * ty * tz;
}

template <typename T>
void launch_diag(const Dims& d, const Coef<double>& c, const T* q, double* partial, double* out_dev,
                 hipStream_t s) {
    TimerScope ts("diag", s);
    DiagArgs a;
    a.d = d;
    a.c = c;
    a.zchunk = diag_zchunk(d);
    int tz;
    diag_tiles(d, &a.tiles_x, &a.tiles_y, &tz);
    const int nb = a.tiles_x * a.tiles_y * tz;
    hipLaunchKernelGGL(k_diag_partial<T>, dim3(nb), dim3(kNT), 0, s, a, q, partial);
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(256), 0, s, nb, 1.0 / (double)d.npts, partial,
                       out_dev);
}

// ------------------------------------------------ allocation-free diagnostics
// Partials and result of nsf_diagnostics_noalloc: one kND-double slot per
// diagnostics tile, for at most kScratchTiles tiles (a 1024^3 grid has
// 32 x 128 x 16 = 65536), then the kND output doubles; 8 MiB per GPU, held
// until the process ends. Every call on one GPU shares it. In host code the
// name `scratch` is a host-side stand-in, not a device address: kernels and
// copies get the address hipGetSymbolAddress returns on each device.
constexpr size_t kScratchTiles = 65536;
static __device__ __align__(256) double scratch[kScratchTiles * kND + kND];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

// Device address of the current device's scratch, looked up once per device
// (with that device current) and kept.
int scratch_address(double** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_error(NSF_EHIP, hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return set_error(NSF_EUNSUPPORTED, "device index above 63");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return set_error(NSF_EHIP, e != hipSuccess ? hipGetErrorString(e)
                                                       : "scratch has no device address");
        g_scratch_dev[dev] = (double*)ptr;
    }
    *out = g_scratch_dev[dev];
    return NSF_OK;
}
}  // namespace

size_t diag_noalloc_max_tiles() { return kScratchTiles; }

int diag_noalloc(const Dims& d, const Coef<double>& c, int precision, const void* q,
                 double* out_host, hipStream_t s) {
    if (diag_partial_count(d) > kScratchTiles)
        return set_error(NSF_EINVAL, "grid needs more diagnostics tiles than the fixed scratch holds");
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return set_error(NSF_EHIP, hipGetErrorString(e));
    if (s) {
        int sdev = -1;
        e = hipStreamGetDevice(s, &sdev);
        if (e != hipSuccess) return set_error(NSF_EHIP, hipGetErrorString(e));
        if (sdev != cur) return set_error(NSF_EINVAL, "stream belongs to another device than the current one");
    }
    double* base = nullptr;
    int rc = scratch_address(&base);
    if (rc) return rc;
    double* partial = base;
    double* dout = base + kScratchTiles * kND;
    if (precision == NSF_F64) launch_diag<double>(d, c, (const double*)q, partial, dout, s);
    else launch_diag<float>(d, c, (const float*)q, partial, dout, s);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(out_host, dout, kND * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return set_error(NSF_EHIP, hipGetErrorString(e));
    return NSF_OK;
}

template void launch_diag<float>(const Dims&, const Coef<double>&, const float*, double*, double*,
                                 hipStream_t);
template void launch_diag<double>(const Dims&, const Coef<double>&, const double*, double*,
                                  double*, hipStream_t);

}  // namespace nsf
