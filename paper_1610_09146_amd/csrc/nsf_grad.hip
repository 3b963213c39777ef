// SS / RS gradient loop (paper Section 2, RS and SS paragraphs): the first
// derivatives of the velocity, G_ab = D_b u_a, of a store set (bit 3a + b
// of the mask GM) stored in work arrays, the stored ones in order of 3a + b:
// all nine (the paper's 3D set), the three diagonal ones, or the four
// in-plane ones of a two-dimensional grid (the paper's 2D count).
// z-marching tiles: the stored velocity of each plane (with a two-point x-y
// halo) enters a five-plane LDS ring once; x, y and z differences of the
// centre plane are taken from the ring.
#include "nsf_internal.h"

namespace nsf {

namespace {

constexpr int kTX = 32, kTY = 8, kNT = kTX * kTY;
constexpr int kLX = kTX + 4, kLY = kTY + 4, kNPL = kLX * kLY, kNHALO = kNPL - kNT;
constexpr int kRing = 5;
constexpr int kXCD = 8;

__device__ __forceinline__ int pmodg(int a, int n) {
    int r = a % n;
    return r < 0 ? r + n : r;
}

__device__ __forceinline__ int xcd_tile_g(int bid, int nb) {
    const int per = nb / kXCD, extra = nb % kXCD;
    const int x = bid % kXCD, k = bid / kXCD;
    return x * per + (x < extra ? x : extra) + k;
}

__device__ __forceinline__ void halo_pos_g(int h, int& hx, int& hy) {
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

template <typename T>
struct GradArgs {
    Dims d;
    Coef<T> c;
    int zchunk, tiles_x, tiles_y;
};

template <typename T, int GM>
__global__ void __launch_bounds__(kNT) k_ss_grad(GradArgs<T> A, const T* __restrict__ prim,
                                                 T* __restrict__ grad) {
    // array of gradient (a, b): the number of stored gradients before it
    auto slot = [](int a, int b) { return __builtin_popcount(GM & ((1 << (3 * a + b)) - 1)); };
    auto stored = [](int a, int b) { return (GM >> (3 * a + b)) & 1; };
    __shared__ T sV[kRing * 3 * kNPL];
    const Dims d = A.d;
    const size_t n = d.npts;
    const size_t plane = (size_t)d.nx * d.ny;
    const int t = xcd_tile_g(blockIdx.x, gridDim.x);
    const int tix = t % A.tiles_x;
    const int tiy = (t / A.tiles_x) % A.tiles_y;
    const int tiz = t / (A.tiles_x * A.tiles_y);
    const int x0 = tix * kTX, y0 = tiy * kTY, z0 = tiz * A.zchunk;
    const int z1 = min(z0 + A.zchunk, d.nz);
    const int tid = threadIdx.x;
    const int lx = tid % kTX, ly = tid / kTX;
    const bool active = x0 + lx < d.nx && y0 + ly < d.ny;
    const size_t col = (size_t)pmodg(y0 + ly, d.ny) * d.nx + pmodg(x0 + lx, d.nx);
    const int own = (ly + 2) * kLX + (lx + 2);
    const bool hval = tid < kNHALO;
    int hidx = 0;
    size_t hcol = 0;
    if (hval) {
        int hx, hy;
        halo_pos_g(tid, hx, hy);
        hidx = hy * kLX + hx;
        hcol = (size_t)pmodg(y0 + hy - 2, d.ny) * d.nx + pmodg(x0 + hx - 2, d.nx);
    }
    // the velocity of plane zz at this thread's point and halo point,
    // fetched one plane ahead of use so the load latency overlaps a plane's
    // work
    struct Raw {
        T own[3], halo[3];
    };
    auto fetch = [&](int zz) {
        Raw r;
        const size_t po = (size_t)pmodg(zz, d.nz) * plane;
#pragma unroll
        for (int a = 0; a < 3; ++a) r.own[a] = prim[a * n + po + col];
        if (hval)
#pragma unroll
            for (int a = 0; a < 3; ++a) r.halo[a] = prim[a * n + po + hcol];
        return r;
    };
    auto enter = [&](int zz, const Raw& r) {
        T* V = sV + pmodg(zz, kRing) * 3 * kNPL;
#pragma unroll
        for (int a = 0; a < 3; ++a) V[a * kNPL + own] = r.own[a];
        if (hval)
#pragma unroll
            for (int a = 0; a < 3; ++a) V[a * kNPL + hidx] = r.halo[a];
    };
    for (int s = 0; s < 4; ++s) enter(z0 - 2 + s, fetch(z0 - 2 + s));
    Raw nxt = fetch(z0 + 2);
    const T a1x = A.c.a1[0], a2x = A.c.a2[0], a1y = A.c.a1[1], a2y = A.c.a2[1];
    const T a1z = A.c.a1[2], a2z = A.c.a2[2];
    for (int z = z0; z < z1; ++z) {
        const Raw cur = nxt;
        if (z + 1 < z1) nxt = fetch(z + 3);
        enter(z + 2, cur);
        __syncthreads();
        if (active) {
            const size_t o = (size_t)z * plane + col;
            const T* Vc = sV + pmodg(z, kRing) * 3 * kNPL;
            const T* Vm2 = sV + pmodg(z - 2, kRing) * 3 * kNPL;
            const T* Vm1 = sV + pmodg(z - 1, kRing) * 3 * kNPL;
            const T* Vp1 = sV + pmodg(z + 1, kRing) * 3 * kNPL;
            const T* Vp2 = sV + pmodg(z + 2, kRing) * 3 * kNPL;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const T* F = Vc + a * kNPL;
                // streamed: the residual sweep reads them back from HBM (7% faster)
                if (stored(a, 0))
                    st_nt(a1x * (F[own + 1] - F[own - 1]) + a2x * (F[own + 2] - F[own - 2]),
                          grad + slot(a, 0) * n + o);
                if (stored(a, 1))
                    st_nt(a1y * (F[own + kLX] - F[own - kLX]) + a2y * (F[own + 2 * kLX] - F[own - 2 * kLX]),
                          grad + slot(a, 1) * n + o);
                if (stored(a, 2))
                    st_nt(a1z * (Vp1[a * kNPL + own] - Vm1[a * kNPL + own]) +
                              a2z * (Vp2[a * kNPL + own] - Vm2[a * kNPL + own]),
                          grad + slot(a, 2) * n + o);
            }
        }
        __syncthreads();
    }
}

}  // namespace

template <typename T>
void launch_ss_grad(const Dims& d, const Coef<T>& c, const T* prim, T* grad, int gmask,
                    hipStream_t s) {
    TimerScope ts("ss_grad", s);
    GradArgs<T> a;
    a.d = d;
    a.c = c;
    a.zchunk = d.nz >= 64 ? 64 : d.nz;
    a.tiles_x = (d.nx + kTX - 1) / kTX;
    a.tiles_y = (d.ny + kTY - 1) / kTY;
    const int tz = (d.nz + a.zchunk - 1) / a.zchunk;
    const dim3 grid(a.tiles_x * a.tiles_y * tz);
    if (gmask == kGradDiag)
        hipLaunchKernelGGL((k_ss_grad<T, kGradDiag>), grid, dim3(kNT), 0, s, a, prim, grad);
    else if (gmask == kGradPlane)
        hipLaunchKernelGGL((k_ss_grad<T, kGradPlane>), grid, dim3(kNT), 0, s, a, prim, grad);
    else
        hipLaunchKernelGGL((k_ss_grad<T, kGradAll>), grid, dim3(kNT), 0, s, a, prim, grad);
}

template void launch_ss_grad<float>(const Dims&, const Coef<float>&, const float*, float*, int,
                                    hipStream_t);
template void launch_ss_grad<double>(const Dims&, const Coef<double>&, const double*, double*, int,
                                     hipStream_t);

}  // namespace nsf
