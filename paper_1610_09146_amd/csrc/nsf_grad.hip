// SS / RS primitive and gradient loops (paper Section 2, RS and SS
// paragraphs) in one pass: the primitives u, v, w, p, T (eqs (9)-(10)) and
// the first derivatives of the velocity, G_ab = D_b u_a, of a store set
// (bit 3a + b of the mask GM) stored in work arrays, the stored ones in
// order of 3a + b: all nine (the paper's 3D set), the three diagonal ones,
// or the four in-plane ones of a two-dimensional grid (the paper's 2D
// count). z-marching tiles: the velocity of each plane (with a two-point x-y
// halo), formed from q, enters a five-plane LDS ring once; x, y and z
// differences of the centre plane are taken from the ring.
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

// Primitives and gradients in one pass: the same tile reads q instead of
// the stored velocity, forms u, v, w, p, T of its own points (the
// primitive loop's arithmetic, so the stored values are the same bits) and
// the velocity of its halo points, and writes the primitives of the chunk's
// planes beside the store set's gradients. 152 bytes per point (double)
// instead of the 80 + 96 of the two loops.
template <typename T, int GM>
__global__ void __launch_bounds__(kNT) k_ss_prims_grad(GradArgs<T> A, const T* __restrict__ q,
                                                       T* __restrict__ prim,
                                                       T* __restrict__ grad) {
    auto slot = [](int a, int b) { return __builtin_popcount(GM & ((1 << (3 * a + b)) - 1)); };
    auto stored = [](int a, int b) { return (GM >> (3 * a + b)) & 1; };
    __shared__ T sV[kRing * 3 * kNPL];
    const Dims d = A.d;
    const Coef<T> c = A.c;
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
    // raw conserved values of plane zz at this thread's point (five) and
    // halo point (density and momenta), fetched one plane ahead of use. The
    // density and momenta of a point are also the neighbouring tiles' halo,
    // so they stay in the L2 (read past it, they came from HBM twice: 2.2x
    // the algorithmic reads at 512^3); the energy, read once, streams past.
    struct Raw {
        T own[5], halo[4];
    };
    auto fetch = [&](int zz) {
        Raw r;
        const size_t po = (size_t)pmodg(zz, d.nz) * plane;
#pragma unroll
        for (int f = 0; f < 4; ++f) r.own[f] = q[f * n + po + col];
        r.own[4] = ld_nt(q + 4 * n + po + col);
        if (hval)
#pragma unroll
            for (int f = 0; f < 4; ++f) r.halo[f] = q[f * n + po + hcol];
        return r;
    };
    // velocity into the ring; the primitives of the chunk's own planes out
    auto enter = [&](int zz, const Raw& r) {
        T* V = sV + pmodg(zz, kRing) * 3 * kNPL;
        const Prim<T> P = primitives(r.own[0], r.own[1], r.own[2], r.own[3], r.own[4], c);
        V[own] = P.u;
        V[kNPL + own] = P.v;
        V[2 * kNPL + own] = P.w;
        if (hval) {
            const T ir = fast_rcp(r.halo[0]);
            V[hidx] = r.halo[1] * ir;
            V[kNPL + hidx] = r.halo[2] * ir;
            V[2 * kNPL + hidx] = r.halo[3] * ir;
        }
        if (active && zz >= z0 && zz < z1) {
            const size_t o = (size_t)zz * plane + col;
            st_nt(P.u, prim + o);
            st_nt(P.v, prim + n + o);
            st_nt(P.w, prim + 2 * n + o);
            st_nt(P.p, prim + 3 * n + o);
            st_nt(P.t, prim + 4 * n + o);
        }
    };
    for (int s = 0; s < 4; ++s) enter(z0 - 2 + s, fetch(z0 - 2 + s));
    Raw nxt = fetch(z0 + 2);
    const T a1x = c.a1[0], a2x = c.a2[0], a1y = c.a1[1], a2y = c.a2[1];
    const T a1z = c.a1[2], a2z = c.a2[2];
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
void launch_ss_prims_grad(const Dims& d, const Coef<T>& c, const T* q, T* prim, T* grad,
                          int gmask, hipStream_t s) {
    TimerScope ts("ss_prims_grad", s);
    GradArgs<T> a;
    a.d = d;
    a.c = c;
    a.zchunk = d.nz >= 64 ? 64 : d.nz;
    a.tiles_x = (d.nx + kTX - 1) / kTX;
    a.tiles_y = (d.ny + kTY - 1) / kTY;
    const int tz = (d.nz + a.zchunk - 1) / a.zchunk;
    const dim3 grid(a.tiles_x * a.tiles_y * tz);
    if (gmask == kGradDiag)
        hipLaunchKernelGGL((k_ss_prims_grad<T, kGradDiag>), grid, dim3(kNT), 0, s, a, q, prim, grad);
    else if (gmask == kGradPlane)
        hipLaunchKernelGGL((k_ss_prims_grad<T, kGradPlane>), grid, dim3(kNT), 0, s, a, q, prim, grad);
    else
        hipLaunchKernelGGL((k_ss_prims_grad<T, kGradAll>), grid, dim3(kNT), 0, s, a, q, prim, grad);
}

template void launch_ss_prims_grad<float>(const Dims&, const Coef<float>&, const float*, float*,
                                          float*, int, hipStream_t);
template void launch_ss_prims_grad<double>(const Dims&, const Coef<double>&, const double*,
                                           double*, double*, int, hipStream_t);

}  // namespace nsf
