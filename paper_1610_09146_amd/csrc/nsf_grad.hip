// SS / RS primitive and gradient loops (paper Section 2, RS and SS
// paragraphs) in one pass: the primitives u, v, w, p, T (eqs (9)-(10)) and
// the first derivatives of the velocity, G_ab = D_b u_a, of a store set
// (bit 3a + b of the mask GM) stored in work arrays, the stored ones in
// order of 3a + b: all nine (the paper's 3D set), the three diagonal ones,
// or the four in-plane ones of a two-dimensional grid (the paper's 2D
// count). z-marching tiles: the velocity of each plane (with a two-point x-y
// halo), formed from q, enters a four-plane LDS ring once; x and y
// differences of the centre plane are taken from the ring, z differences
// from a register queue of the own column.
#include "nsf_internal.h"

namespace nsf {

namespace {

// Tile shape: 32 x TY points, one thread per point of a plane.
template <int TY>
struct PgTile {
    static constexpr int TX = 32, NT = TX * TY;
    static constexpr int LX = TX + 4, LY = TY + 4, NPL = LX * LY, NHALO = NPL - NT;
    static_assert(NHALO <= NT, "one halo point per thread at most");
};
// LDS velocity ring: planes z .. z+2 are in use at iteration z, and the slot
// that plane z+2 enters was last read two iterations before (every thread has
// passed the barrier of the iteration between), so four slots need one
// barrier per plane
constexpr int kRing = 4;
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

template <int TY>
__device__ __forceinline__ void halo_pos_g(int h, int& hx, int& hy) {
    using G = PgTile<TY>;
    constexpr int ROWS2 = 2 * G::LX;
    if (h < ROWS2) {
        hy = h / G::LX;
        hx = h % G::LX;
    } else if (h < 2 * ROWS2) {
        const int t = h - ROWS2;
        hy = TY + 2 + t / G::LX;
        hx = t % G::LX;
    } else {
        const int t = h - 2 * ROWS2;
        hy = 2 + t / 4;
        const int c = t % 4;
        hx = c < 2 ? c : G::TX + c;
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
// instead of the 80 + 96 of the two loops. The in-plane differences of the
// centre plane come from the LDS ring, the z differences from a register
// queue of the own column's velocity (planes z-2 .. z+2).
// MON (double precision): the tile also sums the kinetic energy and the
// enstrophy of its points, 1/2 rho |u|^2 and 1/2 rho |omega|^2 with omega
// from the same fourth-order velocity gradients (Section 3 diagnostics), in
// plane order per thread, then over the block in a fixed order, into
// mpart[2 * tile]: the monitor of a step whose first stage this is, without
// a separate diagnostics pass.
template <typename T, int GM, int TY, bool MON>
__global__ void __launch_bounds__(32 * TY) k_ss_prims_grad(GradArgs<T> A, const T* __restrict__ q,
                                                           T* __restrict__ prim,
                                                           T* __restrict__ grad,
                                                           double* __restrict__ mpart) {
    using G = PgTile<TY>;
    constexpr int kTX = G::TX, kLX = G::LX, kNPL = G::NPL, kNHALO = G::NHALO;
    auto slot = [](int a, int b) { return __builtin_popcount(GM & ((1 << (3 * a + b)) - 1)); };
    auto stored = [](int a, int b) { return (GM >> (3 * a + b)) & 1; };
    __shared__ T sV[kRing * 3 * kNPL];
    __shared__ double sM[MON ? 2 * (G::NT / 64) : 1];
    const Dims d = A.d;
    const Coef<T> c = A.c;
    const size_t n = d.npts;
    const size_t plane = (size_t)d.nx * d.ny;
    const int t = xcd_tile_g(blockIdx.x, gridDim.x);
    const int tix = t % A.tiles_x;
    const int tiy = (t / A.tiles_x) % A.tiles_y;
    const int tiz = t / (A.tiles_x * A.tiles_y);
    const int x0 = tix * kTX, y0 = tiy * TY, z0 = tiz * A.zchunk;
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
        halo_pos_g<TY>(tid, hx, hy);
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
#pragma unroll
        for (int f = 0; f < 4; ++f) r.halo[f] = hval ? q[f * n + po + hcol] : T(1);
        return r;
    };
    // velocity of plane zz into its ring slot and the own column's queue
    // entry vq (density into rq); the primitives of the chunk's own planes out
    auto enter = [&](int zz, const Raw& r, T vq[3], T& rq) {
        rq = r.own[0];
        T* V = sV + pmodg(zz, kRing) * 3 * kNPL;
        const Prim<T> P = primitives(r.own[0], r.own[1], r.own[2], r.own[3], r.own[4], c);
        vq[0] = P.u;
        vq[1] = P.v;
        vq[2] = P.w;
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
    T vq[5][3];  // own column's velocity, planes z-2 .. z+2
    T rq[5];     // and its density
#pragma unroll
    for (int s = 0; s < 4; ++s) enter(z0 - 2 + s, fetch(z0 - 2 + s), vq[s + 1], rq[s + 1]);
    Raw nxt = fetch(z0 + 2);
    const T a1x = c.a1[0], a2x = c.a2[0], a1y = c.a1[1], a2y = c.a2[1];
    const T a1z = c.a1[2], a2z = c.a2[2];
    double mke = 0.0, mens = 0.0;
    for (int z = z0; z < z1; ++z) {
        const Raw cur = nxt;
        if (z + 1 < z1) nxt = fetch(z + 3);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            rq[s] = rq[s + 1];
#pragma unroll
            for (int a = 0; a < 3; ++a) vq[s][a] = vq[s + 1][a];
        }
        enter(z + 2, cur, vq[4], rq[4]);
        __syncthreads();
        if (active) {
            const size_t o = (size_t)z * plane + col;
            const T* Vc = sV + pmodg(z, kRing) * 3 * kNPL;
            T g[3][3];  // g[a][b] = D_b u_a (the monitor needs all nine)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const T* F = Vc + a * kNPL;
                g[a][0] = a1x * (F[own + 1] - F[own - 1]) + a2x * (F[own + 2] - F[own - 2]);
                g[a][1] = a1y * (F[own + kLX] - F[own - kLX]) + a2y * (F[own + 2 * kLX] - F[own - 2 * kLX]);
                g[a][2] = a1z * (vq[3][a] - vq[1][a]) + a2z * (vq[4][a] - vq[0][a]);
#pragma unroll
                for (int b = 0; b < 3; ++b)
                    if (stored(a, b)) st_nt(g[a][b], grad + slot(a, b) * n + o);
            }
            if constexpr (MON) {
                const double rho = rq[2], u = vq[2][0], v = vq[2][1], w = vq[2][2];
                const double ox = g[2][1] - g[1][2], oy = g[0][2] - g[2][0], oz = g[1][0] - g[0][1];
                mke += 0.5 * rho * (u * u + v * v + w * w);
                mens += 0.5 * rho * (ox * ox + oy * oy + oz * oz);
            }
        }
    }
    if constexpr (MON) {
        // fixed order: wave shuffles, then the waves in order
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            mke += __shfl_down(mke, off, 64);
            mens += __shfl_down(mens, off, 64);
        }
        if ((tid & 63) == 0) {
            sM[2 * (tid >> 6)] = mke;
            sM[2 * (tid >> 6) + 1] = mens;
        }
        __syncthreads();
        if (tid == 0) {
            double x = 0.0, y = 0.0;
            for (int w = 0; w < G::NT / 64; ++w) {
                x += sM[2 * w];
                y += sM[2 * w + 1];
            }
            mpart[2 * t] = x;
            mpart[2 * t + 1] = y;
        }
    }
}

}  // namespace

template <typename T, int TY, bool MON>
static void launch_pg(const GradArgs<T>& a, int gmask, const T* q, T* prim, T* grad,
                      double* mpart, hipStream_t s) {
    const int tz = (a.d.nz + a.zchunk - 1) / a.zchunk;
    const dim3 grid(a.tiles_x * a.tiles_y * tz), block(32 * TY);
    if (gmask == kGradDiag)
        hipLaunchKernelGGL((k_ss_prims_grad<T, kGradDiag, TY, MON>), grid, block, 0, s, a, q, prim,
                           grad, mpart);
    else if (gmask == kGradPlane)
        hipLaunchKernelGGL((k_ss_prims_grad<T, kGradPlane, TY, MON>), grid, block, 0, s, a, q, prim,
                           grad, mpart);
    else
        hipLaunchKernelGGL((k_ss_prims_grad<T, kGradAll, TY, MON>), grid, block, 0, s, a, q, prim,
                           grad, mpart);
}

// Compute units of the current device (256 on a whole MI355X), looked up once
// per device.
static int device_cus() {
    static int cus[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cus[dev] == 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1)
            n = 256;
        cus[dev] = n;
    }
    return cus[dev];
}

// Tiles: on large grids 32 x 32 with 128-plane chunks, while that leaves four
// tiles per CU (one workgroup each: its four-plane ring takes 124 KB in
// double precision). Their halo and chunk preamble re-read q 1.13 times at
// 512^3, against 1.44 times for 32 x 16 tiles with 64-plane chunks (3.90
// against 4.12 ms per launch). Smaller grids keep 32 x 8 tiles (three
// workgroups per CU) with chunks of at most 64 planes, halved down to 16
// while the grid has fewer tiles than the GPU has CUs (256^3: 0.53 ms
// against 0.55 ms for the large tiles; 128^3: 32-plane chunks, 0.074 ms
// against 0.101 ms for 64).
template <typename T>
static GradArgs<T> pg_plan(const Dims& d, int* ty) {
    const int cus = device_cus();
    GradArgs<T> a{};
    a.d = d;
    a.tiles_x = (d.nx + 31) / 32;
    if (a.tiles_x * ((d.ny + 31) / 32) * (d.nz / 128) >= 4 * cus) {
        *ty = 32;
        a.tiles_y = (d.ny + 31) / 32;
        a.zchunk = 128;
    } else {
        *ty = 8;
        a.tiles_y = (d.ny + 7) / 8;
        int zc = 64;
        while (zc > 16 && a.tiles_x * a.tiles_y * ((d.nz + zc - 1) / zc) < cus) zc /= 2;
        a.zchunk = d.nz < zc ? d.nz : zc;
    }
    return a;
}

int ss_prims_grad_tiles(const Dims& d) {
    int ty;
    const GradArgs<double> a = pg_plan<double>(d, &ty);
    return a.tiles_x * a.tiles_y * ((d.nz + a.zchunk - 1) / a.zchunk);
}

template <typename T>
void launch_ss_prims_grad(const Dims& d, const Coef<T>& c, const T* q, T* prim, T* grad,
                          int gmask, hipStream_t s, double* mpart) {
    TimerScope ts("ss_prims_grad", s);
    int ty;
    GradArgs<T> a = pg_plan<T>(d, &ty);
    a.c = c;
    if constexpr (sizeof(T) == 8) {
        if (mpart) {
            if (ty == 32) launch_pg<T, 32, true>(a, gmask, q, prim, grad, mpart, s);
            else launch_pg<T, 8, true>(a, gmask, q, prim, grad, mpart, s);
            return;
        }
    }
    if (ty == 32) launch_pg<T, 32, false>(a, gmask, q, prim, grad, nullptr, s);
    else launch_pg<T, 8, false>(a, gmask, q, prim, grad, nullptr, s);
}

template void launch_ss_prims_grad<float>(const Dims&, const Coef<float>&, const float*, float*,
                                          float*, int, hipStream_t, double*);
template void launch_ss_prims_grad<double>(const Dims&, const Coef<double>&, const double*,
                                           double*, double*, int, hipStream_t, double*);

}  // namespace nsf
