// BL (baseline) algorithm kernels (paper Section 2, BL paragraph): each
// derivative is its own grid loop writing a grid-sized work array, and the
// residual loop reads the 60 stored derivatives back.
//
// Work-array numbering of the 60 derivatives (G_ab = D_b u_a):
//    0.. 2 D_b rho          3..11 D_b(rho u_a)       12..14 D_b(rho E)
//   15..23 G_ab             24..32 D_b(rho u_a u_b)  33..35 D_b(rho E u_b)
//   36..38 D_b(p u_b)       39..41 D_b p             42..50 D2_b u_a
//   51..56 D_a(G_kk), (a,k) = (0,1),(0,2),(1,0),(1,2),(2,0),(2,1)
//   57..59 D2_b T
// (index 3a + b within each nine-array group).
#include "nsf_internal.h"

namespace nsf {

namespace {

constexpr int kBX = 64, kBY = 4, kBZ = 4, kRY = 4;

// One derivative loop: out = D_AX f (ORDER 1) or D2_AX f (ORDER 2). Along
// x a block covers a row segment of kBX * kBY points in kBZ consecutive
// planes (four planes per block: 10% faster at 512^3 than one, 2 to 32
// measured alike; the long segment has fewer ends, whose halo reads fetch
// partly used lines: 2% more). Along y and z each thread slides a
// five-point window down its column, one new load per point: over kRY rows
// of one plane (y; 11% faster than the x form) or over kBZ planes (z), as a
// column of kBX x kBY points.
template <typename T, int AX, int ORDER>
__global__ void __launch_bounds__(kBX * kBY) k_bl_deriv(Dims d, Coef<T> c, const T* __restrict__ f,
                                                        T* __restrict__ out) {
    const size_t sy = (size_t)d.nx, sz = (size_t)d.nx * d.ny;
    if constexpr (AX == 1) {
        // one plane per block; each thread slides a five-row window down a
        // segment of kRY rows of its column
        const int i = blockIdx.x * kBX + threadIdx.x;
        const int j0 = (blockIdx.y * kBY + threadIdx.y) * kRY;
        const int k = blockIdx.z;
        if (i >= d.nx || j0 >= d.ny) return;
        const int j1 = min(j0 + kRY, d.ny);
        const size_t base = (size_t)k * sz + i;
        T v[5];
#pragma unroll
        for (int m = -2; m <= 1; ++m) v[m + 2] = f[base + (size_t)wrap(j0 + m, d.ny) * sy];
        T nxt = f[base + (size_t)wrap(j0 + 2, d.ny) * sy];
        for (int j = j0; j < j1; ++j) {
            v[4] = nxt;
            if (j + 1 < j1) nxt = f[base + (size_t)wrap(j + 3, d.ny) * sy];
            T* o = out + base + (size_t)j * sy;
            if (ORDER == 1)
                __builtin_nontemporal_store(d1(v[0], v[1], v[3], v[4], c.a1[AX], c.a2[AX]), o);
            else
                __builtin_nontemporal_store(d2(v[0], v[1], v[2], v[3], v[4], c.b0[AX], c.b1[AX], c.b2[AX]), o);
#pragma unroll
            for (int m = 0; m < 4; ++m) v[m] = v[m + 1];
        }
        return;
    }
    const int i = AX == 0 ? (blockIdx.x * kBY + threadIdx.y) * kBX + threadIdx.x
                          : blockIdx.x * kBX + threadIdx.x;
    const int j = AX == 0 ? blockIdx.y : blockIdx.y * kBY + threadIdx.y;
    const int k0 = blockIdx.z * kBZ;
    const int k1 = min(k0 + kBZ, d.nz);
    if (i >= d.nx || j >= d.ny) return;
    const size_t col = (size_t)j * sy + i;
    auto emit = [&](const T v[5], int k) {
        if (ORDER == 1)
            __builtin_nontemporal_store(d1(v[0], v[1], v[3], v[4], c.a1[AX], c.a2[AX]),
                                        out + (size_t)k * sz + col);
        else
            __builtin_nontemporal_store(d2(v[0], v[1], v[2], v[3], v[4], c.b0[AX], c.b1[AX], c.b2[AX]),
                                        out + (size_t)k * sz + col);
    };
    if (AX == 2) {
        T v[5];
#pragma unroll
        for (int m = -2; m <= 1; ++m) v[m + 2] = f[(size_t)wrap(k0 + m, d.nz) * sz + col];
        T nxt = f[(size_t)wrap(k0 + 2, d.nz) * sz + col];
        for (int k = k0; k < k1; ++k) {
            v[4] = nxt;
            if (k + 1 < k1) nxt = f[(size_t)wrap(k + 3, d.nz) * sz + col];
            emit(v, k);
#pragma unroll
            for (int m = 0; m < 4; ++m) v[m] = v[m + 1];
        }
    } else {
#pragma unroll 4
        for (int k = k0; k < k1; ++k) {
            const size_t base = (size_t)k * sz;
            T v[5];
#pragma unroll
            for (int m = -2; m <= 2; ++m) {
                const size_t idx = AX == 0 ? base + (size_t)j * sy + wrap(i + m, d.nx)
                                           : base + (size_t)wrap(j + m, d.ny) * sy + i;
                v[m + 2] = (ORDER == 2 || m != 0) ? f[idx] : T(0);
            }
            emit(v, k);
        }
    }
}

// Residual loop of BL: every derivative read from its work array. The work
// arrays and the residual are streamed (non-temporal: 13% faster at 512^3),
// as are the derivative loops' outputs (3%).
template <typename T>
__global__ void __launch_bounds__(256) k_bl_assemble(Dims d, Coef<T> c, const T* __restrict__ q,
                                                     const T* __restrict__ prim,
                                                     const T* __restrict__ dv, T* __restrict__ r) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= d.npts) return;
    const size_t n = d.npts;
    Center<T> ce;
    ce.rho = q[e];
    ce.m[0] = q[n + e];
    ce.m[1] = q[2 * n + e];
    ce.m[2] = q[3 * n + e];
    ce.E = q[4 * n + e];
    ce.u[0] = prim[e];
    ce.u[1] = prim[n + e];
    ce.u[2] = prim[2 * n + e];
    Terms<T> t;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        t.Drho[b] = __builtin_nontemporal_load(dv + ((0 + b) * n + e));
        t.DE[b] = __builtin_nontemporal_load(dv + ((12 + b) * n + e));
        t.DEu[b] = __builtin_nontemporal_load(dv + ((33 + b) * n + e));
        t.Dpu[b] = __builtin_nontemporal_load(dv + ((36 + b) * n + e));
        t.Dp[b] = __builtin_nontemporal_load(dv + ((39 + b) * n + e));
        t.D2T[b] = __builtin_nontemporal_load(dv + ((57 + b) * n + e));
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            t.Dm[a][b] = __builtin_nontemporal_load(dv + ((3 + 3 * a + b) * n + e));
            t.G[a][b] = __builtin_nontemporal_load(dv + ((15 + 3 * a + b) * n + e));
            t.Dmu[a][b] = __builtin_nontemporal_load(dv + ((24 + 3 * a + b) * n + e));
            t.D2u[a][b] = __builtin_nontemporal_load(dv + ((42 + 3 * a + b) * n + e));
        }
    }
    t.cross[0] = __builtin_nontemporal_load(dv + (51 * n + e)) + __builtin_nontemporal_load(dv + (52 * n + e));
    t.cross[1] = __builtin_nontemporal_load(dv + (53 * n + e)) + __builtin_nontemporal_load(dv + (54 * n + e));
    t.cross[2] = __builtin_nontemporal_load(dv + (55 * n + e)) + __builtin_nontemporal_load(dv + (56 * n + e));
    T R[5];
    assemble(ce, t, c, R);
#pragma unroll
    for (int f = 0; f < 5; ++f) __builtin_nontemporal_store(R[f], r + f * n + e);
}

template <typename T, int AX, int ORDER>
void launch_one(const Dims& d, const Coef<T>& c, const T* f, T* out, hipStream_t s) {
    const dim3 g(AX == 0 ? (unsigned)((d.nx + kBX * kBY - 1) / (kBX * kBY)) : (unsigned)((d.nx + kBX - 1) / kBX),
                 AX == 1 ? (unsigned)((d.ny + kBY * kRY - 1) / (kBY * kRY))
                         : AX == 0 ? (unsigned)d.ny : (unsigned)((d.ny + kBY - 1) / kBY),
                 AX == 1 ? (unsigned)d.nz : (unsigned)((d.nz + kBZ - 1) / kBZ));
    hipLaunchKernelGGL((k_bl_deriv<T, AX, ORDER>), g, dim3(kBX, kBY), 0, s, d, c, f, out);
}

}  // namespace

template <typename T>
void launch_bl_deriv(const Dims& d, const Coef<T>& c, int axis, int order, const T* f, T* out,
                     hipStream_t s) {
    TimerScope ts("bl_deriv", s);
    if (order == 1) {
        if (axis == 0) launch_one<T, 0, 1>(d, c, f, out, s);
        else if (axis == 1) launch_one<T, 1, 1>(d, c, f, out, s);
        else launch_one<T, 2, 1>(d, c, f, out, s);
    } else {
        if (axis == 0) launch_one<T, 0, 2>(d, c, f, out, s);
        else if (axis == 1) launch_one<T, 1, 2>(d, c, f, out, s);
        else launch_one<T, 2, 2>(d, c, f, out, s);
    }
}

template <typename T>
void launch_bl_assemble(const Dims& d, const Coef<T>& c, const T* q, const T* prim,
                        const T* deriv, T* r, hipStream_t s) {
    TimerScope ts("bl_assemble", s);
    const unsigned blocks = (unsigned)((d.npts + 255) / 256);
    hipLaunchKernelGGL(k_bl_assemble<T>, dim3(blocks), dim3(256), 0, s, d, c, q, prim, deriv, r);
}

#define NSF_INST(T)                                                                             \
    template void launch_bl_deriv<T>(const Dims&, const Coef<T>&, int, int, const T*, T*,      \
                                     hipStream_t);                                             \
    template void launch_bl_assemble<T>(const Dims&, const Coef<T>&, const T*, const T*,       \
                                        const T*, T*, hipStream_t);
NSF_INST(float)
NSF_INST(double)
#undef NSF_INST

}  // namespace nsf
