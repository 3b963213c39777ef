// Pointwise kernels: Taylor-Green initial state, primitive variables, the
// low-storage RK stage update, BL product arrays and a streaming copy.
#include "nsf_internal.h"

namespace nsf {

namespace {

constexpr int kBlock = 256;

// The primitive and stage-update loops stream their arrays (ld_nt / st_nt):
// at 512^3 they ran 5-9% faster so. The BL product loop, whose output the
// next derivative loop re-reads at once, ran 5% slower so and keeps plain
// access.

inline unsigned grid_for(size_t n, int per_block) {
    size_t b = (n + per_block - 1) / per_block;
    return (unsigned)(b < 1 ? 1 : b);
}

// SplitMix64 (Steele, Lea & Flood, OOPSLA 2014), counter-indexed: output
// number counter+1 of the stream whose state starts at seed.
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t counter) {
    uint64_t z = seed + (counter + 1ull) * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Taylor-Green vortex (paper Section 3, DeBonis 2013), evaluated in double.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_init(Dims d, InitParams p, T* __restrict__ q,
                                                 double* __restrict__ qacc) {
    const size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= d.npts) return;
    const int i = (int)(idx % (size_t)d.nx);
    const int j = (int)((idx / (size_t)d.nx) % (size_t)d.ny);
    const int k = (int)(idx / ((size_t)d.nx * d.ny));
    const double two_pi = 6.283185307179586476925286766559;
    const double x = (double)i * (two_pi / d.nx);
    const double y = (double)j * (two_pi / d.ny);
    const double z = (double)k * (two_pi / d.nz);
    double vel[3];
    vel[0] = p.V0 * sin(x) * cos(y) * cos(z);
    vel[1] = -p.V0 * cos(x) * sin(y) * cos(z);
    vel[2] = 0.0;
    const double pr = 1.0 / (p.gamma * p.Ma * p.Ma) +
                      p.V0 * p.V0 * (cos(2.0 * x) + cos(2.0 * y)) * (cos(2.0 * z) + 2.0) / 16.0;
    if (p.kind == 1) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const uint64_t bits = splitmix64(p.seed, (uint64_t)a * d.npts + idx) >> 11;
            const double U = (double)bits * 0x1.0p-53;
            vel[a] = vel[a] * (1.0 + p.amp * (2.0 * U - 1.0));
        }
    } else if (p.kind == 2) {
        const double xs = x + p.phase[0], ys = y + p.phase[1], zs = z + p.phase[2];
        vel[0] += p.amp * sin(xs) * cos(ys) * cos(zs);
        vel[1] += -p.amp * cos(xs) * sin(ys) * cos(zs);
    }
    const double rho = p.gamma * p.Ma * p.Ma * pr;  // T = 1
    const double E = pr / (p.gamma - 1.0) +
                     rho * (vel[0] * vel[0] + vel[1] * vel[1] + vel[2] * vel[2]) / 2.0;
    const double v5[5] = {rho, rho * vel[0], rho * vel[1], rho * vel[2], E};
#pragma unroll
    for (int f = 0; f < 5; ++f) {
        q[f * d.npts + idx] = (T)v5[f];
        if (qacc) qacc[f * d.npts + idx] = v5[f];
    }
}

// Fused primitives, eqs (9)-(10): u, v, w, p, T from q in one pass.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_prims(Dims d, Coef<T> c, const T* __restrict__ q,
                                                  T* __restrict__ prim) {
    const size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= d.npts) return;
    const size_t n = d.npts;
    Prim<T> P = primitives(ld_nt(q + idx), ld_nt(q + n + idx), ld_nt(q + 2 * n + idx),
                           ld_nt(q + 3 * n + idx), ld_nt(q + 4 * n + idx), c);
    st_nt(P.u, prim + idx);
    st_nt(P.v, prim + n + idx);
    st_nt(P.w, prim + 2 * n + idx);
    st_nt(P.p, prim + 3 * n + idx);
    st_nt(P.t, prim + 4 * n + idx);
}

// BL primitives in three loops (Section 2, BL paragraph): no loop both
// writes a variable and reads it. Loop 1: u_a = rho u_a / rho.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_prims_bl_u(Dims d, const T* __restrict__ q,
                                                       T* __restrict__ prim) {
    const size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= d.npts) return;
    const size_t n = d.npts;
    const T ir = T(1) / q[idx];
    prim[idx] = q[n + idx] * ir;
    prim[n + idx] = q[2 * n + idx] * ir;
    prim[2 * n + idx] = q[3 * n + idx] * ir;
}

// Loop 2: p from the stored velocities, eq (6).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_prims_bl_p(Dims d, Coef<T> c, const T* __restrict__ q,
                                                       T* __restrict__ prim) {
    const size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= d.npts) return;
    const size_t n = d.npts;
    const T u = prim[idx], v = prim[n + idx], w = prim[2 * n + idx];
    prim[3 * n + idx] = c.gm1 * (q[4 * n + idx] - T(0.5) * q[idx] * (u * u + v * v + w * w));
}

// Loop 3: T from the stored pressure, eq (7).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_prims_bl_t(Dims d, Coef<T> c, const T* __restrict__ q,
                                                       T* __restrict__ prim) {
    const size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= d.npts) return;
    const size_t n = d.npts;
    prim[4 * n + idx] = c.gM2 * prim[3 * n + idx] / q[idx];
}

// Low-storage RK substep: q = q_acc + A dt r (not on the last substep),
// q_acc = q_acc + B dt r, and q = q_acc on the last substep. q_acc is
// double in both precisions.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_update(size_t n5, StageCoef sc, const T* __restrict__ r,
                                                   T* __restrict__ q, double* __restrict__ qacc) {
    const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= n5) return;
    const double rr = (double)ld_nt(r + e);
    const double a = ld_nt(qacc + e);
    const double na = fma(sc.b_dt, rr, a);
    st_nt(na, qacc + e);
    st_nt(sc.last ? (T)na : (T)fma(sc.a_dt, rr, a), q + e);
}

// BL product ("function") loop: out = f * g into the reused work array.
// Four elements per thread, a block-width apart (9% faster than one at
// 512^3; the primitive and update loops ran 7-12% slower so and keep one).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_product(size_t n, const T* __restrict__ f,
                                                    const T* __restrict__ g, T* __restrict__ out) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const size_t e = (size_t)blockIdx.x * (4 * kBlock) + r * kBlock + threadIdx.x;
        if (e < n) out[e] = f[e] * g[e];
    }
}

// Streaming copy, one 16-byte element per lane with non-temporal hints
// (bandwidth reference and counter calibration): the fastest plain copy
// form measured on gfx950, about 6.5 TB/s at 4 GiB.
typedef unsigned v4u __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(kBlock) k_copy16(size_t n16, const v4u* __restrict__ src,
                                                   v4u* __restrict__ dst) {
    const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (e < n16) __builtin_nontemporal_store(__builtin_nontemporal_load(src + e), dst + e);
}

__global__ void k_copy1(size_t n, const unsigned char* __restrict__ src,
                        unsigned char* __restrict__ dst) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) dst[e] = src[e];
}

}  // namespace

template <typename T>
void launch_init(const Dims& d, const InitParams& p, T* q, double* qacc, hipStream_t s) {
    TimerScope ts("init", s);
    hipLaunchKernelGGL(k_init<T>, dim3(grid_for(d.npts, kBlock)), dim3(kBlock), 0, s, d, p, q, qacc);
}

template <typename T>
void launch_prims(const Dims& d, const Coef<T>& c, const T* q, T* prim, hipStream_t s) {
    TimerScope ts("prims", s);
    hipLaunchKernelGGL(k_prims<T>, dim3(grid_for(d.npts, kBlock)), dim3(kBlock), 0, s, d, c, q, prim);
}

template <typename T>
void launch_prims_bl(const Dims& d, const Coef<T>& c, const T* q, T* prim, hipStream_t s) {
    TimerScope ts("prims", s);
    const dim3 g(grid_for(d.npts, kBlock));
    hipLaunchKernelGGL(k_prims_bl_u<T>, g, dim3(kBlock), 0, s, d, q, prim);
    hipLaunchKernelGGL(k_prims_bl_p<T>, g, dim3(kBlock), 0, s, d, c, q, prim);
    hipLaunchKernelGGL(k_prims_bl_t<T>, g, dim3(kBlock), 0, s, d, c, q, prim);
}

// The five fields of a state can hold more than 2^32 elements (a 1024^3
// grid has 5 * 2^30), more work items than one dispatch can address (its
// grid size is 32-bit), so the update is issued in launches of at most 2^31
// elements.
template <typename T>
void launch_update(const Dims& d, const StageCoef& sc, const T* r, T* q, double* qacc,
                   hipStream_t s) {
    TimerScope ts("update", s);
    const size_t n5 = 5 * d.npts;
    constexpr size_t kPart = (size_t)1 << 31;
    for (size_t base = 0; base < n5; base += kPart) {
        const size_t m = n5 - base < kPart ? n5 - base : kPart;
        hipLaunchKernelGGL(k_update<T>, dim3(grid_for(m, kBlock)), dim3(kBlock), 0, s, m, sc,
                           r + base, q + base, qacc + base);
    }
}

template <typename T>
void launch_product(const Dims& d, const T* f, const T* g, T* out, hipStream_t s) {
    TimerScope ts("bl_product", s);
    hipLaunchKernelGGL(k_product<T>, dim3(grid_for(d.npts, 4 * kBlock)), dim3(kBlock), 0, s, d.npts, f, g, out);
}

void launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s) {
    TimerScope ts("copy", s);
    const size_t n16 = bytes / 16;
    // one lane per element, in launches of at most 2^31 elements (a dispatch
    // addresses fewer than 2^32 work items)
    constexpr size_t kPart = (size_t)1 << 31;
    for (size_t base = 0; base < n16; base += kPart) {
        const size_t m = n16 - base < kPart ? n16 - base : kPart;
        hipLaunchKernelGGL(k_copy16, dim3(grid_for(m, kBlock)), dim3(kBlock), 0, s, m,
                           (const v4u*)src + base, (v4u*)dst + base);
    }
    const size_t tail = bytes - n16 * 16;
    if (tail)
        hipLaunchKernelGGL(k_copy1, dim3(1), dim3(64), 0, s, tail,
                           (const unsigned char*)src + n16 * 16, (unsigned char*)dst + n16 * 16);
}

#define NSF_INST(T)                                                                             \
    template void launch_init<T>(const Dims&, const InitParams&, T*, double*, hipStream_t);    \
    template void launch_prims<T>(const Dims&, const Coef<T>&, const T*, T*, hipStream_t);     \
    template void launch_prims_bl<T>(const Dims&, const Coef<T>&, const T*, T*, hipStream_t);  \
    template void launch_update<T>(const Dims&, const StageCoef&, const T*, T*, double*,       \
                                   hipStream_t);                                               \
    template void launch_product<T>(const Dims&, const T*, const T*, T*, hipStream_t);
NSF_INST(float)
NSF_INST(double)
#undef NSF_INST

}  // namespace nsf
