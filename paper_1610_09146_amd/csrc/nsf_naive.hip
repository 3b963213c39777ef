// Untiled per-point residual kernels: one thread per grid point, every
// stencil value fetched from global memory (the caches supply the reuse).
// RA: all derivatives inline; SS: velocity gradients from the nine stored
// arrays, everything else inline (paper Section 2, RA and SS paragraphs).
#include "nsf_gather.h"
#include "nsf_internal.h"

namespace nsf {

namespace {

constexpr int kBX = 64, kBY = 4;

// Field accessor on global memory with periodic wrap. Fields 0..4 are q,
// 5..9 the primitives, 10..18 the stored gradients G_ab at 10 + 3a + b.
template <typename T>
struct GlobalAt {
    const T* __restrict__ q;
    const T* __restrict__ prim;
    const T* __restrict__ grad;
    Dims d;
    int i, j, k;
    __device__ __forceinline__ T operator()(int f, int dx, int dy, int dz) const {
        const int ii = wrap(i + dx, d.nx), jj = wrap(j + dy, d.ny), kk = wrap(k + dz, d.nz);
        const size_t idx = ((size_t)kk * d.ny + jj) * d.nx + ii;
        if (f < 5) return q[f * d.npts + idx];
        if (f < 10) return prim[(f - 5) * d.npts + idx];
        return grad[(f - 10) * d.npts + idx];
    }
};

template <typename T>
__device__ __forceinline__ Center<T> center_of(const GlobalAt<T>& at) {
    Center<T> c;
    c.rho = at(F_RHO, 0, 0, 0);
    c.m[0] = at(F_MX, 0, 0, 0);
    c.m[1] = at(F_MY, 0, 0, 0);
    c.m[2] = at(F_MZ, 0, 0, 0);
    c.E = at(F_E, 0, 0, 0);
    c.u[0] = at(F_U, 0, 0, 0);
    c.u[1] = at(F_V, 0, 0, 0);
    c.u[2] = at(F_W, 0, 0, 0);
    return c;
}

template <typename T>
__global__ void __launch_bounds__(kBX * kBY) k_ra_naive(Dims d, Coef<T> k, const T* __restrict__ q,
                                                        const T* __restrict__ prim,
                                                        T* __restrict__ r) {
    const int i = blockIdx.x * kBX + threadIdx.x;
    const int j = blockIdx.y * kBY + threadIdx.y;
    const int kz = blockIdx.z;
    if (i >= d.nx || j >= d.ny) return;
    GlobalAt<T> at{q, prim, nullptr, d, i, j, kz};
    Terms<T> t;
    gather_terms(at, k, t, true);
    T R[5];
    assemble(center_of(at), t, k, R);
    const size_t idx = ((size_t)kz * d.ny + j) * d.nx + i;
#pragma unroll
    for (int f = 0; f < 5; ++f) r[f * d.npts + idx] = R[f];
}

// SS gradient kernel: G_ab = D_b u_a into nine work arrays.
template <typename T>
__global__ void __launch_bounds__(kBX * kBY) k_ss_grad_naive(Dims d, Coef<T> k,
                                                             const T* __restrict__ prim,
                                                             T* __restrict__ grad) {
    const int i = blockIdx.x * kBX + threadIdx.x;
    const int j = blockIdx.y * kBY + threadIdx.y;
    const int kz = blockIdx.z;
    if (i >= d.nx || j >= d.ny) return;
    GlobalAt<T> at{nullptr, prim, nullptr, d, i, j, kz};
    const size_t idx = ((size_t)kz * d.ny + j) * d.nx + i;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        grad[(3 * a + 0) * d.npts + idx] = d1_at<T, 0>(at, F_U + a, 0, 0, 0, k);
        grad[(3 * a + 1) * d.npts + idx] = d1_at<T, 1>(at, F_U + a, 0, 0, 0, k);
        grad[(3 * a + 2) * d.npts + idx] = d1_at<T, 2>(at, F_U + a, 0, 0, 0, k);
    }
}

template <typename T>
__global__ void __launch_bounds__(kBX * kBY) k_ss_naive(Dims d, Coef<T> k, const T* __restrict__ q,
                                                        const T* __restrict__ prim,
                                                        const T* __restrict__ grad,
                                                        T* __restrict__ r) {
    const int i = blockIdx.x * kBX + threadIdx.x;
    const int j = blockIdx.y * kBY + threadIdx.y;
    const int kz = blockIdx.z;
    if (i >= d.nx || j >= d.ny) return;
    GlobalAt<T> at{q, prim, grad, d, i, j, kz};
    Terms<T> t;
    gather_terms(at, k, t, false);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) t.G[a][b] = at(10 + 3 * a + b, 0, 0, 0);
    // cross[a] = sum_{c != a} D_a(G_cc), differencing the stored diagonal gradients
    t.cross[0] = d1_at<T, 0>(at, 10 + 4, 0, 0, 0, k) + d1_at<T, 0>(at, 10 + 8, 0, 0, 0, k);
    t.cross[1] = d1_at<T, 1>(at, 10 + 0, 0, 0, 0, k) + d1_at<T, 1>(at, 10 + 8, 0, 0, 0, k);
    t.cross[2] = d1_at<T, 2>(at, 10 + 0, 0, 0, 0, k) + d1_at<T, 2>(at, 10 + 4, 0, 0, 0, k);
    T R[5];
    assemble(center_of(at), t, k, R);
    const size_t idx = ((size_t)kz * d.ny + j) * d.nx + i;
#pragma unroll
    for (int f = 0; f < 5; ++f) r[f * d.npts + idx] = R[f];
}

inline dim3 grid3(const Dims& d) {
    return dim3((unsigned)((d.nx + kBX - 1) / kBX), (unsigned)((d.ny + kBY - 1) / kBY), (unsigned)d.nz);
}

}  // namespace

template <typename T>
void launch_ra_naive(const Dims& d, const Coef<T>& c, const T* q, const T* prim, T* r,
                     hipStream_t s) {
    TimerScope ts("ra_naive", s);
    hipLaunchKernelGGL(k_ra_naive<T>, grid3(d), dim3(kBX, kBY), 0, s, d, c, q, prim, r);
}

template <typename T>
void launch_ss_grad_naive(const Dims& d, const Coef<T>& c, const T* prim, T* grad, hipStream_t s) {
    TimerScope ts("ss_grad_naive", s);
    hipLaunchKernelGGL(k_ss_grad_naive<T>, grid3(d), dim3(kBX, kBY), 0, s, d, c, prim, grad);
}

template <typename T>
void launch_ss_naive(const Dims& d, const Coef<T>& c, const T* q, const T* prim, const T* grad,
                     T* r, hipStream_t s) {
    TimerScope ts("ss_naive", s);
    hipLaunchKernelGGL(k_ss_naive<T>, grid3(d), dim3(kBX, kBY), 0, s, d, c, q, prim, grad, r);
}

#define NSF_INST(T)                                                                            \
    template void launch_ra_naive<T>(const Dims&, const Coef<T>&, const T*, const T*, T*,     \
                                     hipStream_t);                                            \
    template void launch_ss_grad_naive<T>(const Dims&, const Coef<T>&, const T*, T*,          \
                                          hipStream_t);                                       \
    template void launch_ss_naive<T>(const Dims&, const Coef<T>&, const T*, const T*,         \
                                     const T*, T*, hipStream_t);
NSF_INST(float)
NSF_INST(double)
#undef NSF_INST

}  // namespace nsf
