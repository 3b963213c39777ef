// Diagnostics of paper Section 3 (kinetic-energy and enstrophy integrals,
// after DeBonis 2013) plus conservation sums, extrema and a non-finite
// count. Reduced in double in a fixed order: each thread walks a fixed
// point sequence, waves reduce with shuffles in a fixed tree, waves combine
// through LDS, and a second one-block pass folds the per-block partials in
// index order -- no atomics, so results are bitwise reproducible.
#include <math.h>

#include "nsf_internal.h"

namespace nsf {

namespace {

constexpr int kThreads = 256;
constexpr int kMaxBlocks = 2048;
constexpr int kND = 16;

// slot kinds: sums 0..6, 15; maxima 7..11; minima 12, 13; count 14 (a sum)
__device__ __forceinline__ bool is_max(int s) { return s >= 7 && s <= 11; }
__device__ __forceinline__ bool is_min(int s) { return s == 12 || s == 13; }

__device__ __forceinline__ double combine(int s, double a, double b) {
    if (is_max(s)) return fmax(a, b);
    if (is_min(s)) return fmin(a, b);
    return a + b;
}

__device__ __forceinline__ double identity(int s) {
    if (is_max(s)) return 0.0;
    if (is_min(s)) return INFINITY;
    return 0.0;
}

// Reduce acc[kND] over the block in a fixed order; thread 0 returns it.
__device__ void block_reduce(double acc[kND]) {
    __shared__ double sh[kThreads / 64][kND];
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
        for (int s = 0; s < kND; ++s) sh[wave][s] = acc[s];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int s = 0; s < kND; ++s) {
            double v = sh[0][s];
            for (int w = 1; w < kThreads / 64; ++w) v = combine(s, v, sh[w][s]);
            acc[s] = v;
        }
}

template <typename T>
__device__ __forceinline__ void vel_at(const T* __restrict__ q, size_t n, size_t e, double v[3]) {
    const double ir = 1.0 / (double)q[e];
    v[0] = (double)q[n + e] * ir;
    v[1] = (double)q[2 * n + e] * ir;
    v[2] = (double)q[3 * n + e] * ir;
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_diag_partial(Dims d, Coef<double> c, const T* __restrict__ q,
                                                           double* __restrict__ partial) {
    double acc[kND];
#pragma unroll
    for (int s = 0; s < kND; ++s) acc[s] = identity(s);
    const size_t n = d.npts;
    const size_t stride = (size_t)gridDim.x * kThreads;
    const double gm1 = c.gm1;
    for (size_t e = (size_t)blockIdx.x * kThreads + threadIdx.x; e < n; e += stride) {
        const int i = (int)(e % (size_t)d.nx);
        const int j = (int)((e / (size_t)d.nx) % (size_t)d.ny);
        const int k = (int)(e / ((size_t)d.nx * d.ny));
        double qv[5];
#pragma unroll
        for (int f = 0; f < 5; ++f) qv[f] = (double)q[f * n + e];
        double nf = 0.0;
#pragma unroll
        for (int f = 0; f < 5; ++f) nf += isfinite(qv[f]) ? 0.0 : 1.0;
        const double u = qv[1] / qv[0], v = qv[2] / qv[0], w = qv[3] / qv[0];
        const double ke = 0.5 * qv[0] * (u * u + v * v + w * w);
        const double p = gm1 * (qv[4] - ke);
        // vorticity from the fourth-order first derivative of the velocity
        double dvel[3][3];  // dvel[b][a] = D_b u_a
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            double vm2[3], vm1[3], vp1[3], vp2[3];
            size_t em2, em1, ep1, ep2;
            const size_t sx = 1, sy = (size_t)d.nx, sz = (size_t)d.nx * d.ny;
            const size_t base = e;
            if (b == 0) {
                const size_t row = e - i;
                em2 = row + wrap(i - 2, d.nx); em1 = row + wrap(i - 1, d.nx);
                ep1 = row + wrap(i + 1, d.nx); ep2 = row + wrap(i + 2, d.nx);
            } else if (b == 1) {
                const size_t pl = base - (size_t)j * sy;
                em2 = pl + wrap(j - 2, d.ny) * sy; em1 = pl + wrap(j - 1, d.ny) * sy;
                ep1 = pl + wrap(j + 1, d.ny) * sy; ep2 = pl + wrap(j + 2, d.ny) * sy;
            } else {
                const size_t col = base - (size_t)k * sz;
                em2 = col + wrap(k - 2, d.nz) * sz; em1 = col + wrap(k - 1, d.nz) * sz;
                ep1 = col + wrap(k + 1, d.nz) * sz; ep2 = col + wrap(k + 2, d.nz) * sz;
            }
            (void)sx;
            vel_at(q, n, em2, vm2);
            vel_at(q, n, em1, vm1);
            vel_at(q, n, ep1, vp1);
            vel_at(q, n, ep2, vp2);
            const double a1 = c.a1[b], a2 = c.a2[b];
#pragma unroll
            for (int a = 0; a < 3; ++a) dvel[b][a] = a1 * (vp1[a] - vm1[a]) + a2 * (vp2[a] - vm2[a]);
        }
        const double ox = dvel[1][2] - dvel[2][1];
        const double oy = dvel[2][0] - dvel[0][2];
        const double oz = dvel[0][1] - dvel[1][0];
        acc[0] += ke;
        acc[1] += 0.5 * qv[0] * (ox * ox + oy * oy + oz * oz);
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
    block_reduce(acc);
    if (threadIdx.x == 0)
#pragma unroll
        for (int s = 0; s < kND; ++s) partial[(size_t)blockIdx.x * kND + s] = acc[s];
}

__global__ void __launch_bounds__(kThreads) k_diag_final(int nblocks, double inv_n,
                                                         const double* __restrict__ partial,
                                                         double* __restrict__ out) {
    double acc[kND];
#pragma unroll
    for (int s = 0; s < kND; ++s) acc[s] = identity(s);
    for (int b = threadIdx.x; b < nblocks; b += kThreads)
#pragma unroll
        for (int s = 0; s < kND; ++s) acc[s] = combine(s, acc[s], partial[(size_t)b * kND + s]);
    block_reduce(acc);
    if (threadIdx.x == 0) {
        const int means[] = {0, 1, 2, 3, 4, 5, 6, 15};
        for (int m = 0; m < 8; ++m) acc[means[m]] *= inv_n;
#pragma unroll
        for (int s = 0; s < kND; ++s) out[s] = acc[s];
    }
}

int nblocks_for(const Dims& d) {
    size_t b = (d.npts + kThreads - 1) / kThreads;
    if (b > (size_t)kMaxBlocks) b = kMaxBlocks;
    return (int)(b < 1 ? 1 : b);
}

}  // namespace

size_t diag_partial_count(const Dims& d) { return (size_t)nblocks_for(d); }

template <typename T>
void launch_diag(const Dims& d, const Coef<double>& c, const T* q, double* partial, double* out_dev,
                 hipStream_t s) {
    TimerScope ts("diag", s);
    const int nb = nblocks_for(d);
    hipLaunchKernelGGL(k_diag_partial<T>, dim3(nb), dim3(kThreads), 0, s, d, c, q, partial);
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(kThreads), 0, s, nb, 1.0 / (double)d.npts,
                       partial, out_dev);
}

template void launch_diag<float>(const Dims&, const Coef<double>&, const float*, double*, double*,
                                 hipStream_t);
template void launch_diag<double>(const Dims&, const Coef<double>&, const double*, double*,
                                  double*, hipStream_t);

}  // namespace nsf
