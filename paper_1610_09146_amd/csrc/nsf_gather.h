// Evaluation of every derivative term of the residual at one point from a
// field accessor, used by the untiled per-point kernels (RA, SS) and as the
// GPU's own reference path. The accessor is called as at(field, dx, dy, dz)
// with fields 0..4 = rho, rho u, rho v, rho w, rho E and 5..9 = u, v, w, p, T.
#pragma once

#include "nsf_device.h"

namespace nsf {

enum Field { F_RHO = 0, F_MX = 1, F_MY = 2, F_MZ = 3, F_E = 4, F_U = 5, F_V = 6, F_W = 7, F_P = 8, F_T = 9 };

template <int AX>
__device__ __forceinline__ void ax_offset(int m, int& dx, int& dy, int& dz) {
    dx = AX == 0 ? m : 0;
    dy = AX == 1 ? m : 0;
    dz = AX == 2 ? m : 0;
}

// First derivative of field f along AX at offset (ox, oy, oz) from the point.
template <typename T, int AX, typename At>
__device__ __forceinline__ T d1_at(At& at, int f, int ox, int oy, int oz, const Coef<T>& k) {
    int dx, dy, dz;
    T v[4];
    const int ms[4] = {-2, -1, 1, 2};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        ax_offset<AX>(ms[s], dx, dy, dz);
        v[s] = at(f, ox + dx, oy + dy, oz + dz);
    }
    return d1(v[0], v[1], v[2], v[3], k.a1[AX], k.a2[AX]);
}

// First derivative along AX of the product f*g (product formed per point).
template <typename T, int AX, typename At>
__device__ __forceinline__ T d1prod_at(At& at, int f, int g, const Coef<T>& k) {
    int dx, dy, dz;
    T v[4];
    const int ms[4] = {-2, -1, 1, 2};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        ax_offset<AX>(ms[s], dx, dy, dz);
        v[s] = at(f, dx, dy, dz) * at(g, dx, dy, dz);
    }
    return d1(v[0], v[1], v[2], v[3], k.a1[AX], k.a2[AX]);
}

template <typename T, int AX, typename At>
__device__ __forceinline__ T d2_at(At& at, int f, const Coef<T>& k) {
    int dx, dy, dz;
    T v[5];
#pragma unroll
    for (int s = 0; s < 5; ++s) {
        ax_offset<AX>(s - 2, dx, dy, dz);
        v[s] = at(f, dx, dy, dz);
    }
    return d2(v[0], v[1], v[2], v[3], v[4], k.b0[AX], k.b1[AX], k.b2[AX]);
}

// D_OUT(D_IN f): outer first-derivative stencil over inner derivatives.
template <typename T, int OUT, int IN, typename At>
__device__ __forceinline__ T d1d1_at(At& at, int f, const Coef<T>& k) {
    int dx, dy, dz;
    T v[4];
    const int ms[4] = {-2, -1, 1, 2};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        ax_offset<OUT>(ms[s], dx, dy, dz);
        v[s] = d1_at<T, IN>(at, f, dx, dy, dz, k);
    }
    return d1(v[0], v[1], v[2], v[3], k.a1[OUT], k.a2[OUT]);
}

template <typename T, int B, typename At>
__device__ __forceinline__ void gather_axis(At& at, const Coef<T>& k, Terms<T>& d, bool grads) {
    d.Drho[B] = d1_at<T, B>(at, F_RHO, 0, 0, 0, k);
    d.DE[B] = d1_at<T, B>(at, F_E, 0, 0, 0, k);
    d.Dp[B] = d1_at<T, B>(at, F_P, 0, 0, 0, k);
    d.DEu[B] = d1prod_at<T, B>(at, F_E, F_U + B, k);
    d.Dpu[B] = d1prod_at<T, B>(at, F_P, F_U + B, k);
    d.D2T[B] = d2_at<T, B>(at, F_T, k);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        d.Dm[a][B] = d1_at<T, B>(at, F_MX + a, 0, 0, 0, k);
        d.Dmu[a][B] = d1prod_at<T, B>(at, F_MX + a, F_U + B, k);
        d.D2u[a][B] = d2_at<T, B>(at, F_U + a, k);
        if (grads) d.G[a][B] = d1_at<T, B>(at, F_U + a, 0, 0, 0, k);
    }
}

// All terms; when `grads` is false, G and cross are left for the caller
// (stored-gradient algorithms).
template <typename T, typename At>
__device__ __forceinline__ void gather_terms(At& at, const Coef<T>& k, Terms<T>& d, bool grads) {
    gather_axis<T, 0>(at, k, d, grads);
    gather_axis<T, 1>(at, k, d, grads);
    gather_axis<T, 2>(at, k, d, grads);
    if (grads) {
        d.cross[0] = d1d1_at<T, 0, 1>(at, F_V, k) + d1d1_at<T, 0, 2>(at, F_W, k);
        d.cross[1] = d1d1_at<T, 1, 0>(at, F_U, k) + d1d1_at<T, 1, 2>(at, F_W, k);
        d.cross[2] = d1d1_at<T, 2, 0>(at, F_U, k) + d1d1_at<T, 2, 1>(at, F_V, k);
    }
}

}  // namespace nsf
