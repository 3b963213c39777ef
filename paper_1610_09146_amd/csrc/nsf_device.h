// Device-side building blocks shared by the gfx950 kernels: stencil weights,
// periodic indexing, the primitive-variable closure and the residual
// assembly of the compressible Navier-Stokes equations (paper Section 2,
// eqs (1)-(10)).
#pragma once

#ifndef NSF_NEWTON_RCP
#define NSF_NEWTON_RCP 1
#endif

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace nsf {

constexpr int kFields = 5;

// Grid extents and the size of one field.
struct Dims {
    int nx, ny, nz;
    size_t npts;
};

// Stencil weights and physical constants in the arithmetic type T, all
// products and reciprocals formed once on the host (the paper's division
// minimisation, Section 2, BL paragraph).
//   first derivative  D f  = a1 (f[+1] - f[-1]) + a2 (f[+2] - f[-2]),
//                      a1 = 8/(12h), a2 = -1/(12h);
//   second derivative D2 f = b0 f[0] + b1 (f[+1] + f[-1]) + b2 (f[+2] + f[-2]),
//                      b0 = -30/(12h^2), b1 = 16/(12h^2), b2 = -1/(12h^2).
template <typename T>
struct Coef {
    T a1[3], a2[3];
    T b0[3], b1[3], b2[3];
    T inv_Re;      // 1/Re
    T third;       // 1/3
    T two_thirds;  // 2/3
    T gm1;         // gamma - 1
    T gM2;         // gamma Ma^2
    T kappa;       // 1/((gamma-1) Ma^2 Pr Re), eq (5)
    T b0s;         // b0[0] + b0[1] + b0[2]: centre weight of the Laplacian
};

// Streaming (non-temporal) access for grid arrays a loop reads or writes
// once: the arrays are far larger than any cache, and keeping them out of L2
// leaves it to the data that is re-read (stencil neighbours).
template <typename V>
__device__ __forceinline__ V ld_nt(const V* p) { return __builtin_nontemporal_load(p); }
template <typename V>
__device__ __forceinline__ void st_nt(V v, V* p) { __builtin_nontemporal_store(v, p); }

// periodic index for offsets |i - [0, n)| <= 2: one period when n >= 3, a
// full modulo for the single-plane (two-dimensional) axis
__device__ __forceinline__ int wrap(int i, int n) {
    i = i < 0 ? i + n : (i >= n ? i - n : i);
    return (i < 0 || i >= n) ? ((i % n) + n) % n : i;
}

template <typename T>
__device__ __forceinline__ T d1(T fm2, T fm1, T fp1, T fp2, T a1, T a2) {
    return a1 * (fp1 - fm1) + a2 * (fp2 - fm2);
}

template <typename T>
__device__ __forceinline__ T d2(T fm2, T fm1, T f0, T fp1, T fp2, T b0, T b1, T b2) {
    return b0 * f0 + b1 * (fp1 + fm1) + b2 * (fp2 + fm2);
}

// 1/x for the density (normal, far from 0 and infinity): the hardware
// reciprocal estimate refined by Newton-Raphson steps e = 1 - x r, r + r e
// (Markstein). The double estimate carries about 24 bits, so double takes
// two steps (measured on gfx950: equal to the rounded quotient 1/x on 2^20
// densities in [0.9, 1.1]); the single estimate is within an ulp and one
// step gives the rounded quotient on the same sample. About half the
// instructions of the IEEE division sequence.
template <typename T>
__device__ __forceinline__ T fast_rcp(T x) {
#if NSF_NEWTON_RCP
    if constexpr (sizeof(T) == 8) {
        double r = __builtin_amdgcn_rcp(x);
        double e = fma(-x, r, 1.0);
        r = fma(r, e, r);
        e = fma(-x, r, 1.0);
        return fma(r, e, r);
    } else {
        const float r = __builtin_amdgcn_rcpf(x);
        const float e = fmaf(-x, r, 1.0f);
        return fmaf(r, e, r);
    }
#else
    return T(1) / x;
#endif
}

// Primitive variables from one point's conservative values, eqs (9)-(10):
// u_a = (rho u_a)/rho, p = (gamma-1)(rho E - rho|u|^2/2), T = gamma Ma^2 p/rho.
// One reciprocal of rho per point.
template <typename T>
struct Prim {
    T u, v, w, p, t;
};

template <typename T>
__device__ __forceinline__ Prim<T> primitives(T rho, T mx, T my, T mz, T E, const Coef<T>& c) {
    Prim<T> P;
    const T ir = fast_rcp(rho);
    P.u = mx * ir;
    P.v = my * ir;
    P.w = mz * ir;
    P.p = c.gm1 * (E - T(0.5) * rho * (P.u * P.u + P.v * P.v + P.w * P.w));
    P.t = c.gM2 * P.p * ir;
    return P;
}

// Point values entering the residual pointwise.
template <typename T>
struct Center {
    T rho, m[3], E, u[3];
};

// Every derivative the residual needs at one point (paper Section 2;
// G[a][b] = D_b u_a):
//   Drho[b] = D_b rho           Dm[a][b] = D_b(rho u_a)    DE[b] = D_b(rho E)
//   Dmu[a][b] = D_b(rho u_a u_b) DEu[b] = D_b(rho E u_b)   Dpu[b] = D_b(p u_b)
//   Dp[b] = D_b p               D2u[a][b] = D2_b u_a       D2T[b] = D2_b T
//   cross[a] = sum_{k != a} D_a(G_kk)
template <typename T>
struct Terms {
    T Drho[3], Dm[3][3], DE[3], G[3][3];
    T Dmu[3][3], DEu[3], Dpu[3], Dp[3];
    T D2u[3][3], D2T[3];
    T cross[3];
};

// Residual assembly (Section 2): skew-symmetric convection eq (8) with
// phi = 1, u_a, E; pressure gradient and pressure work in divergence form;
// viscous force expanded to second derivatives,
//   V_a = (1/Re)[sum_b D2_b u_a + (D2_a u_a + sum_{k!=a} D_a G_kk)/3];
// heat flux kappa sum_b D2_b T; viscous work tau_ab G_ab + u_a V_a with
//   tau_ab = (1/Re)(G_ab + G_ba - 2/3 delta_ab div).
template <typename T>
__device__ __forceinline__ void assemble(const Center<T>& c, const Terms<T>& d, const Coef<T>& k,
                                         T R[5]) {
    const T div = d.G[0][0] + d.G[1][1] + d.G[2][2];
    // mass
    {
        T s = c.rho * div;
#pragma unroll
        for (int b = 0; b < 3; ++b) s += d.Dm[b][b] + c.u[b] * d.Drho[b];
        R[0] = T(-0.5) * s;
    }
    // momentum
    T V[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const T lap = d.D2u[a][0] + d.D2u[a][1] + d.D2u[a][2];
        V[a] = k.inv_Re * (lap + k.third * (d.D2u[a][a] + d.cross[a]));
        T s = c.m[a] * div;
#pragma unroll
        for (int b = 0; b < 3; ++b) s += d.Dmu[a][b] + c.u[b] * d.Dm[a][b];
        R[1 + a] = T(-0.5) * s - d.Dp[a] + V[a];
    }
    // energy
    {
        T s = c.E * div;
        T pf = T(0), heat = T(0), gg = T(0), gt = T(0);
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            s += d.DEu[b] + c.u[b] * d.DE[b];
            pf += d.Dpu[b];
            heat += d.D2T[b];
        }
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                gg += d.G[a][b] * d.G[a][b];
                gt += d.G[a][b] * d.G[b][a];
            }
        const T work = k.inv_Re * (gg + gt - k.two_thirds * div * div);
        const T vwork = c.u[0] * V[0] + c.u[1] * V[1] + c.u[2] * V[2];
        R[4] = T(-0.5) * s - pf + k.kappa * heat + work + vwork;
    }
}

}  // namespace nsf
