// z-marching residual kernel for the RA / SN algorithms (every derivative
// evaluated in the residual loop, none stored; paper Section 2) on gfx950.
//
// A workgroup owns a TX x TY column tile of the x-y plane and marches its
// threads up a chunk of z-planes. At output plane z:
//   - x and y stencils read LDS: the seven fields rho, rho u_a, rho E, p, T
//     of plane z, and u, v, w from a five-plane ring (z-2 .. z+2), each with
//     a two-point halo (periodic wrap folded into the halo loads);
//   - z stencils read a per-thread register queue of the seven fields at
//     planes z-2 .. z+2 of the thread's own column, and the ring for u, v, w;
//   - the cross derivatives with z are taken as D_z of in-plane derivatives
//     (D_z D_x u, D_z D_y v, D_z D_x w, D_z D_y w: mixed central differences
//     commute), the in-plane derivatives being formed at the leading plane
//     z+2 and queued, so no thread needs a z-halo column;
//   - D_x D_y v and D_y D_x u use the LDS corner halo.
// Terms are folded into running sums direction by direction to keep few
// values live. FUSED = true recomputes the primitives from q inside the tile
// (no primitive arrays) and applies the low-storage RK stage update in the
// epilogue, writing the next stage's state to a different buffer.
#include "nsf_internal.h"

namespace nsf {

namespace {

// Streaming accesses of the fused stage: the accumulator and the stage
// output are touched once per launch and go with the non-temporal hint, so
// they do not displace the q planes that neighbouring tiles re-read as halo
// from the L2. (The unfused residual store stays a plain store: the update
// kernel reads it right after.)
#ifndef NSF_STREAM_NT
#define NSF_STREAM_NT 1
#endif
template <typename V>
__device__ __forceinline__ V stream_load(const V* p) {
    if constexpr (NSF_STREAM_NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <typename V>
__device__ __forceinline__ void stream_store(V v, V* p) {
    if constexpr (NSF_STREAM_NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Buffer view of one z-plane of one field. The base is uniform, so the
// descriptor sits in scalar registers and every lane passes a 32-bit byte
// offset. An offset at or past the plane's size is out of range: the hardware
// then returns 0 for a load and drops a store, which lets lanes outside the
// grid skip their accesses without a branch. (The grid check keeps a plane
// below 2^28 points, so a plane of doubles stays below kOutside bytes.)
constexpr uint32_t kOutside = 0x80000000u;
constexpr int kPolicy = NSF_STREAM_NT ? 2 : 0;  // cache-policy bits: non-temporal
constexpr int kRsrcWord3 = 0x00020000;        // gfx9 family: 32-bit data format
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_view(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                             kRsrcWord3);
}
// cached load of a field value (the q planes are re-read by neighbouring tiles)
template <typename T>
__device__ __forceinline__ T plane_load(__amdgpu_buffer_rsrc_t v, uint32_t off) {
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(v, off, 0, 0));
    else
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(v, off, 0, 0));
}
__device__ __forceinline__ double view_load(__amdgpu_buffer_rsrc_t v, uint32_t off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(v, off, 0, kPolicy));
}
__device__ __forceinline__ void view_store(double x, __amdgpu_buffer_rsrc_t v, uint32_t off) {
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, x), v, off, 0, kPolicy);
}
__device__ __forceinline__ void view_store(float x, __amdgpu_buffer_rsrc_t v, uint32_t off) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), v, off, 0, kPolicy);
}

constexpr int kTX = 32;  // tile width; the tile height is 8 or 16 rows

__device__ __forceinline__ int pmod(int a, int n) {
    int r = a % n;
    return r < 0 ? r + n : r;
}

// Give every XCD a contiguous range of tiles so that neighbouring tiles
// (which share halos) run under the same L2.
__device__ __forceinline__ int xcd_tile(int bid, int nb) {
    const int per = nb / kXCD, extra = nb % kXCD;
    const int x = bid % kXCD, k = bid / kXCD;
    return x * per + (x < extra ? x : extra) + k;
}

template <int TX, int TY>
struct Geom {
    static constexpr int LX = TX + 4, LY = TY + 4;
    static constexpr int NT = TX * TY;
    static constexpr int NPL = LX * LY;
    static constexpr int NHALO = NPL - NT;
    static constexpr int HPT = (NHALO + NT - 1) / NT;
    // cross-derivative ring: D_y v on the tile rows with the x halo, D_x u on
    // the tile columns with the y halo
    static constexpr int DYN = LX * TY, DXN = TX * LY, DSZ = DYN + DXN;
    static constexpr int DHALO = 4 * TY + 4 * TX;  // halo points of the two
};

// Halo position h (0 .. NHALO-1) -> LDS coordinates: two full rows below,
// two above, then the two-column strips left and right of the tile rows.
template <int TX, int TY>
__device__ __forceinline__ void halo_pos(int h, int& hx, int& hy) {
    constexpr int LX = TX + 4;
    constexpr int ROWS2 = 2 * LX;
    if (h < ROWS2) {
        hy = h / LX;
        hx = h % LX;
    } else if (h < 2 * ROWS2) {
        const int t = h - ROWS2;
        hy = TY + 2 + t / LX;
        hx = t % LX;
    } else {
        const int t = h - 2 * ROWS2;
        hy = 2 + t / 4;
        const int c = t % 4;
        hx = c < 2 ? c : TX + c;
    }
}

// Own-column values queued in registers (the velocity lives in the LDS ring).
template <typename T>
struct Pt {
    T rho, m0, m1, m2, E, p, t;
};

// Raw loads of one point: q (and, when primitives are stored, prim).
template <typename T, bool FUSED>
struct Raw {
    T q[5];
    T pr[FUSED ? 1 : 5];
};

template <typename T, bool FUSED>
__device__ __forceinline__ void load_raw(Raw<T, FUSED>& r, const T* __restrict__ q,
                                         const T* __restrict__ prim, size_t n, size_t off) {
#pragma unroll
    for (int f = 0; f < 5; ++f) r.q[f] = q[f * n + off];
    if (!FUSED) {
#pragma unroll
        for (int f = 0; f < 5; ++f) r.pr[f] = prim[f * n + off];
    }
}

template <typename T, bool FUSED>
__device__ __forceinline__ Pt<T> finish(const Raw<T, FUSED>& r, const Coef<T>& k, T uvw[3]) {
    Pt<T> P;
    P.rho = r.q[0];
    P.m0 = r.q[1];
    P.m1 = r.q[2];
    P.m2 = r.q[3];
    P.E = r.q[4];
    if (FUSED) {
        const Prim<T> pv = primitives(r.q[0], r.q[1], r.q[2], r.q[3], r.q[4], k);
        uvw[0] = pv.u;
        uvw[1] = pv.v;
        uvw[2] = pv.w;
        P.p = pv.p;
        P.t = pv.t;
    } else {
        uvw[0] = r.pr[0];
        uvw[1] = r.pr[1];
        uvw[2] = r.pr[2];
        P.p = r.pr[3];
        P.t = r.pr[4];
    }
    return P;
}

// Halo loads for the u, v, w ring plane (velocity only).
template <typename T, bool FUSED>
struct RawV {
    T a[FUSED ? 4 : 3];
};

template <typename T, bool FUSED>
__device__ __forceinline__ void load_rawv(RawV<T, FUSED>& r, const T* __restrict__ q,
                                          const T* __restrict__ prim, size_t n, size_t off) {
    if (FUSED) {
#pragma unroll
        for (int f = 0; f < 4; ++f) r.a[f] = q[f * n + off];
    } else {
#pragma unroll
        for (int f = 0; f < 3; ++f) r.a[f] = prim[f * n + off];
    }
}

template <typename T, bool FUSED>
__device__ __forceinline__ void finish_v(const RawV<T, FUSED>& r, T& u, T& v, T& w) {
    if (FUSED) {
        const T ir = fast_rcp(r.a[0]);
        u = r.a[1] * ir;
        v = r.a[2] * ir;
        w = r.a[3] * ir;
    } else {
        u = r.a[0];
        v = r.a[1];
        w = r.a[2];
    }
}

// Halo loads for the seven-field plane (rho, m, E, p, T).
template <typename T, bool FUSED>
struct RawP {
    T a[FUSED ? 5 : 7];
};

template <typename T, bool FUSED>
__device__ __forceinline__ void load_rawp(RawP<T, FUSED>& r, const T* __restrict__ q,
                                          const T* __restrict__ prim, size_t n, size_t off) {
#pragma unroll
    for (int f = 0; f < 5; ++f) r.a[f] = q[f * n + off];
    if (!FUSED) {
        r.a[5] = prim[3 * n + off];
        r.a[6] = prim[4 * n + off];
    }
}

template <typename T, bool FUSED>
__device__ __forceinline__ void finish_p(const RawP<T, FUSED>& r, const Coef<T>& k, T out[7]) {
#pragma unroll
    for (int f = 0; f < 5; ++f) out[f] = r.a[f];
    if (FUSED) {
        const Prim<T> pv = primitives(r.a[0], r.a[1], r.a[2], r.a[3], r.a[4], k);
        out[5] = pv.p;
        out[6] = pv.t;
    } else {
        out[5] = r.a[5];
        out[6] = r.a[6];
    }
}

template <typename T>
__device__ __forceinline__ T D1(T m2, T m1, T p1, T p2, T a1, T a2) {
    return a1 * (p1 - m1) + a2 * (p2 - m2);
}

// a * b + c with one rounding, whatever the surrounding code: where the same
// value is formed at several call sites and must agree bitwise, the choice
// of which product the compiler fuses is not left to it
template <typename T>
__device__ __forceinline__ T fmadd(T a, T b, T c) {
    if constexpr (sizeof(T) == 8) return __builtin_fma(a, b, c);
    else return __builtin_fmaf(a, b, c);
}

// First difference without its weight: D1 = a1 * D1u, since a2 = -a1 / 8
// exactly (the two weights are 8/(12h) and -1/(12h), and scaling by a power
// of two is exact). Sums of differences along one direction then take the
// weight once.
template <typename T>
__device__ __forceinline__ T D1u(T m2, T m1, T p1, T p2) {
    return T(-0.125) * (p2 - m2) + (p1 - m1);
}

template <typename T>
__device__ __forceinline__ T D2(T m2, T m1, T c, T p1, T p2, T b0, T b1, T b2) {
    return b0 * c + b1 * (p1 + m1) + b2 * (p2 + m2);
}

}  // namespace

namespace {

// Running sums of the residual (paper Section 2, residual assembly), folded
// one direction at a time.
template <typename T>
struct Acc {
    T S0;      // sum_b D_b(rho u_b) + u_b D_b rho
    T Sm[3];   // sum_b D_b(rho u_a u_b) + u_b D_b(rho u_a)
    T SE;      // sum_b D_b((rho E + 2 p) u_b) + u_b D_b(rho E): the skew
               // convection of rho E and, by linearity, twice the pressure work
    T HEAT;    // sum_b D2_b T \ in the split form without the centre term:
    T LAP[3];  // sum_b D2_b u_a / finalize adds the centre value once, times
               //                  the sum of the three centre weights
    T D2aa[3]; // D2_a u_a
    T Dp[3];   // D_a p
    T G[3][3]; // G_ab = D_b u_a
};

// Fold direction B given stencil values (index 0..4 = offsets -2..2) of the
// ten fields along that direction. rho/m/E/p/T arrays: f[field][5];
// ub = velocity component B along the stencil. Two rearrangements, both
// identities of the discrete operators (only rounding changes):
// FACT (the recomputed-derivative forms): the skew sums take the
// first-difference weight once per direction, and D_B p is kept unweighted;
// CENTRE (the same forms, double precision): the centre terms of the second
// differences are left to finalize, which adds them once for the three
// directions. In single precision that sum, b0s * T with T near 1, cancels
// against the off-centre sums in float and the kinetic-energy change of a
// 100-step 512^3 run drifts 3x further from the double-precision run, so
// float keeps the per-direction second differences. The stored-gradient
// form keeps the direct sums: with the centre terms split, its compiled
// schedule waits on its gradient loads early (+29% at 512^3).
// GSKIP: bit a set leaves G[a][B] to the caller, which has it from earlier
// work on the plane (see the tile loop).
template <typename T, int B, bool FACT, bool CENTRE, int GSKIP = 0>
__device__ __forceinline__ void fold_dir(Acc<T>& A, const T rho[5], const T m[3][5], const T E[5],
                                         const T p[5], const T tt[5], const T vel[3][5], T a1,
                                         T a2, T b0, T b1, T b2, const T uc[3]) {
    const T* ub = vel[B];
    // skew sums: D(f u_B) + u_B D(f), with the weight a1 taken once (FACT)
    auto dd = [&](const T f[5]) -> T {
        if constexpr (FACT) return D1u(f[0], f[1], f[3], f[4]);
        else return D1(f[0], f[1], f[3], f[4], a1, a2);
    };
    auto acc = [&](T& sum, T dfu, T df) {
        if constexpr (FACT) sum += a1 * (dfu + uc[B] * df);
        else sum += dfu + uc[B] * df;
    };
    const T Drho = dd(rho);
    acc(A.S0, dd(m[B]), Drho);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const T Dm = dd(m[a]);
        const T mu[5] = {m[a][0] * ub[0], m[a][1] * ub[1], T(0), m[a][3] * ub[3], m[a][4] * ub[4]};
        acc(A.Sm[a], dd(mu), Dm);
        if (!((GSKIP >> a) & 1)) A.G[a][B] = D1(vel[a][0], vel[a][1], vel[a][3], vel[a][4], a1, a2);
        if constexpr (CENTRE) {
            // b2 = -b1 / 16 exactly: off-centre part of D2 = b1 * offu
            const T offu = T(-0.0625) * (vel[a][4] + vel[a][0]) + (vel[a][3] + vel[a][1]);
            A.LAP[a] += b1 * offu;
            if (a == B) A.D2aa[a] = b0 * vel[a][2] + b1 * offu;
        } else {
            const T d2 = D2(vel[a][0], vel[a][1], vel[a][2], vel[a][3], vel[a][4], b0, b1, b2);
            A.LAP[a] += d2;
            if (a == B) A.D2aa[a] = d2;
        }
    }
    // -1/2 D(E u) - D(p u) = -1/2 D((E + 2 p) u): one stencil for both fluxes
    auto H = [&](int s) -> T { return (T(2) * p[s] + E[s]) * ub[s]; };
    const T Eu[5] = {H(0), H(1), T(0), H(3), H(4)};
    acc(A.SE, dd(Eu), dd(E));
    A.Dp[B] = dd(p);  // unweighted in the FACT form: finalize applies a1
    if constexpr (CENTRE) A.HEAT += b1 * (T(-0.0625) * (tt[4] + tt[0]) + (tt[3] + tt[1]));
    else A.HEAT += D2(tt[0], tt[1], tt[2], tt[3], tt[4], b0, b1, b2);
}

// Residual assembly; om2 receives |omega|^2 with omega = curl u from G
// (used by the kinetic-energy / enstrophy monitor). FACT and CENTRE as in
// fold_dir; FACT also selects the compact form of the viscous work.
template <typename T, bool FACT, bool CENTRE>
__device__ __forceinline__ void finalize(const Acc<T>& A, const T cross[3], T rho, const T m[3],
                                         T E, T t, const T u[3], const Coef<T>& k, T R[5], T& om2) {
    const T b0s = CENTRE ? k.b0s : T(0);  // centre weight of the three second differences
    {
        const T ox = A.G[2][1] - A.G[1][2];
        const T oy = A.G[0][2] - A.G[2][0];
        const T oz = A.G[1][0] - A.G[0][1];
        om2 = ox * ox + oy * oy + oz * oz;
    }
    const T div = A.G[0][0] + A.G[1][1] + A.G[2][2];
    R[0] = T(-0.5) * (A.S0 + rho * div);
    T V[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const T lap = CENTRE ? b0s * u[a] + A.LAP[a] : A.LAP[a];
        V[a] = k.inv_Re * (lap + k.third * (A.D2aa[a] + cross[a]));
        const T dp = FACT ? k.a1[a] * A.Dp[a] : A.Dp[a];
        R[1 + a] = T(-0.5) * (A.Sm[a] + m[a] * div) - dp + V[a];
    }
    T ggt;
    if constexpr (FACT) {
        // sum_ab G_ab (G_ab + G_ba) = 2 sum_a G_aa^2 + sum_{a<b} (G_ab + G_ba)^2
        const T s01 = A.G[0][1] + A.G[1][0];
        const T s02 = A.G[0][2] + A.G[2][0];
        const T s12 = A.G[1][2] + A.G[2][1];
        const T dsq = A.G[0][0] * A.G[0][0] + A.G[1][1] * A.G[1][1] + A.G[2][2] * A.G[2][2];
        ggt = T(2) * dsq + s01 * s01 + s02 * s02 + s12 * s12;
    } else {
        T gg = T(0), gt = T(0);
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                gg += A.G[a][b] * A.G[a][b];
                gt += A.G[a][b] * A.G[b][a];
            }
        ggt = gg + gt;
    }
    const T work = k.inv_Re * (ggt - k.two_thirds * div * div);
    const T heat = CENTRE ? b0s * t + A.HEAT : A.HEAT;
    R[4] = T(-0.5) * (A.SE + E * div) + k.kappa * heat + work +
           (u[0] * V[0] + u[1] * V[1] + u[2] * V[2]);
}

// Views of one output plane for the recompute forms: the plane fields of
// plane z and the velocity of planes z-2 .. z+2 in LDS, each plane with its
// two-point x-y halo. Strides in elements.
template <typename T>
struct RcView {
    const T* P;      // plane fields rho, rho E, p, T (stored-gradient form: then rho u_a)
    const T* V[5];   // velocity u, v, w of planes z-2 .. z+2
    int ownP, ownV;  // the output point in the two layouts
    int FOP, RSP;    // field and row strides of the plane fields
    int FOV, RSV;    // field and row strides of the velocity planes
};

// Residual of one point in the recompute forms (paper Section 2): the
// recompute-all algorithm RA, and, with the velocity gradients read from
// their stored arrays, the recompute-some algorithm RS. The five equations
// are evaluated one after another and every derivative a term needs is
// formed where the term uses it, from the grid values staged in LDS (x and
// y stencils, and the cross derivatives with z as nested stencils over the
// velocity planes) or in the own column's register queue Q (z stencils):
// nothing is carried from one equation to the next. The empty asm statement
// with a memory clobber at the start of each equation makes the compiler
// load the staged values again, so it cannot merge the derivatives of
// different equations, which would turn the kernel into the thread-local
// form. A z difference of queue values alone occurs in one equation only, so
// the queue needs no such fence. Same assembly as the oracle: skew-symmetric
// convection eq (8) with phi = 1, u_a, E; pressure work -D_j(p u_j); viscous
// force V_a = (1/Re)[sum_b D2_b u_a + (D2_a u_a + sum_{c != a} D_a G_cc)/3];
// heat flux kappa sum_b D2_b T; viscous work tau_ab G_ab + u_a V_a.
// om2 (monitored stage) receives |curl u|^2 from recomputed gradients.
// Compiler fence for the recompute forms: no load moves across it, so a
// derivative after it reads its grid values again.
__device__ __forceinline__ void rc_fence() { asm volatile("" ::: "memory"); }
// Ties a finished equation's residual to its place between the fences, so the
// compiler does not sink its arithmetic below them (into the store branch),
// which would hold every loaded value live until then.
template <typename T>
__device__ __forceinline__ void rc_pin(T& x) { asm volatile("" : "+v"(x)); }

template <typename T, bool SS, bool MON, int GM, typename PoffF>
__device__ __forceinline__ void recompute_point(const RcView<T>& v, const Pt<T> Q[5], const T uc[3],
                                                const Coef<T>& k, const T* grad, size_t n,
                                                PoffF poff, int z, size_t col, const size_t xnb[4],
                                                const size_t ynb[4], T R[5], T& om2) {
    // plane field f at in-plane offset (dx, dy) of plane z
    auto P = [&](int f, int dx, int dy) -> T { return v.P[f * v.FOP + v.ownP + dx + dy * v.RSP]; };
    // velocity component c at offset (dx, dy, dz), |dz| <= 2
    auto U = [&](int c, int dx, int dy, int dz) -> T {
        return v.V[dz + 2][c * v.FOV + v.ownV + dx + dy * v.RSV];
    };
    auto qf = [&](const Pt<T>& q, int f) -> T {
        switch (f) {
            case 0: return q.rho;
            case 1: return q.E;
            case 2: return q.p;
            case 3: return q.t;
            case 4: return q.m0;
            case 5: return q.m1;
            default: return q.m2;
        }
    };
    // plane field f at stencil position s (0..4 = offsets -2..2) along B
    auto F = [&](int f, int B, int s) -> T {
        if (B == 0) return P(f, s - 2, 0);
        if (B == 1) return P(f, 0, s - 2);
        return qf(Q[s], f);
    };
    auto Us = [&](int c, int B, int s) -> T {
        return U(c, B == 0 ? s - 2 : 0, B == 1 ? s - 2 : 0, B == 2 ? s - 2 : 0);
    };
    // momentum rho u_a at stencil position s along B (the stored-gradient
    // form stages the conserved momenta; the others form rho * u_a)
    auto M = [&](int a, int B, int s) -> T {
        if constexpr (SS) return F(4 + a, B, s);
        else return F(0, B, s) * Us(a, B, s);
    };
    auto D1 = [&](int B, auto g) -> T { return k.a1[B] * (g(3) - g(1)) + k.a2[B] * (g(4) - g(0)); };
    auto D2 = [&](int B, auto g) -> T {
        return k.b0[B] * g(2) + k.b1[B] * (g(3) + g(1)) + k.b2[B] * (g(4) + g(0));
    };
    const size_t pz = poff(z);
    // stored-gradient forms: whether G_ab is in the store set GM, and its array
    auto stored = [](int a, int b) { return SS && ((GM >> (3 * a + b)) & 1); };
    auto slot = [](int a, int b) { return __builtin_popcount(GM & ((1 << (3 * a + b)) - 1)); };
    // velocity gradient G_ab = D_b u_a: its stored array (RS), or its difference
    auto Gab = [&](int a, int b) -> T {
        if (stored(a, b)) return grad[slot(a, b) * n + pz + col];
        return D1(b, [&](int s) { return Us(a, b, s); });
    };
    // D_A(G_cc), A != c: D_A of the stored diagonal gradient (RS), or the
    // nested difference D_A(D_c u_c) over the staged velocity
    auto DG = [&](int A, int c) -> T {
        if (stored(c, c)) {
            const int comp = slot(c, c);
            auto g = [&](int s) -> T {
                const int m = s < 2 ? s : s - 1;  // xnb / ynb slot of offset s - 2
                if (A == 0) return grad[comp * n + pz + xnb[m]];
                if (A == 1) return grad[comp * n + pz + ynb[m]];
                return grad[comp * n + poff(z + s - 2) + col];
            };
            return D1(A, g);
        } else {
            auto inner = [&](int o) -> T {
                return D1(c, [&](int s) -> T {
                    int d[3] = {0, 0, 0};
                    d[A] += o;
                    d[c] += s - 2;
                    return U(c, d[0], d[1], d[2]);
                });
            };
            return k.a1[A] * (inner(1) - inner(-1)) + k.a2[A] * (inner(2) - inner(-2));
        }
    };
    auto Visc = [&](int a) -> T {
        T lap = T(0), d2aa = T(0);
#pragma unroll
        for (int B = 0; B < 3; ++B) {
            const T d2 = D2(B, [&](int s) { return Us(a, B, s); });
            lap += d2;
            if (B == a) d2aa = d2;
        }
        T cross = T(0);
#pragma unroll
        for (int c = 0; c < 3; ++c)
            if (c != a) cross += DG(a, c);
        return k.inv_Re * (lap + k.third * (d2aa + cross));
    };
    const T rho_c = Q[2].rho;
    // mass, eq (1)
    {
        rc_fence();
        T S = T(0), div = T(0);
#pragma unroll
        for (int B = 0; B < 3; ++B) {
            S += D1(B, [&](int s) { return M(B, B, s); }) + uc[B] * D1(B, [&](int s) { return F(0, B, s); });
            div += Gab(B, B);
        }
        R[0] = T(-0.5) * (S + rho_c * div);
        rc_pin(R[0]);
    }
    // momentum, eq (2)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        rc_fence();
        T S = T(0), div = T(0);
#pragma unroll
        for (int B = 0; B < 3; ++B) {
            S += D1(B, [&](int s) { return M(a, B, s) * Us(B, B, s); }) +
                 uc[B] * D1(B, [&](int s) { return M(a, B, s); });
            div += Gab(B, B);
        }
        const T mc = SS ? qf(Q[2], 4 + a) : rho_c * uc[a];
        R[1 + a] = T(-0.5) * (S + mc * div) - D1(a, [&](int s) { return F(2, a, s); }) + Visc(a);
        rc_pin(R[1 + a]);
    }
    // energy, eq (3)
    {
        rc_fence();
        T S = T(0), pw = T(0), heat = T(0);
#pragma unroll
        for (int B = 0; B < 3; ++B) {
            S += D1(B, [&](int s) { return F(1, B, s) * Us(B, B, s); }) +
                 uc[B] * D1(B, [&](int s) { return F(1, B, s); });
            pw += D1(B, [&](int s) { return F(2, B, s) * Us(B, B, s); });
            heat += D2(B, [&](int s) { return F(3, B, s); });
        }
        T G[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) G[a][b] = Gab(a, b);
        const T div = G[0][0] + G[1][1] + G[2][2];
        T gg = T(0), gt = T(0);
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                gg += G[a][b] * G[a][b];
                gt += G[a][b] * G[b][a];
            }
        T vw = T(0);
#pragma unroll
        for (int a = 0; a < 3; ++a) vw += uc[a] * Visc(a);
        R[4] = T(-0.5) * (S + Q[2].E * div) - pw + k.kappa * heat +
               k.inv_Re * (gg + gt - k.two_thirds * div * div) + vw;
        rc_pin(R[4]);
    }
    if constexpr (MON) {
        rc_fence();
        const T ox = Gab(2, 1) - Gab(1, 2);
        const T oy = Gab(0, 2) - Gab(2, 0);
        const T oz = Gab(1, 0) - Gab(0, 1);
        om2 = ox * ox + oy * oy + oz * oz;
        rc_pin(om2);
    }
}

// Whether the tile keeps unweighted D_y v and D_x u of the last three
// leading planes in LDS, so that the nested cross differences D_x D_y v and
// D_y D_x u read four values each instead of forming sixteen-point stencils:
// the double-precision 16-row tiles of the recomputed-derivative forms,
// whose stage is bound by its arithmetic (-5.6% on the fused 512^3 stage).
// Not the 8-row tile, whose LDS must stay under half the CU's for two
// workgroups, and not single precision, whose stage is bound by memory
// (no gain measured, +2% on its monitored build).
// (Not in the recompute forms: they keep no derivative values.)
template <typename T, int TY, bool SS, bool RC = false>
constexpr bool d_ring() {
    return !SS && !RC && sizeof(T) == 8 && TY == 16;
}

// Velocity ring slots. Five, or four where the fused tile keeps the D ring
// and needs the room: then the slot of the leading plane z+2 is that of
// z-2, whose in-plane readers (it was the centre plane two barriers ago)
// are done, and its own column, which the z fold still reads, is copied to
// registers first.
// The recompute forms read the velocity of all five planes with its
// x-y halo (the z cross derivatives as nested stencils), so they keep five.
template <typename T, int TY, bool FUSED, bool SS, bool RC = false>
constexpr int ring_slots() {
    return FUSED && d_ring<T, TY, SS, RC>() ? 4 : 5;
}

// Whether a tile keeps a per-thread halo ring in LDS: each halo point is
// fetched once per plane, with the leading plane z+2 (the plane the
// neighbouring tile fetches as interior in the same iteration, so the
// halo's cache lines are still in the L2); its velocity goes to the ring at
// once and its plane fields are parked until it is the centre plane.
// Without the ring, the fused form fetches every halo point twice per plane,
// and the stored-gradient form fetches the plane fields of plane z+1, two
// planes after the neighbouring tile did: its nineteen fields per point
// fill the L2 within those two planes, so each halo row came from HBM again
// (the x-halo columns as whole 128-byte lines: 1.66x the algorithmic reads
// of that kernel at 512^3). Double-precision 32 x 8 tiles drop the ring:
// without its LDS two workgroups fit on a CU.
#ifndef NSF_SS_HOIST
#define NSF_SS_HOIST 1
#endif
#ifndef NSF_F64_Y8_HALO_RING
#define NSF_F64_Y8_HALO_RING 0
#endif
template <typename T, int TY, bool FUSED, bool MON = false, bool SS = false>
constexpr bool halo_ring() {
    return (FUSED || SS) && (sizeof(T) == 4 || TY != 8 || NSF_F64_Y8_HALO_RING);
}

// Plane fields kept in LDS with their halo: rho, E, p, T (momentum at a
// neighbour is rebuilt as rho * u from the velocity ring). Two buffers
// alternate by plane parity, so the writes of plane z+1 never meet the reads
// of plane z and one barrier per plane suffices: the velocity-ring slot a
// plane recycles is read at that point only for the own column, by the
// thread that writes it (see ring_slots).
constexpr int kPF = 4;
// The stored-gradient form runs at the register limit; rebuilding momentum
// would spill there, so it keeps seven plane fields in one buffer (momentum
// stored) and a second barrier per plane.
template <bool SS>
struct PlaneLds {
    static constexpr int kFields = SS ? 7 : kPF;
    static constexpr int kBuffers = SS ? 1 : 2;
};
// plane fields a halo-ring slot parks per halo point: the plane buffer's
template <bool SS>
constexpr int halo_fields() { return PlaneLds<SS>::kFields; }

// One tile (x-y tile tix, tiy; z-chunk tiz, packed as t) of one grid. sP
// holds kBuffers * kFields * NPL values (the plane fields), sV
// ring_slots * 3 * NPL (the velocity ring). With the halo ring sH holds
// 2 * halo_fields * NHALO values: the plane fields of the raw values each
// thread loaded at its halo point, parked until the point's plane is the
// centre plane (a per-thread ring in LDS, so every halo point is fetched
// once per plane, in the same iteration in which the neighbouring tile
// fetches it as interior; two slots, since each thread reads plane z's
// entry before parking plane z+2's in the same slot). With the D ring, sD holds
// 3 * DSZ values. Ends with a barrier, so the caller may reuse the LDS for
// another tile right away.
template <typename T, int TX, int TY, bool FUSED, bool SS = false, bool MON = false,
          bool RC = false, int GM = kGradAll>
__device__ __forceinline__ void zsweep_tile(const ZArgs<T>& A, int t, T* __restrict__ sP,
                                            T* __restrict__ sV, T* __restrict__ sH,
                                            T* __restrict__ sD,
                                            double2* __restrict__ sM = nullptr) {
    // FUSED: the stage update is applied in the epilogue (q_out, q_acc
    // instead of r). RP: the primitives are recomputed from q in the tile;
    // the stored-gradient forms read them from their stored arrays, fused or
    // not.
    constexpr bool RP = FUSED && !SS;
    static_assert(!(FUSED && SS && (MON || RC)), "the fused stored-gradient stage is SS, unmonitored");
    static_assert(!MON || !SS, "the stored-gradient forms sum the monitor in their gradient pass");
    constexpr bool HR = halo_ring<T, TY, FUSED, MON, SS>();
    constexpr int HF = halo_fields<SS>();
    // Lean form of the fused stage: no branch between the prefetch and the
    // next iteration. Halo prefetches run on every lane and the epilogue uses
    // buffer accesses that drop the lanes outside the grid. With a branch
    // there, the compiler's count of outstanding memory operations takes the
    // path without stores, and the wait for the prefetched plane then also
    // waits for this plane's stores. (The monitored stage keeps the branch
    // where its sums would not fit the registers without it: in single
    // precision and in the 8-row double-precision tile.)
    constexpr bool kLean = RP && !(MON && (sizeof(T) == 4 || TY == 8));
    // Momenta in the z fold: every recomputed-derivative form takes rho * u
    // from the queue and the velocity ring, as the x and y folds do, instead
    // of holding the conserved momenta of five planes in registers (this is
    // where the lean form finds its registers; all forms share the choice so
    // that they round alike). The stored-gradient form keeps the momenta in
    // its plane fields.
    constexpr bool kMomFromVel = !SS;
    // second-difference centre terms summed once (see fold_dir)
    constexpr bool kCentre = !SS && sizeof(T) == 8;
    using G = Geom<TX, TY>;
    constexpr int LX = G::LX, NPL = G::NPL, NT = G::NT, HPT = G::HPT, NHALO = G::NHALO;
    constexpr int RING = ring_slots<T, TY, FUSED, SS, RC>();
    constexpr bool DR = d_ring<T, TY, SS, RC>();
    static_assert(!DR || G::DHALO <= G::NT, "the D-ring halo items need one thread each");
    static_assert(RING == 5 || (RING == 4 && FUSED), "four ring slots rely on the fused loop order");
    // velocity gradients of the centre plane that earlier work already holds
    // unweighted: D_x w and D_y w in the z-cross queues (formed when the plane
    // led), D_x u and D_y v in the D ring; the x and y folds skip them
    constexpr int kGskipX = SS ? 0 : (DR ? 0b101 : 0b100);
    constexpr int kGskipY = SS ? 0 : (DR ? 0b110 : 0b100);
    // stored-gradient forms: array of the stored G_ab (the number of stored
    // gradients before it in the store set GM)
    auto gslot = [](int a, int b) { return __builtin_popcount(GM & ((1 << (3 * a + b)) - 1)); };
    auto gstored = [](int a, int b) { return (GM >> (3 * a + b)) & 1; };
    constexpr int kG00 = 0, kG11 = __builtin_popcount(GM & 0xF);

    const Dims d = A.d;
    const Coef<T> k = A.k;
    const size_t n = d.npts;
    const size_t plane = (size_t)d.nx * d.ny;

    const int tix = t % A.tiles_x;
    const int tiy = (t / A.tiles_x) % A.tiles_y;
    const int tiz = t / (A.tiles_x * A.tiles_y);
    const int x0 = tix * TX, y0 = tiy * TY, z0 = tiz * A.zchunk;
    const int z1 = min(z0 + A.zchunk, d.nz);

    const int tid = threadIdx.x;
    const int lx = tid % TX, ly = tid / TX;
    const int gi = x0 + lx, gj = y0 + ly;
    const bool active = gi < d.nx && gj < d.ny;
    const size_t col = (size_t)pmod(gj, d.ny) * d.nx + pmod(gi, d.nx);
    // LDS planes of the recomputed-derivative forms are stored row by row
    // with the fields of a row side by side ([row][field][column]): all
    // fields of a row then lie within the reach of one ds_read2 base (2040
    // bytes), where field-major planes need a base per field (-1.8% on the
    // FP64 and -4.6% on the FP32 fused stage). The stored-gradient form keeps
    // field-major planes ([field][row][column]): interleaved, its compiled
    // schedule ran 20% slower. RS*: row strides; FO*: field offsets.
    constexpr int PF = PlaneLds<SS>::kFields;
    constexpr int RSV = SS ? LX : 3 * LX, RSP = SS ? LX : PF * LX;
    constexpr int FOV = SS ? NPL : LX, FOP = SS ? NPL : LX;
    const int ownV = (ly + 2) * RSV + (lx + 2);
    const int ownP = (ly + 2) * RSP + (lx + 2);

    int hidxV[HPT], hidxP[HPT];
    size_t hcol[HPT];
    bool hval[HPT];
#pragma unroll
    for (int h = 0; h < HPT; ++h) {
        const int hh = tid + h * NT;
        hval[h] = hh < NHALO;
        int hx = 0, hy = 0;
        if (hval[h]) halo_pos<TX, TY>(hh, hx, hy);
        hidxV[h] = hy * RSV + hx;
        hidxP[h] = hy * RSP + hx;
        hcol[h] = (size_t)pmod(y0 + hy - 2, d.ny) * d.nx + pmod(x0 + hx - 2, d.nx);
    }
    // D ring: the last DHALO threads also form D_y v on the x-halo columns
    // (4 x TY points) and D_x u on the y-halo rows (TX x 4 points)
    int dq = -1, dsrc = 0, ddst = 0;
    if constexpr (DR) {
        const int i = tid - (NT - G::DHALO);
        if (i >= 0 && i < 4 * TY) {
            const int c = i / TY, r = i % TY;
            const int hx = c < 2 ? c : TX + c;
            dq = 0;
            dsrc = (r + 2) * RSV + hx;
            ddst = r * LX + hx;
        } else if (i >= 4 * TY) {
            const int j = i - 4 * TY;
            const int rr = j / TX, c = j % TX;
            const int hy = rr < 2 ? rr : TY + rr;
            dq = 1;
            dsrc = hy * RSV + c + 2;
            ddst = G::DYN + hy * TX + c;
        }
    }
    auto dslot = [&](int z) { return sD + pmod(z, 3) * G::DSZ; };
    auto poff = [&](int z) { return (size_t)pmod(z, d.nz) * plane; };
    // plane-view byte offsets of the own column and the halo points
    const uint32_t pq = (uint32_t)(plane * sizeof(T));
    const uint32_t colq = (uint32_t)(col * sizeof(T));
    uint32_t hcolq[HPT];
#pragma unroll
    for (int h = 0; h < HPT; ++h) hcolq[h] = (uint32_t)(hcol[h] * sizeof(T));
    auto ring = [&](int z) { return sV + pmod(z, RING) * 3 * NPL; };
    // in-plane offsets of the own column's x and y neighbours at -2, -1, +1, +2
    size_t xnb[4], ynb[4];
    if constexpr (SS) {
        const int ms[4] = {-2, -1, 1, 2};
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            xnb[m] = (size_t)pmod(gj, d.ny) * d.nx + pmod(gi + ms[m], d.nx);
            ynb[m] = (size_t)pmod(gj + ms[m], d.ny) * d.nx + pmod(gi, d.nx);
        }
    }

    // register queue of the own column, planes z-2 .. z+2 (velocity in the ring)
    Pt<T> Qz[5];
    T uvw[5][3];
#pragma unroll
    for (int s = 0; s < 5; ++s) {
        Raw<T, RP> raw;
        load_raw<T, RP>(raw, A.q, A.prim, n, poff(z0 - 2 + s) + col);
        Qz[s] = finish<T, RP>(raw, k, uvw[s]);
    }
    T unew[3] = {uvw[4][0], uvw[4][1], uvw[4][2]};  // own velocity of plane z+2

    // queued in-plane derivatives for the z cross terms: Dx u + Dy v, Dx w, Dy w
    // (stored-gradient form: Xs and Xw queue the stored G_xx and G_yy of the
    // own column instead, for D_z of the diagonal gradients)
    T Xs[5], Xw[5], Yw[5];
    if constexpr (SS && !RC) {
#pragma unroll
        for (int s = 0; s < 5; ++s) {
            Xs[s] = A.grad[kG00 * n + poff(z0 - 2 + s) + col];
            Xw[s] = A.grad[kG11 * n + poff(z0 - 2 + s) + col];
        }
    }
    auto leading = [&](const T* V, T& s, T& xw, T& yw, int zz, bool keepD) {
        const T* U = V;
        const T* Vv = V + FOV;
        const T* W = V + 2 * FOV;
        const T dxu = D1u(U[ownV - 2], U[ownV - 1], U[ownV + 1], U[ownV + 2]);
        const T dyv = D1u(Vv[ownV - 2 * RSV], Vv[ownV - RSV], Vv[ownV + RSV], Vv[ownV + 2 * RSV]);
        if constexpr (DR) {
            // unweighted D_y v and D_x u of this plane, for its cross terms two
            // iterations on (written after the barrier, read after the barrier
            // two planes later; the slot it replaces was read last plane)
            if (keepD) {
                T* D = dslot(zz);
                D[ly * LX + lx + 2] = dyv;
                D[G::DYN + (ly + 2) * TX + lx] = dxu;
                if (dq == 0) {
                    const T* f = Vv + dsrc;
                    D[ddst] = D1u(f[-2 * RSV], f[-RSV], f[RSV], f[2 * RSV]);
                } else if (dq == 1) {
                    const T* f = U + dsrc;
                    D[ddst] = D1u(f[-2], f[-1], f[1], f[2]);
                }
            }
        }
        // (queued per plane: on a single-plane grid the z difference of the
        // queue is then exactly zero)
        s = fmadd(k.a1[0], dxu, k.a1[1] * dyv);
        // unweighted: the cross terms apply the weights of both directions
        xw = D1u(W[ownV - 2], W[ownV - 1], W[ownV + 1], W[ownV + 2]);
        yw = D1u(W[ownV - 2 * RSV], W[ownV - RSV], W[ownV + RSV], W[ownV + 2 * RSV]);
    };

    // per-thread halo ring: slot of plane zz, plane field f (the values the
    // plane buffer takes at that halo point: rho, E, p, T, and in the
    // stored-gradient form the momenta after them)
    auto hring = [&](int zz, int f, int h) -> T& {
        return sH[(pmod(zz, 2) * HF + f) * NHALO + tid + h * NT];
    };
    auto park = [&](int zz, int h, const T f7[7]) {
        hring(zz, 0, h) = f7[0];
        hring(zz, 1, h) = f7[4];
        hring(zz, 2, h) = f7[5];
        hring(zz, 3, h) = f7[6];
        if constexpr (HF == 7) {
            hring(zz, 4, h) = f7[1];
            hring(zz, 5, h) = f7[2];
            hring(zz, 6, h) = f7[3];
        }
    };
    auto unpark = [&](int zz, int h, T f7[7]) {
        f7[0] = hring(zz, 0, h);
        f7[4] = hring(zz, 1, h);
        f7[5] = hring(zz, 2, h);
        f7[6] = hring(zz, 3, h);
        if constexpr (HF == 7) {
            f7[1] = hring(zz, 4, h);
            f7[2] = hring(zz, 5, h);
            f7[3] = hring(zz, 6, h);
        }
    };

    // preamble: ring planes z0-2 .. z0+1 and their queued in-plane derivatives
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int zz = z0 - 2 + s;
        T* V = ring(zz);
        V[ownV] = uvw[s][0];
        V[FOV + ownV] = uvw[s][1];
        V[2 * FOV + ownV] = uvw[s][2];
#pragma unroll
        for (int h = 0; h < HPT; ++h)
            if (hval[h]) {
                T u, v, w;
                if constexpr (RP) {
                    RawP<T, RP> rp;
                    load_rawp<T, RP>(rp, A.q, A.prim, n, poff(zz) + hcol[h]);
                    const T ir = fast_rcp(rp.a[0]);
                    u = rp.a[1] * ir;
                    v = rp.a[2] * ir;
                    w = rp.a[3] * ir;
                    if constexpr (HR)
                        if (s >= 2) {
                            T f7[7];
                            finish_p<T, RP>(rp, k, f7);
                            park(zz, h, f7);
                        }
                } else {
                    RawV<T, RP> rv;
                    load_rawv<T, RP>(rv, A.q, A.prim, n, poff(zz) + hcol[h]);
                    finish_v<T, RP>(rv, u, v, w);
                    if constexpr (HR)
                        if (s >= 2) {
                            RawP<T, RP> rp;
                            load_rawp<T, RP>(rp, A.q, A.prim, n, poff(zz) + hcol[h]);
                            T f7[7];
                            finish_p<T, RP>(rp, k, f7);
                            park(zz, h, f7);
                        }
                }
                V[hidxV[h]] = u;
                V[FOV + hidxV[h]] = v;
                V[2 * FOV + hidxV[h]] = w;
            }
        __syncthreads();
        if constexpr (!SS && !RC) leading(V, Xs[s], Xw[s], Yw[s], zz, s >= 2);
    }

    // prefetched halo values for the first iteration: fused form, raw q of
    // plane z0+2; stored-primitive form, velocity of plane z0+2 and the
    // seven plane fields of plane z0 (of plane z0+2 with the halo ring)
    RawP<T, RP> hq[HPT];
    RawV<T, RP> hv[RP ? 1 : HPT];
    RawP<T, RP> hz[RP && !HR ? HPT : 1];  // fused, no ring: raw q of plane z
#pragma unroll
    for (int h = 0; h < HPT; ++h)
        if (hval[h]) {
            if constexpr (RP) {
                load_rawp<T, RP>(hq[h], A.q, A.prim, n, poff(z0 + 2) + hcol[h]);
                if constexpr (!HR) load_rawp<T, RP>(hz[h], A.q, A.prim, n, poff(z0) + hcol[h]);
            } else {
                load_rawv<T, RP>(hv[h], A.q, A.prim, n, poff(z0 + 2) + hcol[h]);
                load_rawp<T, RP>(hq[h], A.q, A.prim, n, poff(HR ? z0 + 2 : z0) + hcol[h]);
            }
        }

    // fused form, monitored stage: per-thread sums of rho|u|^2/2 and
    // rho|omega|^2/2 over the tile's planes (in plane order). Single
    // precision keeps them in a thread-private LDS slot: its register budget
    // (three waves per SIMD) has no room for two more doubles.
    constexpr bool kLdsMon = MON && sizeof(T) == 4;
    double mke = 0.0, mens = 0.0;
    // Lean double-precision 16-row form: the accumulator of plane z+1 is fetched
    // right after plane z's stores, a whole plane of work ahead of its use
    // (-2.8% on the 512^3 stage against fetching it in the epilogue, A/B on
    // one box). Single precision fetches it early in the same iteration
    // instead (kEarlyAcc; one plane ahead was neutral there); the 8-row
    // double-precision tile has no registers for it. This form alone also
    // takes the accumulator-saving substeps (ZArgs::qacc_in, acc_store).
    constexpr bool kAccAhead = kLean && sizeof(T) == 8 && TY == 16;
    double accN[kAccAhead ? 5 : 1];
    if constexpr (kAccAhead) {
        const uint32_t pb0 = (uint32_t)(plane * sizeof(double));
        const uint32_t off0 = (active && z0 < z1) ? (uint32_t)col * 8u : kOutside;
#pragma unroll
        for (int f = 0; f < 5; ++f)
            accN[f] = view_load(plane_view(A.qacc_in + f * n + (size_t)z0 * plane, pb0), off0);
    }
    if constexpr (kLdsMon) sM[tid] = make_double2(0.0, 0.0);

    for (int z = z0; z < z1; ++z) {
        // Halo waves first: the waves that load halo points have more to do
        // before the barrier, and the others wait for them there, so they run
        // at raised priority until it (double precision: -2.6% on the fused
        // 512^3 stage; single precision, which is bound by memory, gains
        // nothing)
        // Stored-gradient form: the in-plane neighbours of the diagonal
        // gradients (D_x of G_yy and G_zz, D_y of G_xx and G_zz) are fetched
        // first thing in the iteration, so their latency overlaps the LDS
        // writes and the barrier, and only their two sums stay live through
        // the folds. (The full store set only: with the diagonal or in-plane
        // sets the hoisted values push those kernels into spills.)
        constexpr bool kHoistG = SS && !RC && GM == kGradAll && NSF_SS_HOIST;
        T gnb[kHoistG ? 4 : 1][4];
        if constexpr (kHoistG) {
            const size_t pz = poff(z);
            const int cx1 = GM == kGradAll ? 4 : gslot(1, 1);
            const int cy0 = GM == kGradAll ? 0 : gslot(0, 0);
            const int c22 = GM == kGradAll ? 8 : gslot(2, 2);
            constexpr bool kZZ = GM == kGradAll || ((GM >> 8) & 1);
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                gnb[0][m] = A.grad[cx1 * n + pz + xnb[m]];
                gnb[1][m] = kZZ ? A.grad[c22 * n + pz + xnb[m]] : T(0);
                gnb[2][m] = A.grad[cy0 * n + pz + ynb[m]];
                gnb[3][m] = kZZ ? A.grad[c22 * n + pz + ynb[m]] : T(0);
            }
        }
        constexpr bool kHaloPrio = RP && sizeof(T) == 8;
        if constexpr (kHaloPrio) {
            if (tid < NHALO) __builtin_amdgcn_s_setprio(2);
        }
        // (a) LDS: ring slot of plane z+2 (velocity) and the plane-z fields.
        // The slot of plane z+2 last held plane z+2-RING, whose in-plane
        // readers are done (see ring_slots); with four slots that is plane
        // z-2, and its own column, still needed by the z fold, is kept first
        T* Vl = ring(z + 2);
        T vm2[3];
        if constexpr (RING == 4) {
            vm2[0] = Vl[ownV];
            vm2[1] = Vl[FOV + ownV];
            vm2[2] = Vl[2 * FOV + ownV];
        }
        Vl[ownV] = unew[0];
        Vl[FOV + ownV] = unew[1];
        Vl[2 * FOV + ownV] = unew[2];
        T* Pz = sP + (PlaneLds<SS>::kBuffers == 2 ? (z & 1) * PF * NPL : 0);  // plane z
        // field slots: rho, E, p, T, then (stored-gradient form) m0, m1, m2
        Pz[ownP] = Qz[2].rho;
        Pz[FOP + ownP] = Qz[2].E;
        Pz[2 * FOP + ownP] = Qz[2].p;
        Pz[3 * FOP + ownP] = Qz[2].t;
        if constexpr (PF == 7) {
            Pz[4 * FOP + ownP] = Qz[2].m0;
            Pz[5 * FOP + ownP] = Qz[2].m1;
            Pz[6 * FOP + ownP] = Qz[2].m2;
        }
#pragma unroll
        for (int h = 0; h < HPT; ++h)
            if (hval[h]) {
                T u, v, w;
                T f7[7];
                if constexpr (RP) {
                    // velocity of the leading plane from the raw values of z+2
                    const T ir = fast_rcp(hq[h].a[0]);
                    u = hq[h].a[1] * ir;
                    v = hq[h].a[2] * ir;
                    w = hq[h].a[3] * ir;
                    if constexpr (HR) {
                        // plane-z fields parked two planes ago; park those of z+2
                        unpark(z, h, f7);
                        T g7[7];
                        finish_p<T, RP>(hq[h], k, g7);
                        park(z + 2, h, g7);
                    } else {
                        // plane-z fields from the raw values fetched in the
                        // previous iteration
                        finish_p<T, RP>(hz[h], k, f7);
                    }
                } else {
                    finish_v<T, RP>(hv[h], u, v, w);
                    if constexpr (HR) {
                        unpark(z, h, f7);
                        T g7[7];
                        finish_p<T, RP>(hq[h], k, g7);
                        park(z + 2, h, g7);
                    } else {
                        finish_p<T, RP>(hq[h], k, f7);
                    }
                }
                Vl[hidxV[h]] = u;
                Vl[FOV + hidxV[h]] = v;
                Vl[2 * FOV + hidxV[h]] = w;
                Pz[hidxP[h]] = f7[0];
                Pz[FOP + hidxP[h]] = f7[4];
                Pz[2 * FOP + hidxP[h]] = f7[5];
                Pz[3 * FOP + hidxP[h]] = f7[6];
                if constexpr (PF == 7) {
                    Pz[4 * FOP + hidxP[h]] = f7[1];
                    Pz[5 * FOP + hidxP[h]] = f7[2];
                    Pz[6 * FOP + hidxP[h]] = f7[3];
                }
            }
        // (b) prefetch the next iteration's loads. The lean form loads
        // through plane views (one 32-bit offset per lane instead of a 64-bit
        // address per field) and on every lane: a halo slot past the end has
        // the wrapped address of the tile's corner and is left unused, since a
        // branch here would make the wait for these loads also wait for this
        // plane's stores.
        // The unfused double-precision recompute forms fetch after the
        // compute instead: the prefetched stored primitives do not fit beside
        // their residual (52-84 B of spills per lane against 19-36).
        constexpr bool kLatePrefetch = RC && !RP && sizeof(T) == 8;
        Raw<T, RP> nxt;
        auto fetch_next = [&]() {
            load_raw<T, RP>(nxt, A.q, A.prim, n, poff(z + 3) + col);
#pragma unroll
            for (int h = 0; h < HPT; ++h)
                if (hval[h]) {
                    if constexpr (RP) {
                        load_rawp<T, RP>(hq[h], A.q, A.prim, n, poff(z + 3) + hcol[h]);
                        if constexpr (!HR)
                            load_rawp<T, RP>(hz[h], A.q, A.prim, n, poff(z + 1) + hcol[h]);
                    } else {
                        load_rawv<T, RP>(hv[h], A.q, A.prim, n, poff(z + 3) + hcol[h]);
                        load_rawp<T, RP>(hq[h], A.q, A.prim, n, poff(HR ? z + 3 : z + 1) + hcol[h]);
                    }
                }
        };
        if constexpr (kLean) {
            const size_t z3 = poff(z + 3);
#pragma unroll
            for (int f = 0; f < 5; ++f) nxt.q[f] = plane_load<T>(plane_view(A.q + f * n + z3, pq), colq);
#pragma unroll
            for (int h = 0; h < HPT; ++h)
#pragma unroll
                for (int f = 0; f < 5; ++f)
                    hq[h].a[f] = plane_load<T>(plane_view(A.q + f * n + z3, pq), hcolq[h]);
            if constexpr (!HR) {
                const size_t z1p = poff(z + 1);
#pragma unroll
                for (int h = 0; h < HPT; ++h)
#pragma unroll
                    for (int f = 0; f < 5; ++f)
                        hz[h].a[f] = plane_load<T>(plane_view(A.q + f * n + z1p, pq), hcolq[h]);
            }
        } else if constexpr (!kLatePrefetch) {
            fetch_next();
        }
        T gnx[SS ? 2 : 1];
        if constexpr (SS && !RC) {
            gnx[0] = A.grad[kG00 * n + poff(z + 3) + col];
            gnx[1] = A.grad[kG11 * n + poff(z + 3) + col];
        }
        // fused form: the accumulator of plane z. The lean single-precision
        // form fetches it here, before the compute, so its latency is
        // covered (the lean double-precision form has it from the previous
        // iteration); the other fused forms fetch it in the epilogue.
        constexpr bool kEarlyAcc = kLean && sizeof(T) == 4;
        const size_t oidx = (size_t)z * plane + col;
        const size_t zo = (size_t)z * plane;
        const uint32_t pb = (uint32_t)(plane * sizeof(double));
        const uint32_t off = active ? (uint32_t)col * 8u : kOutside;
        double acc[FUSED ? 5 : 1];
        if constexpr (kEarlyAcc) {
#pragma unroll
            for (int f = 0; f < 5; ++f) acc[f] = view_load(plane_view(A.qacc + f * n + zo, pb), off);
        }
        __syncthreads();
        if constexpr (kHaloPrio) __builtin_amdgcn_s_setprio(0);

        // (c) leading-plane in-plane derivatives for the z cross terms
        if constexpr (!SS && !RC) leading(Vl, Xs[4], Xw[4], Yw[4], z + 2, true);

        T crossxy[2] = {T(0), T(0)};
        if constexpr (kHoistG) {
            crossxy[0] = D1(gnb[0][0], gnb[0][1], gnb[0][2], gnb[0][3], k.a1[0], k.a2[0]) +
                         D1(gnb[1][0], gnb[1][1], gnb[1][2], gnb[1][3], k.a1[0], k.a2[0]);
            crossxy[1] = D1(gnb[2][0], gnb[2][1], gnb[2][2], gnb[2][3], k.a1[1], k.a2[1]) +
                         D1(gnb[3][0], gnb[3][1], gnb[3][2], gnb[3][3], k.a1[1], k.a2[1]);
        }
        // (d) residual at plane z
        const T* Vc = ring(z);
        const T uc[3] = {Vc[ownV], Vc[FOV + ownV], Vc[2 * FOV + ownV]};
        T R[5];
        T om2 = T(0);
        if constexpr (RC) {
            recompute_point<T, SS, MON, GM>(RcView<T>{Pz, {ring(z - 2), ring(z - 1), Vc, ring(z + 1), ring(z + 2)},
                                                  ownP, ownV, FOP, RSP, FOV, RSV},
                                        Qz, uc, k, A.grad, n, poff, z, col, xnb, ynb, R, om2);
        } else {
        Acc<T> ac;
        ac.S0 = ac.SE = ac.HEAT = T(0);
#pragma unroll
        for (int a = 0; a < 3; ++a) ac.Sm[a] = ac.LAP[a] = T(0);
        {  // x
            T rho[5], m[3][5], E[5], p[5], tt[5], vel[3][5];
#pragma unroll
            for (int s = 0; s < 5; ++s) {
                const int o = ownP + s - 2, ov = ownV + s - 2;
                rho[s] = Pz[o];
                E[s] = Pz[FOP + o];
                p[s] = Pz[2 * FOP + o];
                tt[s] = Pz[3 * FOP + o];
                vel[0][s] = Vc[ov];
                vel[1][s] = Vc[FOV + ov];
                vel[2][s] = Vc[2 * FOV + ov];
                if constexpr (PF == 7) {
#pragma unroll
                    for (int a = 0; a < 3; ++a) m[a][s] = Pz[(4 + a) * FOP + o];
                } else {
#pragma unroll
                    for (int a = 0; a < 3; ++a) m[a][s] = rho[s] * vel[a][s];
                }
            }
            fold_dir<T, 0, !SS, kCentre, kGskipX>(ac, rho, m, E, p, tt, vel, k.a1[0], k.a2[0], k.b0[0], k.b1[0], k.b2[0], uc);
        }
        {  // y
            T rho[5], m[3][5], E[5], p[5], tt[5], vel[3][5];
#pragma unroll
            for (int s = 0; s < 5; ++s) {
                const int o = ownP + (s - 2) * RSP, ov = ownV + (s - 2) * RSV;
                rho[s] = Pz[o];
                E[s] = Pz[FOP + o];
                p[s] = Pz[2 * FOP + o];
                tt[s] = Pz[3 * FOP + o];
                vel[0][s] = Vc[ov];
                vel[1][s] = Vc[FOV + ov];
                vel[2][s] = Vc[2 * FOV + ov];
                if constexpr (PF == 7) {
#pragma unroll
                    for (int a = 0; a < 3; ++a) m[a][s] = Pz[(4 + a) * FOP + o];
                } else {
#pragma unroll
                    for (int a = 0; a < 3; ++a) m[a][s] = rho[s] * vel[a][s];
                }
            }
            fold_dir<T, 1, !SS, kCentre, kGskipY>(ac, rho, m, E, p, tt, vel, k.a1[1], k.a2[1], k.b0[1], k.b1[1], k.b2[1], uc);
        }
        {  // z: register queue, velocity from the ring
            T rho[5], m[3][5], E[5], p[5], tt[5], vel[3][5];
#pragma unroll
            for (int s = 0; s < 5; ++s) {
                const T* Vs = ring(z - 2 + s);
                rho[s] = Qz[s].rho;
                E[s] = Qz[s].E;
                p[s] = Qz[s].p;
                tt[s] = Qz[s].t;
                if (RING == 4 && s == 0) {
#pragma unroll
                    for (int a = 0; a < 3; ++a) vel[a][0] = vm2[a];
                } else {
                    vel[0][s] = Vs[ownV];
                    vel[1][s] = Vs[FOV + ownV];
                    vel[2][s] = Vs[2 * FOV + ownV];
                }
                if constexpr (kMomFromVel) {
#pragma unroll
                    for (int a = 0; a < 3; ++a) m[a][s] = rho[s] * vel[a][s];
                } else {
                    m[0][s] = Qz[s].m0;
                    m[1][s] = Qz[s].m1;
                    m[2][s] = Qz[s].m2;
                }
            }
            fold_dir<T, 2, !SS, kCentre>(ac, rho, m, E, p, tt, vel, k.a1[2], k.a2[2], k.b0[2], k.b1[2], k.b2[2], uc);
        }
        // cross derivatives sum_{c != a} D_a(G_cc)
        T cross[3];
        if constexpr (SS) {
            // stored velocity gradients (G_ab at 3a + b): pointwise values
            // for the assembly, and D_a of the stored diagonal G_cc. Only
            // the diagonal is read again (by the neighbours' differences);
            // the off-diagonal values are read once and streamed past L2
            // (-5% HBM reads of this kernel at 512^3: the neighbours'
            // halo values then stay in L2)
            const T* Gs = A.grad;
            const size_t pz = poff(z);
            auto gat = [&](int comp, size_t off) { return Gs[comp * n + off]; };
            // (the full store set keeps the plain loop: written with the
            // store-set test, its compiled schedule spilled, +14% at 512^3)
            if constexpr (GM == kGradAll) {
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b)
                        ac.G[a][b] = a == b ? gat(3 * a + b, pz + col)
                                            : stream_load(Gs + (3 * a + b) * n + pz + col);
            } else {
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b)
                        if (gstored(a, b))
                            ac.G[a][b] = a == b ? gat(gslot(a, b), pz + col)
                                                : stream_load(Gs + gslot(a, b) * n + pz + col);
            }
            auto dxg = [&](int comp) {
                return D1(gat(comp, pz + xnb[0]), gat(comp, pz + xnb[1]), gat(comp, pz + xnb[2]),
                          gat(comp, pz + xnb[3]), k.a1[0], k.a2[0]);
            };
            auto dyg = [&](int comp) {
                return D1(gat(comp, pz + ynb[0]), gat(comp, pz + ynb[1]), gat(comp, pz + ynb[2]),
                          gat(comp, pz + ynb[3]), k.a1[1], k.a2[1]);
            };
            // (a store set without G_zz belongs to a single-plane grid, where
            // every z difference, hence G_zz, is zero)
            if constexpr (kHoistG) {
                cross[0] = crossxy[0];
                cross[1] = crossxy[1];
            } else if constexpr (GM == kGradAll) {
                cross[0] = dxg(4) + dxg(8);
                cross[1] = dyg(0) + dyg(8);
            } else {
                cross[0] = dxg(gslot(1, 1)) + (gstored(2, 2) ? dxg(gslot(2, 2)) : T(0));
                cross[1] = dyg(gslot(0, 0)) + (gstored(2, 2) ? dyg(gslot(2, 2)) : T(0));
            }
            cross[2] = D1(Xs[0], Xs[1], Xs[3], Xs[4], k.a1[2], k.a2[2]) +
                       D1(Xw[0], Xw[1], Xw[3], Xw[4], k.a1[2], k.a2[2]);
        } else {
            const T* U = Vc;
            const T* Vv = Vc + FOV;
            // nested differences unweighted, the two weights applied once:
            // D_x D_y v + D_z D_x w = a1x (a1y Du_x Du_y v + a1z Du_z Du_x w)
            auto dyv = [&](int mx) {
                const int o = ownV + mx;
                return D1u(Vv[o - 2 * RSV], Vv[o - RSV], Vv[o + RSV], Vv[o + 2 * RSV]);
            };
            auto dxu = [&](int my) {
                const int o = ownV + my * RSV;
                return D1u(U[o - 2], U[o - 1], U[o + 1], U[o + 2]);
            };
            T dxdyv, dydxu;
            if constexpr (DR) {
                // from the D ring: D_y v along the row, D_x u along the column
                const T* Dy = dslot(z) + ly * LX + lx;
                const T* Dx = dslot(z) + G::DYN + ly * TX + lx;
                dxdyv = D1u(Dy[0], Dy[1], Dy[3], Dy[4]);
                dydxu = D1u(Dx[0], Dx[TX], Dx[3 * TX], Dx[4 * TX]);
                ac.G[0][0] = k.a1[0] * Dx[2 * TX];
                ac.G[1][1] = k.a1[1] * Dy[2];
            } else {
                dxdyv = D1u(dyv(-2), dyv(-1), dyv(1), dyv(2));
                dydxu = D1u(dxu(-2), dxu(-1), dxu(1), dxu(2));
            }
            const T a1z = k.a1[2], a2z = k.a2[2];
            ac.G[2][0] = k.a1[0] * Xw[2];
            ac.G[2][1] = k.a1[1] * Yw[2];
            cross[0] = k.a1[0] * (k.a1[1] * dxdyv + a1z * D1u(Xw[0], Xw[1], Xw[3], Xw[4]));
            cross[1] = k.a1[1] * (k.a1[0] * dydxu + a1z * D1u(Yw[0], Yw[1], Yw[3], Yw[4]));
            cross[2] = D1(Xs[0], Xs[1], Xs[3], Xs[4], a1z, a2z);
        }
        {
            T mc[3] = {Qz[2].m0, Qz[2].m1, Qz[2].m2};
            if constexpr (kMomFromVel)
#pragma unroll
                for (int a = 0; a < 3; ++a) mc[a] = Qz[2].rho * uc[a];
            finalize<T, !SS, kCentre>(ac, cross, Qz[2].rho, mc, Qz[2].E, Qz[2].t, uc, k, R, om2);
        }
        }  // thread-local form
        if constexpr (kLatePrefetch) fetch_next();
        if constexpr (MON) {
            if (active) {
                // kinetic energy and enstrophy of the input state (Section 3
                // diagnostics), vorticity from the same fourth-order G
                const double rho = (double)Qz[2].rho;
                const double u0 = uc[0], u1 = uc[1], u2 = uc[2];
                const double ke = 0.5 * rho * (u0 * u0 + u1 * u1 + u2 * u2);
                const double en = 0.5 * rho * (double)om2;
                if constexpr (kLdsMon) {
                    double2 m = sM[tid];
                    m.x += ke;
                    m.y += en;
                    sM[tid] = m;
                } else {
                    mke += ke;
                    mens += en;
                }
            }
        }
        if constexpr (kLean) {
            const uint32_t pbT = (uint32_t)(plane * sizeof(T));
            const uint32_t offT = active ? (uint32_t)(col * sizeof(T)) : kOutside;
            if constexpr (kAccAhead) {
                // the second substep's accumulator from the step's initial
                // state (accN) and its own input state at the point: q0 +
                // (B_1 / A_1)(q1 - q0), which is q0 + B_1 dt R_1 (the first
                // substep stores no accumulator); acc_mix = 0 elsewhere, and
                // fma(0, x, a) = a
                const double rho1 = (double)Qz[2].rho;
                const double q1[5] = {rho1, rho1 * uc[0], rho1 * uc[1], rho1 * uc[2],
                                      (double)Qz[2].E};
#pragma unroll
                for (int f = 0; f < 5; ++f) acc[f] = fma(A.acc_mix, q1[f] - accN[f], accN[f]);
            } else if constexpr (!kEarlyAcc) {
#pragma unroll
                for (int f = 0; f < 5; ++f) acc[f] = view_load(plane_view(A.qacc + f * n + zo, pb), off);
            }
            // the last stage's output is q_acc itself: the same fma with B dt
            const double out_dt = A.last ? A.b_dt : A.a_dt;
            // (a third substep that leaves q_acc alone drops its stores by
            // the out-of-range offset, without a branch)
            const uint32_t offA = A.acc_store ? off : kOutside;
#pragma unroll
            for (int f = 0; f < 5; ++f) {
                const double rr = (double)R[f];
                view_store(fma(A.b_dt, rr, acc[f]), plane_view(A.qacc + f * n + zo, pb), offA);
                view_store((T)fma(out_dt, rr, acc[f]), plane_view(A.qout + f * n + zo, pbT), offT);
            }
            if constexpr (kAccAhead) {
                const uint32_t offN = (active && z + 1 < z1) ? (uint32_t)col * 8u : kOutside;
                const size_t zn = (size_t)(z + 1) * plane;
#pragma unroll
                for (int f = 0; f < 5; ++f) accN[f] = view_load(plane_view(A.qacc_in + f * n + zn, pb), offN);
            }
        } else if (active) {
            if constexpr (FUSED) {
                if constexpr (!kEarlyAcc) {
#pragma unroll
                    for (int f = 0; f < 5; ++f) acc[f] = stream_load(A.qacc + f * n + oidx);
                }
                const double out_dt = A.last ? A.b_dt : A.a_dt;
#pragma unroll
                for (int f = 0; f < 5; ++f) {
                    const double rr = (double)R[f];
                    stream_store(fma(A.b_dt, rr, acc[f]), A.qacc + f * n + oidx);
                    stream_store((T)fma(out_dt, rr, acc[f]), A.qout + f * n + oidx);
                }
            } else {
                // the residual is read once, by the update kernel: streamed
#pragma unroll
                for (int f = 0; f < 5; ++f) stream_store(R[f], A.r + f * n + oidx);
            }
        }
        // Second barrier: single-buffered plane fields (stored-gradient
        // forms), and the recompute forms, whose nested z stencils read the
        // neighbours' columns of ring plane z-2, the slot the next iteration
        // overwrites with plane z+3 before its barrier.
        if constexpr (PlaneLds<SS>::kBuffers == 1 || RC) __syncthreads();
        // (e) rotate the queues (double-buffered plane fields: no barrier, see kPF)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            Qz[s] = Qz[s + 1];
            Xs[s] = Xs[s + 1];
            Xw[s] = Xw[s + 1];
            Yw[s] = Yw[s + 1];
        }
        Qz[4] = finish<T, RP>(nxt, k, unew);
        if constexpr (SS && !RC) {
            Xs[4] = gnx[0];
            Xw[4] = gnx[1];
        }
    }
    __syncthreads();  // every read of the tile's LDS is done
    if constexpr (MON) {
        if constexpr (kLdsMon) {
            mke = sM[tid].x;
            mens = sM[tid].y;
        }
        {
            // fixed-order tile reduction: wave shuffles, then waves in order
            // (the velocity ring, 16-byte aligned, is free after the last
            // barrier of the loop)
            double* red = reinterpret_cast<double*>(sV);
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                mke += __shfl_down(mke, off, 64);
                mens += __shfl_down(mens, off, 64);
            }
            if ((tid & 63) == 0) {
                red[2 * (tid >> 6)] = mke;
                red[2 * (tid >> 6) + 1] = mens;
            }
            __syncthreads();
            if (tid == 0) {
                double a = 0.0, b = 0.0;
                for (int w = 0; w < NT / 64; ++w) {
                    a += red[2 * w];
                    b += red[2 * w + 1];
                }
                A.mpart[2 * t] = a;
                A.mpart[2 * t + 1] = b;
            }
            __syncthreads();
        }
    }
}

#ifndef NSF_ZSWEEP_RC_UNIT
// One block folds the per-tile monitor sums in tile order.
__global__ void __launch_bounds__(256) k_monitor_final(const double* __restrict__ mpart, int ntiles,
                                                      double inv_n, double* __restrict__ out2) {
    __shared__ double red[8];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < ntiles; i += 256) {
        a += mpart[2 * i];
        b += mpart[2 * i + 1];
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        a += __shfl_down(a, off, 64);
        b += __shfl_down(b, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[2 * (threadIdx.x >> 6)] = a;
        red[2 * (threadIdx.x >> 6) + 1] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double x = 0.0, y = 0.0;
        for (int w = 0; w < 4; ++w) {
            x += red[2 * w];
            y += red[2 * w + 1];
        }
        out2[0] = x * inv_n;
        out2[1] = y * inv_n;
    }
}
#endif

// Waves per SIMD the register budget is tuned for: double-precision tiles
// need up to 256 VGPRs (two waves), single precision fits three.
template <typename T, bool RC = false>
struct Occ {
    static constexpr int kWaves = (sizeof(T) == 8 || RC) ? 2 : 3;
};

template <typename T, int TX, int TY, bool FUSED, bool SS, bool MON, bool RC, int GM>
__global__ void __attribute__((amdgpu_flat_work_group_size(TX * TY, TX * TY),
                               amdgpu_waves_per_eu(Occ<T, RC>::kWaves, Occ<T, RC>::kWaves)))
k_ra_zsweep(ZArgs<T> A) {
    using G = Geom<TX, TY>;
    __shared__ T sP[PlaneLds<SS>::kBuffers * PlaneLds<SS>::kFields * G::NPL];
    __shared__ __attribute__((aligned(16))) T sV[ring_slots<T, TY, FUSED, SS, RC>() * 3 * G::NPL];
    __shared__ T sH[halo_ring<T, TY, FUSED, MON, SS>() ? 2 * halo_fields<SS>() * G::NHALO : 1];
    __shared__ T sD[d_ring<T, TY, SS, RC>() ? 3 * G::DSZ : 1];
    __shared__ double2 sM[MON && sizeof(T) == 4 ? TX * TY : 1];
    zsweep_tile<T, TX, TY, FUSED, SS, MON, RC, GM>(A, xcd_tile(blockIdx.x, gridDim.x), sP, sV, sH,
                                                   sD, sM);
}

// Persistent batched stage kernel: the workgroups take (instance, tile)
// items from the host-built bands (one band of neighbouring tiles per XCD,
// longest first) through one counter per band, each its own XCD's band
// first. Every tile is computed the same way whichever workgroup runs it.
// Stage s reads state s of the rotation q -> qb -> qc -> q.
template <typename T, int TX, int TY, bool RC>
__global__ void __attribute__((amdgpu_flat_work_group_size(TX * TY, TX * TY),
                               amdgpu_waves_per_eu(Occ<T, RC>::kWaves, Occ<T, RC>::kWaves)))
k_ra_batch(const BatchDesc<T>* __restrict__ desc, const int2* __restrict__ items,
           const int* __restrict__ boff, int* __restrict__ ctr, int stage, int store_acc) {
    using G = Geom<TX, TY>;
    __shared__ T sP[2 * kPF * G::NPL];
    __shared__ __attribute__((aligned(16))) T sV[ring_slots<T, TY, true, false, RC>() * 3 * G::NPL];
    __shared__ T sH[halo_ring<T, TY, true>() ? 2 * kPF * G::NHALO : 1];
    __shared__ T sD[d_ring<T, TY, false, RC>() ? 3 * G::DSZ : 1];
    __shared__ int sItem;
    const double A_[2] = {2.0 / 3.0, 5.0 / 12.0};
    const double B_[3] = {1.0 / 4.0, 3.0 / 20.0, 3.0 / 5.0};
    // the next stage's counters are free (that stage last ran a full step
    // ago and starts after this launch ends): zero them for it
    if (blockIdx.x == 0 && threadIdx.x < kXCD) ctr[((stage + 1) % 3) * kXCD + threadIdx.x] = 0;
    int* const c = ctr + stage * kXCD;
    // this workgroup's XCD (dispatch deals workgroups to the XCDs in turn):
    // its band first, then the following bands as they run out. A band is
    // left after the first take past its end and never revisited, so every
    // workgroup ends after at most (items it runs) + 8 takes.
    int band = blockIdx.x % kXCD;
    for (int tries = 0; tries < kXCD;) {
        if (threadIdx.x == 0) sItem = atomicAdd(c + band, 1);
        __syncthreads();
        const int k = sItem;
        __syncthreads();  // every thread has read sItem before the next take
        const int i = boff[band] + k;
        if (i >= boff[band + 1]) {
            band = (band + 1) % kXCD;
            ++tries;
            continue;
        }
        const int2 it = items[i];
        const BatchDesc<T>& bd = desc[it.x];
        ZArgs<T> A;
        A.d = bd.d;
        A.k = bd.k;
        A.q = stage == 0 ? bd.q : (stage == 1 ? bd.qb : bd.qc);
        A.qout = stage == 0 ? bd.qb : (stage == 1 ? bd.qc : bd.q);
        A.prim = nullptr;
        A.grad = nullptr;
        A.r = nullptr;
        A.qacc = bd.qacc;
        // double precision, 16-row tiles: the first substep reads the
        // accumulator from q (equal at a step boundary) and leaves q_acc
        // unwritten, the second forms the first's accumulator from the
        // step's initial state, still in q (see ZArgs::acc_mix), and the
        // third leaves q_acc unwritten unless store_acc (a call's last step)
        constexpr bool kSave = sizeof(T) == 8 && TY == 16;
        A.qacc_in = (kSave && stage < 2) ? reinterpret_cast<const double*>(bd.q) : bd.qacc;
        A.acc_store = kSave ? (stage == 0 ? 0 : stage == 2 ? store_acc : 1) : 1;
        A.acc_mix = (kSave && stage == 1) ? B_[0] / A_[0] : 0.0;
        A.a_dt = stage < 2 ? A_[stage] * bd.dt : 0.0;
        A.b_dt = B_[stage] * bd.dt;
        A.last = stage == 2;
        A.zchunk = bd.zchunk;
        A.mpart = nullptr;
        A.tiles_x = bd.tiles_x;
        A.tiles_y = bd.tiles_y;
        zsweep_tile<T, TX, TY, true, false, false, RC>(A, it.y, sP, sV, sH, sD);
    }
}

template <typename T, int TX, int TY, bool FUSED, bool SS = false, bool MON = false,
          bool RC = false, int GM = kGradAll>
void launch_tiles(const ZArgs<T>& a0, int zchunk, hipStream_t s) {
    ZArgs<T> a = a0;
    const Dims& d = a.d;
    a.zchunk = zchunk < 1 ? d.nz : (zchunk > d.nz ? d.nz : zchunk);
    a.tiles_x = (d.nx + TX - 1) / TX;
    a.tiles_y = (d.ny + TY - 1) / TY;
    const int tiles_z = (d.nz + a.zchunk - 1) / a.zchunk;
    const unsigned nb = (unsigned)(a.tiles_x * a.tiles_y * tiles_z);
    hipLaunchKernelGGL((k_ra_zsweep<T, TX, TY, FUSED, SS, MON, RC, GM>), dim3(nb), dim3(TX * TY), 0,
                       s, a);
}

}  // namespace

// The RA instantiations (recompute, no stored gradients) are compiled in a
// unit of their own (nsf_zsweep_rc.hip includes this file with
// NSF_ZSWEEP_RC_UNIT defined), so that each unit can take the scheduler
// setting that suits its kernels: the other forms, RS included, are
// scheduled with the AMDGPU register-pressure trackers (-1% on the fused SN
// stage, -7% on the fused SS stage, -14% on the RS residual at 512^3, whose
// spills halve), which make the RA tiles spill more (80 B per lane in the
// fused RA stage, +21%).
template <typename T, int TY, bool FUSED, bool SS, bool MON, int GM>
void launch_tiles_rc(const ZArgs<T>& a, int zchunk, hipStream_t s);
template <typename T, int TY>
void launch_batch_rc(dim3 g, const BatchDesc<T>* desc, const int2* items, const int* boff,
                     int* ctr, int stage, int store_acc, hipStream_t s);
template <typename T, int TY>
hipError_t batch_occupancy_rc(int* nb);

#ifdef NSF_ZSWEEP_RC_UNIT

template <typename T, int TY, bool FUSED, bool SS, bool MON, int GM>
void launch_tiles_rc(const ZArgs<T>& a, int zchunk, hipStream_t s) {
    launch_tiles<T, kTX, TY, FUSED, SS, MON, true, GM>(a, zchunk, s);
}

template <typename T, int TY>
void launch_batch_rc(dim3 g, const BatchDesc<T>* desc, const int2* items, const int* boff,
                     int* ctr, int stage, int store_acc, hipStream_t s) {
    hipLaunchKernelGGL((k_ra_batch<T, kTX, TY, true>), g, dim3(kTX * TY), 0, s, desc, items, boff,
                       ctr, stage, store_acc);
}

template <typename T, int TY>
hipError_t batch_occupancy_rc(int* nb) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, k_ra_batch<T, kTX, TY, true>,
                                                        kTX * TY, 0);
}

// RA residual and fused RA stage (monitored or not), batched RA stage
#define NSF_RC_INST(T, TY)                                                                      \
    template void launch_tiles_rc<T, TY, false, false, false, kGradAll>(const ZArgs<T>&, int,    \
                                                                        hipStream_t);           \
    template void launch_tiles_rc<T, TY, false, false, true, kGradAll>(const ZArgs<T>&, int,     \
                                                                       hipStream_t);            \
    template void launch_tiles_rc<T, TY, true, false, true, kGradAll>(const ZArgs<T>&, int,      \
                                                                      hipStream_t);             \
    template void launch_tiles_rc<T, TY, true, false, false, kGradAll>(const ZArgs<T>&, int,     \
                                                                       hipStream_t);            \
    template void launch_batch_rc<T, TY>(dim3, const BatchDesc<T>*, const int2*, const int*,     \
                                         int*, int, int, hipStream_t);                          \
    template hipError_t batch_occupancy_rc<T, TY>(int*);
NSF_RC_INST(float, 8)
NSF_RC_INST(float, 16)
NSF_RC_INST(double, 8)
NSF_RC_INST(double, 16)
#undef NSF_RC_INST

#else  // the unit of every other form and the launchers

int default_zchunk(const Dims& d) { return d.nz >= 256 ? 64 : (d.nz >= 64 ? 32 : d.nz); }

// Double precision: 32 x 16 tiles (one 512-thread workgroup per CU, fewest
// halo points per output point); single precision: 32 x 8 (three
// 256-thread workgroups per CU).
int default_tile_y(int precision_bytes, const Dims& d) {
    return (precision_bytes == 8 && d.ny >= 16) ? 16 : 8;
}

void tile_counts(const Dims& d, int zchunk, int tile_y, int* tx, int* ty, int* tz, int* zc) {
    const int c = zchunk < 1 ? d.nz : (zchunk > d.nz ? d.nz : zchunk);
    *zc = c;
    *tx = (d.nx + kTX - 1) / kTX;
    *ty = (d.ny + tile_y - 1) / tile_y;
    *tz = (d.nz + c - 1) / c;
}

template <typename T>
void launch_ra_zsweep(const Dims& d, const Coef<T>& c, const T* q, const T* prim, T* r,
                      int zchunk, int tile_y, hipStream_t s, bool recompute, double* mpart) {
    TimerScope ts(recompute ? "ra_zsweep" : "sn_zsweep", s);
    ZArgs<T> a{};
    a.d = d;
    a.k = c;
    a.q = q;
    a.prim = prim;
    a.r = r;
    a.mpart = mpart;
    // the monitored build (double precision): each tile also sums the
    // kinetic energy and enstrophy of its input points into mpart
    if constexpr (sizeof(T) == 8) {
        if (mpart) {
            if (recompute) {
                if (tile_y == 16) launch_tiles_rc<T, 16, false, false, true, kGradAll>(a, zchunk, s);
                else launch_tiles_rc<T, 8, false, false, true, kGradAll>(a, zchunk, s);
            } else {
                if (tile_y == 16) launch_tiles<T, kTX, 16, false, false, true>(a, zchunk, s);
                else launch_tiles<T, kTX, 8, false, false, true>(a, zchunk, s);
            }
            return;
        }
    }
    if (recompute) {
        if (tile_y == 16) launch_tiles_rc<T, 16, false, false, false, kGradAll>(a, zchunk, s);
        else launch_tiles_rc<T, 8, false, false, false, kGradAll>(a, zchunk, s);
    } else {
        if (tile_y == 16) launch_tiles<T, kTX, 16, false>(a, zchunk, s);
        else launch_tiles<T, kTX, 8, false>(a, zchunk, s);
    }
}

template <typename T, int GM>
void launch_ss_set(const ZArgs<T>& a, int zchunk, int tile_y, hipStream_t s, bool recompute) {
    if (recompute) {
        if (tile_y == 16) launch_tiles<T, kTX, 16, false, true, false, true, GM>(a, zchunk, s);
        else launch_tiles<T, kTX, 8, false, true, false, true, GM>(a, zchunk, s);
    } else {
        if (tile_y == 16) launch_tiles<T, kTX, 16, false, true, false, false, GM>(a, zchunk, s);
        else launch_tiles<T, kTX, 8, false, true, false, false, GM>(a, zchunk, s);
    }
}

template <typename T>
void launch_ss_zsweep(const Dims& d, const Coef<T>& c, const T* q, const T* prim, const T* grad,
                      T* r, int zchunk, int tile_y, hipStream_t s, bool recompute, int gmask) {
    TimerScope ts(recompute ? "rs_zsweep" : "ss_zsweep", s);
    ZArgs<T> a{};
    a.d = d;
    a.k = c;
    a.q = q;
    a.prim = prim;
    a.grad = grad;
    a.r = r;
    if (gmask == kGradDiag) launch_ss_set<T, kGradDiag>(a, zchunk, tile_y, s, recompute);
    else if (gmask == kGradPlane) launch_ss_set<T, kGradPlane>(a, zchunk, tile_y, s, recompute);
    else launch_ss_set<T, kGradAll>(a, zchunk, tile_y, s, recompute);
}

template <typename T, int GM>
void launch_ss_fused_set(const ZArgs<T>& a, int zchunk, int tile_y, hipStream_t s) {
    if (tile_y == 16) launch_tiles<T, kTX, 16, true, true, false, false, GM>(a, zchunk, s);
    else launch_tiles<T, kTX, 8, true, true, false, false, GM>(a, zchunk, s);
}

template <typename T>
void launch_ss_fused(const Dims& d, const Coef<T>& c, const T* q, const T* prim, const T* grad,
                     T* qout, double* qacc, const StageCoef& sc, int zchunk, int tile_y,
                     hipStream_t s, int gmask) {
    TimerScope ts("ss_fused", s);
    ZArgs<T> a{};
    a.d = d;
    a.k = c;
    a.q = q;
    a.prim = prim;
    a.grad = grad;
    a.qout = qout;
    a.qacc = qacc;
    a.qacc_in = qacc;
    a.acc_store = 1;
    a.a_dt = sc.a_dt;
    a.b_dt = sc.b_dt;
    a.last = sc.last;
    if (gmask == kGradDiag) launch_ss_fused_set<T, kGradDiag>(a, zchunk, tile_y, s);
    else if (gmask == kGradPlane) launch_ss_fused_set<T, kGradPlane>(a, zchunk, tile_y, s);
    else launch_ss_fused_set<T, kGradAll>(a, zchunk, tile_y, s);
}

template <typename T>
void launch_ra_batch(const BatchDesc<T>* desc, const int2* items, const int* boff, int* ctr,
                     int stage, int nblocks, int tile_y, hipStream_t s, bool recompute,
                     int store_acc) {
    TimerScope ts("ra_batch", s);
    const dim3 g(nblocks);
    if (recompute) {
        if (tile_y == 16) launch_batch_rc<T, 16>(g, desc, items, boff, ctr, stage, store_acc, s);
        else launch_batch_rc<T, 8>(g, desc, items, boff, ctr, stage, store_acc, s);
    } else if (tile_y == 16) {
        hipLaunchKernelGGL((k_ra_batch<T, kTX, 16, false>), g, dim3(kTX * 16), 0, s, desc, items,
                           boff, ctr, stage, store_acc);
    } else {
        hipLaunchKernelGGL((k_ra_batch<T, kTX, 8, false>), g, dim3(kTX * 8), 0, s, desc, items,
                           boff, ctr, stage, store_acc);
    }
}

template <typename T>
int batch_blocks_per_cu(int tile_y, bool recompute) {
    int nb = 0;
    hipError_t e;
    if (recompute)
        e = tile_y == 16 ? batch_occupancy_rc<T, 16>(&nb) : batch_occupancy_rc<T, 8>(&nb);
    else
        e = tile_y == 16
            ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_ra_batch<T, kTX, 16, false>, kTX * 16, 0)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_ra_batch<T, kTX, 8, false>, kTX * 8, 0);
    return e == hipSuccess ? nb : 0;
}

void launch_monitor_final(const double* mpart, int ntiles, double inv_n, double* out2,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_monitor_final, dim3(1), dim3(256), 0, s, mpart, ntiles, inv_n, out2);
}

int sweep_tiles(const Dims& d, int zchunk, int tile_y) {
    int tx, ty, tz, zc;
    tile_counts(d, zchunk, tile_y, &tx, &ty, &tz, &zc);
    return tx * ty * tz;
}

template <typename T>
void launch_ra_fused(const Dims& d, const Coef<T>& c, const T* q, T* qout, double* qacc,
                     const StageCoef& sc, int zchunk, int tile_y, hipStream_t s, double* mpart,
                     bool recompute) {
    // The accumulator-saving substeps (first reads the accumulator from q,
    // third leaves q_acc unwritten) in the double-precision 16-row form only;
    // elsewhere every substep reads and writes q_acc (same results: q_acc
    // equals q at a step boundary, and the value stored is the new state).
    const bool saving = sizeof(T) == 8 && tile_y == 16;
    const bool first_q = saving && sc.acc_from_q;
    const bool last_ns = saving && !sc.store_acc && !sc.acc_from_q;
    // timer families by what a launch moves: the monitored first substep,
    // an unmonitored first substep that reads the accumulator from q, a
    // third substep that leaves q_acc unwritten, and the full stage
    const char* fam = mpart ? (recompute ? "ra_fused_mon" : "sn_fused_mon")
                      : first_q ? (recompute ? "ra_fused_first" : "sn_fused_first")
                      : last_ns ? (recompute ? "ra_fused_last" : "sn_fused_last")
                                : (recompute ? "ra_fused" : "sn_fused");
    TimerScope ts(fam, s);
    ZArgs<T> a{};
    a.mpart = mpart;
    a.d = d;
    a.k = c;
    a.q = q;
    a.qout = qout;
    a.qacc = qacc;
    // the first substep may read the accumulator from the state (double
    // precision only: there q_acc equals q at a step boundary)
    a.qacc_in = first_q ? reinterpret_cast<const double*>(q)
                : (saving && sc.acc_src) ? reinterpret_cast<const double*>(sc.acc_src) : qacc;
    a.acc_store = saving && !sc.store_acc ? 0 : 1;
    a.acc_mix = saving ? sc.acc_mix : 0.0;
    a.a_dt = sc.a_dt;
    a.b_dt = sc.b_dt;
    a.last = sc.last;
    if (recompute) {
        if (mpart) {
            if (tile_y == 16) launch_tiles_rc<T, 16, true, false, true, kGradAll>(a, zchunk, s);
            else launch_tiles_rc<T, 8, true, false, true, kGradAll>(a, zchunk, s);
        } else {
            if (tile_y == 16) launch_tiles_rc<T, 16, true, false, false, kGradAll>(a, zchunk, s);
            else launch_tiles_rc<T, 8, true, false, false, kGradAll>(a, zchunk, s);
        }
    } else if (mpart) {
        if (tile_y == 16) launch_tiles<T, kTX, 16, true, false, true>(a, zchunk, s);
        else launch_tiles<T, kTX, 8, true, false, true>(a, zchunk, s);
    } else {
        if (tile_y == 16) launch_tiles<T, kTX, 16, true>(a, zchunk, s);
        else launch_tiles<T, kTX, 8, true>(a, zchunk, s);
    }
}

#define NSF_INST(T)                                                                          \
    template void launch_ra_batch<T>(const BatchDesc<T>*, const int2*, const int*, int*, int,    \
                                     int, int, hipStream_t, bool, int);                       \
    template int batch_blocks_per_cu<T>(int, bool);                                           \
    template void launch_ra_zsweep<T>(const Dims&, const Coef<T>&, const T*, const T*, T*,  \
                                      int, int, hipStream_t, bool, double*);                \
    template void launch_ss_zsweep<T>(const Dims&, const Coef<T>&, const T*, const T*,      \
                                      const T*, T*, int, int, hipStream_t, bool, int);      \
    template void launch_ss_fused<T>(const Dims&, const Coef<T>&, const T*, const T*,       \
                                     const T*, T*, double*, const StageCoef&, int, int,     \
                                     hipStream_t, int);                                     \
    template void launch_ra_fused<T>(const Dims&, const Coef<T>&, const T*, T*, double*,    \
                                     const StageCoef&, int, int, hipStream_t, double*, bool);
NSF_INST(float)
NSF_INST(double)
#undef NSF_INST

#endif  // NSF_ZSWEEP_RC_UNIT

}  // namespace nsf
