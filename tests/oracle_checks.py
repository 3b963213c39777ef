"""Checks of the CPU oracle against results fixed by the mathematics, written
as functions that return error measures, so that the same check can pin the
oracle (tests/test_oracle_energy_pins.py) and be shown to fail on copies of
the oracle with a planted mistake (tests/test_oracle_mutants.py).

Two independent routes to the residual of eqs (1)-(3) (Section 2):

  continuum_errors  the exact residual of the continuous equations in
      divergence form, differentiated symbolically (sympy) for a smooth
      state with variable density, pressure and temperature and a
      non-solenoidal velocity. The fourth-order scheme must converge to it
      at fourth order in every field. The skew-symmetric split of eq (8) and
      the expansion of the viscous terms are identities of the continuous
      operators, so this pins every term's sign, coefficient and axis,
      independently of how the discrete form arranges them.

  wave_closed_form_errors  the exact discrete residual of a one-dimensional
      compressive wave: every field is a trigonometric polynomial, products
      are formed exactly, and the fourth-order operators act on each
      harmonic through their modified wavenumbers
          D e^{ikx} = i k'(k) e^{ikx},  k'(k) = (8 sin kh - sin 2kh)/(6h),
          D2 e^{ikx} = -k''2(k) e^{ikx},  k''2(k) = (15 - 16 cos kh + cos 2kh)/(6h^2).
      The discrete product rule does not hold (D(pu) differs from
      u Dp + p Du by O(h^4)), so this pins the discrete arrangement the
      method prescribes: the skew split of eq (8) with phi = E, and the
      pressure work -D_j(p u_j) in divergence form outside that split.
"""
from __future__ import annotations

import functools

import mpmath as mp
import numpy as np

from oracle import oracle as O


# ------------------------------------------------------------ continuum
@functools.lru_cache(maxsize=None)
def _continuum(phys_items):
    import sympy as sp

    phys = dict(phys_items)
    x, y, z = sp.symbols("x y z", real=True)
    X = (x, y, z)
    g, M, Pr, Re = [sp.nsimplify(phys[k]) for k in ("gamma", "Ma", "Pr", "Re")]
    R = sp.Rational
    rho = 1 + R(1, 5) * sp.sin(x + 1) * sp.cos(y) + R(1, 10) * sp.cos(2 * z + R(1, 2))
    u = [R(3, 10) * sp.sin(x) * sp.cos(y + R(1, 3)) + R(1, 5) * sp.cos(z),
         R(1, 4) * sp.cos(x + R(1, 2)) * sp.sin(2 * y) - R(1, 10) * sp.sin(z + 1),
         R(1, 5) * sp.sin(z) * sp.cos(x - y) + R(1, 10) * sp.cos(y)]
    T = 1 + R(1, 5) * sp.cos(x + z) + R(1, 10) * sp.sin(y + 2)
    p = rho * T / (g * M ** 2)                        # eq (7): T = gamma M^2 p / rho
    E = p / ((g - 1) * rho) + sum(a * a for a in u) / 2   # eq (6) solved for E
    G = [[sp.diff(u[i], X[j]) for j in range(3)] for i in range(3)]
    div = G[0][0] + G[1][1] + G[2][2]
    tau = [[(G[i][j] + G[j][i] - R(2, 3) * (1 if i == j else 0) * div) / Re
            for j in range(3)] for i in range(3)]     # eq (4)
    kappa = 1 / ((g - 1) * M ** 2 * Pr * Re)
    qh = [kappa * sp.diff(T, X[j]) for j in range(3)]  # eq (5)
    # eqs (1)-(3) as written: minus the divergence of the fluxes
    R0 = -sum(sp.diff(rho * u[j], X[j]) for j in range(3))
    Rm = [-sum(sp.diff(rho * u[i] * u[j] + (p if i == j else 0) - tau[i][j], X[j])
               for j in range(3)) for i in range(3)]
    RE = -sum(sp.diff(rho * E * u[j] + u[j] * p - qh[j]
                      - sum(u[i] * tau[i][j] for i in range(3)), X[j]) for j in range(3))
    q = [rho, rho * u[0], rho * u[1], rho * u[2], rho * E]
    return sp.lambdify(X, q, "numpy"), sp.lambdify(X, [R0] + Rm + [RE], "numpy")


def _grid(N):
    g1 = 2 * np.pi * np.arange(N) / N
    Z, Y, Xg = np.meshgrid(g1, g1, g1, indexing="ij")
    return Xg, Y, Z


def _fields(f, Xg, Y, Z):
    return np.stack([np.broadcast_to(np.asarray(a, dtype=np.float64), Xg.shape)
                     for a in f(Xg, Y, Z)])


def continuum_errors(phys, Ns=(16, 32, 64)):
    """Per-field max-norm error of the oracle residual against the exact
    continuous residual, relative to the exact field's max, for each N:
    array [len(Ns)][5]."""
    fq, fR = _continuum(tuple(sorted(phys.items())))
    out = []
    for N in Ns:
        Xg, Y, Z = _grid(N)
        q = np.ascontiguousarray(_fields(fq, Xg, Y, Z))
        ex = _fields(fR, Xg, Y, Z)
        r = O.rhs(q, phys)
        out.append([np.abs(r[f] - ex[f]).max() / np.abs(ex[f]).max() for f in range(5)])
    return np.array(out)


# --------------------------------------------------- exact discrete residual
class TrigPoly:
    """sum_k c_k e^{ikx} with exact (40-digit) complex coefficients."""

    def __init__(self, c):
        self.c = {k: v for k, v in c.items() if v != 0}

    @staticmethod
    def const(a):
        return TrigPoly({0: mp.mpc(a)})

    @staticmethod
    def cos(k, a=1):
        return TrigPoly({k: mp.mpc(a) / 2, -k: mp.mpc(a) / 2})

    @staticmethod
    def sin(k, a=1):
        return TrigPoly({k: mp.mpc(0, -1) * a / 2, -k: mp.mpc(0, 1) * a / 2})

    def __add__(self, o):
        o = o if isinstance(o, TrigPoly) else TrigPoly.const(o)
        c = dict(self.c)
        for k, v in o.c.items():
            c[k] = c.get(k, 0) + v
        return TrigPoly(c)

    __radd__ = __add__

    def __neg__(self):
        return TrigPoly({k: -v for k, v in self.c.items()})

    def __sub__(self, o):
        return self + (-(o if isinstance(o, TrigPoly) else TrigPoly.const(o)))

    def __mul__(self, o):
        if not isinstance(o, TrigPoly):
            return TrigPoly({k: v * o for k, v in self.c.items()})
        c = {}
        for k1, v1 in self.c.items():
            for k2, v2 in o.c.items():
                c[k1 + k2] = c.get(k1 + k2, 0) + v1 * v2
        return TrigPoly(c)

    __rmul__ = __mul__

    def D(self, h):
        return TrigPoly({k: v * mp.mpc(0, 1) * (8 * mp.sin(k * h) - mp.sin(2 * k * h)) / (6 * h)
                         for k, v in self.c.items()})

    def D2(self, h):
        return TrigPoly({k: -v * (15 - 16 * mp.cos(k * h) + mp.cos(2 * k * h)) / (6 * h * h)
                         for k, v in self.c.items()})

    def at(self, xs):
        return np.array([mp.re(sum(v * mp.expj(k * x) for k, v in self.c.items())) for x in xs])


def wave_closed_form(N, phys, kind, alpha=0.3, beta=0.4, p0=8.0, dp=0.5):
    """Exact discrete state and residual of a wave along one axis, at the N
    grid points x_i = 2 pi i / N, as 40-digit values.

    kind "isothermal": rho = 1 + alpha cos x, u = beta sin x, p = p0 rho
        (T constant: the heat flux vanishes; density, pressure and the
        dilatation vary);
    kind "pressure": rho = 1, u = beta sin x, p = p0 + dp cos 2x (T varies
        with p, so the heat flux enters).
    The other velocity components are zero. Returns (rho, m, rhoE), (R(rho),
    R(m), R(rhoE)) along the wave; the two transverse momentum residuals are
    exactly zero."""
    with mp.workdps(40):
        g, M, Pr, Re = [mp.mpf(phys[k]) for k in ("gamma", "Ma", "Pr", "Re")]
        h = 2 * mp.pi / N
        P = TrigPoly
        if kind == "isothermal":
            rho = P.const(1) + P.cos(1, alpha)
            p = rho * p0
        elif kind == "pressure":
            rho = P.const(1)
            p = P.const(p0) + P.cos(2, dp)
        else:
            raise ValueError(kind)
        T = p * (g * M * M) if kind == "pressure" else P.const(g * M * M * p0)
        u = P.sin(1, beta)
        m = rho * u
        E = p * (1 / (g - 1)) + rho * u * u * mp.mpf("0.5")
        Du, D2u = u.D(h), u.D2(h)
        kappa = 1 / ((g - 1) * M * M * Pr * Re)
        c43 = mp.mpf(4) / (3 * Re)  # 1D: V = (1 + 1/3) D2u / Re, tau G = (4/3) (Du)^2 / Re
        half = mp.mpf("0.5")
        R0 = -(m.D(h) + u * rho.D(h) + rho * Du) * half
        R1 = -((m * u).D(h) + u * m.D(h) + m * Du) * half - p.D(h) + D2u * c43
        R4 = (-((E * u).D(h) + u * E.D(h) + E * Du) * half - (p * u).D(h) + T.D2(h) * kappa
              + Du * Du * c43 + u * D2u * c43)
        xs = [2 * mp.pi * i / N for i in range(N)]
        return [f.at(xs) for f in (rho, m, E)], [f.at(xs) for f in (R0, R1, R4)]


def wave_closed_form_errors(N, phys, kind, axis, prec="ld"):
    """Relative max-norm errors of the oracle residual against the exact
    discrete one, for the wave along `axis` on an N x 6 x 7 grid (rotated):
    [err R(rho), err R(m along the wave), err R(rho E), max |transverse R(m)|]."""
    (rho, m, E), (R0, R1, R4) = wave_closed_form(N, phys, kind)
    shape = [5, 6, 7]
    shape[axis] = N
    nx, ny, nz = shape
    lay = [1, 1, 1]
    lay[2 - axis] = N

    def put(a):
        a = np.array([float(v) for v in a], dtype=np.float64)
        return np.broadcast_to(a.reshape(lay), (nz, ny, nx))

    t = np.longdouble if prec == "ld" else np.float64
    q = np.zeros((5, nz, ny, nx), dtype=t)
    q[0] = put(rho)
    q[1 + axis] = put(m)
    q[4] = put(E)
    r = O.rhs(q, phys, prec=prec).astype(np.float64)

    def err(got, ex):
        ex = np.array([float(v) for v in ex])
        return float(np.abs(got - put(ex)).max() / np.abs(ex).max())

    other = max(float(np.abs(r[1 + b]).max()) for b in range(3) if b != axis)
    return [err(r[0], R0), err(r[1 + axis], R1), err(r[4], R4), other]


# ------------------------------------------------------ Taylor-Green extrema
def tgv_extrema_errors(N, phys):
    """Differences of the oracle diagnostics from the Taylor-Green extrema
    on a grid whose N is divisible by 4 (so x, y, z = 0 and pi/2 are grid
    points): rho = 1 + gamma M^2 (cos 2x + cos 2y)(cos 2z + 2)/16 spans
    1 -+ 3 gamma M^2 / 8, p spans 1/(gamma M^2) -+ 3/8, and w = 0."""
    g, M = phys["gamma"], phys["Ma"]
    q = O.init((N, N, N), phys, {})
    d = O.diagnostics(q, phys)
    p0 = 1.0 / (g * M * M)
    return {
        "max_rho": abs(d[7] - (1 + 3 * g * M * M / 8)),
        "min_rho": abs(d[12] - (1 - 3 * g * M * M / 8)),
        "min_p": abs(d[13] - (p0 - 3.0 / 8.0)) / p0,
        "max_rhow": abs(d[10]),
        "nonfinite": d[14],
    }


def diag_norm_errors(phys):
    """max |q_f| must be the largest magnitude of each field whatever its
    sign, min rho the smallest density, and the non-finite count the number
    of NaN and Inf entries; returns the number of violated statements."""
    N = 8
    q = O.init((N, N, N), phys, {"pert_kind": 1, "pert_amp": 1e-3, "seed": 4})
    bad = 0
    d = O.diagnostics(q, phys)
    bad += sum(d[7 + f] != np.abs(q[f]).max() for f in range(5))
    bad += d[12] != q[0].min()
    q2 = q.copy()
    q2[1, 3, 2, 1] = -7.5
    q2[3, 0, 0, 0] = np.nan
    q2[4, 5, 5, 5] = np.inf
    d2 = O.diagnostics(q2, phys)
    bad += d2[8] != 7.5
    bad += d2[14] != 2.0
    return int(bad)


def stage_model_mismatch(phys, prec="d"):
    """Largest difference between the slab RK step with float32-rounded
    stage states (numpy) and the full-grid C step with the same model, on
    the slab's output planes (zero when both state the model alike)."""
    shape = (12, 10, 20)
    q = O.init(shape, phys, {"pert_kind": 1, "pert_amp": 0.05, "seed": 23}, prec=prec)
    full = O.rk_step_rounded(q, phys, 0.01, 1, prec=prec)
    idx = [(k % 20) for k in range(-6, 8)]
    got = O.rk_step_slab(q[:, idx], 20, phys, 0.01, prec=prec, stage_dtype=np.float32)
    return float(np.abs((got - full[:, idx[6:8]]).astype(np.float64)).max())


# ---------------------------------------------------------- pass or fail
CONT_RATIO_BOUNDS = ((12.5, 18.0), (14.5, 17.5))


def continuum_ok(phys):
    e = continuum_errors(phys)
    r = e[:-1] / e[1:]
    ok = all(np.all(r[i] > lo) and np.all(r[i] < hi)
             for i, (lo, hi) in enumerate(CONT_RATIO_BOUNDS)) and np.all(e[-1] < 1e-4)
    return bool(ok), e


def wave_ok(N, phys, kind, axis, prec="ld", tol=1e-14):
    e = wave_closed_form_errors(N, phys, kind, axis, prec=prec)
    return bool(max(e[:3]) < tol and e[3] < 1e-16), e


def extrema_ok(N, phys):
    e = tgv_extrema_errors(N, phys)
    ok = (e["max_rho"] < 1e-15 and e["min_rho"] < 1e-15 and e["min_p"] < 1e-15
          and e["max_rhow"] == 0.0 and e["nonfinite"] == 0.0)
    return bool(ok), e
