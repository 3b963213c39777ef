"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these compare the oracle with itself: each checks a closed form, an
invariant, a published test vector or a brute-force construction that a
plausible mistake in the oracle (a dropped term, a wrong sign, a wrong axis
or index) would break.

Closed forms used (h = 2 pi / N, k the integer wavenumber):
  modified wavenumber of the 4th-order first derivative
      k'(k)   = (8 sin kh - sin 2kh) / (6h)
  and of the 4th-order second derivative
      k''2(k) = (15 - 16 cos kh + cos 2kh) / (6 h^2),
so D sin(kx) = k' cos(kx) and D2 sin(kx) = -k''2 sin(kx) exactly on the
periodic grid (Section 2: fourth-order central differences).
"""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1610_09146_amd import workloads as W

PHYS = dict(Re=1600.0, Ma=0.1, Pr=0.71, gamma=1.4)  # Section 3


def kp(k, h):
    return (8 * np.sin(k * h) - np.sin(2 * k * h)) / (6 * h)


def kpp2(k, h):
    return (15 - 16 * np.cos(k * h) + np.cos(2 * k * h)) / (6 * h * h)


def grid(shape):
    nx, ny, nz = shape
    x = 2 * np.pi * np.arange(nx) / nx
    y = 2 * np.pi * np.arange(ny) / ny
    z = 2 * np.pi * np.arange(nz) / nz
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X, Y, Z


def state_from_prims(rho, u, v, w, p, gamma=1.4):
    return np.stack([rho, rho * u, rho * v, rho * w,
                     p / (gamma - 1) + 0.5 * rho * (u * u + v * v + w * w)])


# ---------------------------------------------------------------- generator
def _golden(name):
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    with open(path) as f:
        return [line.split() for line in f if line.strip() and not line.startswith("#")]


def test_splitmix64_published_vectors():
    # first outputs of SplitMix64 from state 0 (tests/golden/splitmix64_vectors.txt)
    rows = _golden("splitmix64_vectors.txt")
    assert len(rows) == 3
    for idx, hexval in rows:
        assert O.splitmix64(0, int(idx)) == int(hexval, 16)


def test_taylor_green_setup_matches_paper():
    # the workload recipes carry the paper's Section 3 parameters
    g = {k: float(v) for k, v in _golden("tgv_setup.txt")}
    for key in ("Re", "Ma", "Pr", "gamma"):
        assert W.TGV_PHYS[key] == g[key], key
    assert W.tgv_dt(64) == g["dt_64"]
    assert W.tgv_dt(128) == g["dt_64"] / 2 and W.tgv_dt(512) == g["dt_64"] / 8


# ---------------------------------------------------------------- operators
@pytest.mark.parametrize("N", [8, 12, 16, 32])
@pytest.mark.parametrize("k", [1, 2, 3])
def test_P1_first_derivative_modified_wavenumber(N, k):
    shape = (N, N + 2, N + 4)  # distinct axis lengths catch axis mix-ups
    X, Y, Z = grid(shape)
    for ax, coord in enumerate((X, Y, Z)):
        n = shape[ax]
        h = 2 * np.pi / n
        rho = 2.0 + 0.5 * np.sin(k * coord)
        q = state_from_prims(rho, 0 * rho, 0 * rho, 0 * rho, 1.0 + 0 * rho)
        d = O.derivs(q, PHYS)
        expect = 0.5 * kp(k, h) * np.cos(k * coord)
        assert np.max(np.abs(d[ax] - expect)) < 1e-13
        for other in range(3):
            if other != ax:
                assert np.max(np.abs(d[other])) < 1e-13


@pytest.mark.parametrize("N", [8, 16, 32])
def test_P1_fourth_order_convergence(N):
    # error of D sin x against cos x shrinks by 2^4 per halving of h
    h1, h2 = 2 * np.pi / N, np.pi / N
    e1 = abs(kp(1, h1) - 1)
    e2 = abs(kp(1, h2) - 1)
    assert 14.5 < e1 / e2 < 16.5
    # and the oracle reproduces k' (checked above), hence this order
    X, Y, Z = grid((N, 8, 8))
    q = state_from_prims(1.5 + 0.25 * np.sin(X), 0 * X, 0 * X, 0 * X, 1 + 0 * X)
    d = O.derivs(q, PHYS)
    err = np.max(np.abs(d[0] - 0.25 * np.cos(X)))
    assert abs(err - 0.25 * e1) < 1e-13


@pytest.mark.parametrize("N", [8, 16, 32])
@pytest.mark.parametrize("k", [1, 3])
def test_P2_second_derivative_modified_wavenumber(N, k):
    shape = (N + 4, N, N + 2)
    X, Y, Z = grid(shape)
    rho = 1.0 + 0 * X
    for ax, coord in enumerate((X, Y, Z)):
        h = 2 * np.pi / shape[ax]
        u = np.sin(k * coord)
        T_field = 1.0 + 0.1 * np.sin(k * coord)
        # T = gamma M^2 p / rho with rho = 1  ->  choose p = T / (gamma M^2)
        p = T_field / (PHYS["gamma"] * PHYS["Ma"] ** 2)
        q = state_from_prims(rho, u, 0 * u, 0 * u, p)
        d = O.derivs(q, PHYS)
        # D2_b u_a at index 42 + 3a + b, D2_b T at 57 + b
        assert np.max(np.abs(d[42 + ax] + kpp2(k, h) * u)) < 1e-12 * kpp2(k, h)
        assert np.max(np.abs(d[57 + ax] + 0.1 * kpp2(k, h) * np.sin(k * coord))) < 1e-12 * kpp2(k, h)
        for other in range(3):
            if other != ax:
                assert np.max(np.abs(d[42 + other])) < 1e-12


@pytest.mark.parametrize("N", [8, 16])
def test_P3_cross_derivatives(N):
    shape = (N, N + 2, N + 4)
    X, Y, Z = grid(shape)
    hs = [2 * np.pi / n for n in shape]
    coords = (X, Y, Z)
    ks = (1, 2, 3)
    # G_kk = D_k u_k; cross group 51.. = D_a(G_kk) for (a,k) in this order
    pairs = [(0, 1), (0, 2), (1, 0), (1, 2), (2, 0), (2, 1)]
    for m, (a, kk) in enumerate(pairs):
        vel = [0 * X, 0 * X, 0 * X]
        vel[kk] = np.sin(ks[a] * coords[a]) * np.sin(ks[kk] * coords[kk])
        q = state_from_prims(1.0 + 0 * X, *vel, 1.0 + 0 * X)
        d = O.derivs(q, PHYS)
        expect = (kp(ks[a], hs[a]) * kp(ks[kk], hs[kk])
                  * np.cos(ks[a] * coords[a]) * np.cos(ks[kk] * coords[kk]))
        assert np.max(np.abs(d[51 + m] - expect)) < 1e-12


def test_product_derivative_closed_form():
    # D_x(rho u u) with rho = 1, u = sin x: u^2 = (1 - cos 2x)/2, so
    # D_x(u u) = k'(2) sin(2x) / 2 (group 24 = D_0(rho u_0 u_0)).
    N = 16
    X, Y, Z = grid((N, N, N))
    h = 2 * np.pi / N
    u = np.sin(X)
    q = state_from_prims(1.0 + 0 * X, u, 0 * u, 0 * u, 1.0 + 0 * X)
    d = O.derivs(q, PHYS)
    assert np.max(np.abs(d[24] - kp(2, h) * np.sin(2 * X) / 2)) < 1e-13


# ------------------------------------------------------------- initial state
@pytest.mark.parametrize("N", [8, 16, 32])
@pytest.mark.parametrize("Ma", [0.1, 0.05])
def test_P4_initial_state_invariants(N, Ma):
    phys = dict(PHYS, Ma=Ma)
    g = phys["gamma"]
    q = O.init((N, N, N), phys, {})
    d = O.diagnostics(q, phys)
    assert abs(d[0] - 1.0 / 8.0) < 1e-13                  # KE = V0^2/8
    assert abs(d[2] - 1.0) < 1e-14                        # <rho> = 1
    assert max(abs(d[3]), abs(d[4]), abs(d[5])) < 1e-16   # <rho u_i> = 0
    p0 = 1.0 / (g * Ma * Ma)
    assert abs(d[15] - p0) < 1e-13 * p0                   # <p> = 1/(gamma M^2)
    assert abs(d[6] - (p0 / (g - 1) + 1.0 / 8.0)) < 1e-12 * p0
    prim = O.prims(q, phys)
    assert np.max(np.abs(prim[4] - 1.0)) < 1e-14          # isothermal T = 1
    assert np.max(np.abs(prim[2])) == 0.0                 # w = 0
    # discretely divergence-free initial velocity
    dd = O.derivs(q, phys)
    assert np.max(np.abs(dd[15] + dd[19] + dd[23])) < 1e-14


@pytest.mark.parametrize("N,Ma", [(8, 0.1), (16, 0.1), (32, 0.1), (16, 0.2)])
def test_P7_initial_enstrophy(N, Ma):
    # <rho |omega|^2 / 2> = k'(1)^2 V0^2 (3/8 - 5 gamma M^2 V0^2 / 128)
    phys = dict(PHYS, Ma=Ma)
    h = 2 * np.pi / N
    q = O.init((N, N, N), phys, {})
    ens = O.diagnostics(q, phys)[1]
    expect = kp(1, h) ** 2 * (3.0 / 8.0 - 5 * phys["gamma"] * Ma * Ma / 128.0)
    assert abs(ens - expect) < 1e-14 * expect * 10


@pytest.mark.parametrize("N", [8, 16, 32])
@pytest.mark.parametrize("Re", [1600.0, 400.0])
def test_P5_initial_kinetic_energy_decay_rate(N, Re):
    # dKE/dt = < u_i R(rho u_i) - |u|^2 R(rho)/2 > at t = 0 equals
    # -(3 k''2 + (k''2 - k'^2)/3) / (4 Re): convection and pressure cancel on
    # the divergence-free discrete state, only the expanded viscous terms
    # remain. Distinguishes the D2 stencil from D(D) and the 1/3 form.
    phys = dict(PHYS, Re=Re)
    h = 2 * np.pi / N
    q = O.init((N, N, N), phys, {})
    r = O.rhs(q, phys, prec="ld").astype(np.float64)
    prim = O.prims(q, phys)
    u = prim[:3]
    rate = np.mean(np.sum(u * r[1:4], axis=0) - 0.5 * np.sum(u * u, axis=0) * r[0])
    expect = -(3 * kpp2(1, h) + (kpp2(1, h) - kp(1, h) ** 2) / 3) / (4 * Re)
    assert abs(rate - expect) < 1e-12 * abs(expect)


@pytest.mark.parametrize("N", [8, 16])
def test_P6_energy_residual_mean(N):
    # <R(rho E)> at t = 0 equals 5 V0^2 (k'^2 - k''2) / (6 Re): the viscous
    # work expanded by the product rule is not a discrete divergence.
    h = 2 * np.pi / N
    q = O.init((N, N, N), PHYS, {}, prec="ld")
    r = O.rhs(q, PHYS, prec="ld")
    expect = 5 * (kp(1, h) ** 2 - kpp2(1, h)) / (6 * PHYS["Re"])
    got = float(np.mean(r[4]))
    assert abs(got - expect) < 1e-10 * abs(expect)


# ------------------------------------------------------------- conservation
@pytest.mark.parametrize("shape", [(8, 8, 8), (12, 10, 9), (16, 16, 16)])
def test_P8_discrete_conservation_any_state(shape):
    # sum R(rho) = sum R(rho u_i) = 0 for any periodic state: D is
    # skew-adjoint and every stencil's weights sum to zero.
    rng = np.random.default_rng(5)
    phys = PHYS
    q = O.init(shape, phys, {"pert_kind": 1, "pert_amp": 0.2, "seed": 3})
    q[0] *= 1 + 0.05 * rng.standard_normal(q[0].shape)
    r = O.rhs(q, phys)
    for f in range(4):
        assert abs(r[f].sum()) < 1e-13 * np.abs(r[f]).sum()
    # energy is not conserved to round-off (viscous work is expanded)
    assert abs(r[4].sum()) > 1e-8 * np.abs(r[4]).sum()


def test_P8_conservation_over_rk_steps():
    N = 12
    q = O.init((N, N, N), PHYS, {"pert_kind": 1, "pert_amp": 1e-2, "seed": 7})
    s0 = q.reshape(5, -1).sum(axis=1)
    q2 = O.rk_step(q, PHYS, dt=1e-2, nsteps=3)
    s1 = q2.reshape(5, -1).sum(axis=1)
    for f in range(4):
        assert abs(s1[f] - s0[f]) < 1e-12 * max(1.0, np.abs(q[f]).sum())


# --------------------------------------------------------------- time order
def test_P9_third_order_in_time():
    # halving dt at fixed final time divides the temporal error by ~8
    N = 12
    q = O.init((N, N, N), PHYS, {"pert_kind": 2, "pert_amp": 0.3, "phase": (0.3, 1.1, 2.0)})
    T = 0.24
    sols = [O.rk_step(q, PHYS, dt=T / n, nsteps=n) for n in (6, 12, 24)]
    e1 = np.max(np.abs(sols[0] - sols[1]))
    e2 = np.max(np.abs(sols[1] - sols[2]))
    assert 6.5 < e1 / e2 < 9.5, e1 / e2


def test_rk_coefficients_third_order_conditions():
    from fractions import Fraction as F
    a1, a2 = F(2, 3), F(5, 12)
    b1, b2, b3 = F(1, 4), F(3, 20), F(3, 5)
    c2, c3 = a1, b1 + a2           # stage times of the two-register form
    a32 = a2
    assert b1 + b2 + b3 == 1
    assert b2 * c2 + b3 * c3 == F(1, 2)
    assert b2 * c2 ** 2 + b3 * c3 ** 2 == F(1, 3)
    assert b3 * a32 * c2 == F(1, 6)
    assert abs(O.RK_A[0] - 2 / 3) < 1e-16 and abs(O.RK_B[2] - 0.6) < 1e-16


# ------------------------------------------------------------ perturbations
def test_pointwise_perturbation_statistics():
    N = 16
    amp = 1e-3
    q0 = O.init((N, N, N), PHYS, {})
    q1 = O.init((N, N, N), PHYS, {"pert_kind": 1, "pert_amp": amp, "seed": 1610})
    assert np.array_equal(q0[0], q1[0])          # rho unchanged (p unchanged)
    mask = np.abs(q0[1]) > 1e-3
    xi = q1[1][mask] / q0[1][mask] - 1
    assert xi.min() >= -amp * (1 + 1e-9) and xi.max() < amp * (1 + 1e-9)
    assert abs(xi.mean()) < 0.1 * amp
    assert abs(xi.std() - amp / np.sqrt(3)) < 0.1 * amp
    # the counter stream for component 0, point 5 is SplitMix64 output 6
    U = O.splitmix64(1610, 5) >> 11
    idx = np.unravel_index(5, q0[1].shape)
    if abs(q0[1][idx]) > 0:
        got = q1[1][idx] / q0[1][idx] - 1
        assert abs(got - amp * (2 * U * 2.0 ** -53 - 1)) < 1e-15


def test_random_phase_perturbation_divergence_free():
    N = 16
    q = O.init((N, N, N), PHYS, {"pert_kind": 2, "pert_amp": 1e-2, "phase": (0.4, 2.2, 5.9)})
    d = O.derivs(q, PHYS)
    assert np.max(np.abs(d[15] + d[19] + d[23])) < 1e-14


# --------------------------------------------------------------- floor
@pytest.mark.parametrize("N", [8, 16])
def test_double_vs_extended_floor(N):
    q = O.init((N, N, N), PHYS, {"pert_kind": 1, "pert_amp": 1e-3, "seed": 11}, prec="ld")
    r_ld = O.rhs(q, PHYS, prec="ld")
    r_d = O.rhs(q.astype(np.float64), PHYS, prec="d")
    for f in range(5):
        ref = np.abs(r_ld[f]).max()
        err = np.abs(r_d[f] - r_ld[f]).max() / ref
        assert err < 2e-12, (f, float(err))


# ------------------------------------------------ pointwise term closed forms
def test_heat_flux_and_pressure_gradient_rest_state():
    # fluid at rest, rho = 1, T = 1 + e sin(k x): every term vanishes except
    #   R(rho u) = -D_x p = -e k'(k) cos(kx) / (gamma M^2)
    #   R(rho E) = kappa D2_x T = -kappa e k''2(k) sin(kx)
    # (eq (5): q_j = kappa dT/dx_j enters the energy equation as +d q_j/dx_j)
    N, k, e = 16, 2, 0.01
    g, M, Pr, Re = PHYS["gamma"], PHYS["Ma"], PHYS["Pr"], PHYS["Re"]
    X, Y, Z = grid((N, 12, 10))
    h = 2 * np.pi / N
    T = 1 + e * np.sin(k * X)
    q = state_from_prims(1 + 0 * X, 0 * X, 0 * X, 0 * X, T / (g * M * M))
    r = O.rhs(q, PHYS, prec="ld").astype(np.float64)
    kappa = 1 / ((g - 1) * M * M * Pr * Re)
    assert np.max(np.abs(r[0])) < 1e-14
    assert np.max(np.abs(r[1] + e * kp(k, h) * np.cos(k * X) / (g * M * M))) < 1e-12
    assert np.max(np.abs(r[2])) < 1e-13 and np.max(np.abs(r[3])) < 1e-13
    assert np.max(np.abs(r[4] + kappa * e * kpp2(k, h) * np.sin(k * X))) < 1e-12 * kappa * e * kpp2(k, h)


def test_shear_wave_viscous_force_and_work():
    # rho = 1, p constant, u = e sin(k y), v = w = 0:
    #   R(rho u) = V_x = -e k''2 sin(ky) / Re
    #   R(rho E) = tau_xy G_xy + u V_x = e^2 (k'^2 cos^2 ky - k''2 sin^2 ky) / Re
    N, k, e = 12, 1, 0.05
    Re = PHYS["Re"]
    X, Y, Z = grid((10, N, 8))
    h = 2 * np.pi / N
    u = e * np.sin(k * Y)
    q = state_from_prims(1 + 0 * X, u, 0 * X, 0 * X, 50.0 + 0 * X)
    r = O.rhs(q, PHYS, prec="ld").astype(np.float64)
    assert np.max(np.abs(r[0])) < 1e-15
    assert np.max(np.abs(r[1] + e * kpp2(k, h) * np.sin(k * Y) / Re)) < 1e-15
    # R(rho v) = -D_y p sees only the rounding of p = 50 recovered from rho E
    assert np.max(np.abs(r[2])) < 1e-13 and np.max(np.abs(r[3])) < 1e-15
    expect = e * e * (kp(k, h) ** 2 * np.cos(k * Y) ** 2 - kpp2(k, h) * np.sin(k * Y) ** 2) / Re
    # absolute slack: kappa D2 T of the rounding of T recovered from rho E
    assert np.max(np.abs(r[4] - expect)) < 1e-15 + 1e-12 * np.max(np.abs(expect))


def test_uniform_translation_convective_terms():
    # rho = 1 + e sin(k z), uniform velocity (0, 0, U), p constant:
    #   R(rho) = -U D_z rho,  R(rho w) = -U^2 D_z rho,  R(rho u) = R(rho v) = 0
    # (skew-symmetric split eq (8) with D_z U = 0)
    N, k, e, U = 16, 3, 0.1, 0.7
    X, Y, Z = grid((8, 10, N))
    h = 2 * np.pi / N
    rho = 1 + e * np.sin(k * Z)
    q = state_from_prims(rho, 0 * X, 0 * X, U + 0 * X, 20.0 + 0 * X)
    r = O.rhs(q, PHYS, prec="ld").astype(np.float64)
    Drho = e * kp(k, h) * np.cos(k * Z)
    assert np.max(np.abs(r[0] + U * Drho)) < 1e-13
    assert np.max(np.abs(r[3] + U * U * Drho)) < 1e-13
    assert np.max(np.abs(r[1])) < 1e-15 and np.max(np.abs(r[2])) < 1e-15


# ------------------------------------------------------------- slab paths
def test_slab_entry_points_match_full_grid():
    # the sampled-plane checks at large grids use slabs cut from the grid;
    # a slab must reproduce the full-grid values on its interior planes
    shape = (12, 10, 16)
    tgv = {"pert_kind": 1, "pert_amp": 0.05, "seed": 21}
    q = O.init(shape, PHYS, tgv)
    r = O.rhs(q, PHYS)
    for k0 in (0, 7, 14):
        qs = O.init_slab(shape, k0 - 2, 6, PHYS, tgv)
        idx = [(k % 16) for k in range(k0 - 2, k0 + 4)]
        assert np.array_equal(qs, q[:, idx])
        rs = O.rhs_slab(qs, 16, PHYS)
        assert np.array_equal(rs, r[:, idx[2:4]])



@pytest.mark.parametrize("prec", ["d", "ld"])
def test_slab_rk_step_matches_full_grid(prec):
    # the full-size check of the timed RK step advances slabs cut from the
    # grid: one slab step must give the full-grid step on its output planes
    shape = (12, 10, 20)
    tgv = {"pert_kind": 1, "pert_amp": 0.05, "seed": 22}
    q = O.init(shape, PHYS, tgv, prec=prec)
    dt = 0.01
    full = O.rk_step(q, PHYS, dt, 1, prec=prec)
    for k0, m in ((0, 2), (9, 3), (18, 2)):
        idx = [(k % 20) for k in range(k0 - 6, k0 + m + 6)]
        got = O.rk_step_slab(q[:, idx], 20, PHYS, dt, prec=prec)
        assert got.shape == (5, m, 10, 12)
        assert np.array_equal(got, full[:, idx[6:6 + m]])
    with pytest.raises(ValueError):
        O.rk_step_slab(q[:, :12], 20, PHYS, dt, prec=prec)
    # the single-precision model: rounding through float64 changes nothing in
    # double precision; through float32 it moves the step's increment by
    # single-precision rounding (relative 1e-8 .. 1e-4), no more
    idx = [(k % 20) for k in range(-6, 8)]
    plain = O.rk_step_slab(q[:, idx], 20, PHYS, dt, prec=prec)
    if prec == "d":
        assert np.array_equal(O.rk_step_slab(q[:, idx], 20, PHYS, dt, prec=prec,
                                             stage_dtype=np.float64), plain)
    r32 = O.rk_step_slab(q[:, idx], 20, PHYS, dt, prec=prec, stage_dtype=np.float32)
    base = q[:, idx[6:8]]
    inc = (plain - base).astype(np.float64).reshape(5, -1)
    d32 = (r32 - plain).astype(np.float64).reshape(5, -1)
    rel = np.abs(d32).max(axis=1) / np.abs(inc).max(axis=1)
    assert np.all(rel > 1e-9) and np.all(rel < 1e-4), rel

# ------------------------------------------------------------ two dimensions
# nz = 1: the z-independent problem (the paper counts its arrays for 2D as
# well as 3D, Section 2). The Taylor-Green initial state is its z = 0 plane,
# u = sin x cos y, v = -cos x sin y, w = 0, p = 1/(gamma M^2) + 3(cos 2x + cos 2y)/16.

@pytest.mark.parametrize("N", [8, 16, 32])
def test_2d_closed_forms(N):
    h = 2 * np.pi / N
    q = O.init((N, N, 1), PHYS, {})
    d = O.diagnostics(q, PHYS)
    # KE = <rho |u|^2 / 2> = 1/4: the density variation is orthogonal to |u|^2
    assert abs(d[0] - 0.25) < 1e-14
    assert abs(d[2] - 1.0) < 1e-14
    # omega = (0, 0, 2 k' sin x sin y) and rho = 1 + 3 gamma M^2 (cos 2x + cos 2y)/16:
    # enstrophy = k'^2 (1/2 - 3 gamma M^2 / 32)
    ens = kp(1, h) ** 2 * (0.5 - 3 * PHYS["gamma"] * PHYS["Ma"] ** 2 / 32)
    assert abs(d[1] - ens) < 1e-13 * ens
    r = O.rhs(q, PHYS, prec="ld")
    # no z-momentum is generated: every z-difference vanishes (to one
    # rounding of the stencil's weighted sum, which the oracle evaluates term
    # by term)
    assert np.abs(r[3]).max() <= 1e-15 * np.abs(r[1]).max()
    # initial rate: two directions of D2 plus the 1/3 cross form; convection
    # and pressure cancel on the divergence-free state as in three dimensions
    prim = O.prims(q, PHYS)
    u = prim[:3]
    rr = r.astype(np.float64)
    rate = np.mean(np.sum(u * rr[1:4], axis=0) - 0.5 * np.sum(u * u, axis=0) * rr[0])
    expect = -(2 * kpp2(1, h) + (kpp2(1, h) - kp(1, h) ** 2) / 3) / (2 * PHYS["Re"])
    assert abs(rate - expect) < 1e-12 * abs(expect)


@pytest.mark.parametrize("shape", [(16, 12, 1), (11, 9, 1)])
def test_2d_equals_z_uniform_3d(shape):
    # the residual of a z-independent state does not depend on nz: nz = 1
    # against the same plane repeated on nz = 5, with a nonzero w so that the
    # z-momentum equation is exercised too
    nx, ny, _ = shape
    q2 = O.init(shape, PHYS, {"pert_kind": 1, "pert_amp": 1e-2, "seed": 3}).astype(np.longdouble)
    x = 2 * np.pi * np.arange(nx) / nx
    y = 2 * np.pi * np.arange(ny) / ny
    w = 0.05 * np.sin(x)[None, :] * np.cos(2 * y)[:, None]
    q2[3, 0] = q2[0, 0] * w
    q2[4, 0] += 0.5 * q2[0, 0] * w * w
    q3 = np.repeat(q2, 5, axis=1)
    r2 = O.rhs(q2, PHYS, prec="ld")
    r3 = O.rhs(q3, PHYS, prec="ld")
    assert np.any(r2[3] != 0)
    for k in range(5):
        # the z second difference of a constant leaves a rounding residue of
        # the stencil weights (their sum is 0 only in exact arithmetic)
        assert np.all(rel_err_ld(r3[:, k:k + 1], r2) <= 1e-15), k


def rel_err_ld(a, b):
    a = np.asarray(a).reshape(a.shape[0], -1)
    b = np.asarray(b).reshape(b.shape[0], -1)
    return (np.abs(a - b).max(axis=1) / np.maximum(np.abs(b).max(axis=1), 1e-300)).astype(np.float64)

