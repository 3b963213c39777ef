"""Brute-force pin of the oracle on small grids with dense operators.

The periodic first- and second-derivative operators are built as dense
matrices: an n x n circulant per axis from the fourth-order central
weights, lifted to the 3D grid by Kronecker products with identities
(index = (k*ny + j)*nx + i). Every derivative group and the residual are then
evaluated by matrix-vector products, term by term, and compared with the C
oracle. Non-cubic grids make an axis mix-up or transposed operand fail.
"""
import numpy as np
import pytest

from oracle import oracle as O

PHYS = dict(Re=1600.0, Ma=0.1, Pr=0.71, gamma=1.4)


def circulant(n, weights):
    """Dense periodic operator: (C f)_i = sum_m w_m f_{(i+m) mod n}."""
    C = np.zeros((n, n))
    for m, w in weights.items():
        for i in range(n):
            C[i, (i + m) % n] += w
    return C


def operators(shape):
    nx, ny, nz = shape
    D, D2 = [], []
    for ax, n in enumerate(shape):
        h = 2 * np.pi / n
        c1 = circulant(n, {-2: 1 / (12 * h), -1: -8 / (12 * h), 1: 8 / (12 * h), 2: -1 / (12 * h)})
        c2 = circulant(n, {-2: -1 / (12 * h * h), -1: 16 / (12 * h * h), 0: -30 / (12 * h * h),
                           1: 16 / (12 * h * h), 2: -1 / (12 * h * h)})
        Ix, Iy, Iz = np.eye(nx), np.eye(ny), np.eye(nz)
        if ax == 0:
            D.append(np.kron(Iz, np.kron(Iy, c1)))
            D2.append(np.kron(Iz, np.kron(Iy, c2)))
        elif ax == 1:
            D.append(np.kron(Iz, np.kron(c1, Ix)))
            D2.append(np.kron(Iz, np.kron(c2, Ix)))
        else:
            D.append(np.kron(c1, np.kron(Iy, Ix)))
            D2.append(np.kron(c2, np.kron(Iy, Ix)))
    return D, D2


def brute(q, phys):
    """Derivative groups and residual with dense operators (flattened)."""
    _, nz, ny, nx = q.shape
    D, D2 = operators((nx, ny, nz))
    g, M, Re, Pr = phys["gamma"], phys["Ma"], phys["Re"], phys["Pr"]
    f = q.reshape(5, -1)
    rho, mom, rhoE = f[0], f[1:4], f[4]
    u = mom / rho
    p = (g - 1) * (rhoE - 0.5 * rho * np.sum(u * u, axis=0))
    T = g * M * M * p / rho
    groups = np.zeros((60, f.shape[1]))
    G = np.zeros((3, 3, f.shape[1]))
    for b in range(3):
        groups[0 + b] = D[b] @ rho
        groups[12 + b] = D[b] @ rhoE
        groups[33 + b] = D[b] @ (rhoE * u[b])
        groups[36 + b] = D[b] @ (p * u[b])
        groups[39 + b] = D[b] @ p
        groups[57 + b] = D2[b] @ T
        for a in range(3):
            groups[3 + 3 * a + b] = D[b] @ mom[a]
            G[a, b] = D[b] @ u[a]
            groups[15 + 3 * a + b] = G[a, b]
            groups[24 + 3 * a + b] = D[b] @ (mom[a] * u[b])
            groups[42 + 3 * a + b] = D2[b] @ u[a]
    pairs = [(0, 1), (0, 2), (1, 0), (1, 2), (2, 0), (2, 1)]
    for m, (a, k) in enumerate(pairs):
        groups[51 + m] = D[a] @ (D[k] @ u[k])
    # residual, Section 2 with the skew-symmetric split and expanded viscous terms
    div = G[0, 0] + G[1, 1] + G[2, 2]
    R = np.zeros((5, f.shape[1]))
    R[0] = -0.5 * sum(D[b] @ mom[b] + u[b] * (D[b] @ rho) + rho * G[b, b] for b in range(3))
    V = []
    for a in range(3):
        cross = sum(D[a] @ (D[k] @ u[k]) for k in range(3) if k != a)
        V.append((sum(D2[b] @ u[a] for b in range(3)) + (D2[a] @ u[a] + cross) / 3) / Re)
        conv = sum(D[b] @ (mom[a] * u[b]) + u[b] * (D[b] @ mom[a]) + mom[a] * G[b, b]
                   for b in range(3))
        R[1 + a] = -0.5 * conv - D[a] @ p + V[a]
    kappa = 1 / ((g - 1) * M * M * Pr * Re)
    conv = sum(D[b] @ (rhoE * u[b]) + u[b] * (D[b] @ rhoE) + rhoE * G[b, b] for b in range(3))
    pflux = sum(D[b] @ (p * u[b]) for b in range(3))
    heat = sum(D2[b] @ T for b in range(3))
    work = sum((G[a, b] + G[b, a] - (2 / 3 * div if a == b else 0)) / Re * G[a, b]
               for a in range(3) for b in range(3))
    vwork = sum(u[a] * V[a] for a in range(3))
    R[4] = -0.5 * conv - pflux + kappa * heat + work + vwork
    return groups, R


@pytest.mark.parametrize("shape", [(8, 8, 8), (8, 10, 12), (12, 9, 8)])
@pytest.mark.parametrize("pert", [{"pert_kind": 1, "pert_amp": 0.05, "seed": 42},
                                  {"pert_kind": 2, "pert_amp": 0.2, "phase": (0.7, 1.9, 4.1)}])
def test_P10_bruteforce_terms_and_residual(shape, pert):
    q = O.init(shape, PHYS, pert)
    # break the TGV symmetries further: perturb density and energy too
    rng = np.random.default_rng(1)
    q[0] *= 1 + 0.02 * rng.standard_normal(q[0].shape)
    q[4] *= 1 + 0.001 * rng.standard_normal(q[4].shape)
    groups_b, R_b = brute(q, PHYS)
    groups_o = O.derivs(q, PHYS).reshape(60, -1)
    for gi in range(60):
        scale = max(np.abs(groups_b[gi]).max(), 1e-30)
        err = np.abs(groups_o[gi] - groups_b[gi]).max() / scale
        assert err < 1e-12, (gi, err)
    R_o = O.rhs(q, PHYS).reshape(5, -1)
    for f in range(5):
        err = np.abs(R_o[f] - R_b[f]).max() / np.abs(R_b[f]).max()
        assert err < 1e-12, (f, err)


def test_P10_bruteforce_rk_step():
    # one RK step assembled from the dense residual and the two-register
    # update, versus the oracle's time loop
    shape = (8, 8, 8)
    q = O.init(shape, PHYS, {"pert_kind": 1, "pert_amp": 0.05, "seed": 9})
    dt = 3.385e-3 * 2
    A, B = (2 / 3, 5 / 12), (1 / 4, 3 / 20, 3 / 5)
    qs = q.reshape(5, -1).copy()
    qacc = qs.copy()
    for s in range(3):
        _, R = brute(qs.reshape(q.shape), PHYS)
        if s < 2:
            qs = qacc + A[s] * dt * R
        qacc = qacc + B[s] * dt * R
    qs = qacc
    q_o = O.rk_step(q, PHYS, dt=dt, nsteps=1).reshape(5, -1)
    for f in range(5):
        err = np.abs(q_o[f] - qs[f]).max() / np.abs(qs[f]).max()
        assert err < 1e-12, (f, err)
