"""Pins of the oracle's point maps against the paper and the mathematics.

Each check reaches the oracle's value by a different route than its own
formula: the Piola stress and tangent by automatic differentiation of the
strain energy (Sec. 4.1, Eq. 62), the equilibria by solving the defining
moment constraints (Sec. 2.3, Eqs. 22-23) as a linear system, the fluxes
against the explicit listings of Eqs. 15 and 17, and the stress against the
values the paper prints for its affine benchmarks.
"""
import os

import numpy as np
import pytest
import torch

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    out = {}
    for line in open(os.path.join(GOLD, name)):
        line = line.split("#")[0].strip()
        if not line:
            continue
        k, *v = line.split()
        out[k] = [float(x) for x in v]
    return out


def _W_torch(F, mu, lam):
    # strain energy of the compressible neo-Hookean solid (Sec. 4.1, Eq. 62)
    D = F.shape[0]
    J = torch.det(F)
    return 0.5 * mu * ((F * F).sum() - D) - (mu + 0.5 * lam) * torch.log(J) + 0.25 * lam * (J * J - 1.0)


def _rand_F(rng, D, scale=0.3):
    while True:
        F = np.eye(D) + scale * rng.standard_normal((D, D))
        if np.linalg.det(F) > 0.2:
            return F


@pytest.mark.parametrize("D", [2, 3])
def test_piola_is_energy_gradient(orc, D):
    rng = np.random.default_rng(1)
    for _ in range(20):
        F = _rand_F(rng, D)
        mu, lam = rng.uniform(0.3, 3.0), rng.uniform(0.1, 20.0)
        Ft = torch.tensor(F, dtype=torch.float64, requires_grad=True)
        (g,) = torch.autograd.grad(_W_torch(Ft, mu, lam), Ft)
        P = orc.piola(F, mu, lam)
        assert np.allclose(P, g.numpy(), rtol=1e-12, atol=1e-12 * np.abs(P).max())


@pytest.mark.parametrize("D", [2, 3])
def test_tangent_is_energy_hessian(orc, D):
    rng = np.random.default_rng(2)
    for _ in range(10):
        F = _rand_F(rng, D)
        dF = rng.standard_normal((D, D))
        mu, lam = rng.uniform(0.3, 3.0), rng.uniform(0.1, 20.0)
        H = torch.autograd.functional.hessian(lambda X: _W_torch(X, mu, lam),
                                              torch.tensor(F, dtype=torch.float64))
        ref = np.einsum("iakb,kb->ia", H.numpy(), dF)
        dP = orc.piola_jvp(F, dF, mu, lam)
        assert np.allclose(dP, ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())


@pytest.mark.parametrize("D", [2, 3])
def test_stress_free_reference_and_acoustic_tensor(orc, D):
    mu, lam = 1.3, 4.1
    assert np.abs(orc.piola(np.eye(D), mu, lam)).max() == 0.0
    # acoustic tensor Q_ik = n_A C_iAkB n_B (Sec. 2.2, Eq. 19) at F = I has the
    # longitudinal speed^2 lam + 2 mu once and the shear speed^2 mu (D-1) times
    rng = np.random.default_rng(3)
    n = rng.standard_normal(D)
    n /= np.linalg.norm(n)
    Q = np.zeros((D, D))
    for k in range(D):
        dF = np.outer(np.eye(D)[k], n)
        Q[:, k] = orc.piola_jvp(np.eye(D), dF, mu, lam) @ n
    ev = np.sort(np.linalg.eigvalsh(0.5 * (Q + Q.T)))
    assert np.allclose(ev, sorted([lam + 2 * mu] + [mu] * (D - 1)), rtol=1e-13)


def test_affine_annulus_printed_stress(orc):
    g = _golden("affine_annulus_terminal_state.txt")
    F = np.array(g["F"]).reshape(2, 2)
    assert abs(np.linalg.det(F) - g["J"][0]) < 5e-4
    sig = orc.cauchy(F, g["mu"][0], g["lambda"][0])
    # printed to four decimals
    assert np.abs(sig.reshape(-1) - np.array(g["sigma"])).max() < 6e-5


def test_ellipsoid_printed_jacobian(orc):
    g = _golden("ellipsoid_terminal_F.txt")
    F = np.eye(3) + g["T"][0] * np.array(g["A"]).reshape(3, 3)
    assert np.abs(F.reshape(-1) - np.array(g["F"])).max() < 5e-5
    # J through the oracle's moment output of a uniform state
    s = orc.Sim(3, (4, 4, 4), 0.25, 0.025, 1.0, 2.0 / 3.0)
    U0 = np.zeros((12, 64))
    U0[3:] = F.reshape(-1)[:, None]
    s.set_state(U0)
    _, _, J = s.moments()
    assert np.abs(J - g["J"][0]).max() < 5e-6


def test_flux_matches_explicit_listings(orc):
    rng = np.random.default_rng(4)
    mu, lam = 1.0, 2.0
    # D = 2 (Eq. 15)
    F = _rand_F(rng, 2)
    v = rng.standard_normal(2)
    U = np.concatenate([v, F.reshape(-1)])
    P = orc.piola(F, mu, lam)
    Phi = orc.flux(U, 2, mu, lam)
    PhiX = [-P[0, 0], -P[1, 0], -v[0], 0, -v[1], 0]
    PhiY = [-P[0, 1], -P[1, 1], 0, -v[0], 0, -v[1]]
    assert np.allclose(Phi[0], PhiX, atol=1e-15) and np.allclose(Phi[1], PhiY, atol=1e-15)
    # D = 3 (Eq. 17)
    F = _rand_F(rng, 3)
    v = rng.standard_normal(3)
    U = np.concatenate([v, F.reshape(-1)])
    P = orc.piola(F, mu, lam)
    Phi = orc.flux(U, 3, mu, lam)
    lst = [
        [-P[0, 0], -P[1, 0], -P[2, 0], -v[0], 0, 0, -v[1], 0, 0, -v[2], 0, 0],
        [-P[0, 1], -P[1, 1], -P[2, 1], 0, -v[0], 0, 0, -v[1], 0, 0, -v[2], 0],
        [-P[0, 2], -P[1, 2], -P[2, 2], 0, 0, -v[0], 0, 0, -v[1], 0, 0, -v[2]],
    ]
    assert np.allclose(Phi, lst, atol=1e-15)


def _evec(q, D):
    e = np.zeros(D)
    e[q // 2] = -1.0 if q & 1 else 1.0
    return e


@pytest.mark.parametrize("D", [2, 3])
def test_equilibrium_solves_moment_constraints(orc, D):
    """feq is the unique solution of the moment constraints and the symmetric
    pair-sum closure (Eqs. 22-23), solved here as a dense linear system."""
    M, Q = D + D * D, 2 * D
    rng = np.random.default_rng(5)
    c, mu, lam, rho0 = 7.0, 1.2, 3.4, 1.7
    for _ in range(5):
        F = _rand_F(rng, D)
        U = np.concatenate([rng.standard_normal(D), F.reshape(-1)])
        Phi = orc.flux(U, D, mu, lam, rho0)
        rows, rhs = [], []
        for r in range(M):
            row = np.zeros((Q, M)); row[:, r] = 1.0
            rows.append(row.reshape(-1)); rhs.append(U[r])
            for A in range(D):
                row = np.zeros((Q, M))
                for q in range(Q):
                    row[q, r] = c * _evec(q, D)[A]
                rows.append(row.reshape(-1)); rhs.append(Phi[A, r])
                row = np.zeros((Q, M)); row[2 * A, r] = row[2 * A + 1, r] = 1.0
                rows.append(row.reshape(-1)); rhs.append(U[r] / D)
        A_ = np.array(rows)
        sol, *_ = np.linalg.lstsq(A_, np.array(rhs), rcond=None)
        assert np.linalg.matrix_rank(A_) == Q * M  # unique
        fe = orc.feq(U, D, c, mu, lam, rho0)
        assert np.allclose(fe.reshape(-1), sol, rtol=1e-12, atol=1e-13)
        # pair identities (Sec. 3.2, Eq. 40)
        for A in range(D):
            d = _evec(2 * A, D)
            assert np.allclose(fe[2 * A] + fe[2 * A + 1], U / D, atol=1e-14)
            assert np.allclose(fe[2 * A] - fe[2 * A + 1], (d @ Phi) / c, atol=1e-14)


@pytest.mark.parametrize("D", [2, 3])
def test_equilibrium_derivative_matches_finite_difference(orc, D):
    rng = np.random.default_rng(6)
    c, mu, lam = 10.0, 1.0, 2.0
    F = _rand_F(rng, D, 0.2)
    U = np.concatenate([rng.standard_normal(D), F.reshape(-1)])
    Z = rng.standard_normal(D + D * D)
    h = 1e-6
    fd = (orc.feq(U + h * Z, D, c, mu, lam) - orc.feq(U - h * Z, D, c, mu, lam)) / (2 * h)
    assert np.allclose(orc.feq_jvp(U, Z, D, c, mu, lam), fd, atol=1e-9)


@pytest.mark.parametrize("D", [2, 3])
def test_damping_source_gives_trapezoid_decay(orc, D):
    """Uniform velocity under B = (-gamma v, 0): with source weights summing to
    1/2 (Eq. 30) and the half-step recovery (Eq. 28) the lattice reproduces the
    trapezoidal decay v^{n+1} = v^n (1 - gamma dt/2)/(1 + gamma dt/2), keeps F,
    and the displacement quadrature (Eq. 34) integrates it by the trapezoid
    rule."""
    n = [4] * D
    N = 4 ** D
    dt, gamma = 0.01, 10.0
    s = orc.Sim(D, n, 0.1, dt, 1.0, 2.0, gamma=gamma)
    rng = np.random.default_rng(7)
    F = _rand_F(rng, D, 0.1)
    v0 = rng.standard_normal(D)
    U0 = np.zeros((D + D * D, N))
    U0[:D] = v0[:, None]
    U0[D:] = F.reshape(-1)[:, None]
    s.set_state(U0)
    fac = (1 - gamma * dt / 2) / (1 + gamma * dt / 2)
    u_ref = np.zeros(D)
    v = v0.copy()
    for k in range(1, 6):
        s.step(1)
        vn = v * fac
        u_ref = u_ref + 0.5 * dt * (v + vn)
        v = vn
        U, u, _ = s.moments()
        assert np.allclose(U[:D], v[:, None], rtol=1e-13, atol=1e-15)
        assert np.allclose(U[D:], F.reshape(-1)[:, None], atol=1e-14)
        assert np.allclose(u, u_ref[:, None], atol=1e-15)
