"""Pins of the oracle's compatibility projection (Sec. 3.5, Eqs. 57-61) by
facts the mathematics fixes, independent of how the oracle is written.

- Damped Jacobi sweeps (the paper's relaxation of the normal equations
  K u = b): on an all-active periodic lattice K is the graph Laplacian of
  the periodic grid, whose eigenvectors are the Fourier modes.  The error
  against the exact least-squares solution therefore shrinks mode by mode:
  after k sweeps of weight w, a mode of wavevector theta has been multiplied
  by (1 - w lambda_theta / 2D)^k exactly, lambda_theta = sum_A 2 (1 - cos
  theta_A).  The exact solution comes from a dense least-squares solve of
  the edge problem built here from the edge relation of Eq. 57.
- Dirichlet anchors (Sec. 3.5 allows prescribed displacement values as
  projection anchors): an affine displacement u = G (X - X0) + a with
  F = I + G satisfies every edge relation and every anchor relation
  u_m + (F_m - I)(X_b - X_m) = u_D(X_b) exactly when u_D is the same affine
  field, so both projection modes must return u unchanged.  A dropped or
  sign-flipped offset (F_m - I)(X_b - X_m), or anchors evaluated at the
  wrong node, moves u.
"""
import numpy as np
import pytest

import workloads as W


def _periodic_edges(n, dx, F):
    """Incidence matrix of the periodic grid's axis edges and the targets of
    Eq. 57 (dense; small grids): edge l -> m = l + e_A has target
    (dx/2) [(F_m - I) + (F_l - I)] e_A for each displacement component."""
    D = len(n)
    N = int(np.prod(n))
    idx = np.arange(N).reshape(n[::-1])  # [z][y][x] with x fastest
    rows, tgt = [], [[] for _ in range(D)]
    for A in range(D):
        ax = D - 1 - A  # axis A of the lattice is array axis D-1-A
        nb = np.roll(idx, -1, axis=ax)
        for l, m in zip(idx.reshape(-1), nb.reshape(-1)):
            r = np.zeros(N)
            r[m] += 1.0
            r[l] -= 1.0
            rows.append(r)
            for i in range(D):
                tgt[i].append(0.5 * dx * (F[i * D + A, m] + F[i * D + A, l] - 2.0 * (i == A)))
    return np.array(rows), [np.array(t) for t in tgt]


@pytest.mark.parametrize("n,kvec", [((8, 6), (1, 2)), ((8, 6), (3, 0)), ((6, 4, 5), (1, 1, 2)),
                                    ((6, 4, 5), (0, 2, 1))])
@pytest.mark.parametrize("w", [2.0 / 3.0, 0.45])
def test_jacobi_sweep_damps_each_fourier_mode_by_its_symbol(orc, n, kvec, w):
    D = len(n)
    N = int(np.prod(n))
    dx = 1.0 / n[0]
    rng = np.random.default_rng(7)
    F = np.eye(D).reshape(-1)[:, None] + 0.2 * rng.standard_normal((D * D, N))
    A_, tgt = _periodic_edges(n, dx, F)
    xs = np.array([np.linalg.lstsq(A_, t, rcond=None)[0] for t in tgt])
    # the Fourier mode over integer node coordinates
    I = np.stack(np.meshgrid(*[np.arange(k) for k in n], indexing="ij"), 0)  # [A][x][y][z]
    I = I.reshape(D, -1, order="F")  # node index x + nx*(y + ny*z)
    theta = [2.0 * np.pi * k / m for k, m in zip(kvec, n)]
    mode = np.cos(sum(t * I[A] for A, t in enumerate(theta)) + 0.3)
    lam = sum(2.0 * (1.0 - np.cos(t)) for t in theta)
    rho = 1.0 - w * lam / (2 * D)
    eps = np.array([1.0, -0.5, 0.25][:D])[:, None]
    for k in (1, 2, 20):
        s = orc.Sim(D, n, dx, dx / 10, 1.0, 2.0, proj_sweeps=k, proj_weight=w)
        uc, _ = s.project(F, xs + eps * mode)
        err = uc - xs - eps * rho ** k * mode
        assert np.abs(err).max() < 1e-13, (k, np.abs(err).max(), rho)


def _annulus_mixed(orc, sweeps, G, a, X0):
    c = W.config_c2(40)
    s = orc.Sim(2, c["n"], c["dx"], c["dt"], c["mu"], c["lam"], omega=c["omega"], gamma=c["gamma"],
                origin=c["origin"], periodic_mask=0, proj_every=20, proj_sweeps=sweeps)
    s.set_levelset(c["phi"], c["bid"])
    s.set_bc(1, orc.DIRICHLET, given_as_displacement=True, a=a, G=G, X0=X0)
    s.set_bc(2, orc.NEUMANN)
    return s, c


@pytest.mark.parametrize("sweeps", [20, 0])
def test_anchored_projection_keeps_affine_displacement(orc, sweeps):
    rng = np.random.default_rng(11)
    G = 0.1 * rng.standard_normal((2, 2))
    a = 0.01 * rng.standard_normal(2)
    X0 = (0.4, 0.55)
    s, c = _annulus_mixed(orc, sweeps, G, a, X0)
    L = s.links()
    assert np.any(L["bid"] == 1) and np.any(L["bid"] == 2)
    X = c["X"]
    u = G @ (X - np.array(X0)[:, None]) + a[:, None]
    F = (np.eye(2) + G).reshape(-1)[:, None] * np.ones((1, s.N))
    act = c["phi"] <= 0
    for t in (0.0, 0.37):
        uc, _ = s.project(F, u, t=t)
        assert np.abs((uc - u)[:, act]).max() < 1e-13


def test_anchored_projection_moves_a_shifted_displacement(orc):
    """Control for the test above: the same affine field shifted by a
    constant no longer meets the anchors, and the projection pulls it back
    towards the prescribed values (the anchors act)."""
    rng = np.random.default_rng(11)
    G = 0.1 * rng.standard_normal((2, 2))
    a = 0.01 * rng.standard_normal(2)
    X0 = (0.4, 0.55)
    s, c = _annulus_mixed(orc, 0, G, a, X0)
    X = c["X"]
    u = G @ (X - np.array(X0)[:, None]) + a[:, None]
    F = (np.eye(2) + G).reshape(-1)[:, None] * np.ones((1, s.N))
    act = c["phi"] <= 0
    uc, _ = s.project(F, u + 0.01, t=0.0)
    # exact mode: anchors make K definite, the minimiser is the affine field
    assert np.abs((uc - u)[:, act]).max() < 1e-12
