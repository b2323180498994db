"""Pins of the oracle's reverse mode (project extension; the paper has no
adjoint) against central finite differences of the forward oracle.

For L = sum dLdU . U + dLdu . u over the moments after n steps, the adjoint
gradients dL/dmu, dL/dlambda, dL/dv0 . dv and dL/du0 . du must agree with
Richardson-extrapolated central differences (error O(h^4)) of L computed by
rerunning the forward oracle.  The cases are chosen so that each part of the
step carries weight in some of them: periodic bulk with damping (collision,
streaming, recovery), Dirichlet-only embedded (Dirichlet closure), Neumann
with and without projection (LSQ, Newton implicit function theorem, the
projection's Jacobi sweeps, or its exact CG solve and gauge, the repair), a
3D sphere, and the fibre-reinforced law in 2D and 3D.
"""
import numpy as np
import pytest

import workloads as W
from oracle import oracle as O


def _make(cfg, mu, lam):
    o = O.Sim(cfg["D"], cfg["n"], cfg["dx"], cfg["dt"], mu, lam, omega=cfg["omega"], gamma=cfg["gamma"],
              origin=cfg.get("origin"), periodic_mask=cfg.get("pm"), proj_every=cfg.get("proj_every", 20),
              proj_sweeps=cfg.get("proj_sweeps", 20))
    if cfg.get("fibre"):
        o.set_fibres(*cfg["fibre"])
    if "phi" in cfg:
        o.set_levelset(cfg["phi"], cfg["bid"])
        kinds = {"dirichlet": O.DIRICHLET, "neumann": O.NEUMANN}
        ramps = {"const": O.RAMP_CONST, "sin2": O.RAMP_SIN2}
        for bid, bc in cfg["bcs"].items():
            bc = dict(bc)
            t = kinds[bc.pop("type")]
            if "ramp" in bc:
                bc["ramp"] = ramps[bc["ramp"]]
            o.set_bc(bid, t, **bc)
    return o


def _loss(cfg, mu, lam, U0, u0, n, wU, wu, dU0=None):
    o = _make(cfg, mu, lam)
    o.set_state(U0, u0=u0, dU0=cfg.get("dU0") if dU0 is None else dU0)
    o.step(n)
    U, u, _ = o.moments()
    return float(np.sum(wU * U) + np.sum(wu * u))


def _richardson(fun, h):
    d1 = (fun(h) - fun(-h)) / (2 * h)
    d2 = (fun(h / 2) - fun(-h / 2)) / h
    return (4 * d2 - d1) / 3


def _disk(pe, neumann_only, N=16):
    g = W.framed_box(N, 2)
    X = W.node_coords(g["n"], g["dx"], g["origin"])
    phi, bid = W.annulus_phi(X, (0.5, 0.5), 0.25, 0.45)
    rng = np.random.default_rng(3)
    v, dv = W.fourier_velocity(X, W.fourier_modes(rng, 2), 1e-2)
    U0, dU0 = W.state_from(v, dv, np.eye(2) + 0.02 * rng.standard_normal((2, 2)))
    if neumann_only:
        bcs = {1: dict(type="neumann"), 2: dict(type="neumann", p_normal=0.01)}
    else:
        bcs = {1: dict(type="dirichlet", a=(0.001, 0.0)),
               2: dict(type="dirichlet", ramp="sin2", T_r=0.05, p_radial=0.01, X0=(0.5, 0.5))}
    return dict(g, D=2, pm=0, phi=phi, bid=bid, bcs=bcs, mu=1.0, lam=3.0, dt=g["dx"] / 10, omega=1.8,
                gamma=0.3, proj_every=pe, U0=U0, dU0=dU0, u0=1e-3 * rng.standard_normal((2, X.shape[1])))


def _periodic(D, N, omega, gamma):
    c = W.periodic_case(D, N, lambda rng: np.eye(D) + 0.05 * rng.standard_normal((D, D)), 1e-2, 7)
    return dict(c, D=D, mu=1.0, lam=2.0, dt=c["dx"] / 10, omega=omega, gamma=gamma)


def _sphere():
    c = W.config_c5(10)
    c["proj_every"] = 3
    c["u0"] = 1e-3 * np.random.default_rng(5).standard_normal((3, c["U0"].shape[1]))
    return dict(c, pm=0)


CASES = {
    "periodic2d_damped": (lambda: _periodic(2, 8, 1.8, 0.5), 10),
    "periodic3d": (lambda: _periodic(3, 4, 1.7, 0.0), 6),
    "dirichlet_annulus": (lambda: _disk(4, False), 9),
    "neumann_annulus_projection": (lambda: _disk(4, True), 9),
    "neumann_annulus_no_projection": (lambda: _disk(0, True), 9),
    "neumann_sphere_projection": (_sphere, 7),
    # the projection solved exactly instead of relaxed by Jacobi sweeps
    "neumann_annulus_projection_exact": (lambda: dict(_disk(4, True), proj_sweeps=0), 9),
    "neumann_sphere_projection_exact": (lambda: dict(_sphere(), proj_sweeps=0), 7),
    # the fibre-reinforced law (anisotropic stress and tangent everywhere)
    "neumann_annulus_fibres": (lambda: dict(_disk(4, True), fibre=(0.6, (0.8, 0.6))), 9),
    "neumann_sphere_fibres": (lambda: dict(_sphere(), fibre=(0.5, (0.0, 0.6, 0.8))), 7),
}


@pytest.mark.parametrize("name", list(CASES))
def test_adjoint_matches_finite_differences(name):
    make, n = CASES[name]
    cfg = make()
    rng = np.random.default_rng(11)
    D, N = cfg["D"], int(np.prod(cfg["n"]))
    M = D + D * D
    act = (cfg["phi"] <= 0).reshape(-1) if "phi" in cfg else np.ones(N, bool)
    U0 = cfg["U0"]
    u0 = cfg.get("u0", np.zeros((D, N)))
    wU = rng.standard_normal((M, N)) * act
    wu = rng.standard_normal((D, N)) * act
    dv = rng.standard_normal((D, N)) * act
    du = rng.standard_normal((D, N)) * act
    dd = rng.standard_normal((D, M, N)) * act
    dU0 = cfg.get("dU0", np.zeros((D, M, N)))
    mu, lam = cfg["mu"], cfg["lam"]
    o = _make(cfg, mu, lam)
    o.set_state(U0, u0=u0, dU0=cfg.get("dU0"))
    gm, gv, g0, gd = o.adjoint(n, wU, wu, with_dU0=True)
    assert o.stats()["step"] == n
    # the adjoint call leaves the forward state at step n
    U, u, _ = o.moments()
    assert abs(float(np.sum(wU * U) + np.sum(wu * u)) - _loss(cfg, mu, lam, U0, u0, n, wU, wu)) < 1e-13 * (
        np.abs(wU * U).sum() + np.abs(wu * u).sum())

    def L_v(h):
        U = U0.copy()
        U[:D] += h * dv
        return _loss(cfg, mu, lam, U, u0, n, wU, wu)

    checks = [
        ("mu", lambda h: _loss(cfg, mu + h, lam, U0, u0, n, wU, wu), gm[0], 1e-3 * mu),
        ("lambda", lambda h: _loss(cfg, mu, lam + h, U0, u0, n, wU, wu), gm[1], 1e-3 * lam),
        ("v0", L_v, float(np.sum(gv * dv)), 1e-3),
        ("u0", lambda h: _loss(cfg, mu, lam, U0, u0 + h * du, n, wU, wu), float(np.sum(g0 * du)), 1e-5),
        # the initial gradient data enter the second-order initialisation
        # (Eqs. 32-33) linearly
        ("dU0", lambda h: _loss(cfg, mu, lam, U0, u0, n, wU, wu, dU0 + h * dd), float(np.sum(gd * dd)), 1e-3),
    ]
    for what, fun, ad, h in checks:
        fd = _richardson(fun, h)
        scale = max(abs(fd), 1e-9 * abs(gm).sum(), 1e-12)
        assert abs(ad - fd) <= 1e-6 * scale, (what, ad, fd)


def test_adjoint_requires_fresh_state():
    cfg = _periodic(2, 4, 1.8, 0.0)
    o = _make(cfg, 1.0, 2.0)
    o.set_state(cfg["U0"], dU0=cfg["dU0"])
    o.step(1)
    with pytest.raises(O.OracleError):
        o.adjoint(2, np.ones((6, 16)))
