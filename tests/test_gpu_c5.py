"""The differentiation configuration as configured, on the 32^3 copy of the
embedded sphere (FP64 GPU build, 60 steps: three projection steps).

Loss: L = 1/2 sum_{m in S} |u_m - u*_m|^2 over the surface nodes S (active
nodes with at least one cut link), u* the final displacement of a forward
run at mu* = 1.3, lambda* = 6.  The loss depends on the final state, so the
reverse mode runs in two calls: record the forward, form dL/du = u - u* on
S, run the backward pass.  Checks:
  - the GPU gradients dL/d(mu, lambda), dL/dv0 and dL/d dU0 equal the
    oracle's reverse mode on the same loss (1e-9 relative);
  - dL/dmu, dL/dlambda and the derivative along a smooth initial-velocity
    direction (v0 + h dv with the gradient data moving by h grad dv, so the
    initial state stays consistent) match central differences at h = 1e-3
    (relative steps) of FP64 forward runs to 1e-4 (the configured bar; FP64
    gives far better), for the FP64 and the FP32 reverse mode.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

STEPS = 60


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def setup():
    import torch
    from paper_2606_20646_amd import tlvlbm as T
    torch.cuda.set_device(0)
    c = W.config_c5(32)
    rng = np.random.default_rng(77)
    dv, ddv = W.fourier_velocity(c["X"], W.fourier_modes(rng, 3), 1e-2)
    return T, c, dv, ddv


def _gpu(T, c, precision, mu, lam, U0, dU0):
    s = T.Solver(3, c["n"], c["dx"], c["dt"], mu, lam, omega=c["omega"], origin=c["origin"], periodic_mask=0,
                 proj_every=c["proj_every"], precision=precision)
    s.set_levelset(c["phi"], c["bid"])
    s.set_boundary(1, "neumann")
    s.set_state(U0, dU0=dU0)
    return s


def _orc(orc, c, mu, lam, U0, dU0):
    o = orc.Sim(3, c["n"], c["dx"], c["dt"], mu, lam, omega=c["omega"], origin=c["origin"], periodic_mask=0,
                proj_every=c["proj_every"])
    o.set_levelset(c["phi"], c["bid"])
    o.set_bc(1, orc.NEUMANN)
    o.set_state(U0, dU0=dU0)
    return o


def _surface(c, links):
    S = np.zeros(c["phi"].size, bool)
    S[links["node"]] = True
    return S


def _target(orc, c):
    o = _orc(orc, c, 1.3, 6.0, c["U0"], c["dU0"])
    o.step(STEPS)
    return o.moments()[1]


def _dU(dU0, ddv):
    out = dU0.copy()
    out[:, :3] += ddv
    return out


@pytest.mark.parametrize("precision,tol_orc", [("fp64", 1e-9), ("fp32", 1e-4)])
def test_c5_loss_gradients(setup, orc, precision, tol_orc):
    T, c, dv, ddv = setup
    _say(f"c5 configured loss 32^3 {precision} {STEPS} steps")
    us = _target(orc, c)
    g = _gpu(T, c, precision, c["mu"], c["lam"], c["U0"], c["dU0"])
    S = _surface(c, g.links())
    g.adjoint_record(STEPS)
    u = g.moments()[1]
    gm, gv, _, gd = g.adjoint_backward(None, (u - us) * S, grad_u0=False, grad_dU0=True)
    # the oracle's reverse mode on its own forward and the same loss
    o = _orc(orc, c, c["mu"], c["lam"], c["U0"], c["dU0"])
    assert np.array_equal(_surface(c, o.links()), S)
    o.step(STEPS)
    uo = o.moments()[1]
    o = _orc(orc, c, c["mu"], c["lam"], c["U0"], c["dU0"])
    gm_o, gv_o, _, gd_o = o.adjoint(STEPS, None, (uo - us) * S, with_dU0=True)
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))  # noqa: E731
    print(f"mu,lam gpu {gm} oracle {gm_o}; v0 {rel(gv, gv_o):.2e}; dU0 {rel(gd, gd_o):.2e}", flush=True)
    assert np.all(np.abs(gm - gm_o) <= tol_orc * np.abs(gm_o).max())
    assert rel(gv, gv_o) <= tol_orc and rel(gd, gd_o) <= tol_orc

    # central differences of FP64 forward runs, h = 1e-3 (relative)
    def L(mu, lam, U0, dU0):
        s = _gpu(T, c, "fp64", mu, lam, U0, dU0)
        s.step(STEPS)
        uu = s.moments()[1]
        return 0.5 * float(np.sum(((uu - us) * S) ** 2))

    mu, lam = c["mu"], c["lam"]
    hm, hl = 1e-3 * mu, 1e-3 * lam
    fd_mu = (L(mu + hm, lam, c["U0"], c["dU0"]) - L(mu - hm, lam, c["U0"], c["dU0"])) / (2 * hm)
    fd_lam = (L(mu, lam + hl, c["U0"], c["dU0"]) - L(mu, lam - hl, c["U0"], c["dU0"])) / (2 * hl)
    h = 1e-3

    def Lv(t):
        U0 = c["U0"].copy()
        U0[:3] += t * dv
        return L(mu, lam, U0, _dU(c["dU0"], t * ddv))

    fd_v = (Lv(h) - Lv(-h)) / (2 * h)
    ad_v = float(np.sum(gv * dv) + np.sum(gd[:, :3] * ddv))
    errs = [abs(gm[0] - fd_mu) / abs(fd_mu), abs(gm[1] - fd_lam) / abs(fd_lam), abs(ad_v - fd_v) / abs(fd_v)]
    print(f"fd mu {fd_mu} lam {fd_lam} v {fd_v}; adjoint {gm[0]} {gm[1]} {ad_v}; rel {errs}", flush=True)
    assert max(errs) <= 1e-4
