"""Body acceleration (Sec. 2.1, Eq. 5) on the GPU path against the oracle.

- Manufactured finite-strain plane wave (tests/refsol.PlaneWaveMMS) with the
  body acceleration updated before every step: GPU = oracle (FP64 1e-12,
  FP32 1e-5 relative), and the GPU errors against the exact solution fall at
  second order at omega = 2 (as the oracle's do).
- Embedded annulus with a ramped constant body acceleration, clamp,
  traction-free surface and projection: GPU = oracle (FP64).
- A context with a body acceleration cannot join a batch nor run the reverse
  mode (error, no silent fallback).
"""
import numpy as np
import pytest

import refsol
import workloads as W
from parity import check

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def T():
    import torch
    from paper_2606_20646_amd import tlvlbm
    torch.cuda.set_device(0)
    return tlvlbm


def _mms(D):
    if D == 2:
        return refsol.PlaneWaveMMS(2, (1, 1), (1, 0.3), 0.02, 2 * np.pi, 1.0, 2.0)
    return refsol.PlaneWaveMMS(3, (1, 0, 1), (1, 0.4, -0.2), 0.02, 2 * np.pi, 1.0, 2.0)


def _run_mms(sim, m, X, dt, nst):
    sim.set_body_force(m.body(X, 0.0))
    U0, u0 = m.fields(X, 0.0)
    sim.set_state(U0, u0=u0, dU0=m.gradients(X, 0.0))
    for it in range(nst):
        sim.set_body_force(m.body(X, it * dt))
        sim.step(1)
    U, u, _ = sim.moments()
    return U, u


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_manufactured_wave_matches_oracle(T, orc, precision, tol):
    D, N = 2, 32
    m = _mms(D)
    dx = 1 / N
    dt = dx / 10
    X = W.node_coords([N] * D, dx, [0.0] * D)
    _say(f"manufactured wave {N}^2 {precision} 64 steps")
    g = T.Solver(D, [N] * D, dx, dt, 1.0, 2.0, omega=2.0, precision=precision, track_u=1)
    Ug, ug = _run_mms(g, m, X, dt, 64)
    o = orc.Sim(D, [N] * D, dx, dt, 1.0, 2.0, omega=2.0)
    Uo, uo = _run_mms(o, m, X, dt, 64)
    check(Ug, Uo, D, tol, ug, uo, label=f"manufactured wave {precision}", pops=o.get_f(), steps=64,
          stress=(1.0, 2.0, 1.0, 10.0, 2.0))


@pytest.mark.parametrize("D,Ns", [(2, (32, 64, 128)), (3, (16, 32))])
def test_manufactured_wave_second_order(T, D, Ns):
    m = _mms(D)
    errs = []
    for N in Ns:
        _say(f"manufactured wave order D={D} N={N} fp64")
        dx = 1 / N
        dt = dx / 10
        X = W.node_coords([N] * D, dx, [0.0] * D)
        g = T.Solver(D, [N] * D, dx, dt, 1.0, 2.0, omega=2.0, precision="fp64", track_u=1)
        nst = int(round(0.2 / dt))
        U, u = _run_mms(g, m, X, dt, nst)
        g.close()
        Ue, ue = m.fields(X, nst * dt)
        Fi = np.eye(D).reshape(-1)[:, None]
        errs.append(np.array([np.linalg.norm(U[:D] - Ue[:D]) / np.linalg.norm(Ue[:D]),
                              np.linalg.norm(U[D:] - Ue[D:]) / np.linalg.norm(Ue[D:] - Fi),
                              np.linalg.norm(u - ue) / np.linalg.norm(ue)]))
    print(errs, flush=True)
    for e0, e1 in zip(errs, errs[1:]):
        assert np.all(np.log2(e0 / e1) > 1.85), errs


def test_embedded_ramped_body_force_matches_oracle(T, orc):
    c = W.config_c2(48)
    N = c["X"].shape[1]
    gfield = np.vstack([0.05 * np.ones(N), -0.03 * np.ones(N)])
    kw = dict(omega=c["omega"], gamma=c["gamma"], origin=c["origin"], periodic_mask=0, proj_every=20)
    g = T.Solver(2, c["n"], c["dx"], c["dt"], c["mu"], c["lam"], precision="fp64", **kw)
    o = orc.Sim(2, c["n"], c["dx"], c["dt"], c["mu"], c["lam"], **kw)
    for s in (g, o):
        s.set_levelset(c["phi"], c["bid"])
    g.set_boundary(1, "dirichlet")
    g.set_boundary(2, "neumann")
    o.set_bc(1, orc.DIRICHLET)
    o.set_bc(2, orc.NEUMANN)
    g.set_body_force(gfield, ramp="sin2", T_r=0.02)
    o.set_body_force(gfield, ramp=orc.RAMP_SIN2, T_r=0.02)
    _say("annulus 48 fp64 ramped body force 90 steps")
    for s in (g, o):
        s.set_state(c["U0"])
        s.step(90)
    Ug, ug, _ = g.moments()
    Uo, uo, _ = o.moments()
    act = c["phi"] <= 0
    check(Ug, Uo, 2, 1e-12, ug, uo, mask=act, label="annulus 48 ramped body force fp64", pops=o.get_f(), steps=90,
          stress=(c["mu"], c["lam"], 1.0, 10.0, c["omega"]))
    assert np.abs(Uo[:2, act]).max() > 1e-4  # the body acceleration moved the body


def test_body_force_excludes_reverse_mode(T):
    import torch
    stream = torch.cuda.Stream()
    c = W.config_c4_instance(0, N=40)
    s = T.Solver(2, c["n"], c["dx"], c["dt"], c["mu"], c["lam"], omega=c["omega"], gamma=c["gamma"],
                 origin=c["origin"], periodic_mask=0, precision="fp64", track_u=1, stream=stream.cuda_stream)
    s.set_levelset(c["phi"], c["bid"])
    for bid, bc in c["bcs"].items():
        bc = dict(bc)
        s.set_boundary(bid, bc.pop("type"), **bc)
    s.set_body_force(np.ones((2, s.N)) * 0.01)
    s.set_state(c["U0"])
    with pytest.raises(T.TlvlbmError):
        s.adjoint(3, np.ones((6, s.N)))


FIBRE = (0.8, (np.cos(0.5), np.sin(0.5)))


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_fibre_law_manufactured_wave_matches_oracle(T, orc, precision, tol):
    """The fibre-reinforced law (law 1) through the whole bulk path: the
    manufactured wave of that law, GPU = oracle."""
    D, N = 2, 32
    m = refsol.PlaneWaveMMS(2, (1, 1), (1, 0.3), 0.02, 2 * np.pi, 1.0, 2.0, fibre=(FIBRE[0], np.array(FIBRE[1])))
    dx = 1 / N
    dt = dx / 10
    X = W.node_coords([N] * D, dx, [0.0] * D)
    _say(f"fibre-law manufactured wave {N}^2 {precision} 64 steps")
    g = T.Solver(D, [N] * D, dx, dt, 1.0, 2.0, omega=2.0, precision=precision, track_u=1, fibre=FIBRE)
    Ug, ug = _run_mms(g, m, X, dt, 64)
    o = orc.Sim(D, [N] * D, dx, dt, 1.0, 2.0, omega=2.0)
    o.set_fibres(*FIBRE)
    Uo, uo = _run_mms(o, m, X, dt, 64)
    check(Ug, Uo, D, tol, ug, uo, label=f"manufactured wave {precision}", pops=o.get_f(), steps=64,
          stress=(1.0, 2.0, 1.0, 10.0, 2.0))
    Ue, _ = m.fields(X, 64 * dt)
    assert np.linalg.norm(Ug[:D] - Ue[:D]) <= 0.02 * np.linalg.norm(Ue[:D])
