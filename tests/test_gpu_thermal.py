"""GPU parity of the thermal stretch (the thermal distortion of the outlook's
thermoelasticity, Sec. 6: P(F) = th^(D-1) P_W(F / th) with a per-node
stretch th from the caller's temperature field), through the C ABI, against
the FP64 oracle.

- periodic 3D, F0 = I + 0.05 A with 8 Fourier velocity modes and a smooth
  non-uniform stretch set before the initialisation: state per part
  (tests/parity.py; FP64 1e-12 plus the rounding floor, FP32 1e-5) and the
  stresses of the final state;
- the embedded annulus (displacement-driven inner surface, traction-free
  outer surface, projection every 20 steps) heated radially after the
  initialisation, with the fibre family: the traction closure's Newton
  solve runs on the node's stretch;
- a traction-free disk under a uniform stretch relaxes to the exact
  stress-free expansion F = th I, u = (th - 1)(X - mean X) on the GPU as in
  the oracle;
- a field handed over from a device tensor every 40 steps, as a temperature
  solver would, against the oracle given the same fields;
- th = 1 everywhere is no stretch (to rounding: the stretched law is its own
  kernel instantiation); the calls that refuse a
  stretch (Maxwell branch, reverse mode) and non-positive values (batches
  with a stretch: tests/test_gpu_batch.py).
"""
import numpy as np
import pytest

import workloads as W
from parity import check
from test_gpu_visco import _stress_check

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def T():
    from paper_2606_20646_amd import tlvlbm
    return tlvlbm


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_thermal_periodic_3d(T, orc, precision, tol):
    c = W.config_c3(32)
    steps = 120
    X = W.node_coords(c["n"], c["dx"], c["origin"])
    th = 1.0 + 0.03 * np.sin(2 * np.pi * X[0]) * np.cos(2 * np.pi * X[1]) + 0.02 * np.cos(2 * np.pi * X[2])
    _say(f"thermal stretch periodic 32^3 {precision} {steps} steps")
    g = T.Solver(3, c["n"], c["dx"], c["dt"], c["mu"], c["lam"], omega=c["omega"], precision=precision)
    o = orc.Sim(3, c["n"], c["dx"], c["dt"], c["mu"], c["lam"], omega=c["omega"])
    g.set_thermal_stretch(th)
    o.set_thermal(th)
    for s in (g, o):
        s.set_state(c["U0"], dU0=c["dU0"])
        s.step(steps)
    Ug, _, _ = g.moments()
    Uo, _, _ = o.moments()
    check(Ug, Uo, 3, tol, label=f"thermal periodic 3D {precision}", pops=o.get_f(), steps=steps,
          stress=(c["mu"], c["lam"], 1.0, 10.0, c["omega"]))
    Pg, Sg = g.stress()
    Po, So = o.stress()
    _stress_check(Pg, Po, Sg, So, tol, np.ones(g.N, bool), f"thermal periodic 3D {precision}", o.get_f(), steps,
                  c["lam"] + 2 * c["mu"])


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_thermal_embedded_annulus_with_fibres(T, orc, precision, tol):
    from oracle import oracle as O
    c = W.config_c2(64)
    steps, k1, a0 = 300, 1.5, (0.6, 0.8)
    X = W.node_coords(c["n"], c["dx"], c["origin"])
    r = np.hypot(X[0] - 0.5, X[1] - 0.5)
    th = 1.0 + 0.04 * np.clip((r - 0.25) / 0.25, 0.0, 1.0)
    _say(f"thermal stretch annulus 64^2 with fibres {precision} {steps} steps")
    g = T.Solver(2, c["n"], c["dx"], c["dt"], c["mu"], c["lam"], omega=c["omega"], gamma=c["gamma"],
                 origin=c["origin"], periodic_mask=0, proj_every=c["proj_every"], precision=precision,
                 fibre=(k1, a0))
    o = O.Sim(2, c["n"], c["dx"], c["dt"], c["mu"], c["lam"], omega=c["omega"], gamma=c["gamma"],
              origin=c["origin"], periodic_mask=0, proj_every=c["proj_every"])
    o.set_fibres(k1, a0)
    kinds = {"dirichlet": O.DIRICHLET, "neumann": O.NEUMANN}
    ramps = {"const": O.RAMP_CONST, "sin2": O.RAMP_SIN2}
    g.set_levelset(c["phi"], c["bid"])
    o.set_levelset(c["phi"], c["bid"])
    for bid, bc in c["bcs"].items():
        bc = dict(bc)
        if "ramp" in bc:
            bc["T_r"] = 0.3
        gb = dict(bc)
        g.set_boundary(bid, gb.pop("type"), **gb)
        t = kinds[bc.pop("type")]
        if "ramp" in bc:
            bc["ramp"] = ramps[bc["ramp"]]
        o.set_bc(bid, t, **bc)
    for s in (g, o):
        s.set_state(c["U0"])
    # heated after the initialisation: the stretch takes effect at the next step
    g.set_thermal_stretch(th)
    o.set_thermal(th)
    for s in (g, o):
        s.step(steps)
    assert g.stats()["newton_failures"] == 0
    Ug, ug, _ = g.moments()
    Uo, uo, _ = o.moments()
    act = c["phi"] <= 0
    stiff_mu = c["mu"] + 2 * k1
    check(Ug[:, act], Uo[:, act], 2, tol, ug[:, act], uo[:, act], label=f"thermal annulus {precision}",
          pops=o.get_f()[:, :, act], steps=steps, stress=(stiff_mu, c["lam"], 1.0, c["c"], c["omega"]))
    Pg, Sg = g.stress()
    Po, So = o.stress()
    _stress_check(Pg, Po, Sg, So, tol, act, f"thermal annulus {precision}", o.get_f(), steps,
                  c["lam"] + 2 * stiff_mu)


def _disk(T, orc, th_field, steps, gpu=True):
    N = 32
    n, dx = N + 2, 1 / N
    X = (np.tile(np.arange(n), n) - 1 + 0.5) * dx
    Y = (np.repeat(np.arange(n), n) - 1 + 0.5) * dx
    phi = np.hypot(X - 0.5, Y - 0.5) - 0.3
    kw = dict(origin=(-dx, -dx), periodic_mask=0, gamma=10.0, proj_every=20)
    if gpu:
        s = T.Solver(2, (n, n), dx, dx / 10, 1.0, 2.0, precision="fp64", **kw)
        s.set_levelset(phi, np.ones(n * n, np.uint8))
        s.set_boundary(1, "neumann")
        if th_field is not None:
            s.set_thermal_stretch(th_field(n * n))
    else:
        s = orc.Sim(2, (n, n), dx, dx / 10, 1.0, 2.0, **kw)
        s.set_levelset(phi, np.ones(n * n, np.uint8))
        s.set_bc(1, orc.NEUMANN)
        if th_field is not None:
            s.set_thermal(th_field(n * n))
    U0 = np.zeros((6, n * n))
    U0[2] = U0[5] = 1.0
    s.set_state(U0)
    s.step(steps)
    return s, X, Y, phi <= 0


def test_thermal_free_disk_expands_stress_free(T, orc):
    th = 1.02
    _say("thermal stretch: free disk 32^2 fp64 1600 steps")
    g, X, Y, act = _disk(T, orc, lambda N: np.full(N, th), 1600)
    o, _, _, _ = _disk(T, orc, lambda N: np.full(N, th), 1600, gpu=False)
    Ug, ug, _ = g.moments()
    Uo, uo, _ = o.moments()
    Xa = np.stack([X[act], Y[act]])
    ue = (th - 1.0) * (Xa - Xa.mean(axis=1, keepdims=True))
    assert np.abs(Ug[2:, act] - th * np.array([1.0, 0.0, 0.0, 1.0])[:, None]).max() < 1e-11
    assert np.abs(Ug[:2, act]).max() < 1e-11
    assert np.abs(ug[:, act] - ue).max() < 1e-11
    assert np.abs(ug[:, act] - uo[:, act]).max() < 1e-12
    assert g.stats()["newton_failures"] == 0


def test_thermal_unit_stretch_and_refusals(T):
    _say("thermal stretch: unit field, refusals")
    a, _, _, _ = _disk(T, None, None, 60)
    b, _, _, _ = _disk(T, None, lambda N: np.ones(N), 60)
    fa, ua, _ = a.get_state()
    fb, ub, _ = b.get_state()
    # the stretched law runs in its own kernel instantiation, whose FMA
    # contraction may differ: equal to rounding (the oracle's pin is bitwise)
    print(f"[parity] unit stretch vs none: f {np.abs(fa - fb).max():.2e}, u* {np.abs(ua - ub).max():.2e}", flush=True)
    assert np.abs(fa - fb).max() <= 1e-14 * np.abs(fa).max()
    assert np.abs(ua - ub).max() <= 1e-14 * np.abs(ua).max()
    with pytest.raises(T.TlvlbmError) as e:
        b.set_thermal_stretch(np.zeros(b.N))
    assert e.value.code == T.ERR_INVALID_ARG
    bad = np.ones(b.N)
    bad[5] = np.nan
    with pytest.raises(T.TlvlbmError):
        b.set_thermal_stretch(bad)
    # no Maxwell branch on a stretched context, and no stretch on a branch
    with pytest.raises(T.TlvlbmError):
        b.set_material(1.0, 2.0, viscous=(0.5, 1.0))
    # no reverse mode
    with pytest.raises(T.TlvlbmError):
        b.adjoint(1, dLdu=np.zeros((2, b.N)))
    # removing the field restores the plain law
    b.set_thermal_stretch(None)
    b.step(1)
    v = T.Solver(2, (8, 8), 1 / 8, 1 / 80, 1.0, 2.0, precision="fp64", viscous=(0.5, 1.0))
    with pytest.raises(T.TlvlbmError):
        v.set_thermal_stretch(np.ones(64))


def test_thermal_field_updated_between_steps_from_device(T, orc):
    """the use the call is made for: a temperature solver advances the field
    and hands it over between steps, here as a device tensor every 40 steps
    (a heating front crossing a periodic 2D body), against the oracle given
    the same fields"""
    import torch
    c = W.config_c1()
    X = W.node_coords(c["n"], c["dx"], c["origin"])
    _say("thermal stretch updated every 40 steps from a device tensor, c1 2D fp64")
    g = T.Solver(2, c["n"], c["dx"], c["dt"], c["mu"], c["lam"], omega=c["omega"], precision="fp64")
    o = orc.Sim(2, c["n"], c["dx"], c["dt"], c["mu"], c["lam"], omega=c["omega"])
    for s in (g, o):
        s.set_state(c["U0"], dU0=c["dU0"])
    for k in range(6):
        front = 0.15 * (k + 1)
        th = 1.0 + 0.03 / (1.0 + np.exp(-(front - X[0]) / 0.05))
        g.set_thermal_stretch(torch.tensor(th, dtype=torch.float64, device="cuda"))
        o.set_thermal(th)
        g.step(40)
        o.step(40)
    Ug, _, _ = g.moments()
    Uo, _, _ = o.moments()
    check(Ug, Uo, 2, 1e-12, label="thermal field updates fp64", pops=o.get_f(), steps=240,
          stress=(c["mu"], c["lam"], 1.0, 10.0, c["omega"]))
    # the heated part has moved: the field did act
    g0 = T.Solver(2, c["n"], c["dx"], c["dt"], c["mu"], c["lam"], omega=c["omega"], precision="fp64")
    g0.set_state(c["U0"], dU0=c["dU0"])
    g0.step(240)
    U0, _, _ = g0.moments()
    assert np.abs(U0[:2] - Ug[:2]).max() > 1e-4
