"""Pins of the oracle's history-dependent law: one viscoelastic (Maxwell)
branch on top of the neo-Hookean solid (the extension that the paper's
outlook names as a local node update, Sec. 6).  The branch carries an
overstress Q in the second Piola stress, P = P_NH(F) + F Q, with

    dQ/dt + Q / tau = beta dS_0/dt,     S_0 = mu (I - C^{-1}),  C = F^T F,

so that Q(t) = beta int_0^t exp(-(t - s)/tau) dS_0/ds ds for a point that
starts relaxed.  The oracle advances Q once per lattice step.  Pinned here:

- the exact hereditary integral: along a prescribed smooth path F(t) the
  stepped overstress converges to the convolution (computed by adaptive
  quadrature) at second order in dt;
- the dissipation per cycle: in simple shear the branch is exactly linear
  (P_12 = mu gamma + Q_12), and over a steady cycle gamma = gamma0 sin(w t)
  the work done is pi gamma0^2 G'' with the loss modulus
  G'' = beta mu w tau / (1 + (w tau)^2); the in-phase part is the storage
  modulus G' = mu (1 + beta (w tau)^2 / (1 + (w tau)^2));
- relaxation to the elastic limit: with F held the overstress decays by
  exp(-dt / tau) per step exactly, and the stress tends to P_NH(F);
- the glassy (tau -> infinity) and relaxed (tau -> 0) limits: from an
  undeformed start the law is the neo-Hookean solid with shear modulus
  mu (1 + beta), resp. mu, along any path;
- the tangent at frozen history is the derivative of the stress map;
- in the full scheme: a branch with tau = infinity reproduces the
  neo-Hookean run at mu (1 + beta) (periodic, and the embedded annulus with
  traction-free surface and projection), tau = 0 the run at mu, and a damped
  body under a static load relaxes to the equilibrium of the elastic solid.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import workloads as W
from parity import check

MU, LAM = 1.0, 10.0


def _S0(F, mu=MU):
    return mu * (np.eye(F.shape[0]) - np.linalg.inv(F.T @ F))


def _dS0(F, dF, mu=MU):
    Ci = np.linalg.inv(F.T @ F)
    dC = dF.T @ F + F.T @ dF
    return mu * Ci @ dC @ Ci


def _path2(t):
    F = np.array([[1.0 + 0.2 * math.sin(t), 0.3 * (1.0 - math.cos(t))],
                  [0.1 * math.sin(2.0 * t), 1.0 - 0.1 * math.sin(t)]])
    dF = np.array([[0.2 * math.cos(t), 0.3 * math.sin(t)],
                   [0.2 * math.cos(2.0 * t), -0.1 * math.cos(t)]])
    return F, dF


def _path3(t):
    A = np.array([[0.2, 0.1, -0.05], [0.0, -0.1, 0.15], [0.05, 0.1, 0.1]])
    B = np.array([[0.0, 0.2, 0.0], [-0.1, 0.0, 0.05], [0.0, 0.1, -0.15]])
    F = np.eye(3) + A * math.sin(t) + B * (1.0 - math.cos(1.5 * t))
    dF = A * math.cos(t) + B * 1.5 * math.sin(1.5 * t)
    return F, dF


def _q_exact(path, t, beta, tau):
    """beta int_0^t exp(-(t - s)/tau) dS_0/ds ds by adaptive quadrature"""
    def integrand(s):
        F, dF = path(s)
        return (math.exp(-(t - s) / tau) * beta * _dS0(F, dF)).ravel()
    val, err = integrate.quad_vec(integrand, 0.0, t, epsabs=1e-14, epsrel=1e-13)
    return val.reshape(_path2(0)[0].shape if path is _path2 else (3, 3))


def _overstress(orc, Fs, beta, tau, dt):
    """Q^k of the stepped law along Fs, from P = P_NH + F Q"""
    P = orc.visco_path(Fs, MU, LAM, beta, tau, dt)
    return np.stack([np.linalg.solve(F, Pk - orc.piola(F, MU, LAM)) for F, Pk in zip(Fs, P)])


@pytest.mark.parametrize("D", [2, 3])
def test_stepped_overstress_converges_to_hereditary_integral(orc, D):
    path = _path2 if D == 2 else _path3
    beta, tau, T = 1.5, 0.4, 2.0
    marks = (0.5, 1.0, 2.0)
    exact = {t: _q_exact(path, t, beta, tau) for t in marks}
    scale = max(np.abs(q).max() for q in exact.values())
    errs = []
    for n in (100, 200, 400):
        dt = T / n
        Fs = np.stack([path(k * dt)[0] for k in range(n + 1)])
        Q = _overstress(orc, Fs, beta, tau, dt)
        e = max(np.abs(Q[int(round(t / dt))] - exact[t]).max() for t in marks) / scale
        errs.append(e)
    print(f"D={D} relative overstress error vs dt: {errs}")
    # second order: halving dt divides the error by ~4
    assert errs[0] < 1e-3
    for a, b in zip(errs, errs[1:]):
        assert 3.6 < a / b < 4.4


def test_dissipation_per_cycle_is_the_loss_modulus(orc):
    beta, tau, w, g0 = 2.0, 0.5, 2.0, 0.01
    period = 2.0 * math.pi / w
    nper = 4000
    dt = period / nper
    ncyc = 12  # 12 periods = 75 tau: the start-up transient is gone
    n = ncyc * nper
    t = np.arange(n + 1) * dt
    g = g0 * np.sin(w * t)
    Fs = np.zeros((n + 1, 2, 2))
    Fs[:, 0, 0] = Fs[:, 1, 1] = 1.0
    Fs[:, 0, 1] = g
    P = orc.visco_path(Fs, MU, LAM, beta, tau, dt)
    # simple shear keeps J = 1 and S_0,12 = mu gamma, S_0,22 = 0: P_12 is
    # exactly mu gamma + Q_12 with Q_12 linear in the history of gamma
    last = slice(n - nper, n + 1)
    P12, gl, tl = P[last, 0, 1], g[last], t[last]
    work = np.sum(0.5 * (P12[1:] + P12[:-1]) * np.diff(gl))
    wt = w * tau
    Gpp = beta * MU * wt / (1.0 + wt * wt)
    Gp = MU * (1.0 + beta * wt * wt / (1.0 + wt * wt))
    assert abs(work / (math.pi * g0 * g0 * Gpp) - 1.0) < 1e-5
    # first harmonic of P_12 = g0 (G' sin + G'' cos)
    wts = np.full(nper + 1, 1.0)
    wts[0] = wts[-1] = 0.5
    s_part = 2.0 / nper * np.sum(wts * P12 * np.sin(w * tl)) / g0
    c_part = 2.0 / nper * np.sum(wts * P12 * np.cos(w * tl)) / g0
    assert abs(s_part / Gp - 1.0) < 1e-5
    assert abs(c_part / Gpp - 1.0) < 1e-5
    # the elastic solid dissipates nothing over the same cycle
    P0 = orc.visco_path(Fs, MU, LAM, 0.0, tau, dt)
    assert abs(np.sum(0.5 * (P0[last, 0, 1][1:] + P0[last, 0, 1][:-1]) * np.diff(gl))) < 1e-12 * work / Gpp


@pytest.mark.parametrize("D", [2, 3])
def test_relaxation_to_the_elastic_limit(orc, D):
    beta, tau, dt = 1.0, 0.2, 0.01
    path = _path2 if D == 2 else _path3
    nramp, nhold = 100, 400
    Fs = [path(k * dt)[0] for k in range(nramp + 1)]
    Fs += [Fs[-1]] * nhold
    Fs = np.stack(Fs)
    P = orc.visco_path(Fs, MU, LAM, beta, tau, dt)
    Pel = orc.piola(Fs[-1], MU, LAM)
    over = P[nramp:] - Pel  # F Q, with F fixed
    ratio = over[2:] / over[1:-1]
    # (where the overstress is well above the rounding of P ~ 1)
    mask = np.abs(over[1:-1]) > 1e-4 * np.abs(over[1]).max()
    assert mask.sum() > 100
    assert np.allclose(ratio[mask], math.exp(-dt / tau), rtol=1e-9, atol=0)
    assert np.abs(over[-1]).max() < 1e-8 * np.abs(over[0]).max()
    assert np.abs(over[0]).max() > 1e-2  # the branch did carry stress at the end of the ramp


@pytest.mark.parametrize("D", [2, 3])
def test_glassy_and_relaxed_limits(orc, D):
    beta, dt = 0.7, 0.01
    path = _path2 if D == 2 else _path3
    Fs = np.stack([np.eye(D)] + [path(k * dt)[0] for k in range(1, 200)])
    Pg = orc.visco_path(Fs, MU, LAM, beta, math.inf, dt)
    Pr = orc.visco_path(Fs, MU, LAM, beta, 0.0, dt)
    for F, a, b in zip(Fs, Pg, Pr):
        ref_g = orc.piola(F, MU * (1.0 + beta), LAM)
        assert np.abs(a - ref_g).max() <= 1e-13 * np.abs(ref_g).max()
        ref_r = orc.piola(F, MU, LAM)
        assert np.abs(b - ref_r).max() <= 1e-14 * np.abs(ref_r).max()


@pytest.mark.parametrize("D", [2, 3])
def test_tangent_is_derivative_of_the_stress_map(orc, D):
    rng = np.random.default_rng(7)
    for _ in range(6):
        F = np.eye(D) + 0.25 * rng.standard_normal((D, D))
        if np.linalg.det(F) < 0.3:
            continue
        Qh = rng.standard_normal((D, D))
        Qh = 0.5 * (Qh + Qh.T)
        S0h = _S0(np.eye(D) + 0.2 * rng.standard_normal((D, D)))
        beta, xi = 1.3, 0.9
        dF = rng.standard_normal((D, D))
        jvp = orc.visco_piola_jvp(F, dF, MU, LAM, beta, xi, Qh, S0h)

        def fd(h):
            return (orc.visco_piola(F + h * dF, MU, LAM, beta, xi, Qh, S0h)
                    - orc.visco_piola(F - h * dF, MU, LAM, beta, xi, Qh, S0h)) / (2 * h)
        rich = (4.0 * fd(1e-4) - fd(2e-4)) / 3.0
        assert np.abs(jvp - rich).max() <= 1e-8 * np.abs(jvp).max()
        # the overstress part alone is beta xi F dS_0 + dF Q
        Q = xi * xi * Qh + beta * xi * (_S0(F) - S0h)
        d_el = orc.piola_jvp(F, dF, MU, LAM)
        ref = dF @ Q + beta * xi * F @ _dS0(F, dF)
        assert np.abs(jvp - d_el - ref).max() <= 1e-12 * np.abs(jvp).max()


# ------------------------------------------------------------------ scheme --

def _periodic(orc, D, N, mu, steps, visco=None, gamma=0.0, body=None):
    case = W.periodic_case(D, N, lambda rng: np.eye(D), 2e-2)
    dx = case["dx"]
    o = orc.Sim(D, case["n"], dx, dx / 10.0, mu, LAM, omega=1.8, gamma=gamma, periodic_mask=(1 << D) - 1)
    if visco is not None:
        o.set_viscous(*visco)
    if body is not None:
        o.set_body_force(body(case), ramp=orc.RAMP_SIN2, T_r=0.5)
    o.set_state(case["U0"], dU0=case["dU0"])
    o.step(steps)
    return o


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _close(a, b, Ua, Ub, steps, mu, c, mask=None):
    """runs a and b agree per part (v, F - I) to 1e-12 of the part's size
    plus the FP64 rounding floor of b's populations and stress"""
    D = 2 if Ua.shape[0] == 6 else 3
    pops = b.get_f()
    if mask is not None:
        Ua, Ub, pops = Ua[:, mask], Ub[:, mask], pops[:, :, mask]
    e = check(Ua, Ub, D, 1e-12, pops=pops, steps=steps, stress=(mu, LAM, 1.0, c, 1.8), label="visco vs NH")
    return e


def test_scheme_glassy_and_relaxed_limits_periodic(orc):
    beta = 0.5
    ref_g = _periodic(orc, 2, 24, MU * (1 + beta), 300)
    vis_g = _periodic(orc, 2, 24, MU, 300, visco=(beta, math.inf))
    ref_r = _periodic(orc, 2, 24, MU, 300)
    vis_r = _periodic(orc, 2, 24, MU, 300, visco=(beta, 0.0))
    Ug, Ur = ref_g.moments()[0], ref_r.moments()[0]
    Vg, Vr = vis_g.moments()[0], vis_r.moments()[0]
    I = np.eye(2).reshape(-1)[:, None]
    # glassy: the same law up to the rounding of P_NH(mu) + F beta S_0
    # against P_NH(mu (1 + beta))
    _close(vis_g, ref_g, Vg, Ug, 300, MU * (1 + beta), 10.0)
    # relaxed: the overstress is exactly zero
    assert np.array_equal(Vr, Ur)
    # and the two moduli do give different runs
    assert _rel(Ug[:2], Ur[:2]) > 1e-2
    # the stress of the current state carries the branch: equal to the
    # glassy solid's
    # (the states differ by rounding, carried to the stress at the
    # stiffness lambda + 2 mu (1 + beta))
    Pg, Sg = ref_g.stress()
    Pv, Sv = vis_g.stress()
    stiff = LAM + 2 * MU * (1 + beta)
    dF = np.abs(Vg[2:] - Ug[2:]).max()
    assert np.abs(Pv - Pg).max() < 2 * stiff * dF + 1e-12 * np.abs(Pg).max()
    assert np.abs(Sv - Sg).max() < 2 * stiff * dF + 1e-12 * np.abs(Sg).max()
    assert np.abs(Sg).max() > 1e-3


def test_scheme_glassy_limit_embedded_annulus(orc):
    """traction-free outer surface (Newton solve with the node's history),
    displacement-driven inner surface, projection with repair every 20 steps"""
    from oracle import oracle as O
    c = W.config_c2(32)
    beta = 0.8
    kinds = {"dirichlet": O.DIRICHLET, "neumann": O.NEUMANN}
    ramps = {"const": O.RAMP_CONST, "sin2": O.RAMP_SIN2}

    def run(mu, visco):
        o = O.Sim(2, c["n"], c["dx"], c["dt"], mu, c["lam"], omega=c["omega"], gamma=c["gamma"],
                  origin=c["origin"], periodic_mask=0, proj_every=c["proj_every"])
        o.set_levelset(c["phi"], c["bid"])
        for bid, bc in c["bcs"].items():
            bc = dict(bc)
            t = kinds[bc.pop("type")]
            if "ramp" in bc:
                bc["ramp"] = ramps[bc["ramp"]]
            bc["T_r"] = 0.3
            o.set_bc(bid, t, **bc)
        if visco:
            o.set_viscous(*visco)
        o.set_state(c["U0"])
        o.step(400)
        assert o.stats()["newton_fail"] == 0
        return o

    ref, vis = run(c["mu"] * (1 + beta), None), run(c["mu"], (beta, math.inf))
    (Ur, ur, _), (Uv, uv, _) = ref.moments(), vis.moments()
    act = c["phi"] <= 0
    e = _close(vis, ref, Uv, Ur, 400, c["mu"] * (1 + beta), c["c"], act)
    assert _rel(uv[:, act], ur[:, act]) < 1e-12 + 4 * max(e["v_floor"], e["F_floor"])
    # the glassy body is stiffer than the relaxed one
    Un, un, _ = run(c["mu"], None).moments()
    assert _rel(un[:, act], ur[:, act]) > 1e-3


def test_scheme_relaxes_to_the_elastic_equilibrium(orc):
    """a damped periodic body under a ramped static load: the branch carries
    stress while the load changes and none at rest, so the viscoelastic body
    settles on the elastic body's steady state (v and F; the displacement
    drifts with the scheme's steady O(dx) velocity, alike in both)"""
    def body(case):
        X = W.node_coords(case["n"], case["dx"], case["origin"])
        g = np.zeros_like(X)
        g[0] = 2.0 * np.sin(2 * np.pi * X[1])
        g[1] = 1.0 * np.cos(2 * np.pi * X[0])
        return g

    N, gam = 16, 10.0
    dt = 1.0 / N / 10.0
    I = np.eye(2).reshape(-1)[:, None]
    out = []
    for t in (1.0, 4.0):
        steps = int(round(t / dt))
        e = _periodic(orc, 2, N, MU, steps, gamma=gam, body=body)
        v = _periodic(orc, 2, N, MU, steps, visco=(2.0, 0.05), gamma=gam, body=body)
        Ue, Uv = e.moments()[0], v.moments()[0]
        Qh, _ = v.viscous_history()
        out.append((_rel(Uv[2:] - I, Ue[2:] - I), _rel(Uv[:2], Ue[:2]), np.abs(Qh).max()))
    (f1, v1, q1), (f4, v4, q4) = out
    print(f"visco vs elastic: t=1 F {f1:.2e} v {v1:.2e} |Q| {q1:.2e}; t=4 F {f4:.2e} v {v4:.2e} |Q| {q4:.2e}")
    assert f1 > 1e-3 and q1 > 1e-3  # the branch does delay the approach
    assert f4 < 1e-4 * f1 and v4 < 1e-4 * v1 and q4 < 1e-4 * q1
