"""Pins of the oracle's body acceleration (Sec. 2.1, Eq. 5; the source
B = (b - gamma v, 0) of Eqs. 12 and 28-33).

- Spatially uniform fields: with no gradients the update reduces, per node,
  to the trapezoidal rule for v' = s(t) b - gamma v (the half-step source of
  Eq. 28 with the damping implicit) and u' = v (Eq. 34); the oracle must
  reproduce that recursion to round-off, for constant and ramped s(t).
- Manufactured finite-strain plane wave (tests/refsol.PlaneWaveMMS): with
  the body acceleration b = dv/dt - Div P(F) the exact u(X, t) is a solution;
  at omega = 2 the errors in v, F and u fall at second order (the
  second-order initialisation of Eqs. 32-33 carries b(X, 0)); at
  omega = 1.8 they fall at first order (the BGK relaxation adds O(dx)
  numerical diffusion at fixed c).
"""
import numpy as np
import pytest

import refsol
import workloads as W


@pytest.mark.parametrize("D", [2, 3])
@pytest.mark.parametrize("gamma", [0.0, 0.7])
@pytest.mark.parametrize("ramp", ["const", "sin2"])
def test_uniform_body_acceleration_is_the_trapezoidal_rule(orc, D, gamma, ramp):
    n = [6] * D
    N = int(np.prod(n))
    dx = 1 / 6
    dt = dx / 10
    Tr = 0.05
    rmp = {"const": orc.RAMP_CONST, "sin2": orc.RAMP_SIN2}[ramp]
    s = orc.Sim(D, n, dx, dt, 1.0, 2.0, omega=1.8, gamma=gamma)
    b = np.array([0.3, -0.2, 0.45][:D])
    s.set_body_force(b[:, None] * np.ones((1, N)), ramp=rmp, T_r=Tr)
    M = D + D * D
    U0 = np.zeros((M, N))
    U0[D:] = np.eye(D).reshape(-1)[:, None]
    s.set_state(U0)
    nst = 37
    s.step(nst)
    U, u, _ = s.moments()

    def sc(t):
        return 1.0 if ramp == "const" or t >= Tr else np.sin(np.pi * t / (2 * Tr)) ** 2
    v = np.zeros(D)
    uu = np.zeros(D)
    for k in range(nst):
        vn = (v * (1 - 0.5 * gamma * dt) + 0.5 * dt * (sc(k * dt) + sc((k + 1) * dt)) * b) / (1 + 0.5 * gamma * dt)
        uu = uu + 0.5 * dt * (v + vn)
        v = vn
    assert np.abs(U[:D] - v[:, None]).max() < 1e-15
    assert np.abs(u - uu[:, None]).max() < 1e-15
    assert np.abs(U[D:] - U0[D:]).max() < 1e-14


def _mms_errors(orc, D, N, omega, k, p, T=0.2, a=0.02, mu=1.0, lam=2.0, c=10.0):
    m = refsol.PlaneWaveMMS(D, k, p, a, 2 * np.pi, mu, lam)
    n = [N] * D
    dx = 1 / N
    dt = dx / c
    X = W.node_coords(n, dx, [0.0] * D)
    s = orc.Sim(D, n, dx, dt, mu, lam, omega=omega)
    U0, u0 = m.fields(X, 0.0)
    s.set_body_force(m.body(X, 0.0))
    s.set_state(U0, u0=u0, dU0=m.gradients(X, 0.0))
    nst = int(round(T / dt))
    for it in range(nst):
        s.set_body_force(m.body(X, it * dt))
        s.step(1)
    U, u, _ = s.moments()
    Ue, ue = m.fields(X, nst * dt)
    Fi = np.eye(D).reshape(-1)[:, None]
    return np.array([np.linalg.norm(U[:D] - Ue[:D]) / np.linalg.norm(Ue[:D]),
                     np.linalg.norm(U[D:] - Ue[D:]) / np.linalg.norm(Ue[D:] - Fi),
                     np.linalg.norm(u - ue) / np.linalg.norm(ue)])


@pytest.mark.parametrize("D,Ns,k,p", [(2, (16, 32, 64), (1, 1), (1, 0.3)),
                                      (3, (16, 32), (1, 0, 1), (1, 0.4, -0.2))])
def test_manufactured_plane_wave_second_order(orc, D, Ns, k, p):
    errs = [_mms_errors(orc, D, N, 2.0, k, p) for N in Ns]
    for e0, e1 in zip(errs, errs[1:]):
        order = np.log2(e0 / e1)
        assert np.all(order > 1.85), (errs, order)
    assert np.all(errs[-1] < 0.05), errs


def test_manufactured_plane_wave_first_order_below_omega_2(orc):
    errs = [_mms_errors(orc, 2, N, 1.8, (1, 1), (1, 0.3)) for N in (32, 64)]
    order = np.log2(errs[0] / errs[1])
    assert np.all((order > 0.7) & (order < 1.3)), (errs, order)
