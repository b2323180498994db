"""Pins of the oracle's twisted end data (the tube of Sec. 5.3, Eqs. 87-88).

The loaded end prescribes u_D = ((R(alpha) - I) X_perp, dL) with
alpha = s(t) Phi, dL = s(t) eps L and the half-cosine ramp s; the cut links
impose its time derivative.  Checked against facts that do not restate the
formula: the imposed velocity is the time derivative of the prescribed
displacement (central differences in t), the deformed point keeps its
distance to the axis at every t (a rotation), a quarter turn maps
X_perp = (r, 0) to (0, r), the ramp reaches its full value at t = T_r and
stays, and the clamped end prescribes nothing.
"""
import math

import numpy as np

import workloads as W
from oracle import oracle as orc


def _tube_sim():
    c = W.config_tube(10)
    o = orc.Sim(3, c["n"], c["dx"], c["dt"], c["mu"], c["lam"], omega=c["omega"], gamma=c["gamma"],
                origin=c["origin"], periodic_mask=0, proj_every=c["proj_every"])
    o.set_levelset(c["phi"], c["bid"])
    o.set_bc(3, orc.DIRICHLET, given_as_displacement=True)
    o.set_bc(4, orc.DIRICHLET, given_as_displacement=True, ramp=orc.RAMP_HALFCOS, T_r=10.0,
             a=(0.0, 0.0, 1.5), twist=math.pi / 4, X0=(0.38, 0.38, 0.0))
    o.set_bc(5, orc.DIRICHLET, given_as_displacement=True, ramp=orc.RAMP_HALFCOS, T_r=10.0,
             twist=math.pi / 2, X0=(0.38, 0.38, 0.0))
    return o


def test_velocity_is_the_rate_of_the_displacement():
    o = _tube_sim()
    N = (0.0, 0.0, 1.0)
    rng = np.random.default_rng(3)
    for _ in range(20):
        X = (0.38 + rng.uniform(-0.3, 0.3), 0.38 + rng.uniform(-0.3, 0.3), 3.0)
        t = rng.uniform(0.5, 9.5)
        h = 1e-4
        v, _ = o.bc_data(4, X, N, t)
        _, up = o.bc_data(4, X, N, t + h)
        _, um = o.bc_data(4, X, N, t - h)
        fd = (up - um) / (2 * h)
        assert np.allclose(v, fd, rtol=1e-6, atol=1e-9)


def test_rotation_keeps_the_distance_to_the_axis():
    o = _tube_sim()
    N = (0.0, 0.0, 1.0)
    for t in (0.0, 2.5, 5.0, 7.5, 10.0, 40.0):
        for X in ((0.68, 0.38, 3.0), (0.38, 0.08, 3.0), (0.55, 0.6, 3.0)):
            _, u = o.bc_data(4, X, N, t)
            d = np.array(X[:2]) - 0.38
            assert abs(np.linalg.norm(d + u[:2]) - np.linalg.norm(d)) < 1e-14


def test_quarter_turn_and_ramp():
    o = _tube_sim()
    N = (0.0, 0.0, 1.0)
    r = 0.2
    X = (0.38 + r, 0.38, 3.0)
    _, u = o.bc_data(5, X, N, 10.0)  # s = 1: a quarter turn
    assert np.allclose(u, [-r, r, 0.0], atol=1e-15)
    _, u = o.bc_data(5, X, N, 5.0)  # s = 1/2: an eighth of a turn
    assert np.allclose(u[:2], [r * (math.cos(math.pi / 4) - 1), r * math.sin(math.pi / 4)], atol=1e-15)
    _, u0 = o.bc_data(4, X, N, 0.0)
    assert np.allclose(u0, 0.0)
    _, u1 = o.bc_data(4, X, N, 10.0)
    _, u2 = o.bc_data(4, X, N, 60.0)
    assert np.allclose(u1, u2, atol=1e-15) and abs(u1[2] - 1.5) < 1e-15
    v2, _ = o.bc_data(4, X, N, 60.0)  # at rest after the ramp
    assert np.allclose(v2, 0.0, atol=1e-15)
    v3, u3 = o.bc_data(3, X, N, 5.0)  # clamped end
    assert np.allclose(v3, 0.0) and np.allclose(u3, 0.0)
