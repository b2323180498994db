"""The oracle's own FP64 rounding, measured against an 80-bit run.

The GPU parity gates in FP64 allow, besides the relative tolerance, the
rounding floor that the oracle's raw FP64 populations and stress evaluation
accumulate (tests/parity.py).  This test measures the oracle's actual
rounding on the 64^2 periodic configuration (1000 steps): the same update
(state recovery Eq. 28, equilibrium Eq. 24 with the neo-Hookean stress of
Eq. 62, BGK collision Eq. 29, pull streaming Eq. 31) evaluated in numpy's
80-bit extended precision from the oracle's own initial populations.  The
oracle must agree with it within the floor, part by part, and its velocity
error must be of the size the floor explains (a few 1e-12: above 1e-12,
which is why the floor is part of the FP64 gate).
"""
import numpy as np
import pytest

import workloads as W
from parity import component_errors

LD = np.longdouble


def _stress(F, D, mu, lam):
    if D == 2:
        C = np.stack([F[3], -F[2], -F[1], F[0]])
        J = F[0] * F[3] - F[1] * F[2]
    else:
        C = np.stack([F[4] * F[8] - F[5] * F[7], F[5] * F[6] - F[3] * F[8], F[3] * F[7] - F[4] * F[6],
                      F[2] * F[7] - F[1] * F[8], F[0] * F[8] - F[2] * F[6], F[1] * F[6] - F[0] * F[7],
                      F[1] * F[5] - F[2] * F[4], F[2] * F[3] - F[0] * F[5], F[0] * F[4] - F[1] * F[3]])
        J = F[0] * C[0] + F[1] * C[1] + F[2] * C[2]
    return mu * F + (LD(0.5) * lam * (J * J - 1) / J - mu / J) * C


def _extended_run(f, D, n, c, omega, mu, lam, steps):
    Q, M = 2 * D, D + D * D
    shape = list(n)[::-1]
    cc, om, mu, lam = LD(c), LD(omega), LD(mu), LD(lam)
    for _ in range(steps):
        U = f.sum(0)
        P = _stress(U[D:], D, mu, lam)
        out = np.empty_like(f)
        for q in range(Q):
            A, sg = q // 2, LD(-1 if q & 1 else 1)
            for r in range(M):
                if r < D:
                    phi = -P[r * D + A]
                else:
                    i, B = (r - D) // D, (r - D) % D
                    phi = -U[i] if A == B else np.zeros_like(U[0])
                feq = U[r] / (2 * D) + sg * phi / (2 * cc)
                out[q, r] = f[q, r] + om * (feq - f[q, r])
        for q in range(Q):  # f_q(X) <- f*_q(X - e_q)
            A, sg = q // 2, -1 if q & 1 else 1
            out[q] = np.roll(out[q].reshape([M] + shape), sg, axis=1 + (D - 1 - A)).reshape(M, -1)
        f = out
    return f.sum(0).astype(np.float64)


@pytest.mark.skipif(np.finfo(np.longdouble).eps >= 1e-18, reason="no extended precision long double here")
def test_oracle_rounding_within_floor(orc):
    c = W.config_c1()
    D, Q, M = 2, 4, 6
    N = int(np.prod(c["n"]))
    o = orc.Sim(D, c["n"], c["dx"], c["dt"], c["mu"], c["lam"], omega=c["omega"])
    o.set_state(c["U0"], dU0=c["dU0"])
    f0 = o.get_f().reshape(Q, M, N).astype(LD)
    o.step(c["steps"])
    Uo = o.moments()[0]
    Ux = _extended_run(f0, D, c["n"], c["dx"] / c["dt"], c["omega"], c["mu"], c["lam"], c["steps"])
    e = component_errors(Uo, Ux, D, pops=o.get_f(), steps=c["steps"],
                         stress=(c["mu"], c["lam"], 1.0, c["dx"] / c["dt"], c["omega"]))
    print(e)
    for k in ("v", "F", "v_max", "F_max"):
        assert e[k] <= e[k + "_floor"], (k, e)
    # the oracle's velocity carries rounding above 1e-12 of its size
    assert 1e-12 < e["v"] < 1e-11
