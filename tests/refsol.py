"""Independent reference solutions used to pin the oracle.

Radial static boundary-value problems of the compressible neo-Hookean solid
(Sec. 4.3, Eqs. 72-75 in 2D; Sec. 5.2, Eqs. 84-85 in 3D), solved with
scipy's collocation BVP solver.  The principal nominal stresses are those of
Eq. 74 with J = lambda_r lambda_t^(D-1).
"""
import numpy as np
from scipy.integrate import solve_bvp


def _principal(lr, lt, mu, lam, D):
    J = lr * lt ** (D - 1)
    Pr = mu * (lr - 1.0 / lr) + 0.5 * lam * (J * J - 1.0) / lr
    Pt = mu * (lt - 1.0 / lt) + 0.5 * lam * (J * J - 1.0) / lt
    return Pr, Pt


def radial_bvp(D, mu, lam, Ri, Ro, r_inner=None, Pr_inner=None, Pr_outer=0.0, n=2001):
    """Solve d P_r/dR + (D-1)(P_r - P_t)/R = 0 for r(R) on [Ri, Ro] with either
    r(Ri) or P_r(Ri) prescribed and P_r(Ro) = Pr_outer.  Returns a dict of
    callables r(R), P_r(R), lambda_r(R), lambda_t(R)."""
    def rhs(R, y):
        r, rp = y
        lt = r / R
        Pr, Pt = _principal(rp, lt, mu, lam, D)
        # partial derivatives of P_r = mu (lr - 1/lr) + lam/2 (lr lt^(2D-2) - 1/lr)
        dPr_dlr = mu * (1.0 + 1.0 / rp ** 2) + 0.5 * lam * (lt ** (2 * D - 2) + 1.0 / rp ** 2)
        dPr_dlt = lam * (D - 1) * rp * lt ** (2 * D - 3)
        # d/dR P_r = dPr/dlr r'' + dPr/dlt (r'/R - r/R^2)
        rpp = (-(D - 1) * (Pr - Pt) / R - dPr_dlt * (rp / R - r / R ** 2)) / dPr_dlr
        return np.vstack([rp, rpp])

    def bc(ya, yb):
        Pr_b = _principal(yb[1], yb[0] / Ro, mu, lam, D)[0]
        if r_inner is not None:
            first = ya[0] - r_inner
        else:
            first = _principal(ya[1], ya[0] / Ri, mu, lam, D)[0] - Pr_inner
        return np.array([first, Pr_b - Pr_outer])

    R = np.linspace(Ri, Ro, n)
    r0 = r_inner if r_inner is not None else Ri
    y0 = np.vstack([r0 + (R - Ri) * 0.0 + (R - Ri), np.ones_like(R)])
    sol = solve_bvp(rhs, bc, R, y0, tol=1e-9, max_nodes=400000)
    assert sol.success, sol.message

    def r(Rq):
        return sol.sol(Rq)[0]

    def lr(Rq):
        return sol.sol(Rq)[1]

    def Pr(Rq):
        y = sol.sol(Rq)
        return _principal(y[1], y[0] / Rq, mu, lam, D)[0]

    return dict(r=r, lr=lr, lt=lambda Rq: r(Rq) / Rq, Pr=Pr, sol=sol)
