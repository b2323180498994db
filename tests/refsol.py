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


def cauchy_nh(F, mu, lam):
    """Cauchy stress sigma = J^-1 P F^T of the compressible neo-Hookean solid
    (Sec. 4.1, Eq. 62; the recovery of Eq. 35), for F of shape [n, D, D]."""
    J = np.linalg.det(F)
    Fit = np.transpose(np.linalg.inv(F), (0, 2, 1))
    P = mu * (F - Fit) + 0.5 * lam * (J * J - 1.0)[:, None, None] * Fit
    return np.einsum("nij,nkj->nik", P, F) / J[:, None, None]


def radial_fields(ref, X, Xc):
    """Displacement [D][n] and deformation gradient [n][D][D] of the radial
    map x = Xc + r(R) e_R (Sec. 5.2: lambda_r along e_R, r/R across it)."""
    d = X - np.asarray(Xc, float)[:, None]
    R = np.linalg.norm(d, axis=0)
    e = d / R
    lr, lt = ref["lr"](R), ref["lt"](R)
    u = (ref["r"](R) - R) * e
    D = X.shape[0]
    ee = np.einsum("in,jn->nij", e, e)
    F = lt[:, None, None] * np.eye(D)[None] + (lr - lt)[:, None, None] * ee
    return u, F


def rel_l2(a, b, scale=None):
    """Relative discrete L2 error over the comparison nodes (Sec. 4.1,
    Eq. 63); `scale` replaces b in the denominator (F - I uses F_ref - I)."""
    s = b if scale is None else scale
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(s)))


def affine_errors(c, U, u, J, t):
    """Errors of an affine velocity Dirichlet run (the annulus of Sec. 4.2,
    Eqs. 64-68, or the ellipsoid of Sec. 5.1, Eqs. 80-82) at time t over the
    active nodes: u against t A (X - Xc), v against A (X - Xc), F against
    I + t A; the Jacobian range and the exact J."""
    D = c["D"]
    act = c["phi"] <= 0
    d = c["X"][:, act] - c["Xc"][:, None]
    A = c["A"]
    Fex = np.eye(D) + t * A
    F = U[D:D + D * D, act].T.reshape(-1, D, D)
    Fb = np.broadcast_to(Fex, F.shape)
    sig, sig_ex = cauchy_nh(F, c["mu"], c["lam"]), cauchy_nh(np.ascontiguousarray(Fb), c["mu"], c["lam"])
    return {"E_u": rel_l2(u[:, act], t * (A @ d)), "E_v": rel_l2(U[:D, act], A @ d), "E_sigma": rel_l2(sig, sig_ex),
            "E_F": rel_l2(F, np.broadcast_to(Fex, F.shape)),
            "E_F_minus_I": rel_l2(F, np.broadcast_to(Fex, F.shape), np.broadcast_to(Fex - np.eye(D), F.shape)),
            "J_range": [float(J[act].min()), float(J[act].max())], "J_exact": float(np.linalg.det(Fex))}


def radial_errors(c, ref, U, u, J):
    """Errors of a radial benchmark run (the 2D annulus of Sec. 4.3, Eqs.
    72-75, or the spherical shell of Sec. 5.2, Eqs. 83-85) against the radial
    BVP state over the active nodes: u, F, F - I, Cauchy stress, the RMS of
    the residual velocity and the Jacobian range."""
    D = c["D"]
    act = c["phi"] <= 0
    u_ref, F_ref = radial_fields(ref, c["X"][:, act], c["Xc"])
    F = U[D:D + D * D, act].T.reshape(-1, D, D)
    s, s_ref = cauchy_nh(F, c["mu"], c["lam"]), cauchy_nh(F_ref, c["mu"], c["lam"])
    v = U[:D, act]
    return {"E_u": rel_l2(u[:, act], u_ref), "E_F": rel_l2(F, F_ref),
            "E_F_minus_I": rel_l2(F, F_ref, F_ref - np.eye(D)), "E_sigma": rel_l2(s, s_ref),
            "v_rms": float(np.sqrt((v * v).sum(0).mean())),
            "J_range": [float(J[act].min()), float(J[act].max())]}


def piola_nh(F, mu, lam):
    """Nominal stress P = dW/dF of the compressible neo-Hookean energy
    (Sec. 4.1, Eq. 62), for F of shape [n, D, D]."""
    J = np.linalg.det(F)
    Fit = np.transpose(np.linalg.inv(F), (0, 2, 1))
    return mu * (F - Fit) + 0.5 * lam * (J * J - 1.0)[:, None, None] * Fit


def piola_fibre(F, mu, lam, k1, a0):
    """Nominal stress of the neo-Hookean solid reinforced by fibres along the
    unit reference direction a0: W = W_NH + k1/2 (|F a0|^2 - 1)^2, so
    P = P_NH + 2 k1 (|F a0|^2 - 1) (F a0) (x) a0 ([n, D, D])."""
    a0 = np.asarray(a0, float)
    fa = np.einsum("nij,j->ni", F, a0)
    I4 = (fa * fa).sum(1)
    return piola_nh(F, mu, lam) + 2 * k1 * (I4 - 1.0)[:, None, None] * np.einsum("ni,j->nij", fa, a0)


class PlaneWaveMMS:
    """Manufactured finite-strain plane wave on a periodic box (body
    acceleration of Sec. 2.1, Eq. 5):

        u(X, t) = a cos(Omega t) sin(2 pi xi) p,   xi = k . X,

    k an integer wave vector, p a unit polarisation (not orthogonal to k, so
    J varies).  Then v = du/dt, F = I + a cos(Omega t) 2 pi cos(2 pi xi)
    p (x) k, and the body acceleration that makes u an exact solution is
    b = dv/dt - Div P(F), with Div P = (dP/dxi) k evaluated by Richardson
    central differences of P in xi (P depends on X through xi only)."""

    def __init__(self, D, k, p, a, Omega, mu, lam, fibre=None):
        self.D, self.k, self.a, self.Om, self.mu, self.lam = D, np.asarray(k, float), a, Omega, mu, lam
        p = np.asarray(p, float)
        self.p = p / np.linalg.norm(p)
        self.fibre = fibre  # None or (k1, unit a0)

    def _P(self, F):
        if self.fibre is None:
            return piola_nh(F, self.mu, self.lam)
        return piola_fibre(F, self.mu, self.lam, *self.fibre)

    def _F(self, xi, t):
        g = self.a * np.cos(self.Om * t) * 2 * np.pi * np.cos(2 * np.pi * xi)
        return np.eye(self.D)[None] + g[:, None, None] * np.einsum("i,j->ij", self.p, self.k)[None]

    def fields(self, X, t):
        """U = (v, F row-major) [M][n] and u [D][n] at time t."""
        xi = self.k @ X
        s = np.sin(2 * np.pi * xi)
        u = self.a * np.cos(self.Om * t) * s * self.p[:, None]
        v = -self.a * self.Om * np.sin(self.Om * t) * s * self.p[:, None]
        F = self._F(xi, t)
        return np.vstack([v, F.reshape(-1, self.D * self.D).T]), u

    def gradients(self, X, t):
        """dU/dX_A [D][M][n] at time t (analytic)."""
        D, M = self.D, self.D + self.D * self.D
        xi = self.k @ X
        c, s = np.cos(2 * np.pi * xi), np.sin(2 * np.pi * xi)
        out = np.zeros((D, M, X.shape[1]))
        dv = -self.a * self.Om * np.sin(self.Om * t) * 2 * np.pi * c       # d v / d xi (per p)
        dF = -self.a * np.cos(self.Om * t) * (2 * np.pi) ** 2 * s           # d g / d xi
        pk = np.einsum("i,j->ij", self.p, self.k).reshape(-1)
        for A in range(D):
            out[A, :D] = dv * self.k[A] * self.p[:, None]
            out[A, D:] = dF * self.k[A] * pk[:, None]
        return out

    def body(self, X, t, h=1e-4):
        xi = self.k @ X
        s = np.sin(2 * np.pi * xi)
        dvdt = -self.a * self.Om ** 2 * np.cos(self.Om * t) * s * self.p[:, None]

        def dP(hh):
            return (self._P(self._F(xi + hh, t)) - self._P(self._F(xi - hh, t))) / (2 * hh)
        dPdxi = (4 * dP(h / 2) - dP(h)) / 3
        divP = np.einsum("nij,j->in", dPdxi, self.k)
        return dvdt - divP
