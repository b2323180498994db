"""ctypes wrapper of the FP64 CPU oracle (``orc.c``).

TEST INFRASTRUCTURE ONLY.  The oracle is the plain reference implementation
of the total-Lagrangian vectorial LBM (Feng & Chu, Secs. 2-3, Algorithm 1)
that the GPU library is checked against.  Only ``tests/``, the smoke check
and the CPU-baseline leg of ``bench.py`` may import this module.  It imports
nothing from the product package.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liborc.so")

DIRICHLET, NEUMANN = 1, 2
RAMP_CONST, RAMP_SIN2, RAMP_HALFCOS, RAMP_LINEAR = 0, 1, 2, 3


def build(force: bool = False) -> str:
    """Compile ``orc.c`` into ``liborc.so`` (gcc, OpenMP)."""
    src = os.path.join(HERE, "orc.c")
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(src):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, src, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        dp, ip, i64p = C.POINTER(C.c_double), C.POINTER(C.c_int), C.POINTER(C.c_int64)
        L.orc_piola.argtypes = [C.c_int, C.c_double, C.c_double, dp, dp]
        L.orc_piola_jvp.argtypes = [C.c_int, C.c_double, C.c_double, dp, dp, dp]
        L.orc_piola_law.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, dp, dp, dp]
        L.orc_piola_law_jvp.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, dp, dp, dp, dp]
        L.orc_cauchy.argtypes = [C.c_int, C.c_double, C.c_double, dp, dp]
        L.orc_energy.argtypes = [C.c_int, C.c_double, C.c_double, dp]
        L.orc_energy.restype = C.c_double
        L.orc_flux.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, dp, dp]
        L.orc_feq.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, C.c_double, dp, dp]
        L.orc_feq_jvp.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, C.c_double, dp, dp, dp]
        L.orc_lsq_weights.argtypes = [C.c_int, C.c_int, dp, dp, C.c_double, dp]
        L.orc_newton.argtypes = [C.c_int, C.c_double, C.c_double, dp, dp, dp, dp, C.c_double, dp, ip]
        L.orc_create.argtypes = [C.c_int, ip, C.c_double, dp, C.c_int, C.c_double, C.c_double,
                                 C.c_double, C.c_double, C.c_double, C.c_double, C.c_double, C.c_int]
        L.orc_create.restype = C.c_void_p
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_set_projection.argtypes = [C.c_void_p, C.c_int, C.c_double]
        L.orc_set_body_force.argtypes = [C.c_void_p, dp, C.c_int, C.c_double]
        L.orc_set_bc_twist.argtypes = [C.c_void_p, C.c_int, C.c_double]
        L.orc_bc_data.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p]
        L.orc_set_fibres.argtypes = [C.c_void_p, C.c_double, dp]
        L.orc_set_levelset.argtypes = [C.c_void_p, dp, C.POINTER(C.c_uint8)]
        L.orc_set_bc.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int, dp, dp,
                                 C.c_double, C.c_double, dp]
        L.orc_set_state.argtypes = [C.c_void_p, dp, dp, dp]
        L.orc_step.argtypes = [C.c_void_p, C.c_int64]
        L.orc_moments.argtypes = [C.c_void_p, dp, dp, dp]
        L.orc_get_f.argtypes = [C.c_void_p, dp]
        L.orc_put_f.argtypes = [C.c_void_p, dp, dp, C.c_int64]
        L.orc_get_fs.argtypes = [C.c_void_p, dp]
        L.orc_num_active.argtypes = [C.c_void_p]
        L.orc_num_active.restype = C.c_int64
        L.orc_num_links.argtypes = [C.c_void_p]
        L.orc_num_links.restype = C.c_int64
        L.orc_get_links.argtypes = [C.c_void_p, i64p, C.POINTER(C.c_int32), dp, dp, C.POINTER(C.c_int32)]
        L.orc_stats.argtypes = [C.c_void_p, i64p]
        L.orc_project.argtypes = [C.c_void_p, dp, dp, C.c_double, i64p]
        L.orc_project_anchored.argtypes = [C.c_void_p, dp, dp, C.c_double, C.c_double, i64p]
        L.orc_compatible_F.argtypes = [C.c_void_p, dp, dp, dp]
        L.orc_adjoint.argtypes = [C.c_void_p, C.c_int64, dp, dp, dp, dp, dp, dp]
        L.orc_num_threads.restype = C.c_int
        L.orc_set_viscous.argtypes = [C.c_void_p, C.c_double, C.c_double]
        L.orc_get_viscous.argtypes = [C.c_void_p, dp, dp]
        L.orc_visco_piola.argtypes = [C.c_int] + [C.c_double] * 4 + [dp] * 4
        L.orc_visco_piola_jvp.argtypes = [C.c_int] + [C.c_double] * 4 + [dp] * 5
        L.orc_visco_path.argtypes = [C.c_int] + [C.c_double] * 5 + [C.c_int64, dp, dp]
        L.orc_stress.argtypes = [C.c_void_p, dp, dp]
        L.orc_set_thermal.argtypes = [C.c_void_p, dp]
        L.orc_thermal_piola.argtypes = [C.c_int] + [C.c_double] * 3 + [dp, C.c_double, dp, dp]
        L.orc_thermal_piola_jvp.argtypes = [C.c_int] + [C.c_double] * 3 + [dp, C.c_double, dp, dp, dp]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


def num_threads():
    return int(lib().orc_num_threads())


# ---- point maps -----------------------------------------------------------

def piola(F, mu, lam):
    F = _f64(F)
    D = F.shape[0]
    P = np.zeros((D, D))
    st = lib().orc_piola(D, mu, lam, _d(F), _d(P))
    if st:
        raise OracleError(st, "piola")
    return P


def piola_jvp(F, dF, mu, lam):
    F, dF = _f64(F), _f64(dF)
    D = F.shape[0]
    dP = np.zeros((D, D))
    lib().orc_piola_jvp(D, mu, lam, _d(F), _d(dF), _d(dP))
    return dP


def piola_law(F, mu, lam, k1, a0):
    """P of the fibre-reinforced neo-Hookean law (a0 a unit vector)."""
    F = _f64(F)
    D = F.shape[0]
    a = _f64(list(a0) + [0.0] * (3 - len(a0)))
    P = np.zeros((D, D))
    st = lib().orc_piola_law(D, mu, lam, k1, _d(a), _d(F), _d(P))
    if st:
        raise OracleError(st, "piola_law")
    return P


def piola_law_jvp(F, dF, mu, lam, k1, a0):
    F, dF = _f64(F), _f64(dF)
    D = F.shape[0]
    a = _f64(list(a0) + [0.0] * (3 - len(a0)))
    dP = np.zeros((D, D))
    st = lib().orc_piola_law_jvp(D, mu, lam, k1, _d(a), _d(F), _d(dF), _d(dP))
    if st:
        raise OracleError(st, "piola_law_jvp")
    return dP


def cauchy(F, mu, lam):
    F = _f64(F)
    D = F.shape[0]
    s = np.zeros((D, D))
    lib().orc_cauchy(D, mu, lam, _d(F), _d(s))
    return s


def visco_piola(F, mu, lam, beta, xi, Qh, S0h):
    """P = P_NH(F) + F Q(F), Q(F) = xi^2 Qh + beta xi (S_0(F) - S0h): the
    stress of a node of the Maxwell-branch law with history (Qh, S0h)."""
    F, Qh, S0h = _f64(F), _f64(Qh), _f64(S0h)
    D = F.shape[0]
    P = np.zeros((D, D))
    st = lib().orc_visco_piola(D, mu, lam, beta, xi, _d(Qh), _d(S0h), _d(F), _d(P))
    if st:
        raise OracleError(st, "visco_piola")
    return P


def visco_piola_jvp(F, dF, mu, lam, beta, xi, Qh, S0h):
    F, dF, Qh, S0h = _f64(F), _f64(dF), _f64(Qh), _f64(S0h)
    D = F.shape[0]
    dP = np.zeros((D, D))
    st = lib().orc_visco_piola_jvp(D, mu, lam, beta, xi, _d(Qh), _d(S0h), _d(F), _d(dF), _d(dP))
    if st:
        raise OracleError(st, "visco_piola_jvp")
    return dP


def thermal_piola(F, mu, lam, th, k1=0.0, a0=(1.0, 0.0, 0.0)):
    """P(F) = th^(D-1) P_W(F / th): the law (fibres k1 along a0) at a node
    with thermal stretch th."""
    F = _f64(F)
    D = F.shape[0]
    a = _f64(list(a0) + [0.0] * (3 - len(a0)))
    P = np.zeros((D, D))
    st = lib().orc_thermal_piola(D, mu, lam, k1, _d(a), float(th), _d(F), _d(P))
    if st:
        raise OracleError(st, "thermal_piola")
    return P


def thermal_piola_jvp(F, dF, mu, lam, th, k1=0.0, a0=(1.0, 0.0, 0.0)):
    F, dF = _f64(F), _f64(dF)
    D = F.shape[0]
    a = _f64(list(a0) + [0.0] * (3 - len(a0)))
    dP = np.zeros((D, D))
    st = lib().orc_thermal_piola_jvp(D, mu, lam, k1, _d(a), float(th), _d(F), _d(dF), _d(dP))
    if st:
        raise OracleError(st, "thermal_piola_jvp")
    return dP


def visco_path(F, mu, lam, beta, tau, dt):
    """Stress [n+1][D][D] of a material point of the Maxwell-branch law driven
    along F [n+1][D][D] (one step dt apart), started relaxed at F[0]."""
    F = _f64(F)
    n1, D = F.shape[0], F.shape[1]
    P = np.zeros_like(F)
    st = lib().orc_visco_path(D, mu, lam, beta, tau, dt, n1 - 1, _d(F), _d(P))
    if st:
        raise OracleError(st, "visco_path")
    return P


def energy(F, mu, lam):
    F = _f64(F)
    return lib().orc_energy(F.shape[0], mu, lam, _d(F))


def flux(U, D, mu, lam, rho0=1.0):
    U = _f64(U)
    Phi = np.zeros((D, D + D * D))
    lib().orc_flux(D, mu, lam, rho0, _d(U), _d(Phi))
    return Phi


def feq(U, D, c, mu, lam, rho0=1.0):
    U = _f64(U)
    f = np.zeros((2 * D, D + D * D))
    lib().orc_feq(D, c, mu, lam, rho0, _d(U), _d(f))
    return f


def feq_jvp(U, Z, D, c, mu, lam, rho0=1.0):
    U, Z = _f64(U), _f64(Z)
    f = np.zeros((2 * D, D + D * D))
    lib().orc_feq_jvp(D, c, mu, lam, rho0, _d(U), _d(Z), _d(f))
    return f


def lsq_weights(xi, tang, dx):
    xi, tang = _f64(xi), _f64(tang)
    npts, D = xi.shape
    w = np.zeros((D - 1, npts))
    basis = lib().orc_lsq_weights(D, npts, _d(xi), _d(tang), dx, _d(w))
    return basis, w


def newton(N, Gt, T, h0, mu, lam, tol=1e-12):
    N, Gt, T, h0 = _f64(N), _f64(Gt), _f64(T), _f64(h0)
    D = N.shape[0]
    h = np.zeros(D)
    its = C.c_int(0)
    ok = lib().orc_newton(D, mu, lam, _d(N), _d(Gt), _d(T), _d(h0), tol, _d(h), C.byref(its))
    return bool(ok), h, its.value


# ---- the simulation --------------------------------------------------------

class Sim:
    """One oracle instance; arrays are planar numpy [component][node]."""

    def __init__(self, D, n, dx, dt, mu, lam, rho0=1.0, omega=1.8, gamma=0.0, theta_F=1.0,
                 proj_every=20, origin=None, periodic_mask=None, proj_sweeps=20, proj_weight=2.0 / 3.0):
        self.D, self.M, self.Q = D, D + D * D, 2 * D
        self.n = tuple(int(v) for v in n)
        self.N = int(np.prod(self.n))
        self.dx, self.dt = dx, dt
        n3 = (C.c_int * 3)(*(list(self.n) + [1] * (3 - D)))
        org = np.zeros(3) if origin is None else _f64(list(origin) + [0.0] * (3 - len(origin)))
        pm = ((1 << D) - 1) if periodic_mask is None else periodic_mask
        self.h = lib().orc_create(D, n3, dx, _d(org), pm, mu, lam, rho0, dt, omega, gamma, theta_F,
                                  proj_every)
        if not self.h:
            raise OracleError(1, "create")
        self._org = org
        st = lib().orc_set_projection(self.h, int(proj_sweeps), float(proj_weight))
        if st:
            raise OracleError(st, "set_projection")

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_destroy(self.h)
            self.h = None

    def set_levelset(self, phi, bid=None):
        phi = _f64(phi).reshape(-1)
        b = np.zeros(self.N, np.uint8) if bid is None else np.ascontiguousarray(bid, np.uint8).reshape(-1)
        st = lib().orc_set_levelset(self.h, _d(phi), b.ctypes.data_as(C.POINTER(C.c_uint8)))
        if st:
            raise OracleError(st, "set_levelset")

    def set_bc(self, bid, type, ramp=RAMP_CONST, T_r=1.0, given_as_displacement=False, a=None, G=None,
               p_radial=0.0, X0=None, p_normal=0.0, twist=0.0):
        a3 = np.zeros(3) if a is None else _f64(list(a) + [0.0] * (3 - len(a)))
        G9 = np.zeros((3, 3))
        if G is not None:
            G = np.asarray(G, float)
            G9[: G.shape[0], : G.shape[1]] = G
        G9 = _f64(G9)
        X03 = np.zeros(3) if X0 is None else _f64(list(X0) + [0.0] * (3 - len(X0)))
        st = lib().orc_set_bc(self.h, bid, type, ramp, T_r, int(given_as_displacement), _d(a3), _d(G9),
                              p_radial, p_normal, _d(X03))
        if st:
            raise OracleError(st, "set_bc")
        if twist:
            st = lib().orc_set_bc_twist(self.h, bid, float(twist))
            if st:
                raise OracleError(st, "set_bc_twist")

    def bc_data(self, bid, X, N, t):
        """(imposed velocity or traction, prescribed displacement) of
        boundary identifier bid at point X with normal N, time t."""
        Xa = _f64(list(X) + [0.0] * (3 - len(X)))
        Na = _f64(list(N) + [0.0] * (3 - len(N)))
        val = np.zeros(3)
        disp = np.zeros(3)
        st = lib().orc_bc_data(self.h, int(bid), _d(Xa), _d(Na), float(t), _d(val), _d(disp))
        if st:
            raise OracleError(st, "bc_data")
        return val[: self.D].copy(), disp[: self.D].copy()

    def set_fibres(self, k1, a0):
        """Fibre-reinforced law: W += k1/2 (|F a0|^2 - 1)^2 (k1 = 0: off)."""
        a = _f64(list(a0) + [0.0] * (3 - len(a0)))
        st = lib().orc_set_fibres(self.h, float(k1), _d(a))
        if st:
            raise OracleError(st, "set_fibres")

    def set_viscous(self, beta, tau):
        """Maxwell branch dQ/dt + Q/tau = beta dS_0/dt on top of the law
        (before set_state; tau = inf: glassy limit, tau = 0: none)."""
        st = lib().orc_set_viscous(self.h, float(beta), float(tau))
        if st:
            raise OracleError(st, "set_viscous")

    def viscous_history(self):
        """(Q^n, S_0^n) of every node, [D*D][N] each"""
        Qh = np.zeros((self.D * self.D, self.N))
        S0 = np.zeros((self.D * self.D, self.N))
        st = lib().orc_get_viscous(self.h, _d(Qh), _d(S0))
        if st:
            raise OracleError(st, "get_viscous")
        return Qh, S0

    def stress(self):
        """(P, sigma) of the current state, [D*D][N] each (Eq. 35)"""
        P = np.zeros((self.D * self.D, self.N))
        S = np.zeros((self.D * self.D, self.N))
        st = lib().orc_stress(self.h, _d(P), _d(S))
        if st:
            raise OracleError(st, "stress")
        return P, S

    def set_thermal(self, th):
        """Thermal stretch th [N] (> 0; None removes it): P = th^(D-1) P_W(F/th)."""
        tp = None if th is None else _d(_keep(self, _f64(th).reshape(self.N)))
        st = lib().orc_set_thermal(self.h, tp)
        self._tmps = []
        if st:
            raise OracleError(st, "set_thermal")

    def set_body_force(self, g, ramp=RAMP_CONST, T_r=1.0):
        """Body acceleration b(X, t) = s(t) g(X), g [D][N] (None clears)."""
        gp = None if g is None else _d(_keep(self, _f64(g).reshape(self.D, self.N)))
        st = lib().orc_set_body_force(self.h, gp, int(ramp), float(T_r))
        self._tmps = []
        if st:
            raise OracleError(st, "set_body_force")

    def set_state(self, U0, u0=None, dU0=None):
        U0 = _f64(U0).reshape(self.M, self.N)
        u0p = None if u0 is None else _d(_keep(self, _f64(u0).reshape(self.D, self.N)))
        dUp = None if dU0 is None else _d(_keep(self, _f64(dU0).reshape(self.D, self.M, self.N)))
        st = lib().orc_set_state(self.h, _d(U0), u0p, dUp)
        self._tmps = []
        if st:
            raise OracleError(st, "set_state")

    def step(self, n=1):
        st = lib().orc_step(self.h, int(n))
        if st:
            raise OracleError(st, "step")

    def moments(self):
        U = np.zeros((self.M, self.N))
        u = np.zeros((self.D, self.N))
        J = np.zeros(self.N)
        st = lib().orc_moments(self.h, _d(U), _d(u), _d(J))
        if st:
            raise OracleError(st, "moments")
        return U, u, J

    def adjoint(self, n, dLdU=None, dLdu=None, with_dU0=False):
        """Advance n steps from the state of set_state and return
        (dL/d(mu, lambda), dL/dv0 [D][N], dL/du0 [D][N]) for
        L = sum dLdU . U + dLdu . u over the moments after the last step;
        with_dU0 appends dL/d dU0 [D][M][N] (the initial gradient data)."""
        gU = None if dLdU is None else _f64(dLdU).reshape(self.M, self.N)
        gu = None if dLdu is None else _f64(dLdu).reshape(self.D, self.N)
        gm = np.zeros(2)
        gv = np.zeros((self.D, self.N))
        g0 = np.zeros((self.D, self.N))
        gd = np.zeros((self.D, self.M, self.N)) if with_dU0 else None
        st = lib().orc_adjoint(self.h, int(n), None if gU is None else _d(gU), None if gu is None else _d(gu),
                               _d(gm), _d(gv), _d(g0), None if gd is None else _d(gd))
        if st:
            raise OracleError(st, "adjoint")
        return (gm, gv, g0, gd) if with_dU0 else (gm, gv, g0)

    def get_f(self):
        f = np.zeros((self.Q, self.M, self.N))
        lib().orc_get_f(self.h, _d(f))
        return f

    def get_fs(self):
        f = np.zeros((self.Q, self.M, self.N))
        lib().orc_get_fs(self.h, _d(f))
        return f

    def put_f(self, f, ustar=None, step=0):
        f = _f64(f).reshape(self.Q, self.M, self.N)
        us = None if ustar is None else _d(_keep(self, _f64(ustar).reshape(self.D, self.N)))
        lib().orc_put_f(self.h, _d(f), us, int(step))
        self._tmps = []

    def num_active(self):
        return int(lib().orc_num_active(self.h))

    def num_links(self):
        return int(lib().orc_num_links(self.h))

    def links(self):
        L = self.num_links()
        node = np.zeros(L, np.int64)
        q = np.zeros(L, np.int32)
        eta = np.zeros(L)
        Nb = np.zeros((L, 3))
        bid = np.zeros(L, np.int32)
        lib().orc_get_links(self.h, node.ctypes.data_as(C.POINTER(C.c_int64)),
                            q.ctypes.data_as(C.POINTER(C.c_int32)), _d(eta), _d(Nb),
                            bid.ctypes.data_as(C.POINTER(C.c_int32)))
        return dict(node=node, q=q, eta=eta, N=Nb[:, : self.D], bid=bid)

    def stats(self):
        st = np.zeros(6, np.int64)
        lib().orc_stats(self.h, st.ctypes.data_as(C.POINTER(C.c_int64)))
        return dict(newton_iters=int(st[0]), newton_fail=int(st[1]), cg_iters=int(st[2]),
                    projections=int(st[3]), step=int(st[4]), status=int(st[5]))

    def project(self, F, u, rtol=1e-15, t=None):
        """Projection of u onto F (Sec. 3.5); with t given, the Dirichlet
        cut links of the boundary conditions set add their anchors at time t."""
        F = _f64(F).reshape(self.D * self.D, self.N)
        u = _f64(u).reshape(self.D, self.N).copy()
        its = C.c_int64(0)
        if t is None:
            lib().orc_project(self.h, _d(F), _d(u), rtol, C.byref(its))
        else:
            lib().orc_project_anchored(self.h, _d(F), _d(u), float(t), rtol, C.byref(its))
        return u, its.value

    def compatible_F(self, u, F):
        u = _f64(u).reshape(self.D, self.N)
        F = _f64(F).reshape(self.D * self.D, self.N)
        Fc = np.zeros((self.D * self.D, self.N))
        lib().orc_compatible_F(self.h, _d(u), _d(F), _d(Fc))
        return Fc


def _keep(obj, arr):
    # keep temporaries alive until the next call that replaces them
    if not hasattr(obj, "_tmps"):
        obj._tmps = []
    obj._tmps.append(arr)
    return arr
