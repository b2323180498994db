"""Pins of the oracle's bulk collide-stream update (Secs. 2.3-2.4).

- patch test: a uniform (v, F) is a fixed point of collide-stream on periodic
  grids and the displacement quadrature integrates u = u0 + t v exactly;
- conservation: sum over nodes of U is constant on periodic grids without
  source (Eq. 12 in flux form, B = 0);
- an exact finite-amplitude neo-Hookean shear wave (derived below) converges
  at second order under 2x refinement;
- brute force: two updates on tiny grids in exact rational arithmetic, with the
  stress from symbolic differentiation of the energy (Eq. 62) and the
  equilibria from solving the moment constraints (Eqs. 22-23);
- failure detection: the literal dt = dx reading (c = 1) is unstable and must
  end in a reported non-positive Jacobian.
"""
from fractions import Fraction

import numpy as np
import pytest
import sympy as sp

import workloads as W


def _uniform_state(D, N, v, F):
    U0 = np.zeros((D + D * D, N))
    U0[:D] = np.asarray(v)[:, None]
    U0[D:] = np.asarray(F).reshape(-1)[:, None]
    return U0


@pytest.mark.parametrize("D", [2, 3])
def test_patch_uniform_state_is_fixed(orc, D):
    rng = np.random.default_rng(11)
    n = [6, 5, 4][:D]
    N = int(np.prod(n))
    F = np.eye(D) + 0.2 * rng.standard_normal((D, D))
    v = 0.1 * rng.standard_normal(D)
    dt = 0.1 / 10
    s = orc.Sim(D, n, 0.1, dt, 1.0, 2.0, omega=1.8)
    s.set_state(_uniform_state(D, N, v, F))
    f0 = s.get_f()
    s.step(50)
    f1 = s.get_f()
    assert np.abs(f1 - f0).max() < 1e-14
    U, u, _ = s.moments()
    assert np.allclose(u, (50 * dt) * v[:, None], rtol=1e-13, atol=1e-16)


def test_conservation_periodic_c1(orc):
    c = W.config_c1()
    s = orc.Sim(2, c["n"], c["dx"], c["dt"], c["mu"], c["lam"], omega=c["omega"])
    s.set_state(c["U0"], dU0=c["dU0"])
    U0, _, _ = s.moments()
    s.step(1000)
    U1, _, J = s.moments()
    scale = np.abs(U0).sum()
    drift = np.abs(U1.sum(1) - U0.sum(1)) / scale
    assert drift.max() < 1e-13
    assert J.min() > 0.8


def _shear_wave(D, N, amp, kvec, p, t, mu=1.0, rho0=1.0):
    """Exact solution for p _|_ n: F = I + g(n.X - c_s t) p (x) n,
    v = -c_s g p, c_s = sqrt(mu/rho0): J = 1, P = mu g (p(x)n + n(x)p),
    Div P = mu g' p = rho0 dv/dt and dF/dt = grad v hold for any amplitude."""
    n = [N] * D
    dx = 1.0 / N
    X = W.node_coords(n, dx, [0.0] * D)
    kvec = np.asarray(kvec, float)
    nrm = np.linalg.norm(kvec)
    nvec = kvec / nrm
    cs = np.sqrt(mu / rho0)
    xi = nvec @ X - cs * t
    g = amp * np.sin(2 * np.pi * nrm * xi)
    dg = amp * 2 * np.pi * nrm * np.cos(2 * np.pi * nrm * xi)
    M = D + D * D
    U = np.zeros((M, X.shape[1]))
    dU = np.zeros((D, M, X.shape[1]))
    U[:D] = -cs * g * np.asarray(p)[:, None]
    pn = np.outer(p, nvec).reshape(-1)
    U[D:] = np.eye(D).reshape(-1)[:, None] + g * pn[:, None]
    for A in range(D):
        dU[A, :D] = -cs * dg * nvec[A] * np.asarray(p)[:, None]
        dU[A, D:] = dg * nvec[A] * pn[:, None]
    return n, dx, U, dU


def _shear_errors(orc, D, kvec, p, omega, Ns, mu=1.0, lam=2.0, amp=0.15, T=0.2):
    errs = []
    for N in Ns:
        n, dx, U0, dU0 = _shear_wave(D, N, amp, kvec, p, 0.0, mu)
        dt = dx / 10.0
        steps = int(round(T / dt))
        s = orc.Sim(D, n, dx, dt, mu, lam, omega=omega)
        s.set_state(U0, dU0=dU0)
        s.step(steps)
        U, _, J = s.moments()
        _, _, Uex, _ = _shear_wave(D, N, amp, kvec, p, steps * dt, mu)
        ref = Uex.copy()
        ref[D:] -= np.eye(D).reshape(-1)[:, None]
        errs.append(np.linalg.norm(U - Uex) / np.linalg.norm(ref))
    return np.array(errs)


SHEAR_CASES = [(2, (1, 0), (0, 1)), (2, (1, 1), (1, -1)), (3, (0, 1, 1), (1, 0, 0))]


@pytest.mark.parametrize("D,kvec,p", SHEAR_CASES)
def test_exact_shear_wave_second_order_without_relaxation_diffusion(orc, D, kvec, p):
    """omega = 2 (the paper's setting for its exact affine benchmark) leaves no
    relaxation diffusion: the scheme with second-order initialisation
    (Eqs. 32-33) converges at second order."""
    p = np.asarray(p, float) / np.linalg.norm(p)
    errs = _shear_errors(orc, D, kvec, p, 2.0, [16, 32, 64] if D == 2 else [8, 16, 32])
    orders = np.log2(errs[:-1] / errs[1:])
    assert orders.min() > 1.9, (errs, orders)


@pytest.mark.parametrize("D,kvec,p", SHEAR_CASES)
def test_shear_wave_relaxation_diffusion_matches_chapman_enskog(orc, D, kvec, p):
    """For omega < 2 the BGK relaxation adds the diffusion
    (1/omega - 1/2) dt (c^2/D - c_s^2) (second moment of the pair-sum closed
    equilibrium, Eq. 23, minus the squared flux Jacobian, Eq. 18).  At fixed
    c it is O(dx), so the error of a shear wave with |k| is
    1 - exp(-kappa |k|^2 T), which the lattice must reproduce."""
    p = np.asarray(p, float) / np.linalg.norm(p)
    N = 128 if D == 2 else 32
    omega, T, mu, c = 1.8, 0.2, 1.0, 10.0
    err = _shear_errors(orc, D, kvec, p, omega, [N], T=T)[0]
    dt = (1.0 / N) / c
    kappa = (1.0 / omega - 0.5) * dt * (c * c / D - mu)
    k2 = (2 * np.pi) ** 2 * float(np.dot(kvec, kvec))
    pred = 1.0 - np.exp(-kappa * k2 * T)
    assert abs(err / pred - 1.0) < 0.03, (err, pred)


# ---------------------------------------------------------- brute force -----

def _exact_piola(D):
    Fs = sp.Matrix(D, D, lambda i, j: sp.Symbol(f"F{i}{j}"))
    mu, lam = sp.Symbol("mu"), sp.Symbol("lam")
    J = Fs.det()
    Wsym = mu / 2 * (sum(x ** 2 for x in Fs) - D) - (mu + lam / 2) * sp.log(J) + lam / 4 * (J ** 2 - 1)
    P = [[sp.simplify(sp.diff(Wsym, Fs[i, j])) for j in range(D)] for i in range(D)]
    return Fs, mu, lam, P


def _frac_solve(A, b):
    """exact solution of a consistent overdetermined system by elimination"""
    A = [row[:] + [bb] for row, bb in zip(A, b)]
    nr, nc = len(A), len(A[0]) - 1
    piv_rows, r = [], 0
    for c in range(nc):
        p = next((i for i in range(r, nr) if A[i][c] != 0), None)
        if p is None:
            continue
        A[r], A[p] = A[p], A[r]
        inv = 1 / A[r][c]
        A[r] = [x * inv for x in A[r]]
        for i in range(nr):
            if i != r and A[i][c] != 0:
                fct = A[i][c]
                A[i] = [x - fct * y for x, y in zip(A[i], A[r])]
        piv_rows.append(c)
        r += 1
    assert r == nc
    for i in range(r, nr):
        assert A[i][-1] == 0  # consistent
    x = [Fraction(0)] * nc
    for i, c in enumerate(piv_rows):
        x[c] = A[i][-1]
    return x


@pytest.mark.parametrize("D,n", [(2, (3, 2)), (3, (2, 2, 2))])
def test_brute_force_exact_rational(orc, D, n):
    M, Q = D + D * D, 2 * D
    N = int(np.prod(n))
    mu, lam, rho0 = Fraction(1), Fraction(2), Fraction(1)
    dx, dt = Fraction(1, 4), Fraction(1, 40)
    c = dx / dt
    om = Fraction(9, 5)
    rng = np.random.default_rng(12)
    U0 = []
    for i in range(N):
        v = [Fraction(int(x), 1000) for x in rng.integers(-50, 50, D)]
        F = [[Fraction(int(i == j)) + Fraction(int(x), 100) for j, x in enumerate(rng.integers(-10, 10, D))]
             for i in range(D)]
        U0.append(v + [F[i][j] for i in range(D) for j in range(D)])
    Fs, msym, lsym, Psym = _exact_piola(D)

    def piola(F):
        sub = {Fs[i, j]: sp.Rational(F[i * D + j].numerator, F[i * D + j].denominator)
               for i in range(D) for j in range(D)}
        sub[msym], sub[lsym] = sp.Rational(1), sp.Rational(2)
        out = []
        for i in range(D):
            for j in range(D):
                val = sp.Rational(Psym[i][j].subs(sub))
                out.append(Fraction(int(val.p), int(val.q)))
        return out

    def evec(q):
        e = [0] * D
        e[q // 2] = -1 if q & 1 else 1
        return e

    def feq(U):
        P = piola(U[D:])
        Phi = [[(-P[r * D + A] / rho0) if r < D else
                (-U[(r - D) // D] if (r - D) % D == A else Fraction(0)) for r in range(M)] for A in range(D)]
        out = [[None] * M for _ in range(Q)]
        for r in range(M):
            rows, rhs = [], []
            rows.append([Fraction(1)] * Q); rhs.append(U[r])
            for A in range(D):
                rows.append([c * evec(q)[A] for q in range(Q)]); rhs.append(Phi[A][r])
                row = [Fraction(0)] * Q
                row[2 * A] = row[2 * A + 1] = Fraction(1)
                rows.append(row); rhs.append(U[r] / D)
            sol = _frac_solve(rows, rhs)
            for q in range(Q):
                out[q][r] = sol[q]
        return out

    def idx(cc):
        return cc[0] + n[0] * (cc[1] + (n[1] * cc[2] if D == 3 else 0))

    coords = [tuple(int(x) for x in np.unravel_index(i, n[::-1])[::-1]) for i in range(N)]
    f = [feq(U0[i]) for i in range(N)]  # equilibrium start (no gradients, no source)
    for _ in range(2):
        fs = []
        for i in range(N):
            U = [sum(f[i][q][r] for q in range(Q)) for r in range(M)]
            fe = feq(U)
            fs.append([[f[i][q][r] + om * (fe[q][r] - f[i][q][r]) for r in range(M)] for q in range(Q)])
        fn = [[None] * Q for _ in range(N)]
        for i in range(N):
            for q in range(Q):
                cc = list(coords[i])
                cc[q // 2] = (cc[q // 2] + evec(q)[q // 2]) % n[q // 2]
                fn[idx(cc)][q] = fs[i][q]
        f = fn
    s = orc.Sim(D, n, float(dx), float(dt), 1.0, 2.0, omega=float(om))
    s.set_state(np.array([[float(U0[i][r]) for i in range(N)] for r in range(M)]))
    s.step(2)
    fo = s.get_f()
    ref = np.array([[[float(f[i][q][r]) for i in range(N)] for r in range(M)] for q in range(Q)])
    assert np.abs(fo - ref).max() < 1e-14


def test_unstable_lattice_speed_reports_nonpositive_jacobian(orc):
    """c = 1 (dt = dx) is below the stability threshold of the scheme for
    mu = 1, lam = 2 at omega = 1.8; the run must stop with a J <= 0 or
    non-finite status instead of returning garbage."""
    c = W.config_c1()
    s = orc.Sim(2, c["n"], c["dx"], c["dx"], c["mu"], c["lam"], omega=c["omega"])
    s.set_state(c["U0"], dU0=c["dU0"])
    with pytest.raises(orc.OracleError) as ei:
        s.step(2000)
    assert ei.value.code in (4, 6)
