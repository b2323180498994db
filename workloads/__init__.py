"""Seeded synthetic inputs shaped like the paper's workloads.

This module is shared by the GPU path's tests/benchmark and by the oracle's
tests.  It holds no arithmetic of the method itself: only grids, level-set
samples, boundary identifiers, initial fields (and their analytic spatial
derivatives) and the per-configuration parameters.

Grids are cell centred: node i sits at origin + (i + 1/2) dx.  Embedded
domains live in the unit box [0,1]^D with dx = 1/N and one inactive frame
layer on each non-periodic side, so that every cut link of the body ends on a
grid node.  Flattened arrays use x fastest: index = x + nx*(y + ny*z).
"""
from __future__ import annotations

import itertools
import math

import numpy as np

SEED = 20646


# ---------------------------------------------------------------- grids -----

def node_coords(n, dx, origin):
    """Flattened node coordinates [D][N] (x fastest)."""
    D = len(n)
    axes = [origin[a] + (np.arange(n[a]) + 0.5) * dx for a in range(D)]
    mesh = np.meshgrid(*axes[::-1], indexing="ij")  # (z, y, x) order
    return np.stack([m.reshape(-1) for m in mesh[::-1]])


def framed_box(N, D, pad=1):
    """Unit box with N cells per axis plus `pad` inactive frame layers."""
    n = [N + 2 * pad] * D
    dx = 1.0 / N
    origin = [-pad * dx] * D
    return dict(n=n, dx=dx, origin=origin, periodic_mask=0)


# ------------------------------------------------------ initial fields -------

def fourier_modes(rng, D, nmodes=8, kmax=4.0):
    """Integer wave vectors 1 <= |k| <= kmax drawn without replacement, and
    normal amplitude vectors a_m, b_m."""
    r = int(math.floor(kmax))
    cand = [k for k in itertools.product(range(-r, r + 1), repeat=D)
            if 1.0 <= math.sqrt(sum(c * c for c in k)) <= kmax]
    cand = np.array(cand, dtype=np.int64)
    idx = rng.choice(len(cand), size=nmodes, replace=False)
    k = cand[idx]
    a = rng.standard_normal((nmodes, D))
    b = rng.standard_normal((nmodes, D))
    return k, a, b


def fourier_velocity(X, modes, amp):
    """v(X) = amp * sum_m [a_m cos(2 pi k_m.X) + b_m sin(2 pi k_m.X)] and its
    analytic gradient dv[A][i] = d v_i / d X_A."""
    k, a, b = modes
    D, N = X.shape
    v = np.zeros((D, N))
    dv = np.zeros((D, D, N))
    for m in range(k.shape[0]):
        th = 2.0 * np.pi * (k[m] @ X)
        c, s = np.cos(th), np.sin(th)
        for i in range(D):
            v[i] += amp * (a[m, i] * c + b[m, i] * s)
            for A in range(D):
                dv[A, i] += amp * 2.0 * np.pi * k[m, A] * (-a[m, i] * s + b[m, i] * c)
    return v, dv


def state_from(v, dv, F0):
    """Planar state U0[M][N] for uniform F0 and its gradient dU0[D][M][N]
    (the state ordering is (v, F row-major))."""
    D, N = v.shape
    M = D + D * D
    U0 = np.empty((M, N))
    U0[:D] = v
    U0[D:] = np.asarray(F0, float).reshape(-1)[:, None]
    dU0 = np.zeros((D, M, N))
    dU0[:, :D, :] = dv
    return U0, dU0


def periodic_case(D, N, F0_fn, amp, seed=SEED):
    """Periodic unit box, N^D nodes, uniform F0 plus Fourier velocity modes."""
    rng = np.random.default_rng(seed)
    modes = fourier_modes(rng, D)
    F0 = F0_fn(rng)
    n = [N] * D
    dx = 1.0 / N
    X = node_coords(n, dx, [0.0] * D)
    v, dv = fourier_velocity(X, modes, amp)
    U0, dU0 = state_from(v, dv, F0)
    return dict(D=D, n=n, dx=dx, origin=[0.0] * D, periodic_mask=(1 << D) - 1, U0=U0, dU0=dU0,
                F0=np.asarray(F0), modes=modes)


# --------------------------------------------------------- level sets -------

def annulus_phi(X, center, r_in, r_out):
    """Annulus r_in <= r <= r_out as {phi <= 0}; bid 1 inside the hole, 2
    outside the outer circle."""
    d = X - np.asarray(center, float)[:, None]
    r = np.sqrt((d * d).sum(0))
    phi = np.maximum(r_in - r, r - r_out)
    bid = np.where(r < 0.5 * (r_in + r_out), 1, 2).astype(np.uint8)
    return phi, bid


def superellipse_phi(X, center, a, b, theta_deg, p=4.0):
    th = math.radians(theta_deg)
    d = X - np.asarray(center, float)[:, None]
    xi = math.cos(th) * d[0] + math.sin(th) * d[1]
    ze = -math.sin(th) * d[0] + math.cos(th) * d[1]
    return np.abs(xi / a) ** p + np.abs(ze / b) ** p - 1.0


def rot_y(deg):
    t = math.radians(deg)
    return np.array([[math.cos(t), 0, math.sin(t)], [0, 1, 0], [-math.sin(t), 0, math.cos(t)]])


def rot_z(deg):
    t = math.radians(deg)
    return np.array([[math.cos(t), -math.sin(t), 0], [math.sin(t), math.cos(t), 0], [0, 0, 1]])


def ellipsoid_phi(X, center, axes, Q):
    xi = Q.T @ (X - np.asarray(center, float)[:, None])
    return sum((xi[a] / axes[a]) ** 2 for a in range(3)) - 1.0


def sphere_phi(X, center, R):
    d = X - np.asarray(center, float)[:, None]
    return np.sqrt((d * d).sum(0)) - R


# ---------------------------------------------------- paper geometries ------

def geom_affine_annulus(N=384):
    g = framed_box(N, 2)
    X = node_coords(g["n"], g["dx"], g["origin"])
    phi, bid = annulus_phi(X, (0.5, 0.5), 0.18, 0.42)
    return dict(g, phi=phi, bid=bid, X=X)


def geom_radial_annulus(N=196):
    g = framed_box(N, 2)
    X = node_coords(g["n"], g["dx"], g["origin"])
    phi, bid = annulus_phi(X, (0.5, 0.5), 0.18, 0.42)
    return dict(g, phi=phi, bid=bid, X=X)


def geom_superellipse(N=384):
    g = framed_box(N, 2)
    X = node_coords(g["n"], g["dx"], g["origin"])
    po = superellipse_phi(X, (0.5, 0.5), 0.42, 0.30, 20.0)
    pi = superellipse_phi(X, (0.5, 0.5), 0.16, 0.10, -15.0)
    phi = np.maximum(po, -pi)
    bid = np.where(pi < 0, 1, 2).astype(np.uint8)
    return dict(g, phi=phi, bid=bid, X=X)


def geom_ellipsoid(N=320):
    g = framed_box(N, 3)
    X = node_coords(g["n"], g["dx"], g["origin"])
    phi = ellipsoid_phi(X, (0.5, 0.5, 0.5), (0.34, 0.25, 0.18), rot_z(25.0) @ rot_y(18.0))
    return dict(g, phi=phi, bid=np.ones(phi.shape, np.uint8), X=X)


def geom_spherical_shell(N=200):
    g = framed_box(N, 3)
    X = node_coords(g["n"], g["dx"], g["origin"])
    d = X - 0.5
    r = np.sqrt((d * d).sum(0))
    phi = np.maximum(0.20 - r, r - 0.38)
    bid = np.where(r < 0.29, 1, 2).astype(np.uint8)
    return dict(g, phi=phi, bid=bid, X=X)


def geom_tube():
    """Hollow cylinder R_i=0.15..R_o=0.30 about (0.38, 0.38), 0 <= Z <= 3,
    on the 76x76x300 lattice with dx = 0.01 (plus a frame)."""
    dx = 0.01
    n = [78, 78, 302]
    origin = [-dx, -dx, -dx]
    X = node_coords(n, dx, origin)
    R = np.sqrt((X[0] - 0.38) ** 2 + (X[1] - 0.38) ** 2)
    phi = np.maximum.reduce([0.15 - R, R - 0.30, -X[2], X[2] - 3.0])
    bid = np.full(phi.shape, 2, np.uint8)
    bid[R < 0.225] = 1
    bid[X[2] < 0] = 3
    bid[X[2] > 3.0] = 4
    return dict(n=n, dx=dx, origin=origin, periodic_mask=0, phi=phi, bid=bid, X=X)


# ------------------------------------------------------------ configs -------

def config_c1(seed=SEED):
    """2D D2Q4x6 periodic 64^2 FP64: mu=1, lam=2, F0 = I + 0.1 e1(x)e2,
    v0 = 1e-3 * 8 Fourier modes; c = 10 (dt = dx/10), omega = 1.8."""
    F0 = np.array([[1.0, 0.1], [0.0, 1.0]])
    case = periodic_case(2, 64, lambda rng: F0, 1e-3, seed)
    return dict(case, mu=1.0, lam=2.0, rho0=1.0, c=10.0, dt=case["dx"] / 10.0, omega=1.8, gamma=0.0,
                steps=1000)


def config_c3(N=256, seed=SEED):
    """3D D3Q6x12 periodic N^3 FP32: mu=1, lam=2, F0 = I + 0.05 A (A seeded
    Gaussian), v0 = 1e-3 * 8 Fourier modes; c = 10, omega = 1.8."""
    def F0_fn(rng):
        A = rng.standard_normal((3, 3))
        F0 = np.eye(3) + 0.05 * A
        assert np.linalg.det(F0) > 0
        return F0
    case = periodic_case(3, N, F0_fn, 1e-3, seed)
    return dict(case, mu=1.0, lam=2.0, rho0=1.0, c=10.0, dt=case["dx"] / 10.0, omega=1.8, gamma=0.0,
                steps=1000)


def config_c2(N=512):
    """2D embedded annulus 0.25 <= r <= 0.5 about (0.5, 0.5); inner surface
    radial displacement 0.05 s(t) e_R (sine-squared ramp, T_r = 2), outer
    surface traction free; mu=1, lam=10, c=10, omega=1.8, gamma=10,
    projection every 20 steps."""
    g = framed_box(N, 2)
    X = node_coords(g["n"], g["dx"], g["origin"])
    phi, bid = annulus_phi(X, (0.5, 0.5), 0.25, 0.5)
    dt = g["dx"] / 10.0
    bcs = {
        1: dict(type="dirichlet", ramp="sin2", T_r=2.0, given_as_displacement=True, p_radial=0.05,
                X0=(0.5, 0.5)),
        2: dict(type="neumann"),
    }
    M = 6
    Npts = X.shape[1]
    U0 = np.zeros((M, Npts))
    U0[2] = 1.0
    U0[5] = 1.0
    return dict(g, D=2, X=X, phi=phi, bid=bid, bcs=bcs, mu=1.0, lam=10.0, rho0=1.0, c=10.0, dt=dt,
                omega=1.8, gamma=10.0, proj_every=20, U0=U0, steps=20000)


def config_c5(N=192, seed=SEED, mu=1.0, lam=2.0):
    """3D embedded sphere of radius 0.35 about the box centre, traction-free
    surface; v0 = 1e-2 * 8 Fourier modes, F0 = I."""
    g = framed_box(N, 3)
    X = node_coords(g["n"], g["dx"], g["origin"])
    phi = sphere_phi(X, (0.5, 0.5, 0.5), 0.35)
    rng = np.random.default_rng(seed)
    modes = fourier_modes(rng, 3)
    v, dv = fourier_velocity(X, modes, 1e-2)
    U0, dU0 = state_from(v, dv, np.eye(3))
    return dict(g, D=3, X=X, phi=phi, bid=np.ones(phi.shape, np.uint8), bcs={1: dict(type="neumann")},
                mu=mu, lam=lam, rho0=1.0, c=10.0, dt=g["dx"] / 10.0, omega=1.8, gamma=0.0,
                proj_every=20, U0=U0, dU0=dU0, steps=4000)


def config_c4_instance(k, seed=SEED, N=None, redraw=True):
    """One instance of the batched 2D workload: unit square with 1-5 random
    circular holes, clamped left edge, traction (0.02 mu, 0) on the right
    edge (sine-squared ramp over 500 steps), other surfaces traction free.
    A hole that would leave a ligament narrower than 4 cells to another hole,
    or cut into one at a grazing depth (< 0.03), is drawn again: the
    embedding needs a few active nodes across every ligament (sub-cell
    slivers fail the local traction solve).  redraw=False keeps the first
    draw (the geometry with slivers, for the failure path)."""
    rng = np.random.default_rng(seed + k)
    Nk = int(rng.integers(64, 513)) if N is None else N
    nh = int(rng.integers(1, 6))
    centres = rng.uniform(0.25, 0.75, size=(nh, 2))
    radii = rng.uniform(0.05, 0.15, size=nh)

    def bad(j):
        for i in range(j):
            gap = float(np.linalg.norm(centres[i] - centres[j])) - radii[i] - radii[j]
            if -0.03 < gap < 4.0 / Nk:
                return True
        return False

    for j in range(1, nh if redraw else 1):
        for _ in range(1000):
            if not bad(j):
                break
            centres[j] = rng.uniform(0.25, 0.75, size=2)
            radii[j] = rng.uniform(0.05, 0.15)
    mu = float(rng.uniform(0.5, 2.0))
    lam = float(mu * math.exp(rng.uniform(0.0, math.log(50.0))))
    g = framed_box(Nk, 2)
    X = node_coords(g["n"], g["dx"], g["origin"])
    phi = np.maximum.reduce([-X[0], X[0] - 1.0, -X[1], X[1] - 1.0])
    hole = np.full(X.shape[1], -np.inf)
    for c, r in zip(centres, radii):
        hole = np.maximum(hole, r - np.sqrt((X[0] - c[0]) ** 2 + (X[1] - c[1]) ** 2))
    phi = np.maximum(phi, hole)
    bid = np.full(X.shape[1], 3, np.uint8)
    bid[X[0] < 0.0] = 1
    bid[X[0] > 1.0] = 2
    cmax = math.sqrt(lam + 2.0 * mu)
    c = max(10.0, 1.25 * 2 * cmax)
    dt = g["dx"] / c
    bcs = {1: dict(type="dirichlet"),
           2: dict(type="neumann", ramp="sin2", T_r=500 * dt, a=(0.02 * mu, 0.0)),
           3: dict(type="neumann")}
    U0 = np.zeros((6, X.shape[1]))
    U0[2] = 1.0
    U0[5] = 1.0
    return dict(g, D=2, X=X, phi=phi, bid=bid, bcs=bcs, mu=mu, lam=lam, rho0=1.0, c=c, dt=dt, omega=1.8,
                gamma=10.0, proj_every=20, U0=U0, steps=2000, N_cells=Nk, hole_centres=centres,
                hole_radii=radii)


def config_ellipsoid(N=320):
    """Rotated ellipsoid (Sec. 5.1): semi-axes (0.34, 0.25, 0.18), Q = R_z(25)
    R_y(18) about the box centre; velocity Dirichlet data v = A (X - X_c) on
    the whole surface, the same affine velocity as initial state (u0 = 0,
    F0 = I); mu = 1, lambda = 2/3, omega = 1.8, no damping, no projection
    (Dirichlet only), final time 0.4599."""
    g = geom_ellipsoid(N)
    A = np.array([[0.0, 0.80, 0.0], [0.0, 0.0, -0.60], [0.45, 0.0, 0.08]])
    Xc = np.array([0.5, 0.5, 0.5])
    X = g["X"]
    v0 = A @ (X - Xc[:, None])
    M = 12
    U0 = np.zeros((M, X.shape[1]))
    U0[:3] = v0
    for k in range(3):
        U0[3 + 4 * k] = 1.0
    dU0 = np.zeros((3, M, X.shape[1]))
    for B in range(3):
        for i in range(3):
            dU0[B, i] = A[i, B]
    dt = g["dx"] / 10.0
    T = 0.4599
    return dict(g, D=3, A=A, Xc=Xc, mu=1.0, lam=2.0 / 3.0, rho0=1.0, c=10.0, dt=dt, omega=1.8, gamma=0.0,
                proj_every=20, U0=U0, dU0=dU0, T=T, steps=int(round(T / dt)),
                bcs={1: dict(type="dirichlet", G=A, X0=tuple(Xc))})


def config_shell(N=200, Pr_inner=-1.15242):
    """Spherical shell R_i = 0.20 <= R <= R_o = 0.38 (Sec. 5.2): both
    surfaces Neumann; the cavity receives the nominal traction -P_r(R_i) e_R
    of the radial reference state (sine-squared ramp, T_r = 2), the outer
    surface is traction free; mu = 1, lambda = 2/3, omega = 1.8, gamma = 10,
    projection every 20 steps, run to t = 5 from rest."""
    g = geom_spherical_shell(N)
    X = g["X"]
    M = 12
    U0 = np.zeros((M, X.shape[1]))
    for k in range(3):
        U0[3 + 4 * k] = 1.0
    dt = g["dx"] / 10.0
    Xc = (0.5, 0.5, 0.5)
    return dict(g, D=3, mu=1.0, lam=2.0 / 3.0, rho0=1.0, c=10.0, dt=dt, omega=1.8, gamma=10.0, proj_every=20,
                U0=U0, T=5.0, steps=int(round(5.0 / dt)), Xc=np.array(Xc),
                bcs={1: dict(type="neumann", ramp="sin2", T_r=2.0, p_radial=-Pr_inner, X0=Xc),
                     2: dict(type="neumann")})


def config_radial_annulus(N=196):
    """Radial traction annulus (Sec. 4.3): R_i = 0.18 <= R <= R_o = 0.42
    about (0.5, 0.5); inner surface clamped, outer surface loaded by the
    nominal radial traction p0 s(t) e_R, p0 = 1 (sine-squared ramp, T_r = 2),
    run to t = 5 from rest; mu = 1, lambda = 2/3, omega = 1.8, gamma = 10,
    projection every 20 steps."""
    g = geom_radial_annulus(N)
    X = g["X"]
    U0 = np.zeros((6, X.shape[1]))
    U0[2] = U0[5] = 1.0
    dt = g["dx"] / 10.0
    return dict(g, D=2, mu=1.0, lam=2.0 / 3.0, rho0=1.0, c=10.0, dt=dt, omega=1.8, gamma=10.0, proj_every=20,
                U0=U0, T=5.0, steps=int(round(5.0 / dt)), Xc=np.array([0.5, 0.5]),
                bcs={1: dict(type="dirichlet"),
                     2: dict(type="neumann", ramp="sin2", T_r=2.0, p_radial=1.0, X0=(0.5, 0.5))})


def config_affine_annulus(N=384):
    """Affine Dirichlet annulus (Sec. 4.2): R_i = 0.18 <= R <= R_o = 0.42
    about (0.5, 0.5); both surfaces carry the velocity v = A (X - Xc) / T,
    T = 0.2, A = [[0.35, 0.18], [-0.10, 0.24]], which is also the initial
    velocity (u0 = 0, F0 = I); mu = 1, lambda = 2/3, omega = 2, no damping,
    no projection (Dirichlet only)."""
    g = geom_affine_annulus(N)
    X = g["X"]
    A = np.array([[0.35, 0.18], [-0.10, 0.24]])
    T = 0.2
    Xc = np.array([0.5, 0.5])
    G = A / T
    U0 = np.zeros((6, X.shape[1]))
    U0[:2] = G @ (X - Xc[:, None])
    U0[2] = U0[5] = 1.0
    dU0 = np.zeros((2, 6, X.shape[1]))
    for B in range(2):
        for i in range(2):
            dU0[B, i] = G[i, B]
    dt = g["dx"] / 10.0
    return dict(g, D=2, A=G, Xc=Xc, mu=1.0, lam=2.0 / 3.0, rho0=1.0, c=10.0, dt=dt, omega=2.0, gamma=0.0,
                proj_every=20, U0=U0, dU0=dU0, T=T, steps=int(round(T / dt)),
                bcs={1: dict(type="dirichlet", G=G, X0=(0.5, 0.5)), 2: dict(type="dirichlet", G=G, X0=(0.5, 0.5))})


def config_tube(cells_per_unit=100):
    """Finite tube under end stretch and twist (Sec. 5.3): R_i = 0.15 <= R <=
    R_o = 0.30 about the axis (0.38, 0.38), 0 <= Z <= 3 (the paper's lattice
    is 76 x 76 x 300 nodes at dx = 0.01, cells_per_unit = 100); both walls
    traction free, the end Z = 0 clamped, the end Z = 3 displaced by
    u_D = ((R(alpha) - I) X_perp, dL) with alpha = s(t) 45 deg,
    dL = s(t) 0.5 L (half-cosine ramp, T_r = 10), relaxed to t = 100;
    mu = 1, lambda = 2/3, omega = 1.8, gamma = 10, projection every 20 steps."""
    dx = 1.0 / cells_per_unit
    nxy = int(round(0.76 / dx))
    nz = int(round(3.0 / dx))
    n = [nxy + 2, nxy + 2, nz + 2]
    origin = [-dx, -dx, -dx]
    X = node_coords(n, dx, origin)
    R = np.sqrt((X[0] - 0.38) ** 2 + (X[1] - 0.38) ** 2)
    phi = np.maximum.reduce([0.15 - R, R - 0.30, -X[2], X[2] - 3.0])
    bid = np.full(phi.shape, 2, np.uint8)
    bid[R < 0.225] = 1
    bid[X[2] < 0] = 3
    bid[X[2] > 3.0] = 4
    U0 = np.zeros((12, X.shape[1]))
    for k in range(3):
        U0[3 + 4 * k] = 1.0
    dt = dx / 10.0
    return dict(n=n, dx=dx, origin=origin, periodic_mask=0, phi=phi, bid=bid, X=X, D=3, mu=1.0, lam=2.0 / 3.0,
                rho0=1.0, c=10.0, dt=dt, omega=1.8, gamma=10.0, proj_every=20, U0=U0, T=100.0,
                steps=int(round(100.0 / dt)),
                bcs={1: dict(type="neumann"), 2: dict(type="neumann"),
                     3: dict(type="dirichlet", given_as_displacement=True),
                     4: dict(type="dirichlet", given_as_displacement=True, ramp="halfcos", T_r=10.0,
                             a=(0.0, 0.0, 1.5), twist=math.pi / 4, X0=(0.38, 0.38, 0.0))})
