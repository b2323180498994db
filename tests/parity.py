"""Per-component state comparison of the GPU path against the oracle.

The state U = (v, F) mixes two scales: F is close to the identity (about
sqrt(D) per node) while v and F - I are small.  A relative error over the
whole of U is dominated by the identity part and hides errors in v and in
the deformation; every parity test therefore gates each part on its own
scale:
  ||v_gpu - v_orc|| / ||v_orc||,
  ||F_gpu - F_orc|| / ||F_orc - I||,
  ||u_gpu - u_orc|| / ||u_orc||          (when the displacement is compared),
and the largest pointwise error of each part against that part's largest
magnitude (max|dv| / max|v_orc|, max|dF| / max|F_orc - I|, max|du| /
max|u_orc|).  Norms run over the active nodes given by the mask.

FP64 floor.  The oracle keeps the raw populations f_q in FP64; each is
rounded once per step, so after n steps a moment row r carries up to
n * eps * sum_q |f_q^r| of rounding at every node (eps = 2^-52).  The stress
P = mu F + (b - a) cof F (b - a = lambda (J^2 - 1)/(2J) - mu/J) is a sum of
O(1) terms whose rounding enters the velocity rows through the flux,
omega P/(2c rho0) per population: a further n * eps * (omega / (c rho0))
sum_A (|mu F_iA| + |b - a| |cof F_iA|) per node for velocity row i.  Where a
part is small against these (the velocity rows carry the static stress, the
deformation rows carry F ~ I), the floor exceeds 1e-12 of the part.  The
dynamics carry an error of one part into the other along the characteristics
(dv = c_p dF, c_p = sqrt((lambda + 2 mu) / rho0)), so each part's floor also
includes the other's, converted.  On the
64^2 periodic run after 1000 steps the oracle's own velocity differs from an
80-bit extended-precision run of the same update by 2.9e-12 relative.  Given
the raw populations and the step count (and the material for the stress
terms), each gate is tol * |part| + 4 * floor: the floor counts the stored
populations and the stress; the cut-link closures (interpolation, boundary
stress, the Newton solve's stopping point) and the displacement quadrature
round at the same scale, and each side is allowed twice the counted floor.
Measured at the pointwise maxima of embedded runs early in a load ramp
(where |F - I| is small): up to 2.9 times the counted floor.  For the FP32
tolerance the floor is negligible.
"""
import numpy as np

EPS64 = 2.0 ** -52
FLOOR_FACTOR = 4.0


def _split(U, D):
    v = U[:D]
    F = U[D:D + D * D]
    return v, F


def _stress_terms(F, D, mu, lam):
    """|mu F| + |b - a| |cof F| entrywise [D*D][nodes] for the planar F rows"""
    Fm = np.ascontiguousarray(F.T).reshape(-1, D, D)
    J = np.linalg.det(Fm)
    C = np.linalg.inv(Fm).transpose(0, 2, 1) * J[:, None, None]
    ba = np.abs(0.5 * lam * (J * J - 1.0) / J - mu / J)
    T = np.abs(mu * Fm) + ba[:, None, None] * np.abs(C)
    return T.reshape(-1, D * D).T


def component_errors(Ug, Uo, D, ug=None, uo=None, mask=None, pops=None, steps=0, stress=None, acoustic_v=False):
    """Relative errors per part; with the raw populations pops [Q][M][N] and
    the step count, also each part's FP64 floor on the same scale (keys
    'v_floor', 'F_floor', 'v_max_floor', 'F_max_floor'); stress = (mu,
    lambda, rho0, c, omega) adds the stress terms to the velocity floor.
    acoustic_v (needs stress): the velocity is measured on the scale of the
    velocities the deformation carries, c_p |F - I| (c_p = sqrt((lambda +
    2 mu) / rho0)), when that is larger than its own size: for a body at
    quasi-static equilibrium, whose remaining velocity is a decaying
    remainder far below that scale."""
    if mask is not None:
        Ug, Uo = Ug[:, mask], Uo[:, mask]
        if ug is not None:
            ug, uo = ug[:, mask], uo[:, mask]
        if pops is not None:
            pops = pops[:, :, mask]
    vg, Fg = _split(Ug, D)
    vo, Fo = _split(Uo, D)
    I = np.eye(D).reshape(-1)[:, None]
    dF = Fo - I
    nv, nF, mv, mF = np.linalg.norm(vo), np.linalg.norm(dF), np.abs(vo).max(), np.abs(dF).max()
    if acoustic_v:
        cp = np.sqrt((stress[1] + 2.0 * stress[0]) / stress[2])
        nv, mv = max(nv, cp * nF), max(mv, cp * mF)
    e = {
        "U": np.linalg.norm(Ug - Uo) / np.linalg.norm(Uo),
        "v": np.linalg.norm(vg - vo) / nv,
        "F": np.linalg.norm(Fg - Fo) / nF,
        "v_max": np.abs(vg - vo).max() / mv,
        "F_max": np.abs(Fg - Fo).max() / mF,
    }
    if ug is not None:
        e["u"] = np.linalg.norm(ug - uo) / np.linalg.norm(uo)
        e["u_max"] = np.abs(ug - uo).max() / np.abs(uo).max()
    if pops is not None:
        a = np.abs(pops).sum(0)  # [M][nodes]
        if stress is not None:
            mu, lam, rho0, c, om = stress
            T = _stress_terms(Fo, D, mu, lam)
            for i in range(D):
                a[i] += om / (c * rho0) * T[i * D:(i + 1) * D].sum(0)
        k = steps * EPS64
        fv, fF = k * np.linalg.norm(a[:D]), k * np.linalg.norm(a[D:])
        mvf, mFf = k * a[:D].max(), k * a[D:].max()
        if stress is not None:
            cp = np.sqrt((lam + 2.0 * mu) / rho0)
            fv, fF = fv + cp * fF, fF + fv / cp
            mvf, mFf = mvf + cp * mFf, mFf + mvf / cp
        e["v_floor"] = fv / nv
        e["F_floor"] = fF / nF
        e["v_max_floor"] = mvf / mv
        e["F_max_floor"] = mFf / mF
    return {k: float(v) for k, v in e.items()}


def check(Ug, Uo, D, tol, ug=None, uo=None, utol=None, mask=None, label="", max_tol=None, pops=None, steps=0,
          stress=None, acoustic_v=False):
    """Assert every per-component error is within tol (utol for the
    displacement, max_tol for the pointwise ratios; both default to tol),
    plus four times the FP64 floor of the part when the raw populations pops
    and the step count are given (stress: see component_errors)."""
    e = component_errors(Ug, Uo, D, ug, uo, mask, pops, steps, stress, acoustic_v)
    print(f"[parity] {label} " + " ".join(f"{k}={v:.2e}" for k, v in e.items()), flush=True)
    utol = tol if utol is None else utol
    max_tol = tol if max_tol is None else max_tol
    bad = []
    for k in ("v", "F"):
        if not e[k] <= tol + FLOOR_FACTOR * e.get(k + "_floor", 0.0):
            bad.append(k)
        if not e[k + "_max"] <= max_tol + FLOOR_FACTOR * e.get(k + "_max_floor", 0.0):
            bad.append(k + "_max")
    if "u" in e:
        # u integrates v and the projection rebuilds it from F: its floor is
        # the larger of theirs
        uf = max(e.get("v_floor", 0.0), e.get("F_floor", 0.0))
        ufm = max(e.get("v_max_floor", 0.0), e.get("F_max_floor", 0.0))
        if not e["u"] <= utol + FLOOR_FACTOR * uf:
            bad.append("u")
        if not e["u_max"] <= max(utol, max_tol) + FLOOR_FACTOR * ufm:
            bad.append("u_max")
    assert not bad, f"{label}: {bad} above tolerance ({tol:g}/{utol:g}/{max_tol:g}): {e}"
    return e
