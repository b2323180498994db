"""Write the full-length oracle goldens of the two embedded 2D configurations.

  c2_512_20000_samples.txt    the annulus 0.25 <= R <= 0.5 on 512^2 (+frame):
                              inner surface displaced radially by 0.05 s(t)
                              (sine-squared ramp, T_r = 2), outer surface
                              traction free, mu = 1, lambda = 10, gamma = 10,
                              projection every 20 steps, 20000 steps
  c4_2000_samples.txt         three instances of the batched random-hole
                              recipe (the smallest, a middle and the largest
                              grid of the 64), 2000 steps each

Only the oracle (FP64) and the seeded input generators run here.  Each file
holds, per case, the oracle's state at seeded sample nodes (half drawn from
all active nodes, half from the active nodes that own a cut link):
  node U_0..U_{M-1} u_0..u_{D-1} a_0..a_{M-1}
with U = (v, F), u the displacement and a_r = sum_q |f_q^r| the magnitude of
the raw populations of row r there (the FP64 rounding floor of the parity
gates), and the norms of v, F - I and u over all active nodes.

    python tests/golden/make_embedded_golden.py [c2|c4|all]
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import oracle as O  # noqa: E402

C4_INSTANCES = (45, 7, 63)  # 65^2, 292^2 and 512^2 cells
NSAMPLE = 192


def _sim(c):
    o = O.Sim(2, c["n"], c["dx"], c["dt"], c["mu"], c["lam"], omega=c["omega"], gamma=c["gamma"],
              origin=c["origin"], periodic_mask=0, proj_every=c["proj_every"])
    o.set_levelset(c["phi"], c["bid"])
    kinds = {"dirichlet": O.DIRICHLET, "neumann": O.NEUMANN}
    ramps = {"const": O.RAMP_CONST, "sin2": O.RAMP_SIN2}
    for bid, bc in c["bcs"].items():
        bc = dict(bc)
        t = kinds[bc.pop("type")]
        if "ramp" in bc:
            bc["ramp"] = ramps[bc["ramp"]]
        o.set_bc(bid, t, **bc)
    o.set_state(c["U0"])
    return o


def _samples(c, o, seed):
    act = np.flatnonzero(c["phi"] <= 0)
    link_nodes = np.unique(o.links()["node"])
    rng = np.random.default_rng(seed)
    a = rng.choice(act, NSAMPLE, replace=False)
    b = rng.choice(link_nodes, NSAMPLE, replace=False)
    return np.unique(np.concatenate([a, b]))


def _write_case(f, name, c, steps, seed):
    print(f"[golden] {name}: {steps} steps", flush=True)
    o = _sim(c)
    o.step(steps)
    U, u, _ = o.moments()
    fr = o.get_f()
    act = c["phi"] <= 0
    idx = _samples(c, o, seed)
    a = np.abs(fr).sum(0)
    I = np.eye(2).reshape(-1)[:, None]
    f.write(f"case {name} steps {steps} nodes {len(idx)}\n")
    f.write("norms {:.17e} {:.17e} {:.17e}\n".format(np.linalg.norm(U[:2, act]), np.linalg.norm((U[2:] - I)[:, act]),
                                                     np.linalg.norm(u[:, act])))
    f.write("pops_norms {:.6e} {:.6e} {:.6e} {:.6e}\n".format(np.linalg.norm(a[:2, act]), np.linalg.norm(a[2:, act]),
                                                               a[:2, act].max(), a[2:, act].max()))
    for i in idx:
        f.write(f"{i} " + " ".join(f"{x:.17e}" for x in U[:, i]) + " " +
                " ".join(f"{x:.17e}" for x in u[:, i]) + " " + " ".join(f"{x:.6e}" for x in a[:, i]) + "\n")
    f.flush()


def main(which):
    if which in ("c2", "all"):
        with open(os.path.join(HERE, "c2_512_20000_samples.txt"), "w") as f:
            f.write("# FP64 oracle, the embedded annulus configuration (Sec. 4.3 geometry, 512^2 + frame),\n"
                    "# written by tests/golden/make_embedded_golden.py from the oracle alone\n")
            _write_case(f, "c2", W.config_c2(512), 20000, 1)
    if which in ("c4", "all"):
        with open(os.path.join(HERE, "c4_2000_samples.txt"), "w") as f:
            f.write("# FP64 oracle, three instances of the batched random-hole recipe, 2000 steps each,\n"
                    "# written by tests/golden/make_embedded_golden.py from the oracle alone\n")
            for k in C4_INSTANCES:
                _write_case(f, f"c4_{k}", W.config_c4_instance(k), 2000, 100 + k)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "all")
