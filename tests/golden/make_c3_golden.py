"""Write the full-size reference samples of the 256^3 periodic D3Q6x12
configuration after 1000 steps, computed by the FP64 oracle only.

Output: c3_256_1000_samples.txt with, for 256 seeded random nodes, the node
index and the 12 state components U = (v, F); and the per-component sums of U
over all nodes (conservation check).  Run: python tests/golden/make_c3_golden.py
(about 40 minutes on 8 cores, ~30 GB of memory).
"""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle import oracle as O  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_256_1000_samples.txt")


def main(N=256, steps=1000, nsamp=256):
    c = W.config_c3(N)
    s = O.Sim(3, c["n"], c["dx"], c["dt"], c["mu"], c["lam"], omega=c["omega"])
    s.set_state(c["U0"], dU0=c["dU0"])
    del c["dU0"]
    t0 = time.time()
    for k in range(0, steps, 50):
        s.step(50)
        print(f"step {k + 50} {time.time() - t0:.0f}s", flush=True)
    U, _, _ = s.moments()
    rng = np.random.default_rng(20646)
    idx = np.sort(rng.choice(N ** 3, size=nsamp, replace=False))
    with open(OUT, "w") as f:
        f.write("# FP64 oracle, 256^3 periodic D3Q6x12 configuration (seed 20646), state after 1000 steps.\n")
        f.write("# written by tests/golden/make_c3_golden.py from oracle/ only\n")
        f.write("sums " + " ".join(f"{v:.17g}" for v in U.sum(axis=1)) + "\n")
        for i in idx:
            f.write(f"{i} " + " ".join(f"{v:.17g}" for v in U[:, i]) + "\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
