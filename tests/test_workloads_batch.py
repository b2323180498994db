"""The batched random-hole recipe draws no ligament the lattice cannot
resolve: every pair of holes is either separated by at least 4 cells or
overlaps by at least 0.03 (a merged hole), for all 64 instances at their
drawn resolution and for the reduced resolutions the tests use."""
import numpy as np

import workloads as W


def _gaps(c):
    ce, r = c["hole_centres"], c["hole_radii"]
    return [float(np.linalg.norm(ce[i] - ce[j])) - r[i] - r[j] for i in range(len(r)) for j in range(i + 1, len(r))]


def test_no_subresolution_ligaments():
    for k in range(64):
        for N in (None, 40, 64):
            c = W.config_c4_instance(k, N=N)
            for gap in _gaps(c):
                assert not (-0.03 < gap < 4.0 / c["N_cells"]), (k, N, gap)


def test_holes_stay_inside_the_square():
    for k in range(64):
        c = W.config_c4_instance(k)
        ce, r = c["hole_centres"], c["hole_radii"]
        assert np.all(ce - r[:, None] >= 0.25 - 0.15) and np.all(ce + r[:, None] <= 0.75 + 0.15)
        act = c["phi"] <= 0
        assert act.sum() > 0.4 * c["N_cells"] ** 2
