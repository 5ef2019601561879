"""The FP64 oracle's B-ADMM restarted from its own converged centroid.

A documented property of the method (not a parity pin): with the product
start and rho = rho0 * mean C recomputed at the converged centroid
(Eq. (rho)), a second run settles measurably above the first run's
rounded-plan objective.  This is why a centroid-only warm start cannot
reach the plain run's objective faster."""
import numpy as np
import pytest

import oracle
from synth.generators import warmstart_clusters


@pytest.mark.slow
def test_restart_from_converged_centroid_settles_higher():
    wl = warmstart_clusters("gmm3", 2, seed=400, nc_lo=64, nc_hi=100)
    for c in range(2):
        mem = np.nonzero(wl["labels"] == c)[0]
        x0, w0 = oracle.init_centroids(wl, [wl["first"][c]], 16)
        o = oracle.barycenter(wl, mem, x0[0], w0[0], T=2000, tau=10)
        F = oracle.feasible_objective(wl, mem, o["x"], o["w"], o["plans"])
        o2 = oracle.barycenter(wl, mem, o["x"], o["w"], T=2000, tau=10)
        F2 = oracle.feasible_objective(wl, mem, o2["x"], o2["w"],
                                       o2["plans"])
        assert o2["rho"] < o["rho"]          # rho taken at a better centroid
        assert F2 > F * (1 + 1e-2), (F, F2)
