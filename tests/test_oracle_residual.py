"""Pins of the oracle's primal residual trace (1/N) sum_k |Pi1 - Pi2|_1.

The residual of the splitting constraint Pi1 = Pi2 (the constraint whose
multiplier the dual step Eq. (badmm2) updates) is checked against its
definition on the returned plans, and against the convergence that
Sec. 3.2's B-ADMM guarantees with the support held fixed: the two plans
approach each other."""
import numpy as np

import oracle
from synth.generators import make_workload


def test_residual_matches_returned_plans():
    wl = make_workload("gmm_d3_n65536_k16", N=300)
    off = wl["offsets"]
    mem = np.arange(0, 300, 3)
    x0, w0 = oracle.init_centroids(wl, [mem[0]] if np.diff(off)[mem[0]] >= 16
                                   else [int(np.argmax(np.diff(off)))], 16)
    for T in (1, 7, 40):
        o = oracle.barycenter(wl, mem, x0[0], w0[0], T=T, tau=10)
        r = 0.0
        for k in mem:
            P1, P2, _ = o["plans"].block(off, k)
            r += np.abs(P1 - P2).sum()
        assert abs(o["rtrace"][-1] - r / len(mem)) < 1e-12 * max(1.0, r)
        assert np.all(o["rtrace"] >= 0)
        assert len(o["rtrace"]) == T


def test_residual_vanishes_with_fixed_support():
    wl = make_workload("gmm_d3_n256", N=40)
    x0, w0 = oracle.init_centroids(wl, [0], 8)
    o = oracle.barycenter(wl, np.arange(40), x0[0], w0[0], T=3000, tau=5000)
    r = o["rtrace"]
    assert r[-1] < 1e-3 * r[0]
    assert r[2999] < r[1000] < r[100]
