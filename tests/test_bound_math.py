"""Pins of the inequalities behind the exact assignment pruning (no GPU).

The assignment skips a centroid c for instance k when a lower bound of the
B-ADMM transport value D(k, c) = <C, Pi1> clears the best value found.
Pi1's columns sum to the instance weights (Eq. (badmmc0)), so
LB = sum_j w_j min_i ||y_j - x_i||^2 <= D; moving every support point of the
centroid by at most delta lowers sqrt(LB) by at most delta (each
min_i ||y_j - x_i|| falls by at most delta, and the w-weighted 2-norm over j
is 1-Lipschitz).  Checked here against the oracle's transport value and by
brute force on random supports."""
import numpy as np

import oracle


def _lb(x, y, wy):
    d2 = ((x[:, None, :] - y[None, :, :]) ** 2).sum(-1)
    return float((wy * d2.min(0)).sum())


def test_lower_bound_below_transport_value(oracle_mod):
    rng = np.random.default_rng(11)
    for _ in range(30):
        m, mk, d = rng.integers(1, 9), rng.integers(1, 12), rng.integers(1, 6)
        x, w = rng.random((m, d)), rng.dirichlet(np.ones(m))
        y, wy = rng.random((mk, d)), rng.dirichlet(np.ones(mk))
        v = oracle.badmm_ot(x, w, y, wy, T=100)
        assert _lb(x, y, wy) <= v * (1 + 1e-12) + 1e-15
        ex, _ = oracle.exact_w2(x, w, y, wy)
        assert _lb(x, y, wy) <= ex * (1 + 1e-9) + 1e-12


def test_bound_decays_at_most_by_the_drift():
    rng = np.random.default_rng(12)
    worst = np.inf
    for _ in range(2000):
        m, mk, d = rng.integers(1, 9), rng.integers(1, 12), rng.integers(1, 6)
        x = rng.standard_normal((m, d))
        y, wy = rng.standard_normal((mk, d)), rng.dirichlet(np.ones(mk))
        step = rng.standard_normal((m, d)) * rng.random() * 2
        x2 = x + step
        delta = np.sqrt((step ** 2).sum(1)).max()
        slack = np.sqrt(_lb(x2, y, wy)) - (np.sqrt(_lb(x, y, wy)) - delta)
        worst = min(worst, slack)
        assert slack >= -1e-12
    # the bound is tight enough to be useful: it is attained up to rounding
    # by some random move
    assert worst < 0.5
