"""Pins of the subgradient-descent reference (Appendix A, Algorithm
"Centroid Update with Subgradient Descent"): the LP duals are subgradients
(finite differences of separately solved LPs), the exact transport value
agrees with the assignment problem, the softmax chain rule agrees with
finite differences of the objective, the step-size rule Eq. (stepsize)
fixes the length of a step, steps descend, and at fixed support the
iterations approach the full-batch LP optimum (Eq. fullbatch-lp)."""
import numpy as np
from scipy.optimize import linear_sum_assignment, linprog
from scipy.spatial.distance import cdist

from oracle import subgradient as sg


def _rand(rng, m, mk, d=2):
    x = rng.random((m, d))
    y = rng.random((mk, d))
    return x, rng.dirichlet(np.ones(m)), y, rng.dirichlet(np.ones(mk))


def test_lp_value_matches_assignment_problem():
    rng = np.random.default_rng(1)
    for _ in range(5):
        x, _, y, _ = _rand(rng, 6, 6)
        C = cdist(x, y, "sqeuclidean")
        r, c = linear_sum_assignment(C)
        v, P, _ = sg.transport_lp(C, np.full(6, 1 / 6), np.full(6, 1 / 6))
        assert abs(v - C[r, c].mean()) < 1e-12
        assert np.allclose(P.sum(1), 1 / 6) and np.allclose(P.sum(0), 1 / 6)


def test_row_duals_are_subgradients():
    """Moving mass delta from row b to row a changes the LP value by
    delta (lambda_a - lambda_b) (the LP is linear in its right-hand side
    near a generic point)."""
    rng = np.random.default_rng(2)
    for _ in range(6):
        x, w, y, wy = _rand(rng, 4, 5)
        C = cdist(x, y, "sqeuclidean")
        v0, _, lam = sg.transport_lp(C, w, wy)
        for a, b in ((0, 1), (2, 3), (1, 3)):
            dlt = 1e-7
            wp = w.copy()
            wp[a] += dlt
            wp[b] -= dlt
            v1, _, _ = sg.transport_lp(C, wp, wy)
            assert abs((v1 - v0) / dlt - (lam[a] - lam[b])) < 1e-5


def _objective(blocks, wys, w):
    return np.mean([sg.transport_lp(C, w, wy)[0] for C, wy in zip(blocks, wys)])


def test_softmax_chain_rule_matches_finite_differences():
    rng = np.random.default_rng(3)
    m = 4
    ys, wys, x = [], [], rng.random((m, 2))
    for _ in range(5):
        _, _, y, wy = _rand(rng, m, 5)
        ys.append(y)
        wys.append(wy)
    blocks = [cdist(x, y, "sqeuclidean") for y in ys]
    w0 = rng.dirichlet(np.ones(m))
    out = sg.subgradient_barycenter(lambda _: blocks, ys, wys, x, w0, T=1,
                                    fixed_support=True)
    gs = out["grads"][0]
    s = np.log(w0) - np.log(w0).mean()
    for i in range(m):
        h = 1e-6
        e = np.zeros(m)
        e[i] = h
        fp = _objective(blocks, wys, sg._softmax(s + e))
        fm = _objective(blocks, wys, sg._softmax(s - e))
        assert abs((fp - fm) / (2 * h) - gs[i]) < 1e-6


def test_step_length_and_descent():
    """Eq. (stepsize): with alpha / ||grad|| below zeta the centred log
    weights move by exactly alpha; with zeta binding by zeta ||grad||; a
    small step lowers the objective."""
    rng = np.random.default_rng(4)
    m = 5
    x = rng.random((m, 2))
    ys, wys = [], []
    for _ in range(6):
        _, _, y, wy = _rand(rng, m, 4)
        ys.append(y)
        wys.append(wy)
    blocks = [cdist(x, y, "sqeuclidean") for y in ys]
    w0 = rng.dirichlet(np.ones(m))
    s0 = np.log(w0) - np.log(w0).mean()
    for alpha, zeta in ((1e-3, 1e9), (1e9, 1e-3)):
        out = sg.subgradient_barycenter(lambda _: blocks, ys, wys, x, w0, T=1,
                                        alpha=alpha, zeta=zeta,
                                        fixed_support=True)
        s1 = np.log(out["w"]) - np.log(out["w"]).mean()
        gn = np.linalg.norm(out["grads"][0])
        want = alpha if alpha / gn < zeta else zeta * gn
        assert abs(np.linalg.norm(s1 - s0) - want) < 1e-9 * max(want, 1)
        if alpha < 1:
            assert _objective(blocks, wys, out["w"]) < out["ftrace"][0]


def test_fixed_support_iterations_approach_the_full_lp():
    """At fixed support the objective is convex in w; after 300 steps the
    best objective on the trace is within 1 % of the full-batch LP
    optimum and never below it (a hard bound)."""
    rng = np.random.default_rng(5)
    for _ in range(3):
        m, N = 3, 5
        x = rng.random((m, 2))
        ys, wys = [], []
        for _ in range(N):
            _, _, y, wy = _rand(rng, m, int(rng.integers(2, 5)))
            ys.append(y)
            wys.append(wy)
        blocks = [cdist(x, y, "sqeuclidean") for y in ys]
        out = sg.subgradient_barycenter(lambda _: blocks, ys, wys, x,
                                        np.full(m, 1 / m), T=300, alpha=0.05,
                                        zeta=1.0, fixed_support=True)
        # Eq. (fullbatch-lp) at fixed x
        nv = m + sum(C.size for C in blocks)
        c = np.zeros(nv)
        rows, rhs = [], []
        col = m
        for C, wy in zip(blocks, wys):
            mk = C.shape[1]
            c[col:col + m * mk] = C.ravel()
            for i in range(m):
                r = np.zeros(nv); r[col + i * mk:col + (i + 1) * mk] = 1
                r[i] = -1; rows.append(r); rhs.append(0.0)
            for j in range(mk):
                r = np.zeros(nv); r[col + j:col + m * mk:mk] = 1
                rows.append(r); rhs.append(wy[j])
            col += m * mk
        r = np.zeros(nv); r[:m] = 1; rows.append(r); rhs.append(1.0)
        res = linprog(c, A_eq=np.array(rows), b_eq=rhs, bounds=(0, None),
                      method="highs")
        lp = res.fun / N
        best = out["ftrace"].min()
        assert best >= lp - 1e-10
        assert best <= lp * 1.01, (best, lp)


def test_support_step_minimises_the_plan_cost():
    """The support step (Eq. (updatex)) with the exact plans minimises
    sum_k <C(x), Pi^(k)> over x: the objective with the updated support
    and the previous plans is below that of any perturbed support."""
    rng = np.random.default_rng(6)
    m = 3
    ys, wys = [], []
    for _ in range(4):
        _, _, y, wy = _rand(rng, m, 4)
        ys.append(y)
        wys.append(wy)
    x0 = rng.random((m, 2))
    out = sg.subgradient_barycenter(
        lambda x: [cdist(x, y, "sqeuclidean") for y in ys], ys, wys, x0,
        np.full(m, 1 / m), T=2, tau=1)
    # the support used by iteration 1 is the update from iteration 0's plans
    plans0 = sg.subgradient_barycenter(
        lambda x: [cdist(x, y, "sqeuclidean") for y in ys], ys, wys, x0,
        np.full(m, 1 / m), T=1, tau=1)["plans"]
    x1 = out["x"]

    def cost(x):
        return sum((cdist(x, y, "sqeuclidean") * P).sum()
                   for y, P in zip(ys, plans0))
    c1 = cost(x1)
    for _ in range(20):
        assert cost(x1 + 1e-3 * rng.standard_normal(x1.shape)) > c1
