"""FP64 reference of the subgradient-descent centroid update (Appendix A,
Algorithm "Centroid Update with Subgradient Descent"; Eq. (dualvar),
Eq. (stepsize)).

TEST INFRASTRUCTURE ONLY (like the rest of oracle/): imported by tests/,
never by the product package.  Every transport problem is solved exactly as
the LP Eq. (primal) by scipy's HiGHS, which also gives the dual variables
of the row constraints.

Steps of one iteration n (readings where the appendix is loose are marked):
  1. support update Eq. (updatex) from the previous iteration's plans,
     every tau iterations (n > 0, n % tau == 0);
  2. for every member k: the exact transport plan Pi^(k) between the
     centroid (x, w) and P^(k), and the duals lambda^(k) of its row
     constraints sum_j pi_ij = w_i;
  3. gradient Eq. (dualvar): lambda^(k) minus its mean (reading: the
     printed "(sum_i lambda_i)(1, ..., 1)" is the projection onto the
     simplex's tangent space, i.e. the mean; under the softmax
     parametrisation below any constant shift drops out anyway), averaged
     over the members: g;
  4. with w = softmax(s): grad_s = w * (g - <w, g>) (chain rule of the
     softmax), step size Eq. (stepsize) sigma = min(alpha / ||grad_s||,
     zeta), s <- s - sigma grad_s;
  5. rescaling: s <- s - mean(s) (reading of "rescaled such that
     sum_i s_i = 0"), w = softmax(s).
The objective trace records (1/N) sum_k W^2 at the iteration's (x, w),
i.e. the exact Eq. (centroid) value before the step.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import linprog


def transport_lp(C, w, wy):
    """Eq. (primal) for the cost block C (m x mk) between weights w (rows)
    and wy (columns): (value, plan (m x mk), row duals (m))."""
    C = np.asarray(C, dtype=np.float64)
    m, mk = C.shape
    A = np.zeros((m + mk, m * mk))
    for i in range(m):
        A[i, i * mk:(i + 1) * mk] = 1.0
    for j in range(mk):
        A[m + j, j::mk] = 1.0
    # feasibility tolerances far below HiGHS's defaults (1e-7), so that the
    # plan and duals are exact to FP64 rounding
    res = linprog(C.ravel(), A_eq=A, b_eq=np.concatenate([w, wy]),
                  bounds=(0, None), method="highs",
                  options={"primal_feasibility_tolerance": 1e-10,
                           "dual_feasibility_tolerance": 1e-10})
    if res.status != 0:
        raise RuntimeError("transport LP failed: " + res.message)
    return res.fun, res.x.reshape(m, mk), np.asarray(res.eqlin.marginals[:m])


def _softmax(s):
    e = np.exp(s - s.max())
    return e / e.sum()


def subgradient_barycenter(blocks_of, ys, wys, x, w, T, tau=10, alpha=0.5,
                           zeta=1.0, fixed_support=False):
    """Alg. "Centroid Update with Subgradient Descent" for one cluster.

    blocks_of(x) gives the members' cost blocks at support x (a list of
    m x m_k arrays); ys / wys are the members' support points / weights
    (ys may be None with fixed_support).  Returns dict(x, w, ftrace, plans,
    grads) where plans are the last iteration's exact plans."""
    x = None if x is None else np.array(x, dtype=np.float64)
    w = np.array(w, dtype=np.float64)
    s = np.log(np.maximum(w, 1e-300))
    s -= s.mean()
    w = _softmax(s)
    N = len(wys)
    plans = None
    ftrace, grads = [], []
    for n in range(T):
        if not fixed_support and n > 0 and n % tau == 0:
            # Eq. (updatex) from the previous iteration's plans
            num = np.zeros_like(x)
            den = np.zeros(len(w))
            for P, y in zip(plans, ys):
                num += P @ y
                den += P.sum(1)
            ok = den > 1e-300
            x[ok] = num[ok] / den[ok, None]
        blocks = blocks_of(x)
        g = np.zeros(len(w))
        f = 0.0
        plans = []
        for C, wy in zip(blocks, wys):
            val, P, lam = transport_lp(C, w, wy)
            plans.append(P)
            g += lam - lam.mean()
            f += val
        g /= N
        ftrace.append(f / N)
        gs = w * (g - w @ g)
        nrm = float(np.sqrt(gs @ gs))
        grads.append(gs)
        sigma = min(alpha / nrm, zeta) if nrm > 0 else 0.0
        s = s - sigma * gs
        s -= s.mean()
        w = _softmax(s)
    return {"x": x, "w": w, "ftrace": np.array(ftrace), "plans": plans,
            "grads": grads}
