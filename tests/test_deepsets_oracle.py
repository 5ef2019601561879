"""Pins of the FP64 warm-start network reference (oracle/deepsets.py).

Its gradient is checked against central finite differences of its own loss,
its loss against closed forms (perfect prediction, permutation invariance)
and its proposal against the symmetries the standardised inputs give it
(translation and scale equivariance, member-order invariance)."""
import numpy as np
import pytest

from oracle import deepsets as ds
from synth.generators import make_workload

M, D, H = 3, 2, 8


def _clusters(seed, m=M, d=D, n_cl=2, with_targets=True):
    wl = make_workload("gmm_d3_n256", seed=seed, N=12)
    rng = np.random.Generator(np.random.PCG64(seed + 5))
    out = []
    for c in range(n_cl):
        mem = [2 * c, 2 * c + 1, 2 * c + 5]
        y, w, mw, pw = ds.cluster_points(wl, mem)
        y = y[:, :d].copy()
        cl = dict(y=y, w=w, mw=mw, pw=pw)
        if with_targets:
            cl["xt"] = rng.standard_normal((m, d)) * 0.7
            wt = rng.random(m) + 0.2
            cl["wt"] = wt / wt.sum()
        out.append(cl)
    return out


def test_param_layout():
    din, out, outp = ds.dims(M, D, H)
    assert din == 16 and out == M * (D + 1) and outp == 32
    th = ds.init_params(M, D, H, seed=3)
    assert th.size == ds.param_count(M, D, H)
    P = ds.unpack(th, M, D, H)
    # padding rows / columns start at zero
    assert np.all(P["W1"][D + 1:] == 0) and np.all(P["V3"][:, out:] == 0)
    np.testing.assert_array_equal(ds.pack(P, M, D, H), th)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_gradient_matches_finite_differences(seed):
    cls = _clusters(seed)
    th = ds.init_params(M, D, H, seed=seed)
    # non-zero biases so that every parameter block is exercised
    th = th + 0.05 * np.random.Generator(np.random.PCG64(seed)).standard_normal(
        th.size)
    din, out, outp = ds.dims(M, D, H)
    P = ds.unpack(th, M, D, H)
    P["W1"][D + 1:] = 0.0          # padded feature rows see zero input anyway
    th = ds.pack(P, M, D, H)
    _, g = ds.forward_backward(th, cls, M, D, H)
    h = 1e-6
    live = np.ones(th.size, bool)
    # padded output columns do not enter the loss: their gradient is zero
    Pm = ds.unpack(np.arange(th.size, dtype=float), M, D, H)
    for idx in Pm["V3"][:, out:].reshape(-1).astype(int):
        live[idx] = False
    for idx in Pm["e3"][out:].astype(int):
        live[idx] = False
    assert np.all(g[~live] == 0)
    rng = np.random.Generator(np.random.PCG64(seed + 11))
    pick = rng.choice(np.nonzero(live)[0], size=120, replace=False)
    fd = np.empty(pick.size)
    for t, i in enumerate(pick):
        e = np.zeros_like(th)
        e[i] = h
        fp, _ = ds.forward_backward(th + e, cls, M, D, H)
        fm, _ = ds.forward_backward(th - e, cls, M, D, H)
        fd[t] = (fp - fm) / (2 * h)
    np.testing.assert_allclose(g[pick], fd, rtol=1e-5, atol=1e-7)


def test_perfect_prediction_loss_is_entropy():
    """Targets equal to the proposal: Chamfer 0, cross-entropy = H(w)."""
    cls = _clusters(4, with_targets=False)
    th = ds.init_params(M, D, H, seed=4)
    tot = 0.0
    for cl in cls:
        x, w = ds.propose(th, cl, M, D, H)
        cl["xt"], cl["wt"] = x, w
        tot += -float(w @ np.log(w))
    loss, _ = ds.forward_backward(th, cls, M, D, H)
    assert abs(loss - tot / len(cls)) < 1e-12


def test_proposal_equivariance_and_set_invariance():
    cl = _clusters(5, with_targets=False)[0]
    th = ds.init_params(M, D, H, seed=5)
    x0, w0 = ds.propose(th, cl, M, D, H)
    sh = dict(cl, y=cl["y"] * 2.5 + np.array([3.0, -1.0]))
    x1, w1 = ds.propose(th, sh, M, D, H)
    np.testing.assert_allclose(x1, x0 * 2.5 + np.array([3.0, -1.0]),
                               rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(w1, w0, rtol=1e-12)
    perm = np.random.Generator(np.random.PCG64(9)).permutation(len(cl["y"]))
    pm = {k: v[perm] for k, v in cl.items()}
    x2, w2 = ds.propose(th, pm, M, D, H)
    np.testing.assert_allclose(x2, x0, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(w2, w0, rtol=1e-12)
    assert abs(w0.sum() - 1) < 1e-14 and np.all(w0 > 0)


def test_forward_loss_agrees_with_proposal():
    """The loss is the Chamfer + cross-entropy of propose()'s output,
    evaluated here by brute force in the original coordinates."""
    cls = _clusters(6)
    th = ds.init_params(M, D, H, seed=6)
    ref = 0.0
    for cl in cls:
        x, w = ds.propose(th, cl, M, D, H)
        wsum = cl["w"].sum()
        mu = cl["w"] @ cl["y"] / wsum
        s = np.sqrt((cl["w"] * ((cl["y"] - mu) ** 2).sum(1)).sum() / wsum)
        lx = 0.0
        q = np.zeros(M)
        for j in range(M):
            dists = [np.sum((x[i] - cl["xt"][j]) ** 2) for i in range(M)]
            i = int(np.argmin(dists))
            lx += cl["wt"][j] * dists[i] / s ** 2
            q[i] += cl["wt"][j]
        for i in range(M):
            lx += w[i] * min(np.sum((x[i] - cl["xt"][j]) ** 2)
                             for j in range(M)) / s ** 2
        ref += lx - float(q @ np.log(w))
    loss, _ = ds.forward_backward(th, cls, M, D, H)
    assert abs(loss - ref / len(cls)) < 1e-10 * max(1.0, abs(ref))


def test_bf16_mode_is_a_small_perturbation():
    cls = _clusters(7)
    th = ds.init_params(M, D, H, seed=7)
    l0, g0 = ds.forward_backward(th, cls, M, D, H)
    l1, g1 = ds.forward_backward(th, cls, M, D, H, bf16=True)
    assert abs(l1 - l0) < 3e-2 * abs(l0)
    assert np.linalg.norm(g1 - g0) < 5e-2 * np.linalg.norm(g0)
    r = ds.round_bf16(np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -3.3]))
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2 ** -6
    assert abs(r[3] + 3.3) < 3.3 * 2 ** -8
