"""The allocation-free assignment entry point (d2_assign_noalloc) against
the context's d2_assign on the same device data.

Both read the same instance buffers (torch tensors handed to the context
with d2_load_instances_device and to d2_assign_noalloc directly) and the
same centroids, so labels must be equal and minimal distances equal to
FP rounding (they run the same kernels).  Calls follow each other on one
GPU with shrinking and then differently shaped inputs, so each call runs on
the scratch contents the previous one left.
"""
import ctypes
import os

import numpy as np
import pytest

from synth.generators import make_workload


@pytest.fixture(scope="module")
def d2():
    from paper_1510_00012_amd import d2 as mod
    mod.load_library()
    return mod


def _centroids(wl, K, m, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    Xc = wl["X"][rng.choice(len(wl["X"]), size=(K, m))]
    Wc = rng.random((K, m)) + 0.05
    return np.ascontiguousarray(Xc), Wc / Wc.sum(1, keepdims=True)


def _run_pair(d2, torch, name, N, K, m, dtype, prune, seed):
    wl = make_workload(name, N=N)
    off, X, W = wl["offsets"], wl["X"], wl["W"]
    d = X.shape[1]
    xs = (d + 3) // 4 * 4
    npdt = np.float32 if dtype == "f32" else np.float64
    Xp = np.zeros((len(X), xs))
    Xp[:, :d] = X
    dev = torch.device("cuda", 0)
    X_t = torch.from_numpy(Xp.astype(npdt)).to(dev)
    W_t = torch.from_numpy(W.astype(npdt)).to(dev)
    off_t = torch.from_numpy(off.astype(np.int64)).to(dev)
    Xc, Wc = _centroids(wl, K, m, seed)
    Xc_t = torch.from_numpy(Xc).to(dev)
    Wc_t = torch.from_numpy(Wc).to(dev)
    lab_t = torch.full((N,), -7, dtype=torch.int32, device=dev)
    dist_t = torch.full((N,), -1.0, dtype=torch.float64, device=dev)
    mk_max = int(np.diff(off).max())
    stream = torch.cuda.current_stream(dev)
    print(f"[noalloc {name} N={N} K={K} m={m} d={d} {dtype} prune={prune}]",
          flush=True)
    d2.assign_noalloc(N, d, mk_max, off_t.data_ptr(), X_t.data_ptr(),
                      W_t.data_ptr(), K, m, Xc_t.data_ptr(), Wc_t.data_ptr(),
                      lab_t.data_ptr(), dist_t.data_ptr(), dtype=dtype,
                      iters=50, prune=prune, stream=stream.cuda_stream)
    stream.synchronize()
    lab_n = lab_t.cpu().numpy()
    dist_n = dist_t.cpu().numpy()
    with d2.D2Context(0, dtype) as ctx:
        ctx.load_instances_device(off, X_t.data_ptr(), W_t.data_ptr(), d)
        ctx.centroids_set(Xc, Wc)
        lab_r, dist_r, _ = ctx.assign(iters=50, prune=prune)
    rel = float(np.max(np.abs(dist_n - dist_r) / np.abs(dist_r)))
    print(f"  labels equal {np.array_equal(lab_n, lab_r)}, distance rel "
          f"{rel:.3g}, bitwise {np.array_equal(dist_n, dist_r)}", flush=True)
    assert np.array_equal(lab_n, lab_r)
    assert rel <= (1e-6 if dtype == "f32" else 1e-12)


@pytest.mark.gpu
def test_noalloc_assign_matches_context_assign(d2):
    import torch
    # a call, then a smaller one on the scratch it left, then other shapes
    _run_pair(d2, torch, "gmm_d16_n2000000_k256", 3000, 100, 16, "f32", True,
              1)
    _run_pair(d2, torch, "gmm_d16_n2000000_k256", 1000, 30, 16, "f32", True,
              2)
    _run_pair(d2, torch, "topic_d64_n200000_k64", 700, 12, 32, "f32", True,
              3)
    _run_pair(d2, torch, "gmm_d3_n65536_k16", 1500, 16, 16, "f64", False, 4)
    _run_pair(d2, torch, "gmm_d3_n65536_k16", 500, 5, 9, "f64", True, 5)


def test_noalloc_rejects_sizes_beyond_its_scratch(d2):
    """Argument errors come back before any device call (so this runs
    without a GPU): centroids that do not fit the fixed scratch array, an
    m outside [1, 64], an mk_max beyond the tile limit."""
    if not os.path.exists(d2.LIB_PATH):
        pytest.skip("libd2.so not built")
    with pytest.raises(d2.D2Error) as e:
        d2.assign_noalloc(10, 64, 16, 1, 1, 1, 4096, 64, 1, 1, 1, 1)
    assert e.value.status == d2.D2_EINVAL and "scratch" in str(e.value)
    with pytest.raises(d2.D2Error) as e:
        d2.assign_noalloc(10, 3, 16, 1, 1, 1, 4, 65, 1, 1, 1, 1)
    assert e.value.status == d2.D2_EINVAL
    with pytest.raises(d2.D2Error) as e:
        d2.assign_noalloc(10, 3, 1000, 1, 1, 1, 4, 16, 1, 1, 1, 1)
    assert e.value.status == d2.D2_EINVAL
    # nothing to do: no device needed either
    d2.assign_noalloc(0, 3, 16, None, None, None, 4, 16, None, None, None,
                      None)
    assert ctypes.sizeof(d2.OtParams) == 24
