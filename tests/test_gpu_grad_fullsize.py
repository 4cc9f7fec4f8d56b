"""Gradient parity (Proposition 4) where the matrix-core inner products flush their FP32 sums into
FP64 mid-range, and at the differentiable workload's size.

* real F, N = 512, L = 48, 64 orders x 64 signals: 4096 position stages of 64 over 256 workgroups,
  16 stages per workgroup, i.e. four FP32 -> FP64 flushes each (every 4 stages) before the end;
* sphere2048: kNN (k = 10) graph on 2048 jittered points of the unit sphere, L = 48, 64 orders (one
  per channel) x 64 real signals, the launch the benchmark times (256 stages per workgroup, 64
  flushes); dalpha of 8 orders and their dX against the FP64 oracle.
"""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_common import TOL_FP32, announce, rel_fro, torch_cuda

pytestmark = pytest.mark.gpu


def _real_orthogonal(n, seed):
    """Real orthogonal F with two eigenvalues at -1 (two reflected directions) and rotation pairs."""
    rng = np.random.default_rng(seed)
    pairs = (n - 2) // 2
    d = np.zeros((n, n))
    d[: 2 * pairs, : 2 * pairs] = synth.rotation_blocks(rng.uniform(0.05, np.pi - 0.3, pairs))
    for i in range(2 * pairs, n):
        d[i, i] = -1.0
    v, rr = np.linalg.qr(rng.standard_normal((n, n)))
    v = v * np.sign(np.diag(rr))[None, :]
    return v @ d @ v.T


def _check(torch, F, L, alphas, X, GY, sample, plan_route="schur"):
    from paper_2602_20870_amd import Plan
    dev = torch.device("cuda:0")
    plan = Plan(torch.from_numpy(F).to(dev), L)
    dal, dX = plan.grad(alphas, torch.from_numpy(X).to(dev), torch.from_numpy(GY).to(dev))
    dX = dX[torch.as_tensor(sample, device=dev)].cpu().numpy()
    ref = O.Plan(F, L, route=plan_route)
    assert plan.r_minus1 == ref.r_minus1
    dal_ref, dX_ref = O.grad(ref.P, ref.M, alphas[sample], X[sample].astype(np.float64),
                             GY[sample].astype(np.complex128), x_real=True)
    scale = np.max(np.abs(dal_ref))
    err = np.abs(dal[sample] - dal_ref)
    announce(f"  dalpha worst error {np.max(err) / scale:.2e} of max |dalpha|; "
             f"dX worst {max(rel_fro(dX[i], dX_ref[i]) for i in range(len(sample))):.2e}")
    assert np.max(err) <= TOL_FP32 * scale, (dal[sample], dal_ref)
    for i in range(len(sample)):
        assert rel_fro(dX[i], dX_ref[i]) <= TOL_FP32, i


@pytest.mark.timeout(300)
def test_grad_flushes_mid_range_n512():
    torch = torch_cuda()
    announce("grad N=512 L=48 64 orders x 64 signals (16 stages per workgroup, 4 flushes)")
    rng = np.random.default_rng(512)
    N, L, n, B = 512, 48, 64, 64
    F = _real_orthogonal(N, 9)
    alphas = rng.uniform(-1.8, 1.8, n)
    alphas[:3] = [1.0, 0.0, -0.5]
    X = synth.real_signals((n, N, B), rng).astype(np.float32)
    GY = (rng.standard_normal((n, N, B)) + 1j * rng.standard_normal((n, N, B))).astype(np.complex64)
    sample = np.array([0, 1, 2, 7, 20, 33, 50, 63])
    _check(torch, F, L, alphas, X, GY, sample)


@pytest.mark.timeout(600)
@pytest.mark.slow
def test_grad_sphere2048_bench_launch():
    torch = torch_cuda()
    announce("grad sphere2048 N=2048 L=48 64 orders x 64 signals (the benchmark's launch)")
    cfg = synth.make_config("sphere2048", seed=0, with_signals=False)
    F, L, N = cfg["F"], cfg["L"], cfg["N"]
    n, B = 64, 64
    rng = np.random.default_rng(3)
    alphas = rng.uniform(-1.5, 1.5, n)
    X = rng.standard_normal((n, N, B)).astype(np.float32)
    GY = (rng.standard_normal((n, N, B)) + 1j * rng.standard_normal((n, N, B))).astype(np.complex64)
    sample = np.array([0, 5, 17, 31, 32, 40, 58, 63])
    _check(torch, F, L, alphas, X, GY, sample, plan_route="symmetric")
