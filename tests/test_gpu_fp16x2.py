"""GPU tests of the FP16X2 stack: each entry stored as the fp16 pair (hi, lo) of float(x) 2^12, exactly
the operands the FP32 stack is split into when the matrix-core kernels read it.  On every matrix-core
path (update, apply through both routes, direct route, order and signal gradients) the FP16X2 plan's
results must therefore equal the FP32 plan's bit for bit; the plain direct kernel (complex F) and the
per-tile gradient kernel (N % 8 != 0) decode the pairs and are held to the oracle's FP32 bar."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_common import TOL_FP32, announce, rel_fro, torch_cuda

pytestmark = pytest.mark.gpu


def _orth_with_minus1(n, r, seed, margin=0.3):
    rng = np.random.default_rng(seed)
    rest = n - r
    pairs = rest // 2
    d = np.zeros((n, n))
    d[: 2 * pairs, : 2 * pairs] = synth.rotation_blocks(rng.uniform(0.05, np.pi - margin, size=pairs))
    k = 2 * pairs
    if rest % 2:
        d[k, k] = 1.0
        k += 1
    for i in range(k, n):
        d[i, i] = -1.0
    v, rr = np.linalg.qr(rng.standard_normal((n, n)))
    v = v * np.sign(np.diag(rr))[None, :]
    return v @ d @ v.T


def _same(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return a.shape == b.shape and np.array_equal(a.view(np.uint8), b.view(np.uint8))


def _plans(torch, F, L):
    from paper_2602_20870_amd import Plan
    Ft = torch.from_numpy(F).cuda()
    return Plan(Ft, L, stacktype="fp32"), Plan(Ft, L, stacktype="fp16x2")


@pytest.mark.parametrize("N,r,L", [(96, 3, 12), (128, 0, 33)])
def test_fp16x2_equals_fp32_bitwise_real_F(N, r, L):
    torch = torch_cuda()
    from paper_2602_20870_amd import apply_operator
    announce(f"fp16x2 vs fp32 real F N={N} r={r} L={L}")
    F = _orth_with_minus1(N, r, seed=N + L)
    p32, p16 = _plans(torch, F, L)
    rng = np.random.default_rng(5)
    alphas = np.concatenate([[0.0, 1.0, -0.5], rng.uniform(-2, 2, 37)])
    n = len(alphas)
    Q32, Q16 = p32.update(alphas), p16.update(alphas)
    assert _same(Q32.cpu().numpy(), Q16.cpu().numpy())
    X = torch.from_numpy(synth.real_signals((n, N, 64), rng).astype(np.float32)).cuda()
    assert _same(apply_operator(Q32, X).cpu().numpy(), apply_operator(Q16, X).cpu().numpy())
    assert _same(p32.apply(alphas, X, chunk=16).cpu().numpy(), p16.apply(alphas, X, chunk=16).cpu().numpy())
    # direct route: 40 orders x 3 signals side by side
    Xd = torch.from_numpy(synth.real_signals((N, 3 * n), rng).astype(np.float32)).cuda()
    cols = np.repeat(np.arange(n, dtype=np.int32), 3)
    Yd32, Yd16 = p32.apply_direct(alphas, cols, Xd).cpu().numpy(), p16.apply_direct(alphas, cols, Xd).cpu().numpy()
    assert _same(Yd32, Yd16)
    # gradients: 8 orders, 40 real signals
    GY = torch.from_numpy(synth.complex_signals((8, N, 40), rng).astype(np.complex64)).cuda()
    Xg = X[:8, :, :40].contiguous()
    d32, dx32 = p32.grad(alphas[:8], Xg, GY)
    d16, dx16 = p16.grad(alphas[:8], Xg, GY)
    assert _same(d32, d16) and _same(dx32.cpu().numpy(), dx16.cpu().numpy())
    # and the oracle, for the record
    ref = O.Plan(F, L)
    for a in (0, 3, n - 1):
        assert rel_fro(Q16[a].cpu().numpy(), ref.combine(float(alphas[a]))) <= TOL_FP32


def test_fp16x2_complex_F_update_bitwise_direct_and_grad_against_oracle():
    torch = torch_cuda()
    announce("fp16x2 complex F (DFT N=64, L=10)")
    F = synth.dft_matrix(64)
    L = 10
    p32, p16 = _plans(torch, F, L)
    rng = np.random.default_rng(9)
    alphas = rng.uniform(-2, 2, 6)
    assert _same(p32.update(alphas).cpu().numpy(), p16.update(alphas).cpu().numpy())
    ref = O.Plan(F, L)
    # direct route (plain kernel for complex F): decoded pairs, FP32 bar
    X = synth.complex_signals((64, 6), rng).astype(np.complex64)
    Y = p16.apply_direct(alphas, np.arange(6, dtype=np.int32), torch.from_numpy(X).cuda()).cpu().numpy()
    for c in range(6):
        yr = ref.combine(float(alphas[c])) @ X[:, c].astype(np.complex128)
        assert rel_fro(Y[:, c], yr) <= TOL_FP32
    # gradient on the matrix cores (N % 8 == 0): bitwise equal to the FP32 stack's
    Xg = torch.from_numpy(synth.complex_signals((6, 64, 16), rng).astype(np.complex64)).cuda()
    GY = torch.from_numpy(synth.complex_signals((6, 64, 16), rng).astype(np.complex64)).cuda()
    d32, dx32 = p32.grad(alphas, Xg, GY)
    d16, dx16 = p16.grad(alphas, Xg, GY)
    assert _same(d32, d16) and _same(dx32.cpu().numpy(), dx16.cpu().numpy())


def test_fp16x2_per_tile_gradient_against_oracle():
    torch = torch_cuda()
    announce("fp16x2 per-tile gradient (N = 50)")
    F = _orth_with_minus1(50, 2, seed=50)
    L = 9
    _, p16 = _plans(torch, F, L)
    rng = np.random.default_rng(11)
    alphas = rng.uniform(-1.5, 1.5, 5)
    X = synth.real_signals((5, 50, 7), rng)
    GY = synth.complex_signals((5, 50, 7), rng)
    Xt = torch.from_numpy(X.astype(np.float32)).cuda()
    Gt = torch.from_numpy(GY.astype(np.complex64)).cuda()
    d16, dx16 = p16.grad(alphas, Xt, Gt)
    ref = O.Plan(F, L)
    dref, dxref = O.grad(ref.P, ref.M, alphas, X.astype(np.float32).astype(np.float64),
                         GY.astype(np.complex64).astype(np.complex128))
    assert np.max(np.abs(d16 - dref)) <= TOL_FP32 * np.max(np.abs(dref))
    assert rel_fro(dx16.cpu().numpy(), dxref) <= TOL_FP32


def test_fp16x2_direct_bench_launch_knn4096():
    torch = torch_cuda()
    announce("fp16x2 vs fp32 direct route, knn4096 plan, 32 orders x 2 signals")
    cfg = synth.make_config("knn4096", seed=0, with_signals=False)
    F, L = cfg["F"], cfg["L"]
    p32, p16 = _plans(torch, F, L)
    rng = np.random.default_rng(12)
    X = torch.from_numpy(synth.real_signals((4096, 64), rng).astype(np.float32)).cuda()
    cols = np.repeat(np.arange(32, dtype=np.int32), 2)
    al = cfg["alphas"][:32]
    assert _same(p32.apply_direct(al, cols, X).cpu().numpy(), p16.apply_direct(al, cols, X).cpu().numpy())
