"""GPU parity of the real-F route of the apply call: for a real orthogonal F and real signals the
library writes only R = Re Q and adds the imaginary part sin(pi alpha) W (W^T X) from the -1
eigenspace basis (Definition 1 with real powers, Definition 2).  Against the FP64 oracle's Q X, per
order, at the FP32 bar; against the complex-operator route of the same call; and on the cases that
must leave the route (complex signals, ragged signal counts, N % 32 != 0, r_-1 above the kept basis)."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_common import TOL_FP32, announce, rel_fro, torch_cuda

pytestmark = pytest.mark.gpu


def _orth_with_minus1(n, r, seed, margin=0.3):
    """Real orthogonal V D V^T with r eigenvalues at -1 and the rest in rotation blocks away from -1."""
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


def _run(torch, F, L, alphas, X, chunk=0, form="split", stacktype="fp32"):
    from paper_2602_20870_amd import Plan
    plan = Plan(torch.from_numpy(F).cuda(), L, form=form, stacktype=stacktype)
    Xt = torch.from_numpy(X).cuda()
    Y = plan.apply(alphas, Xt, chunk=chunk).cpu().numpy()
    return plan, Y


def _check(F, L, alphas, X, Y, shared, form="split", tol=TOL_FP32):
    ref = O.Plan(F, L) if form == "split" else None
    worst = 0.0
    for a, al in enumerate(alphas):
        Q = ref.combine(float(al)) if ref else O.fgfrft_operator_standard(F, float(al), L)
        Xa = (X if shared else X[a]).astype(np.float64)
        e = rel_fro(Y[a], Q @ Xa)
        worst = max(worst, e)
        assert e <= tol, (a, al, e)
    return worst


@pytest.mark.parametrize("N,r,B,shared,n", [(96, 3, 64, False, 7),     # rank-3 imaginary part
                                            (128, 0, 128, False, 5),   # no -1 eigenvalue: Q real
                                            (64, 1, 64, True, 9),      # shared signal block
                                            (160, 32, 64, False, 4),   # largest basis the plan keeps
                                            (192, 2, 128, False, 4),   # 64-wide stages, ragged row block
                                            (96, 40, 64, False, 3)])   # r_-1 > 32: complex route
def test_real_route_against_oracle(N, r, B, shared, n):
    torch = torch_cuda()
    announce(f"real-F apply N={N} r={r} B={B} shared={shared} orders={n}")
    F = _orth_with_minus1(N, r, seed=N + r)
    L = 12
    rng = np.random.default_rng(N * 7 + r)
    alphas = rng.uniform(-2, 2, n)
    alphas[0] = 0.5                               # sin(pi alpha) = 1: the full imaginary part
    X = (synth.real_signals((N, B) if shared else (n, N, B), rng) * 300.0).astype(np.float32)
    plan, Y = _run(torch, F, L, alphas, X, chunk=3)
    assert plan.r_minus1 == r
    worst = _check(F, L, alphas, X, Y, shared)
    print(f"worst {worst:.2e}")


def test_real_route_matches_complex_route_and_integer_orders():
    torch = torch_cuda()
    from paper_2602_20870_amd import apply_operator
    announce("real-F apply vs update + complex apply, integer orders")
    N, L, B = 128, 10, 64
    F = _orth_with_minus1(N, 5, seed=3)
    alphas = np.array([0.0, 1.0, -1.0, 2.0, 0.5, -0.5, 1.37])
    rng = np.random.default_rng(4)
    X = synth.real_signals((len(alphas), N, B), rng).astype(np.float32)
    plan, Y = _run(torch, F, L, alphas, X)
    Q = plan.update(alphas)
    Y2 = apply_operator(Q, torch.from_numpy(X).cuda()).cpu().numpy()
    for a in range(len(alphas)):
        assert rel_fro(Y[a], Y2[a]) <= 2e-6, a
    X64 = X.astype(np.float64)
    assert rel_fro(Y[0], X64[0]) <= TOL_FP32                 # Q^0 = I
    assert rel_fro(Y[1], F @ X64[1]) <= TOL_FP32             # Q^1 = F
    assert rel_fro(Y[2], F.T @ X64[2]) <= TOL_FP32           # Q^-1 = F^T
    assert rel_fro(Y[3], F @ F @ X64[3]) <= TOL_FP32         # Q^2 = F^2
    assert np.max(np.abs(Y[:4].imag)) < 1e-5 * np.max(np.abs(Y[:4].real))


@pytest.mark.parametrize("case", ["complex_x", "ragged_B", "ragged_N", "standard_form", "bf16x2"])
def test_cases_around_the_real_route(case):
    torch = torch_cuda()
    announce(f"real-F apply neighbour case {case}")
    rng = np.random.default_rng(hash(case) % 1000)
    N, B, n, form, st, tol = 96, 64, 4, "split", "fp32", TOL_FP32
    if case == "ragged_B":
        B = 70
    if case == "ragged_N":
        N = 100
    if case == "standard_form":
        form = "standard"
    if case == "bf16x2":
        st, tol = "bf16x2", 5e-5
    F = _orth_with_minus1(N, 2, seed=N)
    L = 9
    alphas = rng.uniform(-2, 2, n)
    if case == "complex_x":
        X = synth.complex_signals((n, N, B), rng).astype(np.complex64)
    else:
        X = synth.real_signals((n, N, B), rng).astype(np.float32)
    _, Y = _run(torch, F, L, alphas, X, form=form, stacktype=st)
    ref = O.Plan(F, L)
    for a, al in enumerate(alphas):
        Q = ref.combine(float(al)) if form == "split" else O.fgfrft_operator_standard(F, float(al), L)
        assert rel_fro(Y[a], Q @ X[a].astype(np.complex128)) <= tol, (case, a)


@pytest.mark.parametrize("case", ["real_route", "complex_F", "complex_x"])
def test_apply_dev_matches_apply_and_replays(case):
    """fgfrft_apply_dev (orders on the device, one update launch) gives bitwise the result of
    fgfrft_apply with all orders in one chunk, on the real-F route and on the complex-operator
    route; captured in a graph it replays to the same result with eager work between replays."""
    torch = torch_cuda()
    from paper_2602_20870_amd import Plan
    announce(f"apply_dev {case}")
    N, L, n, B = 128, 12, 5, 64
    rng = np.random.default_rng(21)
    F = synth.haar_unitary(N, rng) if case == "complex_F" else _orth_with_minus1(N, 3, seed=7)
    alphas = np.array([0.5, -1.3, 0.0, 1.75, -0.2])
    X = synth.complex_signals((n, N, B), rng).astype(np.complex64) if case == "complex_x" else \
        synth.real_signals((n, N, B), rng).astype(np.float32)
    plan = Plan(torch.from_numpy(F).cuda(), L)
    Xt = torch.from_numpy(X).cuda()
    ref = plan.apply(alphas, Xt, chunk=n)
    ad = torch.from_numpy(alphas).cuda()
    xc = case == "complex_x"
    ws = torch.empty(plan.apply_dev_workspace_bytes(n, B, x_complex=xc), dtype=torch.uint8, device="cuda")
    Y = torch.empty_like(ref)
    plan.apply_dev(ad, Xt, out=Y, ws=ws)
    torch.cuda.synchronize()
    assert torch.equal(Y, ref)
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.apply_dev(ad, Xt, out=Y, ws=ws)      # warm-up on the capture stream
    s.synchronize()
    with torch.cuda.graph(g, stream=s):
        plan.apply_dev(ad, Xt, out=Y, ws=ws)
    for _ in range(3):
        Y.zero_()
        junk = plan.apply(alphas[::-1].copy(), Xt, chunk=n)   # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(Y, ref)
    del junk
    O_ref = O.Plan(F, L)
    Xd = X.astype(np.complex128) if xc else X.astype(np.float64)
    Yh = Y.cpu().numpy()
    for a, al in enumerate(alphas):
        assert rel_fro(Yh[a], O_ref.combine(float(al)) @ Xd[a]) <= TOL_FP32, a
