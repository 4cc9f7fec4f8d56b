"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the same
seeded inputs.  Bar: relative Frobenius error per order <= 1e-5 (FP32 path)."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_common import TOL_BF16X2, TOL_FP32, announce, rel_fro, torch_cuda

pytestmark = pytest.mark.gpu


def _real_orthogonal_with_minus1(n, r, seed, margin=0.3):
    rng = np.random.default_rng(seed)
    rest = n - r
    pairs = rest // 2
    ph = rng.uniform(0.05, np.pi - margin, size=pairs)
    d = np.zeros((n, n))
    d[: 2 * pairs, : 2 * pairs] = synth.rotation_blocks(ph)
    k = 2 * pairs
    if rest % 2:
        d[k, k] = 1.0
        k += 1
    for i in range(k, n):
        d[i, i] = -1.0
    v, rr = np.linalg.qr(rng.standard_normal((n, n)))
    v = v * np.sign(np.diag(rr))[None, :]
    return v @ d @ v.T


def _gpu_plan(torch, F, L, stacktype="fp32"):
    from paper_2602_20870_amd import Plan
    return Plan(torch.from_numpy(np.ascontiguousarray(F)).cuda(), L, stacktype=stacktype)


def _check_update(torch, F, L, alphas, tol=TOL_FP32, stacktype="fp32", sample=None, r_expect=None):
    plan = _gpu_plan(torch, F, L, stacktype)
    ref = O.Plan(F, L)
    if r_expect is not None:
        assert plan.r_minus1 == r_expect == ref.r_minus1
    else:
        assert plan.r_minus1 == ref.r_minus1
    Q = plan.update(alphas).cpu().numpy()
    idx = range(len(alphas)) if sample is None else sample
    worst = 0.0
    for a in idx:
        e = rel_fro(Q[a], ref.combine(float(alphas[a])))
        worst = max(worst, e)
        assert e <= tol, (a, alphas[a], e)
    return worst, plan, ref, Q


# ----------------------------------------------------------------------------
# plan (offline stage)
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("case", ["er64", "orth_r3", "dft64", "orth_r1_odd"])
def test_plan_projector_and_stack(case):
    torch = torch_cuda()
    announce(f"plan {case}")
    if case == "er64":
        F, L = synth.make_config("er64", with_signals=False)["F"], 10
    elif case == "orth_r3":
        F, L = _real_orthogonal_with_minus1(48, 3, 5), 12
    elif case == "orth_r1_odd":
        F, L = _real_orthogonal_with_minus1(37, 1, 6), 7
    else:
        F, L = synth.dft_matrix(64), 9
    plan = _gpu_plan(torch, F, L)
    ref = O.Plan(F, L)
    info = plan.info()
    assert info["r_minus1"] == ref.r_minus1
    assert info["unitarity_defect"] < 1e-12
    assert info["drift"] < 1e-12
    stack, P = plan.buffers()
    assert np.max(np.abs(P.cpu().numpy() - ref.P)) < 1e-6
    S = stack.cpu().numpy()
    assert S.shape[0] == 2 * L
    for n in range(1, L + 1):
        assert np.max(np.abs(S[n - 1] - ref.M[n])) < 1e-6, n
        assert np.max(np.abs(S[L + n - 1] - ref.M[n].conj().T)) < 1e-6, n


def test_plan_rejects_non_unitary():
    torch = torch_cuda()
    from paper_2602_20870_amd import FGFRFTError
    F = synth.make_config("er64", with_signals=False)["F"].copy()
    F[3, 5] += 1e-6
    with pytest.raises(FGFRFTError) as ei:
        _gpu_plan(torch, F, 10)
    assert ei.value.name == "FGFRFT_ENOTUNITARY"


# ----------------------------------------------------------------------------
# update (a-1, a-2)
# ----------------------------------------------------------------------------
def test_update_er64_config():
    torch = torch_cuda()
    announce("update er64 N=64 L=10 16 orders")
    c = synth.make_config("er64", with_signals=False)
    worst, *_ = _check_update(torch, c["F"], c["L"], c["alphas"])
    print("worst rel err", worst)


def test_update_dft256_complex_minus1():
    torch = torch_cuda()
    announce("update dft256 L=32 256 orders")
    c = synth.make_config("dft256", with_signals=False)
    _check_update(torch, c["F"], c["L"], c["alphas"], sample=range(0, 256, 9), r_expect=64)


def test_update_grid1024_launch_config():
    torch = torch_cuda()
    announce("update grid1024 L=32 256 orders (sampled)")
    c = synth.make_config("grid1024", with_signals=False)
    _check_update(torch, c["F"], c["L"], c["alphas"], sample=[0, 1, 77, 128, 255])


@pytest.mark.parametrize("N,L,n_alpha", [(1, 3, 5), (2, 4, 1), (17, 5, 33), (50, 40, 3), (100, 64, 40),
                                         (17, 5, 70), (100, 64, 70), (33, 20, 65)])
def test_update_ragged_and_edge_sizes(N, L, n_alpha):
    torch = torch_cuda()
    announce(f"update ragged N={N} L={L} n_alpha={n_alpha}")
    rng = np.random.default_rng(N * 100 + L)
    F = _real_orthogonal_with_minus1(N, min(N, 1 + N // 10), N) if N > 1 else np.array([[-1.0]])
    alphas = rng.uniform(-min(L, 3) + 0.01, min(L, 3) - 0.01, n_alpha)
    _check_update(torch, F, L, alphas)


# The paired-block path (real F, 2L padded to 64 matrix rows) at whole-strip sizes: odd L (stack rows
# 2L..63 zero), order counts off a multiple of 32 (a partial last group of stores), several strips per
# CU (N >= 512), and more than 256 orders (the order table in two LDS chunks).
@pytest.mark.parametrize("N,L,n_alpha,seed", [(128, 17, 33, 1), (512, 25, 64, 2), (192, 32, 300, 3),
                                              (256, 31, 1, 4), (512, 32, 256, 5)])
def test_update_paired_path_sizes(N, L, n_alpha, seed):
    torch = torch_cuda()
    announce(f"update paired path N={N} L={L} n_alpha={n_alpha}")
    rng = np.random.default_rng(seed)
    F = _real_orthogonal_with_minus1(N, 1 + N // 16, seed)
    alphas = rng.uniform(-2, 2, n_alpha)
    sample = None if N * n_alpha <= 256 * 128 else sorted(set(range(0, n_alpha, 7)) | {n_alpha - 1})
    worst, *_ = _check_update(torch, F, L, alphas, sample=sample)
    print("worst rel err", worst)


def test_update_integer_and_near_integer_orders():
    """Orders at and next to integers, where c_n(alpha) tends to a Kronecker delta (Definition 1 at
    integer orders): |alpha - m| down to 1e-12."""
    torch = torch_cuda()
    announce("update: integer and near-integer orders")
    F = _real_orthogonal_with_minus1(128, 9, 6)
    alphas = np.array([0.0, 1.0, -1.0, 2.0, 1 + 1e-9, 1 - 1e-7, -2 + 3e-8, 1e-12, -1e-12, 0.5, -0.5, 1.999999,
                       3 - 2e-6, -2.5, 0.25, 31.0 / 32.0])
    worst, plan, ref, Q = _check_update(torch, F, 32, alphas)
    print("worst rel err", worst)
    assert np.max(np.abs(Q[0] - np.eye(128))) < 2e-6
    assert np.max(np.abs(Q[1] - F)) < 2e-6
    assert np.max(np.abs(Q[2] - F.T)) < 2e-6


def test_update_paired_path_bf16x2():
    torch = torch_cuda()
    announce("update paired path: bf16x2 stack N=256 L=32 40 orders")
    F = _real_orthogonal_with_minus1(256, 17, 7)
    alphas = np.random.default_rng(7).uniform(-2, 2, 40)
    worst, *_ = _check_update(torch, F, 32, alphas, tol=TOL_BF16X2, stacktype="bf16x2")
    print("bf16x2 worst rel err", worst)


def test_update_complex_haar_L10():
    torch = torch_cuda()
    announce("update haar N=96 L=10")
    F = synth.haar_unitary(96, np.random.default_rng(4))
    alphas = np.array([0.5, -1.7, 0.15, 0.999, -0.001])
    _check_update(torch, F, 10, alphas)


@pytest.mark.parametrize("case,L", [("haar96", 10), ("dft64", 20)])
def test_update_complex_f_bf16x2(case, L):
    """BF16 hi/lo stack of a complex F (both complex strip shapes: 2L padded to 32 and to 64; the
    DFT matrix has a 16-dimensional -1 eigenspace, so P is exercised too)."""
    torch = torch_cuda()
    announce(f"update complex F bf16x2 {case} L={L}")
    F = synth.haar_unitary(96, np.random.default_rng(40 + L)) if case == "haar96" else synth.dft_matrix(64)
    alphas = np.array([0.5, -1.7, 0.15, 2.3, -0.001, 1.0])
    worst, *_ = _check_update(torch, F, L, alphas, tol=TOL_BF16X2, stacktype="bf16x2")
    print(case, "bf16x2 worst rel err", worst)


def test_update_integer_orders_and_adjoint_symmetry():
    torch = torch_cuda()
    announce("update integer orders / adjoint symmetry")
    F = _real_orthogonal_with_minus1(40, 3, 8)
    plan = _gpu_plan(torch, F, 8)
    alphas = np.array([0.0, 1.0, -1.0, 2.0, -3.0, 0.37, -0.37])
    Q = plan.update(alphas).cpu().numpy().astype(np.complex128)
    ref = [np.eye(40), F, F.T, F @ F, (F @ F @ F).T]
    for a, R in enumerate(ref):
        assert np.max(np.abs(Q[a] - R)) < 2e-6, alphas[a]
    assert rel_fro(Q[6], Q[5].conj().T) < 2e-6


def test_update_bf16x2_precision_form():
    torch = torch_cuda()
    announce("update bf16x2 grid1024 (sampled)")
    c = synth.make_config("grid1024", with_signals=False, n_alpha=64)
    worst, *_ = _check_update(torch, c["F"], c["L"], c["alphas"], tol=TOL_BF16X2, stacktype="bf16x2",
                              sample=[0, 5, 31, 63])
    print("bf16x2 worst rel err", worst)


def test_update_rejects_out_of_range_orders():
    torch = torch_cuda()
    from paper_2602_20870_amd import FGFRFTError
    plan = _gpu_plan(torch, synth.rotation_blocks([0.3, 1.2]), 3)
    for bad in ([3.0], [-3.5], [np.nan]):
        with pytest.raises(FGFRFTError) as ei:
            plan.update(bad)
        assert ei.value.name == "FGFRFT_EALPHA"


# ----------------------------------------------------------------------------
# apply (a-3)
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("xc,shared,N,B", [(False, False, 64, 32), (True, False, 80, 37), (False, True, 50, 5),
                                           (True, True, 130, 70),
                                           (False, True, 96, 128),      # pre-split signals: shared block
                                           (False, False, 160, 256),    # pre-split signals: wide blocks
                                           # 64-wide k stages split over two wave halves (N % 64 == 0):
                                           (False, False, 192, 64),     # ragged row block, 3 stages
                                           (False, False, 64, 64),      # one stage, half a row block
                                           (False, True, 320, 128),     # pre-split shared block, ragged
                                           (False, False, 256, 320)])   # pre-split wide blocks, 5 column blocks
def test_apply_against_oracle(xc, shared, N, B):
    torch = torch_cuda()
    announce(f"apply xc={xc} shared={shared} N={N} B={B}")
    F = _real_orthogonal_with_minus1(N, 2, N)
    L = 10
    rng = np.random.default_rng(N + B)
    alphas = rng.uniform(-2, 2, 6)
    shape = (N, B) if shared else (6, N, B)
    X = synth.complex_signals(shape, rng) if xc else synth.real_signals(shape, rng)
    X = X * 1e3  # exercise the per-signal scaling
    plan = _gpu_plan(torch, F, L)
    ref = O.Plan(F, L)
    Xt = torch.from_numpy(X.astype(np.complex64 if xc else np.float32)).cuda()
    Y = plan.apply(alphas, Xt, chunk=4).cpu().numpy()
    for a, al in enumerate(alphas):
        Xa = X if shared else X[a]
        Xa32 = Xa.astype(np.complex64 if xc else np.float32).astype(np.complex128)
        assert rel_fro(Y[a], ref.combine(al) @ Xa32) <= TOL_FP32, a


def test_apply_operator_adjoint_and_real_output():
    torch = torch_cuda()
    from paper_2602_20870_amd import apply_operator
    announce("apply_operator adjoint / y_real")
    rng = np.random.default_rng(3)
    n, N, B = 3, 72, 24
    Q = (rng.standard_normal((n, N, N)) + 1j * rng.standard_normal((n, N, N))) / np.sqrt(N)
    X = rng.standard_normal((n, N, B)) + 1j * rng.standard_normal((n, N, B))
    Qt = torch.from_numpy(Q.astype(np.complex64)).cuda()
    Xt = torch.from_numpy(X.astype(np.complex64)).cuda()
    Q32 = Q.astype(np.complex64).astype(np.complex128)
    X32 = X.astype(np.complex64).astype(np.complex128)
    Y = apply_operator(Qt, Xt, adjoint=True).cpu().numpy()
    Yr = apply_operator(Qt, Xt, adjoint=False, y_real=True).cpu().numpy()
    for a in range(n):
        assert rel_fro(Y[a], Q32[a].conj().T @ X32[a]) <= TOL_FP32
        assert rel_fro(Yr[a], (Q32[a] @ X32[a]).real) <= TOL_FP32


@pytest.mark.parametrize("xc,N,B", [(True, 144, 64),    # complex signals, ragged 128-column block
                                     (True, 16, 64),     # one block narrower than a load row
                                     (False, 192, 128)])  # real signals, two signal blocks
def test_apply_operator_adjoint_streaming(xc, N, B):
    """Y = Q^H X through the streaming kernel's adjoint form (Q's columns as operand rows, imaginary
    parts negated), for complex and real-part outputs, against the FP64 product per order."""
    torch = torch_cuda()
    from paper_2602_20870_amd import apply_operator
    announce(f"apply_operator adjoint xc={xc} N={N} B={B}")
    rng = np.random.default_rng(N + B + (7 if xc else 0))
    n = 3
    Q = (rng.standard_normal((n, N, N)) + 1j * rng.standard_normal((n, N, N))) / np.sqrt(N)
    X = (rng.standard_normal((n, N, B)) + 1j * rng.standard_normal((n, N, B))) if xc else rng.standard_normal((n, N, B))
    X = X * np.exp(rng.uniform(-3, 3, (1, 1, B)))                       # columns over decades
    Qt = torch.from_numpy(Q.astype(np.complex64)).cuda()
    Xt = torch.from_numpy(X.astype(np.complex64 if xc else np.float32)).cuda()
    Q32 = Q.astype(np.complex64).astype(np.complex128)
    X32 = X.astype(np.complex64 if xc else np.float32).astype(np.complex128)
    Y = apply_operator(Qt, Xt, adjoint=True).cpu().numpy()
    Yr = apply_operator(Qt, Xt, adjoint=True, y_real=True).cpu().numpy()
    for a in range(n):
        ref = Q32[a].conj().T @ X32[a]
        for b in range(B):
            assert rel_fro(Y[a][:, b], ref[:, b]) <= TOL_FP32, (a, b)
            assert rel_fro(Yr[a][:, b], ref[:, b].real) <= TOL_FP32, (a, b)


@pytest.mark.parametrize("N,B", [(192, 64), (128, 128)])
def test_apply_operator_real_signals_both_outputs(N, B):
    """Real signals through the streaming apply with 64-wide k stages (the two wave halves'
    sums added at the end) for a complex and a real-part output."""
    torch = torch_cuda()
    from paper_2602_20870_amd import apply_operator
    announce(f"apply_operator real signals N={N} B={B}")
    rng = np.random.default_rng(N + 7 * B)
    n = 3
    Q = (rng.standard_normal((n, N, N)) + 1j * rng.standard_normal((n, N, N))) / np.sqrt(N)
    X = rng.standard_normal((n, N, B)) * np.exp(rng.uniform(-4, 4, (1, 1, B)))   # columns over decades
    Qt = torch.from_numpy(Q.astype(np.complex64)).cuda()
    Xt = torch.from_numpy(X.astype(np.float32)).cuda()
    Q32 = Q.astype(np.complex64).astype(np.complex128)
    X32 = X.astype(np.float32).astype(np.float64)
    Y = apply_operator(Qt, Xt).cpu().numpy()
    Yr = apply_operator(Qt, Xt, y_real=True).cpu().numpy()
    for a in range(n):
        ref = Q32[a] @ X32[a]
        for b in range(B):   # per column: the columns' magnitudes span eight decades
            assert rel_fro(Y[a][:, b], ref[:, b]) <= TOL_FP32, (a, b)
            assert rel_fro(Yr[a][:, b], ref[:, b].real) <= TOL_FP32, (a, b)


# ----------------------------------------------------------------------------
# gradients (a-4)
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("xc,shared,cplxF", [(False, False, False), (True, False, False), (False, True, False),
                                             (True, False, True)])
def test_grad_against_oracle(xc, shared, cplxF):
    torch = torch_cuda()
    announce(f"grad xc={xc} shared={shared} complexF={cplxF}")
    rng = np.random.default_rng(11)
    N, L, B, n = 48, 9, 6, 5
    F = synth.haar_unitary(N, rng) if cplxF else _real_orthogonal_with_minus1(N, 2, 12)
    alphas = np.array([0.55, -1.3, 1.0, 0.02, -2.2])
    shape = (N, B) if shared else (n, N, B)
    X = synth.complex_signals(shape, rng) if xc else synth.real_signals(shape, rng)
    X = X.astype(np.complex64 if xc else np.float32)
    GY = (rng.standard_normal((n, N, B)) + 1j * rng.standard_normal((n, N, B))).astype(np.complex64)
    plan = _gpu_plan(torch, F, L)
    ref = O.Plan(F, L)
    Xd = X.astype(np.complex128) if xc else X.astype(np.float64)
    Xs = np.broadcast_to(Xd, (n, N, B)) if shared else Xd
    dal_ref, dX_ref = O.grad(ref.P, ref.M, alphas, Xs, GY.astype(np.complex128), x_real=not xc)
    dal, dX = plan.grad(alphas, torch.from_numpy(X).cuda(), torch.from_numpy(GY).cuda())
    scale = np.max(np.abs(dal_ref))
    assert np.max(np.abs(dal - dal_ref)) <= TOL_FP32 * scale, (dal, dal_ref)
    dX = dX.cpu().numpy()
    dX_ref = dX_ref.sum(axis=0) if shared else dX_ref
    assert rel_fro(dX, dX_ref) <= TOL_FP32


@pytest.mark.parametrize("xc,B", [(False, 64), (True, 64), (False, 65), (True, 33)])
def test_grad_outer_product_row_scales(xc, B):
    """G = GY X^H over two and three 32-signal chunks (33, 64, 65 signals), ragged 64 x 64 tiles
    (N = 200), and GY / X rows whose magnitudes span eight decades (the per-order scale of the
    split inner products must follow G's range)."""
    torch = torch_cuda()
    announce(f"grad outer product xc={xc} B={B}")
    rng = np.random.default_rng(100 + B + xc)
    N, L, n = 200, 12, 3
    F = _real_orthogonal_with_minus1(N, 7, 14)
    alphas = np.array([0.37, -1.6, 2.05])
    X = synth.complex_signals((n, N, B), rng) if xc else synth.real_signals((n, N, B), rng)
    X = X * np.logspace(-4, 4, N)[rng.permutation(N)][None, :, None]
    X = X.astype(np.complex64 if xc else np.float32)
    GY = (rng.standard_normal((n, N, B)) + 1j * rng.standard_normal((n, N, B))) * np.logspace(-4, 4, N)[None, :, None]
    GY = GY.astype(np.complex64)
    plan = _gpu_plan(torch, F, L)
    ref = O.Plan(F, L)
    Xd = X.astype(np.complex128) if xc else X.astype(np.float64)
    dal_ref, dX_ref = O.grad(ref.P, ref.M, alphas, Xd, GY.astype(np.complex128), x_real=not xc)
    dal, dX = plan.grad(alphas, torch.from_numpy(X).cuda(), torch.from_numpy(GY).cuda())
    scale = np.max(np.abs(dal_ref))
    assert np.max(np.abs(dal - dal_ref)) <= TOL_FP32 * scale, (dal, dal_ref)
    assert rel_fro(dX.cpu().numpy(), dX_ref) <= TOL_FP32


@pytest.mark.parametrize("N,L,n,xc,shared,B,stacktype", [
    (32, 4, 3, True, False, 64, "fp32"),       # one diagonal 32 x 32 block, complex signals
    (96, 9, 5, False, False, 64, "fp16x2"),    # a 64-tile cut at N: partial diagonal and edge tiles
    (160, 20, 4, False, True, 128, "fp32"),    # shared signals, two 64-signal chunks
    (64, 64, 3, False, False, 64, "fp16x2"),   # five k-blocks: two passes over the segments
    (256, 33, 70, True, False, 64, "fp16x2"),   # two chunks of orders
    (64, 6, 3, True, True, 64, "fp32")])       # complex signals shared by the orders
def test_grad_paired_layout(N, L, n, xc, shared, B, stacktype):
    """Real F with N % 32 == 0 and B % 64 == 0: G is written in the paired layout (a segment's values
    beside their mirror images) and each stack matrix is read on half of its positions; Proposition 4
    with M_n^H = M_n^T (Proposition 2) against the oracle."""
    torch = torch_cuda()
    announce(f"grad paired layout N={N} L={L} n={n} xc={xc} shared={shared} B={B} stack {stacktype}")
    rng = np.random.default_rng(N + 7 * L + n)
    F = _real_orthogonal_with_minus1(N, 3, N + L)
    alphas = rng.uniform(-min(L - 0.5, 2.5), min(L - 0.5, 2.5), n)
    alphas[0] = 1.0
    shape = (N, B) if shared else (n, N, B)
    X = synth.complex_signals(shape, rng) if xc else synth.real_signals(shape, rng)
    X = X.astype(np.complex64 if xc else np.float32)
    GY = ((rng.standard_normal((n, N, B)) + 1j * rng.standard_normal((n, N, B)))
          * np.logspace(-2, 2, n)[:, None, None]).astype(np.complex64)
    plan = _gpu_plan(torch, F, L, stacktype)
    ref = O.Plan(F, L)
    Xd = X.astype(np.complex128) if xc else X.astype(np.float64)
    Xs = np.broadcast_to(Xd, (n, N, B)) if shared else Xd
    dal_ref, dX_ref = O.grad(ref.P, ref.M, alphas, Xs, GY.astype(np.complex128), x_real=not xc)
    dal, dX = plan.grad(alphas, torch.from_numpy(X).cuda(), torch.from_numpy(GY).cuda())
    for a in range(n):   # each order against its own magnitude
        assert abs(dal[a] - dal_ref[a]) <= TOL_FP32 * max(abs(dal_ref[a]), 1e-3 * np.max(np.abs(GY[a]))), a
    dX = dX.cpu().numpy()
    dX_ref = dX_ref.sum(axis=0) if shared else dX_ref
    assert rel_fro(dX, dX_ref) <= TOL_FP32


@pytest.mark.parametrize("N,L,n,xc,shared,B,stacktype", [
    (96, 12, 5, False, False, 64, "fp32"),     # Haar with one eigenvalue at -1, real signals
    (64, 40, 3, True, False, 64, "fp16x2"),    # two passes over the segments (four k-blocks of 32 + ...)
    (128, 20, 4, True, True, 128, "fp32")])    # the unitary DFT (r_-1 = 32), shared complex signals
def test_grad_paired_layout_complex_F(N, L, n, xc, shared, B, stacktype):
    """Complex F in the paired layout: the partner rows enter conjugated (M_n(j, i) = conj(M_n^H(i, j)),
    P Hermitian), Proposition 4 against the oracle."""
    torch = torch_cuda()
    announce(f"grad paired layout complex F N={N} L={L} n={n} xc={xc} shared={shared} B={B} stack {stacktype}")
    rng = np.random.default_rng(3 * N + L)
    if N == 128:
        F = synth.dft_matrix(N)
    else:
        V = synth.haar_unitary(N, rng)
        th = rng.uniform(-np.pi * 0.9, np.pi * 0.9, N)
        th[5] = np.pi
        F = (V * np.exp(1j * th)[None, :]) @ V.conj().T
    alphas = rng.uniform(-2.0, 2.0, n)
    alphas[0] = 1.0
    shape = (N, B) if shared else (n, N, B)
    X = synth.complex_signals(shape, rng) if xc else synth.real_signals(shape, rng)
    X = X.astype(np.complex64 if xc else np.float32)
    GY = synth.complex_signals((n, N, B), rng).astype(np.complex64)
    plan = _gpu_plan(torch, F, L, stacktype)
    ref = O.Plan(F, L)
    Xd = X.astype(np.complex128) if xc else X.astype(np.float64)
    Xs = np.broadcast_to(Xd, (n, N, B)) if shared else Xd
    dal_ref, dX_ref = O.grad(ref.P, ref.M, alphas, Xs, GY.astype(np.complex128), x_real=not xc)
    dal, dX = plan.grad(alphas, torch.from_numpy(X).cuda(), torch.from_numpy(GY).cuda())
    assert np.max(np.abs(dal - dal_ref)) <= TOL_FP32 * np.max(np.abs(dal_ref)), (dal, dal_ref)
    dX = dX.cpu().numpy()
    dX_ref = dX_ref.sum(axis=0) if shared else dX_ref
    assert rel_fro(dX, dX_ref) <= TOL_FP32


@pytest.mark.parametrize("N,L,n,cplxF", [(50, 9, 5, False),    # N % 8 != 0: per-tile inner products
                                         # the same kernel after it, needing more LDS than 64 KB (69 KB,
                                         # 90 KB): the limit set by the first call must be raised
                                         (50, 30, 4, False), (42, 20, 3, True),
                                         (64, 64, 3, False),   # five k-blocks: two passes over the positions
                                         (40, 5, 70, False),   # two chunks of orders
                                         (56, 32, 4, True)])   # complex stack, three k-blocks
def test_grad_paths(N, L, n, cplxF):
    torch = torch_cuda()
    announce(f"grad paths N={N} L={L} n={n} complexF={cplxF}")
    rng = np.random.default_rng(N + L + n)
    F = synth.haar_unitary(N, rng) if cplxF else _real_orthogonal_with_minus1(N, 3, 13)
    alphas = rng.uniform(-min(L - 0.5, 3.0), min(L - 0.5, 3.0), n)
    alphas[0] = 1.0
    B = 7
    X = synth.real_signals((n, N, B), rng).astype(np.float32)
    # G = GY X^H spans several decades across orders: the per-order operand scale must follow it
    GY = ((rng.standard_normal((n, N, B)) + 1j * rng.standard_normal((n, N, B)))
          * np.logspace(-3, 3, n)[:, None, None]).astype(np.complex64)
    plan = _gpu_plan(torch, F, L)
    ref = O.Plan(F, L)
    dal_ref, dX_ref = O.grad(ref.P, ref.M, alphas, X.astype(np.float64), GY.astype(np.complex128), x_real=True)
    dal, dX = plan.grad(alphas, torch.from_numpy(X).cuda(), torch.from_numpy(GY).cuda())
    for a in range(n):   # each order against its own magnitude
        assert abs(dal[a] - dal_ref[a]) <= TOL_FP32 * max(abs(dal_ref[a]), 1e-3 * np.max(np.abs(GY[a]))), a
    assert rel_fro(dX.cpu().numpy(), dX_ref) <= TOL_FP32


@pytest.mark.parametrize("L,stacktype", [(40, "fp32"), (64, "fp32"), (64, "fp16x2"), (48, "bf16x2")])
def test_update_complex_F_beyond_L32(L, stacktype):
    """Complex F with 32 < L <= 64 (one-row strips of the update kernel, 96 or 128 terms per k extent):
    a Haar unitary with one eigenvalue moved to -1, against the oracle; the gradient and the direct route
    (plain kernel for complex F) on the same plan."""
    torch = torch_cuda()
    announce(f"complex F N=96 L={L} stack {stacktype}")
    rng = np.random.default_rng(L)
    V = synth.haar_unitary(96, rng)
    th = rng.uniform(-np.pi * 0.9, np.pi * 0.9, 96)
    th[7] = np.pi
    F = (V * np.exp(1j * th)[None, :]) @ V.conj().T
    tol = TOL_BF16X2 if stacktype == "bf16x2" else TOL_FP32
    alphas = np.concatenate([[0.0, 1.0, -1.0], rng.uniform(-2, 2, 40)])
    worst, plan, ref, Q = _check_update(torch, F, L, alphas, tol=tol, stacktype=stacktype, r_expect=1)
    X = synth.complex_signals((96, 5), rng).astype(np.complex64)
    Y = plan.apply_direct(alphas[:5], np.arange(5, dtype=np.int32), torch.from_numpy(X).cuda()).cpu().numpy()
    for c in range(5):
        assert rel_fro(Y[:, c], ref.combine(float(alphas[c])) @ X[:, c].astype(np.complex128)) <= tol
    if stacktype != "bf16x2":
        Xg = synth.complex_signals((4, 96, 8), rng)
        GY = synth.complex_signals((4, 96, 8), rng)
        da, dX = plan.grad(alphas[3:7], torch.from_numpy(Xg.astype(np.complex64)).cuda(),
                           torch.from_numpy(GY.astype(np.complex64)).cuda())
        dref, dxref = O.grad(ref.P, ref.M, alphas[3:7], Xg.astype(np.complex64).astype(np.complex128),
                             GY.astype(np.complex64).astype(np.complex128))
        assert np.max(np.abs(da - dref)) <= TOL_FP32 * np.max(np.abs(dref))
        assert rel_fro(dX.cpu().numpy(), dxref) <= TOL_FP32
