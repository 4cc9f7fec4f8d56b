"""GPU parity of the direct route (Y[:, c] = Q_L^{alpha(c)} X[:, c] straight from the resident
stack, no operator formed) against the FP64 oracle's Q X on the same seeded inputs.

Bar: relative Frobenius error per order (over that order's columns) <= 1e-5 on the FP32 stack,
5e-5 on the BF16 hi/lo stack.  The matrix-core kernel takes real F with an FP32 stack, real
signals and N % 32 == 0; the other cases exercise the plain kernel."""
import time

import numpy as np
import pytest

import oracle as O
import synth
from gpu_common import TOL_BF16X2, TOL_FP32, announce, rel_fro, torch_cuda

pytestmark = pytest.mark.gpu


def _plan(torch, F, L, stacktype="fp32", form="split"):
    from paper_2602_20870_amd import Plan
    return Plan(torch.from_numpy(np.ascontiguousarray(F)).cuda(), L, stacktype=stacktype, form=form)


def _columns(rng, n_orders, counts):
    """col_order for `counts[a]` columns of order a, interleaved so orders mix inside a tile."""
    cols = np.concatenate([np.full(c, a, dtype=np.int32) for a, c in enumerate(counts)])
    return cols[rng.permutation(cols.size)]


def _check(torch, plan, ref_Q, alphas, cols, X, ldx=None, tol=TOL_FP32, ncols=None):
    """Run the direct route on X [N, ncols] (padded to ldx with NaN) and compare per order."""
    N, nc = X.shape
    ncols = nc if ncols is None else ncols
    ldx = nc if ldx is None else ldx
    xc = np.iscomplexobj(X)
    Xp = np.full((N, ldx), np.nan, dtype=np.complex64 if xc else np.float32)
    Xp[:, :nc] = X
    Xt = torch.from_numpy(Xp).cuda()
    Y = plan.apply_direct(alphas, cols, Xt, ncols=ncols).cpu().numpy()
    X64 = Xp[:, :ncols].astype(np.complex128)
    worst = 0.0
    for a, al in enumerate(alphas):
        sel = np.nonzero(cols[:ncols] == a)[0]
        if sel.size == 0:
            continue
        want = ref_Q(al) @ X64[:, sel]
        e = rel_fro(Y[:, sel], want)
        worst = max(worst, e)
        assert e <= tol, (a, al, e)
    return worst, Y


@pytest.mark.parametrize("N,L,ncols,ldx", [(160, 32, 100, 104),   # ragged row block and column block
                                           (256, 12, 37, 40),     # one column block, padded
                                           (64, 10, 5, 8)])        # er64-sized, few columns
def test_direct_matrix_core_path(N, L, ncols, ldx):
    torch = torch_cuda()
    announce(f"direct matrix-core N={N} L={L} ncols={ncols} ldx={ldx}")
    F = synth.make_config("knn4096", seed=3, N=N, with_signals=False)["F"]
    rng = np.random.default_rng(N + ncols)
    n_orders = min(7, ncols)
    alphas = rng.uniform(-2, 2, n_orders)
    alphas[:3] = [0.0, 1.0, -0.5]
    counts = rng.multinomial(ncols - n_orders, np.ones(n_orders) / n_orders) + 1
    cols = _columns(rng, n_orders, counts)
    X = synth.real_signals((N, ncols), rng)
    X[:, ::3] *= 1e3            # per-column scales differ by orders of magnitude
    X[:, 1::5] *= 1e-4
    plan = _plan(torch, F, L)
    ref = O.Plan(F, L)
    worst, Y = _check(torch, plan, ref.combine, alphas, cols, X.astype(np.float32), ldx=ldx)
    print("worst rel err", worst)
    # order 0 is the identity (Definition 1 at an integer order): Y = X on its columns
    sel = np.nonzero(cols == 0)[0]
    assert rel_fro(Y[:, sel], X[:, sel].astype(np.float32)) <= TOL_FP32


def test_direct_agrees_with_update_then_apply():
    torch = torch_cuda()
    from paper_2602_20870_amd import apply_operator
    announce("direct vs update + apply, grid1024 L=32")
    c = synth.make_config("grid1024", with_signals=False, n_alpha=8)
    F, L, alphas = c["F"], c["L"], c["alphas"]
    rng = np.random.default_rng(11)
    B = 8
    X = synth.real_signals((8, F.shape[0], B), rng).astype(np.float32)
    plan = _plan(torch, F, L)
    Xt = torch.from_numpy(X).cuda()
    Y1 = apply_operator(plan.update(alphas), Xt).cpu().numpy()
    cols = np.repeat(np.arange(8, dtype=np.int32), B)
    Xd = torch.from_numpy(np.ascontiguousarray(X.transpose(1, 0, 2).reshape(F.shape[0], 8 * B))).cuda()
    Y2 = plan.apply_direct(alphas, cols, Xd).cpu().numpy().reshape(F.shape[0], 8, B).transpose(1, 0, 2)
    for a in range(8):
        assert rel_fro(Y2[a], Y1[a]) <= 2 * TOL_FP32, a


@pytest.mark.parametrize("case", ["dft64_complex_x", "haar96_real_x", "real_n70", "real_f_complex_x", "bf16x2",
                                  "bf16x2_n70", "haar96_bf16x2"])
def test_direct_other_configurations(case):
    """Complex F, complex signals and N % 32 != 0 take the plain kernel; a BF16X2 stack with
    N % 32 == 0 takes the bf16 matrix-core kernel, with N = 70 or a complex F the plain one."""
    torch = torch_cuda()
    announce(f"direct plain kernel: {case}")
    seeds = {"dft64_complex_x": 21, "haar96_real_x": 22, "real_n70": 23, "real_f_complex_x": 24, "bf16x2": 25,
             "bf16x2_n70": 26, "haar96_bf16x2": 27}
    rng = np.random.default_rng(seeds[case])
    stacktype, tol, L = "fp32", TOL_FP32, 10
    if case == "dft64_complex_x":
        F = synth.dft_matrix(64)
        X = synth.complex_signals((64, 19), rng)
    elif case == "haar96_real_x":
        F = synth.haar_unitary(96, rng)
        X = synth.real_signals((96, 9), rng)
    elif case == "real_n70":
        F = synth.make_config("knn4096", seed=5, N=70, with_signals=False)["F"]
        X = synth.real_signals((70, 13), rng)
    elif case == "real_f_complex_x":
        F = synth.make_config("knn4096", seed=6, N=96, with_signals=False)["F"]
        X = synth.complex_signals((96, 11), rng)
    elif case == "haar96_bf16x2":       # complex F with the BF16 hi/lo stack: plain kernel
        F = synth.haar_unitary(96, rng)
        X = synth.real_signals((96, 9), rng)
        stacktype, tol = "bf16x2", TOL_BF16X2
    else:
        n = 128 if case == "bf16x2" else 70
        F = synth.make_config("knn4096", seed=7, N=n, with_signals=False)["F"]
        X = synth.real_signals((n, 40), rng)
        X[:, ::4] *= 1e3
        stacktype, tol, L = "bf16x2", TOL_BF16X2, 16
    alphas = rng.uniform(-2, 2, 4)
    cols = _columns(rng, 4, [1, 2, 3, X.shape[1] - 6])
    X = X.astype(np.complex64 if np.iscomplexobj(X) else np.float32)
    plan = _plan(torch, F, L, stacktype=stacktype)
    ref = O.Plan(F, L)
    worst, _ = _check(torch, plan, ref.combine, alphas, cols, X, tol=tol)
    print(case, "worst rel err", worst)


def test_direct_standard_form():
    torch = torch_cuda()
    announce("direct route, standard form (P = 0, M_0 = I)")
    F = synth.make_config("knn4096", seed=8, N=96, with_signals=False)["F"]
    rng = np.random.default_rng(8)
    L = 12
    alphas = rng.uniform(-2, 2, 3)
    cols = _columns(rng, 3, [4, 4, 8])
    X = synth.real_signals((96, 16), rng).astype(np.float32)
    plan = _plan(torch, F, L, form="standard")
    _check(torch, plan, lambda al: O.fgfrft_operator_standard(F, al, L), alphas, cols, X)


def test_direct_bad_orders_give_nan_columns_only():
    torch = torch_cuda()
    announce("direct route: out-of-range orders and order indices")
    F = synth.make_config("knn4096", seed=9, N=64, with_signals=False)["F"]
    rng = np.random.default_rng(9)
    L = 4
    alphas = np.array([0.3, 4.0, -1.2])                   # order 1 has |alpha| >= L
    cols = np.array([0, 1, 2, 5, 0, -1, 2, 1], dtype=np.int32)   # indices 5 and -1 do not exist
    X = synth.real_signals((64, 8), rng).astype(np.float32)
    plan = _plan(torch, F, L)
    Y = plan.apply_direct(alphas, cols, torch.from_numpy(X).cuda()).cpu().numpy()
    bad = np.array([False, True, False, True, False, True, False, True])
    assert np.all(np.isnan(Y[:, bad]))
    assert np.all(np.isfinite(Y[:, ~bad]))
    ref = O.Plan(F, L)
    for c in np.nonzero(~bad)[0]:
        assert rel_fro(Y[:, c], ref.combine(alphas[cols[c]]) @ X[:, c].astype(np.float64)) <= TOL_FP32


def test_direct_zero_columns_is_a_no_op():
    torch = torch_cuda()
    F = synth.rotation_blocks([0.3, 1.2])
    plan = _plan(torch, F, 3)
    out = torch.full((4, 2), 7.0, dtype=torch.complex64, device="cuda")
    X = torch.zeros((4, 4), dtype=torch.float32, device="cuda")
    plan.apply_direct([0.5], torch.zeros(4, dtype=torch.int32, device="cuda"), X, ncols=0, out=out)
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())


@pytest.mark.slow
@pytest.mark.timeout(600)
def test_direct_knn4096_launch_config_sampled_rows():
    """The benchmark's direct-route launch: N = 4096, L = 32, 32 orders x 2 real signals."""
    torch = torch_cuda()
    t0 = time.time()
    announce("direct knn4096: building F (N=4096)")
    cfg = synth.make_config("knn4096", seed=0, with_signals=False)
    F, L, N = cfg["F"], cfg["L"], cfg["N"]
    alphas = cfg["alphas"][:32].copy()
    alphas[:4] = [0.0, 1.0, -1.0, 0.5]
    cols = np.repeat(np.arange(32, dtype=np.int32), 2)
    rng = synth.streams(0, 3)[2]
    X = synth.real_signals((N, 64), rng).astype(np.float32)
    plan = _plan(torch, F, L)
    Y = plan.apply_direct(alphas, cols, torch.from_numpy(X).cuda()).cpu().numpy()
    rows = np.sort(np.concatenate([[0, N - 1], np.random.default_rng(4).choice(np.arange(1, N - 1), 62, replace=False)]))
    announce(f"direct knn4096: oracle sampled rows [{time.time() - t0:.0f}s]")
    P, _, r, _ = O.projectors_symmetric_route(F)
    assert plan.r_minus1 == r
    ref = O.sampled_rows(F, P, alphas, L, rows)                 # [32, 64 rows, N]
    errs = []
    for a in range(32):
        sel = np.nonzero(cols == a)[0]
        errs.append(rel_fro(Y[rows][:, sel], ref[a] @ X[:, sel].astype(np.float64)))
    announce(f"direct knn4096: worst sampled-row error {max(errs):.2e} [{time.time() - t0:.0f}s]")
    assert max(errs) <= TOL_FP32, errs
    # properties with no oracle: order 0 gives X, order 1 gives F X, order -1 gives F^T X
    assert rel_fro(Y[:, 0:2], X[:, 0:2]) <= TOL_FP32
    assert rel_fro(Y[:, 2:4], F @ X[:, 2:4].astype(np.float64)) <= TOL_FP32
    assert rel_fro(Y[:, 4:6], F.T @ X[:, 4:6].astype(np.float64)) <= TOL_FP32


@pytest.mark.parametrize("case", ["real_mfma", "complex_plain_two_groups", "fp16x2_cut_tile"])
def test_apply_batched_requests(case):
    """fgfrft_apply_batched: each request with its own order and signal count (zero, one, ragged,
    more than 64) gets Q(alpha_r) X_r, against the oracle per request; 70 requests take two
    groups of 64 and 6."""
    torch = torch_cuda()
    announce(f"apply_batched {case}")
    rng = np.random.default_rng({"real_mfma": 41, "complex_plain_two_groups": 42, "fp16x2_cut_tile": 43}[case])
    stacktype = "fp32"
    if case == "real_mfma":                  # real F, real signals, N % 32 == 0: matrix-core kernel
        F = synth.make_config("knn4096", seed=8, N=96, with_signals=False)["F"]
        L, counts, xc = 12, [3, 0, 1, 64, 17, 100, 2], False
    elif case == "complex_plain_two_groups":  # complex F, complex signals: plain kernel
        F = synth.haar_unitary(40, rng)
        L, xc = 9, True
        counts = list(rng.integers(0, 6, 70))
    else:                                    # FP16X2 stack, N = 160 (a 64-row block cut at N)
        F = synth.make_config("knn4096", seed=9, N=160, with_signals=False)["F"]
        L, counts, xc, stacktype = 20, [65, 1, 7, 0, 31], False, "fp16x2"
    N, n = F.shape[0], len(counts)
    alphas = rng.uniform(-min(L - 0.5, 2.5), min(L - 0.5, 2.5), n)
    alphas[0] = 1.0
    mk = synth.complex_signals if xc else synth.real_signals
    Xs = [mk((N, int(b)), rng).astype(np.complex64 if xc else np.float32) for b in counts]
    plan = _plan(torch, F, L, stacktype=stacktype)
    ref = O.Plan(F, L)
    outs = plan.apply_batched(alphas, [torch.from_numpy(X).cuda() for X in Xs])
    worst = 0.0
    for r, (X, Y) in enumerate(zip(Xs, outs)):
        assert tuple(Y.shape) == X.shape
        if X.shape[1] == 0:
            continue
        e = rel_fro(Y.cpu().numpy(), ref.combine(float(alphas[r])) @ X.astype(np.complex128))
        worst = max(worst, e)
        assert e <= TOL_FP32, (r, alphas[r], e)
    print(case, "worst rel err", worst)


def test_apply_batched_refusals():
    """Host-side refusals of fgfrft_apply_batched on a real plan: counts out of range, a NULL or
    misaligned request pointer, an order out of range and a short workspace; nothing is enqueued."""
    import ctypes
    torch = torch_cuda()
    from paper_2602_20870_amd._lib import lib
    announce("apply_batched refusals")
    F = synth.make_config("knn4096", seed=8, N=64, with_signals=False)["F"]
    plan = _plan(torch, F, 8)
    L_ = lib()
    X = torch.zeros((64, 8), dtype=torch.float32, device="cuda")
    Y = torch.zeros((64, 8), dtype=torch.complex64, device="cuda")
    ws = torch.zeros(1 << 22, dtype=torch.uint8, device="cuda")

    def call(al, counts, xs, ys, wsb=ws.numel(), wsp=None):
        n = len(counts)
        a = (ctypes.c_double * n)(*al)
        b = (ctypes.c_int * n)(*counts)
        xp = (ctypes.c_void_p * n)(*xs)
        yp = (ctypes.c_void_p * n)(*ys)
        return L_.fgfrft_apply_batched(plan._h, a, n, b, xp, 0, yp, wsp or ws.data_ptr(), wsb, None)

    x, y = X.data_ptr(), Y.data_ptr()
    assert call([0.5, 0.1], [4, -1], [x, x], [y, y]) == -1
    assert call([0.5, 0.1], [4, 5000], [x, x], [y, y]) == -1
    assert call([0.5, 0.1], [4, 2], [x, None], [y, y]) == -1
    assert call([0.5, 0.1], [4, 2], [x, x + 2], [y, y]) == -1
    assert call([0.5, 0.1], [4, 2], [x, x], [y, y + 4]) == -1
    assert call([0.5, 9.0], [4, 2], [x, x], [y, y]) == -3
    assert call([0.5, 0.1], [4, 2], [x, x], [y, y], wsb=256) == -4
    assert call([0.5, 0.1], [4, 2], [x, x], [y, y], wsp=ws.data_ptr() + 128) == -1
    # a request with no signals may pass NULL pointers
    assert call([0.5, 0.1], [4, 0], [x, None], [y, None]) == 0
    torch.cuda.synchronize()
