"""GPU tests of the differentiable form, the device-order update and the serving loop,
all through the C ABI and compared with the FP64 oracle."""
import json
import os

import numpy as np
import pytest

import oracle as O
import synth
from gpu_common import TOL_FP32, announce, rel_fro, torch_cuda

pytestmark = pytest.mark.gpu


def _orth(n, r, seed):
    rng = np.random.default_rng(seed)
    rest = n - r
    d = np.zeros((n, n))
    d[: 2 * (rest // 2), : 2 * (rest // 2)] = synth.rotation_blocks(rng.uniform(0.05, np.pi - 0.3, rest // 2))
    k = 2 * (rest // 2)
    if rest % 2:
        d[k, k] = 1.0
        k += 1
    for i in range(k, n):
        d[i, i] = -1.0
    v, rr = np.linalg.qr(rng.standard_normal((n, n)))
    v = v * np.sign(np.diag(rr))[None, :]
    return v @ d @ v.T


# ----------------------------------------------------------------------------
# differentiable form
# ----------------------------------------------------------------------------
def test_autograd_function_matches_oracle_gradient():
    torch = torch_cuda()
    from paper_2602_20870_amd import FGFRFTFunction, Plan
    announce("autograd N=48 L=8")
    N, L, B = 48, 8, 5
    F = _orth(N, 2, 3)
    rng = np.random.default_rng(0)
    alphas = np.array([0.55, -1.2, 0.3])
    X = rng.standard_normal((3, N, B)).astype(np.float32)
    T = (rng.standard_normal((3, N, B)) + 1j * rng.standard_normal((3, N, B))).astype(np.complex64)
    plan = Plan(torch.from_numpy(F).cuda(), L)
    Xt = torch.from_numpy(X).cuda().requires_grad_(True)
    at = torch.tensor(alphas, dtype=torch.float64, requires_grad=True)
    Y = FGFRFTFunction.apply(Xt, at, plan)
    loss = (Y - torch.from_numpy(T).cuda()).abs().pow(2).sum()
    loss.backward()
    ref = O.Plan(F, L)
    GY = np.stack([2 * (ref.combine(a) @ X[i].astype(np.float64) - T[i]) for i, a in enumerate(alphas)])
    dal_ref, dX_ref = O.grad(ref.P, ref.M, alphas, X.astype(np.float64), GY)
    assert np.max(np.abs(at.grad.numpy() - dal_ref)) <= TOL_FP32 * np.max(np.abs(dal_ref))
    assert rel_fro(Xt.grad.cpu().numpy(), dX_ref) <= TOL_FP32

    # the order gradient also matches the eigenbasis form of Proposition 4 and finite differences
    for i, a in enumerate(alphas):
        D = O.dQ_dalpha_eigen(F, a, L, decomposition=ref.decomposition)
        g_eig = float(np.real(np.sum((GY[i] @ X[i].astype(np.float64).T).conj() * D)))
        assert abs(g_eig - dal_ref[i]) < 1e-9 * max(1, abs(g_eig))
        h = 1e-3
        lp = np.sum(np.abs(ref.combine(a + h) @ X[i] - T[i]) ** 2)
        lm = np.sum(np.abs(ref.combine(a - h) @ X[i] - T[i]) ** 2)
        assert abs((lp - lm) / (2 * h) - dal_ref[i]) < 1e-5 * max(1, abs(dal_ref[i]))


def test_spectral_mask_pipeline_gradient():
    """Per-channel orders in Q^{-a_c} diag(h_c) Q^{a_c} x_c on a kNN sphere graph (L=48)."""
    torch = torch_cuda()
    from paper_2602_20870_amd.autograd import fgfrft
    from paper_2602_20870_amd import Plan
    announce("mask pipeline sphere N=256 L=48, 4 channels")
    rng = np.random.default_rng(5)
    F = synth.gft_from_shift(synth.laplacian(synth.knn_adjacency(synth.sphere_points(256, rng), 10)))
    N, L, C, B = 256, 48, 4, 6
    plan = Plan(torch.from_numpy(F).cuda(), L)
    ref = O.Plan(F, L)
    X = rng.standard_normal((C, N, B)).astype(np.float32)
    H = rng.uniform(0.2, 1.0, (C, N, 1)).astype(np.float32)
    Tgt = rng.standard_normal((C, N, B)).astype(np.float32)
    alphas = np.array([0.4, -0.7, 1.1, 0.05])

    def loss_oracle(al):
        tot = 0.0
        for c in range(C):
            Z = ref.combine(al[c]) @ X[c]
            Yc = ref.combine(-al[c]) @ (H[c] * Z)
            tot += np.sum(np.abs(Yc - Tgt[c]) ** 2)
        return tot

    at = torch.tensor(alphas, dtype=torch.float64, requires_grad=True)
    Xt = torch.from_numpy(X).cuda()
    Z = fgfrft(Xt, at, plan)
    Ht = torch.from_numpy(H).cuda()
    Y = fgfrft((Ht * Z).contiguous(), -at, plan)
    loss = (Y - torch.from_numpy(Tgt).cuda()).abs().pow(2).sum()
    loss.backward()
    g = at.grad.numpy()

    # FP64 chain rule through both applications (Prop. 4 for Q'(alpha), Prop. 3 for the adjoint)
    g_ref = np.empty(C)
    for c in range(C):
        a = alphas[c]
        Xc = X[c].astype(np.float64)
        Zc = ref.combine(a) @ Xc
        Wc = H[c] * Zc
        Yc = ref.combine(-a) @ Wc
        GY = 2 * (Yc - Tgt[c])
        d2 = -np.real(np.sum((GY @ Wc.conj().T).conj() * O.dQ_dalpha(ref.P, ref.M, -a)))
        GZ = H[c] * (ref.combine(-a).conj().T @ GY)
        d1 = np.real(np.sum((GZ @ Xc.T).conj() * O.dQ_dalpha(ref.P, ref.M, a)))
        g_ref[c] = d1 + d2
    # the FP64 reference agrees with Richardson-extrapolated central differences (h = 1e-3, 5e-4)
    for c in range(C):
        def fd(h):
            ap, am = alphas.copy(), alphas.copy()
            ap[c] += h
            am[c] -= h
            return (loss_oracle(ap) - loss_oracle(am)) / (2 * h)
        rich = (4 * fd(5e-4) - fd(1e-3)) / 3
        assert abs(rich - g_ref[c]) <= 1e-6 * max(1.0, np.max(np.abs(g_ref))), (c, rich, g_ref[c])
    assert np.max(np.abs(g - g_ref)) <= TOL_FP32 * np.max(np.abs(g_ref)), (g, g_ref)


# ----------------------------------------------------------------------------
# device-order update (capturable entry point)
# ----------------------------------------------------------------------------
def test_update_dev_matches_host_orders_and_flags_out_of_range():
    torch = torch_cuda()
    from paper_2602_20870_amd import Plan
    announce("update_dev")
    F = _orth(70, 3, 9)
    plan = Plan(torch.from_numpy(F).cuda(), 6)
    al = np.array([0.3, -5.9, 2.0, 1.7])
    Q1 = plan.update(al)
    Q2 = torch.empty_like(Q1)
    plan.update_dev(torch.from_numpy(al).cuda(), out=Q2)
    assert torch.equal(Q1, Q2)
    bad = np.array([0.3, 6.0, -7.5])
    Q3 = torch.empty((3, 70, 70), dtype=torch.complex64, device="cuda")
    plan.update_dev(torch.from_numpy(bad).cuda(), out=Q3)
    q = Q3.cpu().numpy()
    assert np.isfinite(q[0]).all() and np.isnan(q[1]).all() and np.isnan(q[2]).all()


# ----------------------------------------------------------------------------
# serving loop
# ----------------------------------------------------------------------------
def _server(torch, use_graphs, Ns=(64, 100, 256), L=10, route="auto"):
    from paper_2602_20870_amd.serve import Server
    srv = Server(hbm_budget=8 << 30, K=8, bmax=16, slot_sets=2, use_graphs=use_graphs, route=route)
    Fs = {}
    for i, N in enumerate(Ns):
        F = _orth(N, i, 20 + i)
        srv.add_plan(i, F, L)
        Fs[i] = F
    return srv, Fs


@pytest.mark.parametrize("route", ["auto", "operator", "direct"])
def test_serving_result_alone_equals_result_in_mix_and_oracle(route):
    torch = torch_cuda()
    announce(f"serving alone vs mix, route={route}")
    srv, Fs = _server(torch, use_graphs=True, route=route)
    rng = np.random.default_rng(2)
    reqs = [(int(rng.integers(0, 3)), float(rng.uniform(-2, 2)), int(rng.integers(1, 17))) for _ in range(40)]
    sig = {g: rng.standard_normal((F.shape[0], 16)).astype(np.float32) for g, F in Fs.items()}
    # alone: one request at a time
    alone = []
    for g, a, b in reqs[:6]:
        f = srv.submit(g, a, sig[g][:, :b])
        srv.drain()
        alone.append(f.result())
    # in the mix: all requests at once (several batches per plan, overlapping streams)
    fut = [srv.submit(g, a, sig[g][:, :b]) for g, a, b in reqs]
    srv.drain()
    mixed = [f.result() for f in fut]
    for i in range(6):
        assert np.array_equal(alone[i], mixed[i]), i
    refs = {g: O.Plan(F, 10) for g, F in Fs.items()}
    for (g, a, b), y in zip(reqs, mixed):
        yr = refs[g].combine(a) @ sig[g][:, :b].astype(np.float64)
        assert rel_fro(y, yr) <= TOL_FP32
    # graph replays equal eager launches (several replays, eager work in between)
    eager, _ = _server(torch, use_graphs=False, route=route)
    fut_e = [eager.submit(g, a, sig[g][:, :b]) for g, a, b in reqs]
    eager.drain()
    for fe, y in zip(fut_e, mixed):
        assert np.array_equal(fe.result(), y)


def test_serving_admission_counts_every_allocated_byte():
    """A complex-F plan: the server's count is the plan's stack and projector plus every slot-set
    tensor; a budget one byte short is refused after the plan exists (nothing stays counted or
    resident), the exact budget is admitted, requests on it match the oracle, and complex signal
    blocks are refused."""
    torch = torch_cuda()
    announce("serving admission, complex F N=64 L=8")
    from paper_2602_20870_amd.serve import AdmissionError, Server
    F = synth.haar_unitary(64, np.random.default_rng(5))
    kw = dict(K=4, bmax=8, slot_sets=2, use_graphs=False)
    probe = Server(hbm_budget=1 << 40, **kw)
    probe.add_plan(0, F, 8)
    need = probe.used
    assert need == probe.plans[0].persistent.numel() + sum(s.nbytes() for s in probe.slots[0])
    assert probe.footprint(64, 8, complex_F=True) < need
    tight = Server(hbm_budget=need - 1, **kw)
    with pytest.raises(AdmissionError):
        tight.add_plan(0, F, 8)
    assert tight.used == 0 and not tight.plans
    srv = Server(hbm_budget=need, **kw)
    srv.add_plan(0, F, 8)
    assert srv.used == need
    rng = np.random.default_rng(6)
    X = rng.standard_normal((64, 5)).astype(np.float32)
    fut = [srv.submit(0, a, X) for a in (0.4, -1.7, 1.0)]
    srv.drain()
    ref = O.Plan(F, 8)
    for a, f in zip((0.4, -1.7, 1.0), fut):
        assert rel_fro(f.result(), ref.combine(a) @ X.astype(np.float64)) <= TOL_FP32, a
    with pytest.raises(TypeError):
        srv.submit(0, 0.5, X.astype(np.complex64))


# ----------------------------------------------------------------------------
# standard-form ablation (Sec. IV-F, Table VI) on the GPU
# ----------------------------------------------------------------------------
def test_table6_standard_form_and_split_on_gpu():
    """N = 2000 unitary with 32 eigenvalues at -1 (the size of Table VI), alpha = 0.55.

    The standard truncated series (no split) leaves an error on the -1 block that depends
    only on r_-1, alpha and L; the printed values 5.590316 (L = 10) and 5.588024 (L = 20)
    are reproduced by the GPU's standard-form plan.  The split plan removes that block's
    error down to FP32 rounding, and both forms have the same complementary block."""
    torch = torch_cuda()
    from paper_2602_20870_amd import Plan
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table6_lambda_minus1.json")))
    N, r, alpha = 2000, g["r_minus1"], g["alpha"]
    announce(f"table6 N={N} r={r} alpha={alpha}")
    rng = np.random.default_rng(2000)
    V = synth.haar_unitary(N, rng)
    theta = np.concatenate([np.full(r, np.pi), rng.uniform(-0.9 * np.pi, 0.9 * np.pi, N - r)])
    F = (V * np.exp(1j * theta)[None, :]) @ V.conj().T
    dec = (V, theta, np.arange(N) < r)
    W, Wc = V[:, :r], V[:, r:]
    e_m1 = lambda Q: float(np.linalg.norm(W.conj().T @ Q @ W - np.exp(1j * np.pi * alpha) * np.eye(r)))
    e_c = lambda Q: float(np.linalg.norm(Wc.conj().T @ Q @ Wc - np.diag(np.exp(1j * alpha * theta[r:]))))
    Ft = torch.from_numpy(F).cuda()
    for row in g["rows"]:
        L = row["L"]
        std, spl = Plan(Ft, L, form="standard"), Plan(Ft, L)
        assert std.r_minus1 == 0 and spl.r_minus1 == r
        Qs = std.update([alpha])[0].cpu().numpy().astype(np.complex128)
        Qp = spl.update([alpha])[0].cpu().numpy().astype(np.complex128)
        del std, spl
        es, ep = e_m1(Qs), e_m1(Qp)
        cs, cp = e_c(Qs), e_c(Qp)
        announce(f"table6 L={L}: standard E_-1 {es:.6f} (printed {row['standard_E_m1']}), split E_-1 {ep:.2e}, "
                 f"E_c {cs:.6f} / {cp:.6f}")
        assert abs(es - row["standard_E_m1"]) <= 1e-4 * row["standard_E_m1"]
        assert ep <= 1e-4
        assert abs(cs - cp) <= 1e-4 * cp
        assert rel_fro(Qs, O.fgfrft_operator_standard(F, alpha, L)) <= TOL_FP32
        assert rel_fro(Qp, O.fgfrft_operator_eigen(F, alpha, L, decomposition=dec)) <= TOL_FP32


# ----------------------------------------------------------------------------
# exact GFRFT on the GPU (the comparison method) and the Table IV workload
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("N,kind", [(96, "orth_minus1"), (300, "haar")])
def test_gfrft_exact_against_oracle(N, kind):
    torch = torch_cuda()
    from paper_2602_20870_amd import gfrft_exact
    announce(f"gfrft_exact N={N} {kind}")
    rng = np.random.default_rng(N)
    F = _orth(N, 4, 31).astype(np.complex128) if kind == "orth_minus1" else synth.haar_unitary(N, rng)
    Z, theta, m1 = O.spectral_decomposition(F)
    V = torch.from_numpy(np.ascontiguousarray(Z)).cuda()
    Vh = torch.from_numpy(np.ascontiguousarray(Z.conj().T)).cuda()
    th = torch.from_numpy(theta).cuda()
    for alpha in (0.5, -1.3, 2.7, 1.0):
        got = gfrft_exact(V, Vh, th, alpha).cpu().numpy()
        ref = O.gfrft_exact(F, alpha, (Z, theta, m1))
        assert rel_fro(got, ref) <= 1e-12, (alpha, rel_fro(got, ref))
        if alpha == 1.0:
            assert rel_fro(got, F) <= 1e-12


def test_table4_accuracy_on_gpu():
    """FGFRFT (GPU update, complex stack) against the exact GFRFT (GPU) on a Haar matrix, N = 1000,
    L = 10, alpha = 0.5: the same metrics as the oracle for the same draw, and Table IV's level."""
    torch = torch_cuda()
    from paper_2602_20870_amd import Plan, gfrft_exact
    announce("table4 N=1000")
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table4_online.json")))
    L, alpha, N = g["L"], g["alpha"], 1000
    F = synth.haar_unitary(N, np.random.default_rng(4))
    dec = O.spectral_decomposition(F)
    Z, theta, _ = dec
    Ft = torch.from_numpy(F).cuda()
    Q = Plan(Ft, L).update([alpha])[0].to(torch.complex128)
    Fa = gfrft_exact(torch.from_numpy(np.ascontiguousarray(Z)).cuda(),
                     torch.from_numpy(np.ascontiguousarray(Z.conj().T)).cuda(), torch.from_numpy(theta).cuda(), alpha)
    m_gpu = O.error_metrics((Q - Fa).cpu().numpy())
    m_ref = O.error_metrics(O.fgfrft_operator_eigen(F, alpha, L, decomposition=dec) - O.gfrft_exact(F, alpha, dec))
    for key in ("MSE", "MAE", "NMSE"):
        assert abs(m_gpu[key] - m_ref[key]) <= 1e-4 * m_ref[key], (key, m_gpu[key], m_ref[key])
    nmse_printed = np.mean([r["NMSE"] for r in g["rows"]])
    assert abs(m_gpu["NMSE"] - nmse_printed) <= g["rel_tol"] * nmse_printed


# ----------------------------------------------------------------------------
# learnable-order pipelines (order learning and fractional-domain denoising)
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("K", [1, 2, 3])
def test_order_cascade_learns_the_target_total_order(K):
    """K FGFRFT layers from alpha = 0.1 each, target F^{1.5} (exact GFRFT), X = I, loss ||.||_F^2 / N^2,
    Adam lr 0.01 for 200 steps (the cascade setup of Sec. IV) on the ER graph N = 64, L = 10."""
    torch = torch_cuda()
    from paper_2602_20870_amd import Plan
    from paper_2602_20870_amd.learn import OrderCascade, train
    announce(f"order cascade K={K}")
    cfg = synth.make_config("er64", seed=0, with_signals=False)
    F, N = cfg["F"], cfg["N"]
    plan = Plan(torch.from_numpy(F).cuda(), 10)
    dec = O.spectral_decomposition(F)
    target = torch.from_numpy(O.gfrft_exact(F, 1.5, dec).astype(np.complex64)).cuda()
    X = torch.eye(N, dtype=torch.float32, device="cuda")
    model = OrderCascade(plan, K, alpha_init=0.1)
    hist = train(model, lambda m: (m(X) - target).abs().pow(2).sum() / N ** 2, steps=200, lr=0.01)
    announce(f"K={K}: loss {hist[0]:.3e} -> {hist[-1]:.3e}, total order {model.total_order():.4f}")
    assert hist[-1] < 0.05 * hist[0]
    assert abs(model.total_order() - 1.5) < 0.05


def test_fractional_mask_denoiser_reduces_the_error():
    """Q^{-a} diag(h) Q^{a} y on a 16 x 16 grid graph (L = 10, a from 0.9): smooth signals
    (20 lowest graph frequencies) plus white noise; the learned order and mask must cut the error."""
    torch = torch_cuda()
    from paper_2602_20870_amd import Plan
    from paper_2602_20870_amd.learn import FractionalMaskDenoiser, train
    announce("fractional mask denoiser")
    rng = np.random.default_rng(8)
    A = synth.grid_adjacency(16, 16, lambda m: rng.uniform(0.5, 1.5, m))
    F = synth.gft_from_shift(synth.laplacian(A))
    N = F.shape[0]
    x = (F.T[:, :20] @ rng.standard_normal((20, 8))).astype(np.float32)     # 8 smooth signals
    y = (x + 0.3 * x.std() * rng.standard_normal(x.shape)).astype(np.float32)
    plan = Plan(torch.from_numpy(F).cuda(), 10)
    xt, yt = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    model = FractionalMaskDenoiser(plan, alpha_init=0.9)
    noisy = float(((yt - xt) ** 2).sum())
    groups = [{"params": [model.alpha], "lr": 0.01}, {"params": [model.h], "lr": 0.05}]
    hist = train(model, lambda m: (m(yt) - xt).abs().pow(2).sum(), steps=200, params=groups)
    announce(f"denoiser: noisy {noisy:.3e}, loss {hist[0]:.3e} -> {hist[-1]:.3e}, "
             f"alpha {float(model.alpha.detach()):.3f}")
    assert hist[-1] < 0.5 * noisy
    assert np.isfinite(float(model.alpha.detach()))


def test_binding_refuses_buffers_the_kernels_cannot_use():
    """Host tensors, workspaces that are not device bytes and mis-shaped outputs are refused on the
    host before anything is launched; the plan still works afterwards."""
    torch = torch_cuda()
    from paper_2602_20870_amd import Plan, apply_operator, gfrft_exact
    announce("binding refuses foreign buffers")
    N, L = 40, 6
    plan = Plan(torch.from_numpy(_orth(N, 2, 9)).cuda(), L)
    al = [0.3, -0.8]
    with pytest.raises(ValueError, match="cuda"):
        plan.update(al, out=torch.empty((2, N, N), dtype=torch.complex64))
    ald = torch.tensor(al, dtype=torch.float64, device="cuda")
    Q = torch.empty((2, N, N), dtype=torch.complex64, device="cuda")
    with pytest.raises(ValueError, match="cuda"):
        plan.update_dev(ald, out=Q, ws=torch.empty(1 << 16, dtype=torch.uint8))
    with pytest.raises(ValueError, match="uint8"):
        plan.update_dev(ald, out=Q, ws=torch.empty(1 << 16, dtype=torch.float32, device="cuda"))
    X = torch.randn((2, N, 3), device="cuda")
    with pytest.raises(ValueError, match="cuda"):
        plan.grad(al, X, torch.zeros((2, N, 3), dtype=torch.complex64))
    with pytest.raises(ValueError, match="cuda"):
        apply_operator(Q, X, out=torch.empty((2, N, 3), dtype=torch.complex64))
    with pytest.raises(ValueError, match="cuda"):
        plan.apply_direct(ald, torch.zeros(3, dtype=torch.int32, device="cuda"), X[0].contiguous(),
                          out=torch.empty((N, 3), dtype=torch.complex64))
    V = torch.eye(N, dtype=torch.complex128, device="cuda")
    th = torch.zeros(N, dtype=torch.float64, device="cuda")
    for bad in (torch.empty((N, N), dtype=torch.complex64, device="cuda"),
                torch.empty((N, N - 1), dtype=torch.complex128, device="cuda")):
        with pytest.raises(ValueError, match="out"):
            gfrft_exact(V, V, th, 0.5, out=bad)
    Qr = plan.update(al).cpu().numpy()
    ref = O.Plan(_orth(N, 2, 9), L)
    for a, q in zip(al, Qr):
        assert rel_fro(q, ref.combine(a)) <= TOL_FP32


def test_calls_on_an_explicit_stream_match_the_current_stream():
    """update, apply, the direct route and the gradient queued on a side stream (the binding's
    temporaries are kept for that stream) give bitwise the results of the same calls on the
    current stream."""
    torch = torch_cuda()
    from paper_2602_20870_amd import Plan
    announce("explicit stream")
    rng = np.random.default_rng(41)
    F = synth.make_config("knn4096", seed=12, N=128, with_signals=False)["F"]
    plan = Plan(torch.from_numpy(F).cuda(), 12)
    alphas = rng.uniform(-2, 2, 5)
    X = torch.from_numpy(synth.real_signals((5, 128, 8), rng).astype(np.float32)).cuda()
    GY = torch.from_numpy((rng.standard_normal((5, 128, 8)) + 1j * rng.standard_normal((5, 128, 8)))
                          .astype(np.complex64)).cuda()
    Xd = X.permute(1, 0, 2).reshape(128, 40).contiguous()
    cols = np.repeat(np.arange(5, dtype=np.int32), 8)
    ref = (plan.update(alphas), plan.apply(alphas, X), plan.apply_direct(alphas, cols, Xd), plan.grad(alphas, X, GY))
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    got = (plan.update(alphas, stream=side), plan.apply(alphas, X, stream=side),
           plan.apply_direct(alphas, cols, Xd, stream=side), plan.grad(alphas, X, GY, stream=side))
    side.synchronize()
    for a, b in zip(ref[:3], got[:3]):
        assert torch.equal(a, b)
    assert np.array_equal(ref[3][0], got[3][0]) and torch.equal(ref[3][1], got[3][1])
