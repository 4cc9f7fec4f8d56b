"""Gradient parity (Proposition 4) where the matrix-core inner products flush their FP32 sums into
FP64 mid-range, and at the differentiable workload's size.

* real F, N = 512, L = 48, 64 orders x 64 signals: 4096 position stages of 64 over 256 workgroups,
  16 stages per workgroup, i.e. four FP32 -> FP64 flushes each (every 4 stages) before the end;
* sphere2048: kNN (k = 10) graph on 2048 jittered points of the unit sphere, L = 48, 64 orders (one
  per channel) x 64 real signals, the launch the benchmark times (256 stages per workgroup, 64
  flushes); dalpha of 8 orders and their dX against the FP64 oracle.
"""
import time

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


def _denoiser_fp64(F, L, Y, clean, W_in, W_out, alphas, h, check, fd_channels):
    """FP64 forward and backward of the point-cloud denoiser (Def. 2, Prop. 3 and Prop. 4 by the
    chain rule, every operator from the oracle's power stack): loss, dW_out, and for the channels in
    `check` dalpha, dh and the columns of dW_in; central differences of the FP64 loss in alpha for
    `fd_channels` (Richardson-extrapolated, h = 1e-3 and 5e-4)."""
    ref = O.Plan(F, L, route="symmetric")
    T = O.term_matrix(ref.M)                                       # [(2L+1), N^2]
    P = ref.P
    C = alphas.size
    nb, N, _ = Y.shape
    X = np.einsum("bni,ic->cnb", Y, W_in)                          # [C, N, clouds]
    Re = np.empty((C, N, nb))
    Zs, Ms = {}, {}
    for c0 in range(0, C, 16):                                     # operators in chunks of 16 channels
        Qs = O.fgfrft_combine_many(P, T, alphas[c0:c0 + 16])
        for k, Q in enumerate(Qs):
            c = c0 + k
            Z = Q @ X[c]
            M = h[c][:, None] * Z
            Re[c] = np.real(Q.conj().T @ M)                        # Q(-a) = Q(a)^H (Prop. 3)
            if c in check:
                Zs[c], Ms[c] = Z, M
    out = np.einsum("cnb,co->bno", Re, W_out)
    diff = out - clean[None]
    loss = np.mean(diff ** 2)
    gout = 2.0 * diff / diff.size
    dW_out = np.einsum("cnb,bno->co", Re, gout)
    chk = sorted(check)
    Qc = O.fgfrft_combine_many(P, T, alphas[chk])
    G1, G2, dal, dh, dWin = [], [], {}, {}, {}
    for k, c in enumerate(chk):
        Q = Qc[k]
        GY2 = np.einsum("bno,o->nb", gout, W_out[c]).astype(np.complex128)   # d loss / d Zi (real part only)
        dM = Q @ GY2                                                 # adjoint of Zi = Q^H M
        dh[c] = np.real(np.sum(dM.conj() * Zs[c], axis=1))
        dZ = h[c][:, None] * dM
        dX = np.real(Q.conj().T @ dZ)
        dWin[c] = np.einsum("bni,nb->i", Y, dX)
        G1.append((dZ @ X[c].T).reshape(-1))                        # G for Z = Q(a) X
        G2.append((GY2 @ Ms[c].conj().T).reshape(-1))               # G for Zi = Q(b) M, b = -a
    # <G, dQ/da> = j pi e^{j pi a} <G, P> + sum_k c_k'(a) <G, T_k>, all channels at once over the terms
    G1, G2 = np.stack(G1, 1), np.stack(G2, 1)
    def inner(Gm):
        return T @ Gm.real - 1j * (T @ Gm.imag), P.reshape(-1) @ Gm.real - 1j * (P.reshape(-1) @ Gm.imag)
    t1, p1 = inner(G1)
    t2, p2 = inner(G2)
    for k, c in enumerate(chk):
        def dq(t, p, a):
            d = O.coefficient_derivatives(a, L)                      # d[L + n] = c_n'
            dv = np.concatenate([[d[L]], d[L + 1:], d[L - 1::-1]])
            return np.real(1j * np.pi * np.exp(1j * np.pi * a) * p + dv @ t)
        dal[c] = dq(t1[:, k], p1[k], alphas[c]) - dq(t2[:, k], p2[k], -alphas[c])
    fd = {}
    for c in fd_channels:
        def loss_at(a):
            Q = O.fgfrft_combine_many(P, T, [a])[0]
            r = np.real(Q.conj().T @ (h[c][:, None] * (Q @ X[c])))
            o = out + np.einsum("nb,o->bno", r - Re[c], W_out[c])
            return np.mean((o - clean[None]) ** 2)
        def cd(hh):
            return (loss_at(alphas[c] + hh) - loss_at(alphas[c] - hh)) / (2 * hh)
        fd[c] = (4 * cd(5e-4) - cd(1e-3)) / 3
    return loss, dW_out, dal, dh, dWin, fd


@pytest.mark.timeout(900)
@pytest.mark.slow
def test_point_cloud_denoiser_at_workload_size():
    """The differentiable workload end to end: N = 2048 sphere graph (kNN k = 10), L = 48, a 3 -> 64
    channel lift, per-channel learnable orders and masks, 64 noisy clouds, FP32 forward and backward on
    the GPU (every transform and its gradient through the library) against the FP64 chain rule with the
    oracle's operators (loss, dW_out; dalpha, dh and dW_in on 16 channels), whose order gradient in turn
    matches central differences of the FP64 loss on 4 channels."""
    torch = torch_cuda()
    from paper_2602_20870_amd import Plan
    from paper_2602_20870_amd.learn import PointCloudDenoiser
    t0 = time.time()
    announce("denoiser: sphere2048, 64 channels, 64 clouds, L = 48")
    d = synth.point_cloud_denoising(seed=0)
    F, L, N = d["F"], d["L"], d["N"]
    dev = torch.device("cuda:0")
    plan = Plan(torch.from_numpy(F).to(dev), L)
    model = PointCloudDenoiser(plan, channels=64)
    with torch.no_grad():                    # a mask that is not all ones, so dh and the mask path matter
        model.h.mul_(torch.from_numpy(np.random.default_rng(4).uniform(0.5, 1.5, (64, N, 1))).to(dev, torch.float32))
    Y = torch.from_numpy(d["noisy"].astype(np.float32)).to(dev)
    clean = torch.from_numpy(d["clean"].astype(np.float32)).to(dev)
    loss = ((model(Y) - clean[None]) ** 2).mean()
    loss.backward()
    torch.cuda.synchronize()
    g_al = model.alpha.grad.numpy()
    g_h = model.h.grad.squeeze(-1).cpu().numpy()
    g_win, g_wout = model.W_in.grad.cpu().numpy(), model.W_out.grad.cpu().numpy()
    announce(f"denoiser: GPU loss {float(loss.detach()):.6e} [{time.time() - t0:.0f}s]")
    check = list(range(0, 64, 4))
    fd_ch = [0, 20, 40, 60]
    p = lambda t: t.detach().cpu().numpy().astype(np.float64)
    lr, dW_out, dal, dh, dWin, fd = _denoiser_fp64(F, L, d["noisy"].astype(np.float32).astype(np.float64),
                                                   d["clean"].astype(np.float32).astype(np.float64),
                                                   p(model.W_in), p(model.W_out), model.alpha.detach().numpy(),
                                                   p(model.h).squeeze(-1), set(check), fd_ch)
    announce(f"denoiser: FP64 loss {lr:.6e} [{time.time() - t0:.0f}s]")
    assert abs(float(loss.detach()) - lr) <= TOL_FP32 * lr
    assert rel_fro(g_wout, dW_out) <= TOL_FP32
    ref_al = np.array([dal[c] for c in check])
    scale = np.max(np.abs(ref_al))
    err_al = np.max(np.abs(g_al[check] - ref_al)) / scale
    err_h = max(rel_fro(g_h[c], dh[c]) for c in check)
    err_w = max(rel_fro(g_win[:, c], dWin[c]) for c in check)
    err_fd = max(abs(fd[c] - dal[c]) for c in fd_ch) / scale
    announce(f"denoiser: dalpha {err_al:.2e}, dh {err_h:.2e}, dW_in {err_w:.2e} (of max), "
             f"FP64 chain rule vs differences {err_fd:.2e} [{time.time() - t0:.0f}s]")
    assert err_fd <= 1e-6
    assert err_al <= TOL_FP32
    assert err_h <= TOL_FP32
    assert err_w <= TOL_FP32
