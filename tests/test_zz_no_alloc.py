"""The allocation-free update (fgfrft_update_dev_static, tables in the library's fixed per-GPU
array) against the workspace update (fgfrft_update_dev) and the FP64 oracle: two calls in a row
on one plan, the second with fewer orders, then a call on a plan of another L and a complex F.
Both entries run the same kernels, so their operators must agree bit for bit."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_common import TOL_FP32, announce, rel_fro, torch_cuda

pytestmark = pytest.mark.gpu


def _calls(torch, plan, ref, alphas):
    dev = plan.device
    al = torch.from_numpy(np.ascontiguousarray(alphas, dtype=np.float64)).to(dev)
    n, N = len(alphas), plan.N
    q_ws = torch.empty((n, N, N), dtype=torch.complex64, device=dev)
    q_st = torch.full((n, N, N), float("nan"), dtype=torch.complex64, device=dev)
    plan.update_dev(al, out=q_ws)
    plan.update_dev_static(al, out=q_st)
    torch.cuda.synchronize()
    a, b = q_ws.cpu().numpy(), q_st.cpu().numpy()
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), "static-scratch update differs from update_dev"
    for i in sorted({0, n // 2, n - 1}):
        e = rel_fro(b[i], ref.combine(float(alphas[i])))
        assert e <= TOL_FP32, (i, alphas[i], e)


def test_update_dev_static_matches_workspace_update():
    torch = torch_cuda()
    from paper_2602_20870_amd import Plan

    rng = np.random.default_rng(41)
    c = synth.make_config("er64", seed=3)
    F = c["F"]
    # real F, L = 40 (the wider coefficient table): 70 orders, then 9 (smaller) on the same GPU array
    L = 40
    announce("update_dev_static: er64 F, L=40, 70 then 9 orders")
    plan = Plan(torch.from_numpy(F).cuda(), L)
    ref = O.Plan(F, L)
    _calls(torch, plan, ref, rng.uniform(-2.0, 2.0, 70))
    _calls(torch, plan, ref, np.concatenate([[0.0, 1.0, -1.0], rng.uniform(-2.0, 2.0, 6)]))
    # complex F with a -1 eigenspace (unitary DFT), L = 10: 5 orders
    announce("update_dev_static: DFT N=64, L=10, 5 orders")
    Fd = synth.dft_matrix(64)
    plan_c = Plan(torch.from_numpy(Fd).cuda(), 10)
    ref_c = O.Plan(Fd, 10)
    assert plan_c.r_minus1 == ref_c.r_minus1 == 16
    _calls(torch, plan_c, ref_c, rng.uniform(-2.0, 2.0, 5))


def test_update_dev_static_refuses_oversized_batches():
    torch = torch_cuda()
    from paper_2602_20870_amd import Plan
    from paper_2602_20870_amd._lib import FGFRFTError

    announce("update_dev_static: 4097 orders refused on the host")
    c = synth.make_config("er64", seed=0)
    plan = Plan(torch.from_numpy(c["F"]).cuda(), c["L"])
    al = torch.zeros(4097, dtype=torch.float64, device=plan.device)
    out = torch.empty((1, plan.N, plan.N), dtype=torch.complex64, device=plan.device)
    with pytest.raises(ValueError):          # the binding refuses the undersized output first
        plan.update_dev_static(al, out=out)
    out = torch.empty((4097, plan.N, plan.N), dtype=torch.complex64, device=plan.device)
    with pytest.raises(FGFRFTError) as ei:   # the library refuses the batch before any launch
        plan.update_dev_static(al, out=out)
    assert ei.value.name == "FGFRFT_EINVAL" and "4096" in str(ei.value)
