"""Failure paths of the plan that need the GPU's FP64 recurrence, forced from the host by the input
alone (every kernel runs to its normal end):

* FGFRFT_EDRIFT: F = (1 + eps) U with U real orthogonal passes the unitarity gate
  (max|F^T F - I| = 2 eps + eps^2 <= 1e-10) while the powers drift: M_n^T M_n - P_c = ((1 + eps)^{2n} - 1) I,
  so the drift measured at n = L is about 2 L eps.  With eps = 4.5e-11 that is 5.8e-9 at L = 64, above the
  1e-9 gate, and 3.6e-10 at L = 4, below it.
* FGFRFT_ENOTUNITARY: the same F with eps = 1e-8 fails the unitarity gate before any power is formed.
"""
import numpy as np
import pytest

import synth
from gpu_common import announce, torch_cuda

pytestmark = pytest.mark.gpu


def _scaled_rotation(N, eps, seed=0):
    rng = np.random.default_rng(seed)
    U = synth.rotation_blocks(rng.uniform(0.1, 2.8, N // 2))        # no eigenvalue near -1
    v, rr = np.linalg.qr(rng.standard_normal((N, N)))
    v = v * np.sign(np.diag(rr))[None, :]
    return (1.0 + eps) * (v @ U @ v.T)


def test_drift_gate_is_reached_by_a_slightly_non_unitary_F():
    torch = torch_cuda()
    from paper_2602_20870_amd import FGFRFTError, Plan
    N, eps = 64, 4.5e-11
    F = _scaled_rotation(N, eps)
    defect = np.max(np.abs(F.T @ F - np.eye(N)))
    assert defect <= 1e-10                                          # passes the unitarity gate
    announce("EDRIFT: (1 + 4.5e-11) U, L = 64")
    with pytest.raises(FGFRFTError) as ei:
        Plan(torch.from_numpy(F).cuda(), 64)
    assert ei.value.name == "FGFRFT_EDRIFT" and "drift" in str(ei.value)
    announce("EDRIFT control: the same F at L = 4, and U itself at L = 64")
    p4 = Plan(torch.from_numpy(F).cuda(), 4)
    assert 1e-10 < p4.info()["drift"] < 1e-9
    p0 = Plan(torch.from_numpy(_scaled_rotation(N, 0.0)).cuda(), 64)
    assert p0.info()["drift"] < 1e-12


def test_unitarity_gate_refuses_before_the_recurrence():
    torch = torch_cuda()
    from paper_2602_20870_amd import FGFRFTError, Plan
    announce("ENOTUNITARY: (1 + 1e-8) U")
    with pytest.raises(FGFRFTError) as ei:
        Plan(torch.from_numpy(_scaled_rotation(64, 1e-8)).cuda(), 8)
    assert ei.value.name == "FGFRFT_ENOTUNITARY"
