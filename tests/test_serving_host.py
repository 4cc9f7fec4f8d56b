"""Host-side behaviour of the serving loop that needs no GPU: admission by HBM
footprint and the Poisson trace generator."""
import os

import numpy as np
import pytest

from paper_2602_20870_amd import _lib


@pytest.fixture(scope="module")
def built():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libfgfrft.so not built")


def test_admission_refuses_plans_beyond_the_budget(built):
    from paper_2602_20870_amd.serve import AdmissionError, Server
    srv = Server(hbm_budget=1 << 20, K=4, bmax=8, slot_sets=1, use_graphs=False, device="cpu")
    need = srv.footprint(128, 10)
    assert need > 1 << 20
    # stack (2L matrices), P and one slot set of operators and signal blocks
    assert need >= 2 * 10 * 128 * 128 * 4 + 4 * 128 * 128 * 8
    with pytest.raises(AdmissionError):
        srv.add_plan(0, np.eye(128), 10)
    assert srv.used == 0 and not srv.plans


def test_footprint_of_a_complex_plan_and_bad_requests(built):
    import ctypes
    from types import SimpleNamespace
    from paper_2602_20870_amd.serve import Server
    srv = Server(hbm_budget=1 << 40, K=4, bmax=8, slot_sets=2, use_graphs=False, device="cpu")
    N, L = 96, 10
    pb, sb = ctypes.c_size_t(), ctypes.c_size_t()
    assert _lib.lib().fgfrft_plan_bytes(N, L, 0, 0, ctypes.byref(pb), ctypes.byref(sb)) == 0
    # complex stack (8 bytes per entry) and no direct-route blocks for complex F
    assert pb.value >= 2 * L * N * N * 8 + N * N * 8
    assert srv.footprint(N, L, complex_F=True) == pb.value + 2 * (4 * N * N * 8 + 4 * N * 8 * 12)
    with pytest.raises(ValueError):        # L <= 64
        srv.footprint(N, 65, complex_F=True)
    srv.plans[0] = SimpleNamespace(N=8, L=4)
    with pytest.raises(TypeError):
        srv.submit(0, 0.5, np.zeros((8, 2), np.complex64))
    with pytest.raises(ValueError):
        srv.submit(0, 0.5, np.zeros(8, np.float32))
    with pytest.raises(ValueError):
        srv.submit(0, 4.0, np.zeros((8, 2), np.float32))
    assert not srv.pending[0]


def test_route_choice_boundary():
    """Direct iff the batch fits DIRECT_BLOCKS x 64 columns and the extra column blocks cost less
    than the operators the batch would otherwise write and read: one block always goes direct,
    each further block needs 0.15 (2L+1) more orders (L = 32: 9.75 per block)."""
    from paper_2602_20870_amd.serve import DIRECT_BLOCKS, prefer_direct
    assert DIRECT_BLOCKS == 4
    assert all(prefer_direct(n, 1, 32) for n in (1, 2, 16))
    assert not prefer_direct(9, 2, 32) and prefer_direct(10, 2, 32)
    assert not prefer_direct(19, 3, 32) and prefer_direct(20, 3, 32)
    assert not prefer_direct(29, 4, 32) and prefer_direct(30, 4, 32)
    assert not prefer_direct(1000, 5, 32)
    # a shorter stack makes the operator route's per-order bytes relatively dearer
    assert prefer_direct(4, 2, 10) and not prefer_direct(3, 2, 10)
    # the real-F operator route writes and reads half the bytes per order: twice the orders per block
    assert not prefer_direct(19, 2, 32, True) and prefer_direct(20, 2, 32, True)
    assert not prefer_direct(39, 3, 32, True) and prefer_direct(40, 3, 32, True)
    assert all(prefer_direct(n, 1, 32, True) for n in (1, 2, 16))


def test_poisson_trace_statistics():
    from paper_2602_20870_amd.serve import poisson_trace
    t, g, a, b = poisson_trace(20000, 5000.0, list(range(8)), 64, seed=1)
    gaps = np.diff(t)
    assert abs(gaps.mean() - 2e-4) < 1e-5
    assert np.all(gaps > 0)
    assert set(g) == set(range(8)) and a.min() >= -2 and a.max() <= 2
    assert b.min() == 1 and b.max() == 64


def test_slot_sets_grouped_by_size_on_hardware_queues(built):
    """The trace's eight plans on four queues: the two N = 4096 plans share one, the two 2048, the
    two 1024 and the 256 / 512 pair the others, so no small plan waits behind a large plan's batch."""
    from types import SimpleNamespace
    from paper_2602_20870_amd.serve import Server
    srv = Server(hbm_budget=1 << 40, K=4, bmax=8, slot_sets=1, use_graphs=False, device="cpu")
    srv.streams = [f"q{i}" for i in range(4)]
    Ns = [256, 512, 1024, 1024, 2048, 2048, 4096, 4096]
    for gid, N in enumerate(Ns):
        srv.plans[gid] = SimpleNamespace(N=N, L=32)
        srv.slots[gid] = [SimpleNamespace(stream=None)]
    srv._balance()
    q = {gid: srv.slots[gid][0].stream for gid in srv.plans}
    assert q[6] == q[7] and q[4] == q[5] and q[2] == q[3] and q[0] == q[1]
    assert len({q[0], q[2], q[4], q[6]}) == 4
    # fewer slot sets than queues: one each
    srv.plans = {0: SimpleNamespace(N=64, L=8), 1: SimpleNamespace(N=128, L=8)}
    srv.slots = {0: [SimpleNamespace(stream=None)], 1: [SimpleNamespace(stream=None)]}
    srv._balance()
    assert srv.slots[0][0].stream != srv.slots[1][0].stream
