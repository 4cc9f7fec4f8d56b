"""The seeded input recipe: the named workloads have the stated shapes and structure, F is
orthogonal (real graphs) or unitary, and a seed fixes every input.  CPU only."""
import numpy as np
import pytest

import synth


def _defect(F):
    return float(np.max(np.abs(F.conj().T @ F - np.eye(F.shape[0]))))


@pytest.mark.parametrize("name,N", [("er64", None), ("dft256", None), ("knn4096", 300), ("sphere2048", 240)])
def test_named_workloads(name, N):
    c = synth.make_config(name, seed=3, N=N)
    spec = synth.CONFIGS[name]
    n = c["N"]
    assert n == (N or spec["N"]) and c["F"].shape == (n, n) and c["L"] == spec["L"]
    assert _defect(c["F"]) < 1e-10
    assert np.isrealobj(c["F"]) == (name != "dft256")
    assert c["alphas"].shape == (spec["n_alpha"],) and np.all(np.abs(c["alphas"]) <= 2.0)
    X = c["X"]
    assert X.shape == (spec["n_alpha"], n, spec["B"]) and np.iscomplexobj(X) == spec["x_complex"]
    again = synth.make_config(name, seed=3, N=N)
    assert np.array_equal(again["F"], c["F"]) and np.array_equal(again["alphas"], c["alphas"])
    assert np.array_equal(again["X"], X)
    other = synth.make_config(name, seed=4, N=N, with_signals=False)
    assert not np.array_equal(other["alphas"], c["alphas"]) and other["X"] is None


def test_dft_minus_one_multiplicity():
    """The unitary DFT of size 256 has eigenvalues +-1, +-j with multiplicities 65, 64, 64, 63
    (-1 appears 64 times), the r_-1 the dft256 workload is chosen for."""
    r, gap = synth.phase_gap_to_minus_one(synth.dft_matrix(256))
    assert r == 64 and gap > 0.5


def test_knn_graph_is_symmetric_with_at_least_k_neighbours():
    pts = synth.gmm_points(200, 5, np.random.default_rng(1))
    a = synth.knn_adjacency(pts, 10)
    assert np.array_equal(a, a.T) and np.all(np.diag(a) == 0)
    assert np.all((a > 0).sum(axis=1) >= 10) and np.all((a >= 0) & (a <= 1))
