"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This module builds graphs, graph Fourier matrices, transform orders and
graph signals.  It holds none of the fractional-transform arithmetic
(no coefficients, projectors, powers or operators): only the inputs that
the method takes, per the paper's problem statement (a unitary GFT
matrix F, orders alpha, a truncation order L and graph signals).

Graph Fourier matrices follow Sec. II-A: a symmetric graph shift operator
Z = U diag(lambda) U^H gives the GFT matrix F = U^H (= U^T for real Z).
Eigenvalues are taken in ascending order and each eigenvector's sign is
fixed so that its largest-magnitude entry (first index on ties) is
positive, so F is a deterministic function of the graph.

Every generator takes an explicit integer seed; sub-streams are derived
with ``numpy.random.SeedSequence(seed).spawn`` so that the graph, the
orders and the signals of one configuration are independent draws.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "streams", "er_adjacency", "grid_adjacency", "knn_adjacency",
    "gmm_points", "sphere_points", "laplacian", "gft_from_shift",
    "dft_matrix", "haar_unitary", "prescribed_spectrum_unitary",
    "rotation_blocks", "orders", "real_signals", "complex_signals",
    "phase_gap_to_minus_one", "CONFIGS", "make_config",
]


# ----------------------------------------------------------------------------
# random streams
# ----------------------------------------------------------------------------
def streams(seed: int, n: int) -> list[np.random.Generator]:
    """n independent generators derived from one integer seed."""
    return [np.random.default_rng(s) for s in np.random.SeedSequence(int(seed)).spawn(n)]


# ----------------------------------------------------------------------------
# graphs
# ----------------------------------------------------------------------------
def er_adjacency(n: int, p: float, rng: np.random.Generator) -> np.ndarray:
    """Erdos-Renyi G(n, p), undirected, unweighted, no self loops."""
    u = rng.random((n, n))
    a = np.triu(u < p, k=1).astype(np.float64)
    return a + a.T


def grid_adjacency(rows: int, cols: int, weights) -> np.ndarray:
    """4-neighbour grid graph with one weight per undirected edge.

    ``weights`` is a callable ``w(m)`` returning m positive edge weights
    (drawn once per undirected edge, row-major edge order: all horizontal
    edges, then all vertical edges).
    """
    n = rows * cols
    idx = np.arange(n).reshape(rows, cols)
    h = np.stack([idx[:, :-1].ravel(), idx[:, 1:].ravel()], axis=1)
    v = np.stack([idx[:-1, :].ravel(), idx[1:, :].ravel()], axis=1)
    edges = np.concatenate([h, v], axis=0)
    w = np.asarray(weights(edges.shape[0]), dtype=np.float64)
    a = np.zeros((n, n))
    a[edges[:, 0], edges[:, 1]] = w
    a[edges[:, 1], edges[:, 0]] = w
    return a


def gmm_points(n: int, components: int, rng: np.random.Generator,
               spread: float = 0.15) -> np.ndarray:
    """3-D points from an equal-weight isotropic Gaussian mixture.

    Means are uniform in [-1, 1]^3 and each component has standard
    deviation ``spread``.
    """
    means = rng.uniform(-1.0, 1.0, size=(components, 3))
    comp = rng.integers(0, components, size=n)
    return means[comp] + spread * rng.standard_normal((n, 3))


def sphere_points(n: int, rng: np.random.Generator, jitter: float = 0.02) -> np.ndarray:
    """Points uniform on the unit sphere plus N(0, jitter^2) jitter."""
    g = rng.standard_normal((n, 3))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    return g + jitter * rng.standard_normal((n, 3))


def knn_adjacency(points: np.ndarray, k: int) -> np.ndarray:
    """Symmetric kNN graph with Gaussian weights exp(-d^2/sigma^2).

    sigma is the median distance over all k-nearest-neighbour pairs; the
    directed kNN relation is symmetrised by union (an edge exists if
    either endpoint lists the other), with the weight of the pair.
    """
    from scipy.spatial import cKDTree

    n = points.shape[0]
    tree = cKDTree(points)
    d, j = tree.query(points, k=k + 1)
    d, j = d[:, 1:], j[:, 1:]
    sigma = float(np.median(d))
    w = np.exp(-(d / sigma) ** 2)
    a = np.zeros((n, n))
    rows = np.repeat(np.arange(n), k)
    a[rows, j.ravel()] = w.ravel()
    return np.maximum(a, a.T)


def laplacian(a: np.ndarray) -> np.ndarray:
    """Combinatorial Laplacian D - A."""
    return np.diag(a.sum(axis=1)) - a


def gft_from_shift(z: np.ndarray) -> np.ndarray:
    """GFT matrix F = U^T of a real symmetric shift operator (Sec. II-A).

    Ascending eigenvalues; each eigenvector is signed so that its
    largest-magnitude entry (first index on ties) is positive.
    """
    z = 0.5 * (z + z.T)
    _, u = np.linalg.eigh(z)
    piv = np.argmax(np.abs(u), axis=0)
    sgn = np.sign(u[piv, np.arange(u.shape[1])])
    sgn[sgn == 0] = 1.0
    u = u * sgn[None, :]
    return np.ascontiguousarray(u.T)


# ----------------------------------------------------------------------------
# unitary matrices with known structure
# ----------------------------------------------------------------------------
def dft_matrix(n: int) -> np.ndarray:
    """Unitary DFT, F[k, m] = exp(-2 pi j k m / n) / sqrt(n): the GFT of the directed n-cycle."""
    k = np.arange(n)
    km = np.outer(k, k) % n
    return np.exp(-2j * np.pi * km / n) / np.sqrt(n)


def haar_unitary(n: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed unitary: QR of a complex Gaussian with the R-diagonal phases removed."""
    g = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2.0)
    q, r = np.linalg.qr(g)
    d = np.diag(r)
    return q * (d / np.abs(d))[None, :]


def prescribed_spectrum_unitary(phases: np.ndarray, rng: np.random.Generator,
                                real_basis: bool = False) -> np.ndarray:
    """V diag(exp(j phases)) V^H with a random unitary (or orthogonal) V."""
    n = len(phases)
    if real_basis:
        g = rng.standard_normal((n, n))
        v, r = np.linalg.qr(g)
        v = v * np.sign(np.diag(r))[None, :]
    else:
        v = haar_unitary(n, rng)
    return (v * np.exp(1j * np.asarray(phases))[None, :]) @ v.conj().T


def rotation_blocks(angles) -> np.ndarray:
    """Block-diagonal real orthogonal matrix of 2x2 rotations R(phi)."""
    angles = list(angles)
    n = 2 * len(angles)
    f = np.zeros((n, n))
    for b, phi in enumerate(angles):
        c, s = np.cos(phi), np.sin(phi)
        f[2 * b:2 * b + 2, 2 * b:2 * b + 2] = [[c, -s], [s, c]]
    return f


def phase_gap_to_minus_one(f: np.ndarray, tau: float = 1e-6) -> tuple[int, float]:
    """(number of eigenvalues within tau of -1, smallest |lambda+1| among the rest).

    Used only to reject generated matrices whose spectrum sits in the
    grey zone around -1.  Real F uses the symmetric part, whose eigenvalues
    are cos(theta): |lambda+1| = sqrt(2 + 2 cos(theta)).
    """
    if np.isrealobj(f):
        c = np.linalg.eigvalsh(0.5 * (f + f.T))
        dist = np.sqrt(np.maximum(2.0 + 2.0 * c, 0.0))
    else:
        dist = np.abs(np.linalg.eigvals(f) + 1.0)
    inside = dist <= tau
    rest = dist[~inside]
    return int(inside.sum()), float(rest.min()) if rest.size else float("inf")


# ----------------------------------------------------------------------------
# orders and signals
# ----------------------------------------------------------------------------
def orders(n: int, rng: np.random.Generator, lo: float = -2.0, hi: float = 2.0) -> np.ndarray:
    return rng.uniform(lo, hi, size=n)


def real_signals(shape, rng: np.random.Generator) -> np.ndarray:
    return rng.standard_normal(shape)


def complex_signals(shape, rng: np.random.Generator) -> np.ndarray:
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------
CONFIGS = {
    # ER G(64, 0.1), combinatorial Laplacian, L=10, 16 orders, 32 real signals
    "er64": dict(N=64, L=10, n_alpha=16, B=32, x_complex=False),
    # 32x32 grid, U[0.5,1.5] weights, L=32, 256 orders, 64 complex signals per order
    "grid1024": dict(N=1024, L=32, n_alpha=256, B=64, x_complex=True),
    # directed 256-cycle, unitary DFT (lambda=-1 multiplicity 64)
    "dft256": dict(N=256, L=32, n_alpha=256, B=64, x_complex=True),
    # kNN (k=10) on a 5-component 3-D Gaussian mixture, L=32, 256 orders, 64 real signals per order
    "knn4096": dict(N=4096, L=32, n_alpha=256, B=64, x_complex=False),
    # points on the sphere, kNN k=10, L=48, 64 channels, 64 clouds
    "sphere2048": dict(N=2048, L=48, n_alpha=64, B=64, x_complex=False),
    # 128x64 grid, lognormal(0, 0.5) weights, L=64, 1024 orders, 1024 real signals
    "grid8192": dict(N=8192, L=64, n_alpha=1024, B=1024, x_complex=False),
}


def _graph_F(name: str, rng: np.random.Generator, N: int | None = None) -> np.ndarray:
    if name == "er64":
        return gft_from_shift(laplacian(er_adjacency(64, 0.1, rng)))
    if name == "grid1024":
        return gft_from_shift(laplacian(grid_adjacency(32, 32, lambda m: rng.uniform(0.5, 1.5, m))))
    if name == "dft256":
        return dft_matrix(256)
    if name == "knn4096":
        return gft_from_shift(laplacian(knn_adjacency(gmm_points(N or 4096, 5, rng), 10)))
    if name == "sphere2048":
        return gft_from_shift(laplacian(knn_adjacency(sphere_points(N or 2048, rng), 10)))
    if name == "grid8192":
        return gft_from_shift(laplacian(grid_adjacency(128, 64, lambda m: rng.lognormal(0.0, 0.5, m))))
    raise KeyError(name)


def point_cloud_denoising(seed: int = 0, N: int = 2048, clouds: int = 64, noise: float = 0.05) -> dict:
    """Data of the differentiable workload: N points uniform on the unit sphere plus N(0, 0.02^2)
    jitter, the graph of ``sphere2048`` (kNN k = 10, combinatorial Laplacian, F = U^T, the same F as
    ``make_config("sphere2048", seed)``), the clean coordinates as a 3-channel graph signal
    [N, 3], and `clouds` noisy copies [clouds, N, 3] with N(0, noise^2) added per coordinate."""
    g_graph, _, g_sig = streams(seed, 3)
    pts = sphere_points(N, g_graph)
    F = gft_from_shift(laplacian(knn_adjacency(pts, 10)))
    noisy = pts[None, :, :] + noise * g_sig.standard_normal((clouds, N, 3))
    return dict(F=F, clean=pts, noisy=noisy, L=CONFIGS["sphere2048"]["L"], N=N)


def make_config(name: str, seed: int = 0, n_alpha: int | None = None,
                B: int | None = None, N: int | None = None,
                with_signals: bool = True) -> dict:
    """Build one named workload: F (float64 or complex128), orders, signals.

    Returns a dict with keys F, alphas, X (shape [n_alpha, N, B] or None),
    L, N, name, seed.  ``N`` overrides the node count of the kNN workloads
    (used for the serving plans of uneven size).
    """
    spec = dict(CONFIGS[name])
    g_graph, g_alpha, g_sig = streams(seed, 3)
    F = _graph_F(name, g_graph, N)
    n = F.shape[0]
    na = spec["n_alpha"] if n_alpha is None else n_alpha
    b = spec["B"] if B is None else B
    alphas = orders(na, g_alpha)
    X = None
    if with_signals:
        X = complex_signals((na, n, b), g_sig) if spec["x_complex"] else real_signals((na, n, b), g_sig)
    return dict(name=name, seed=seed, F=F, alphas=alphas, X=X, L=spec["L"], N=n)
