"""FP64 reference implementation of the exact GFRFT and of FGFRFT.

TEST INFRASTRUCTURE ONLY: imported by tests, smoke() and the CPU-baseline
leg of the benchmark, never by the GPU library.

Notation follows the paper (arXiv 2602.20870):
  F            unitary GFT matrix, F = V diag(e^{j theta}) V^H, theta in (-pi, pi]
  I_{-1}       indices with theta_k = pi (eigenvalue -1)
  P, P_c       projector onto the -1 eigenspace and its complement, P_c = I - P
  c_n(alpha)   Fourier coefficients of e^{j alpha theta} on (-pi, pi)
  M_n          cached powers F^n P_c, n = 0..L (Algorithm 1, offline stage)
  Q            the L-order FGFRFT operator Q_L^alpha (Definition 1)

Readings where the paper is silent (listed with their reasons in the
design notes of the repository):
  * "theta_k = pi" is decided as |lambda_k + 1| <= tau (default 1e-6) and
    such phases are snapped to exactly pi.
  * Negative powers are always taken as M_n^H (Proposition 2); no separate
    F^{-n} recurrence.
  * dc_n/dalpha at alpha = n uses the smooth limit 0 (Proposition 4 is
    stated for non-integer alpha; the formula is continuous).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

__all__ = [
    "TAU_SNAP", "unitarity_defect", "spectral_decomposition", "coefficients",
    "coefficient_derivatives", "gfrft_exact", "gfrft_exact_grad",
    "split_projectors", "projectors_symmetric_route", "power_stack",
    "fgfrft_combine", "term_matrix", "fgfrft_combine_many", "fgfrft_operator", "fgfrft_operator_standard",
    "fgfrft_operator_eigen", "dQ_dalpha", "dQ_dalpha_eigen", "apply",
    "grad", "truncation_residual", "pointwise_bound", "frobenius_error_exact",
    "frobenius_bound_tight", "frobenius_bound_simplified",
    "worst_case_nmse_bound", "parseval_tail", "parseval_nmse_prediction",
    "error_metrics", "block_errors", "sampled_rows", "sampled_term_rows", "Plan",
]

TAU_SNAP = 1e-6


# ----------------------------------------------------------------------------
# Sec. III-A: spectral representation of a unitary F
# ----------------------------------------------------------------------------
def unitarity_defect(F: np.ndarray) -> float:
    """max_ij |(F^H F - I)_ij|."""
    n = F.shape[0]
    return float(np.max(np.abs(F.conj().T @ F - np.eye(n))))


def spectral_decomposition(F: np.ndarray, tau: float = TAU_SNAP):
    """F = Z diag(e^{j theta}) Z^H with theta in (-pi, pi] (Sec. III-A).

    The unitary Z comes from a complex Schur form; F is normal, so the
    triangular factor is diagonal up to rounding (checked).  Eigenvalues
    within ``tau`` of -1 are put in I_{-1} and their phase set to pi (the
    principal branch puts the endpoint at +pi).

    Returns (Z, theta, in_minus1) with in_minus1 a boolean mask.
    """
    F = np.asarray(F, dtype=np.complex128)
    n = F.shape[0]
    T, Z = scipy.linalg.schur(F, output="complex")
    off = np.linalg.norm(np.triu(T, 1))
    if off > 1e-9 * max(1.0, np.sqrt(n)):
        raise ValueError(f"F is not normal enough for a diagonal Schur form (off={off:.3e})")
    lam = np.diag(T)
    theta = np.angle(lam)
    m1 = np.abs(lam + 1.0) <= tau
    theta[m1] = np.pi
    return Z, theta, m1


def coefficients(alpha: float, L: int) -> np.ndarray:
    """c_n(alpha), n = -L..L: sin(pi(alpha-n)) / (pi(alpha-n)), 1 at alpha = n (Sec. III-A)."""
    n = np.arange(-L, L + 1, dtype=np.float64)
    x = alpha - n
    out = np.ones_like(x)
    nz = x != 0.0
    out[nz] = np.sin(np.pi * x[nz]) / (np.pi * x[nz])
    return out


def coefficient_derivatives(alpha: float, L: int) -> np.ndarray:
    """dc_n/dalpha, n = -L..L (Proposition 4).

    With x = alpha - n, d/dx [sin(pi x)/(pi x)] = (cos(pi x) - sin(pi x)/(pi x)) / x.
    For |x| < 1e-4 the Taylor series -pi^2 x/3 + pi^4 x^3/30 is used (0 at x = 0).
    """
    n = np.arange(-L, L + 1, dtype=np.float64)
    x = alpha - n
    out = np.empty_like(x)
    small = np.abs(x) < 1e-4
    xs = x[small]
    out[small] = -(np.pi ** 2) * xs / 3.0 + (np.pi ** 4) * xs ** 3 / 30.0
    xb = x[~small]
    out[~small] = (np.cos(np.pi * xb) - np.sin(np.pi * xb) / (np.pi * xb)) / xb
    return out


def gfrft_exact(F: np.ndarray, alpha: float, decomposition=None) -> np.ndarray:
    """Exact GFRFT F^alpha = V diag(e^{j alpha theta}) V^H, principal branch (Sec. II-B, III-A)."""
    Z, theta, _ = decomposition if decomposition is not None else spectral_decomposition(F)
    return (Z * np.exp(1j * alpha * theta)[None, :]) @ Z.conj().T


def gfrft_exact_grad(F: np.ndarray, alpha: float, decomposition=None) -> np.ndarray:
    """d F^alpha / d alpha = V diag(j theta e^{j alpha theta}) V^H."""
    Z, theta, _ = decomposition if decomposition is not None else spectral_decomposition(F)
    return (Z * (1j * theta * np.exp(1j * alpha * theta))[None, :]) @ Z.conj().T


# ----------------------------------------------------------------------------
# Sec. III-B / Algorithm 1, offline stage
# ----------------------------------------------------------------------------
def split_projectors(F: np.ndarray, tau: float = TAU_SNAP, decomposition=None):
    """P = W W^H over the orthonormal -1 eigenvectors W, P_c = I - P (Algorithm 1).

    Returns (P, P_c, r_minus1).
    """
    Z, theta, m1 = decomposition if decomposition is not None else spectral_decomposition(F, tau)
    W = Z[:, m1]
    P = W @ W.conj().T
    n = F.shape[0]
    return P, np.eye(n) - P, int(m1.sum())


def projectors_symmetric_route(F: np.ndarray, cos_tol: float = 1e-10):
    """P for a large real orthogonal F from eigh of its symmetric part.

    (F + F^T)/2 = V diag(cos theta) V^T shares F's eigenvectors; the -1
    eigenspace is the cos(theta) = -1 eigenspace.  Used where a complex
    Schur form of F is too slow (N >= 4096).  Returns (P, P_c, r, next_cos)
    where next_cos is the smallest cos(theta) outside the -1 cluster.
    """
    F = np.asarray(F, dtype=np.float64)
    w, V = np.linalg.eigh(0.5 * (F + F.T))
    m1 = w <= -1.0 + cos_tol
    W = V[:, m1]
    P = W @ W.T
    nxt = float(w[~m1].min()) if (~m1).any() else float("nan")
    return P, np.eye(F.shape[0]) - P, int(m1.sum()), nxt


def power_stack(F: np.ndarray, Pc: np.ndarray, L: int) -> list[np.ndarray]:
    """M_0 = P_c, M_n = F M_{n-1}, n = 1..L (Algorithm 1, offline loop)."""
    M = [np.array(Pc, dtype=np.result_type(F, Pc))]
    for _ in range(L):
        M.append(F @ M[-1])
    return M


# ----------------------------------------------------------------------------
# Definition 1 / Proposition 2 / Algorithm 1, online stage
# ----------------------------------------------------------------------------
def fgfrft_combine(P: np.ndarray, M: list[np.ndarray], alpha: float) -> np.ndarray:
    """Q = e^{j pi alpha} P + c_0 P_c + sum_{n=1}^L (c_n M_n + c_{-n} M_n^H).

    The online linear combination of Algorithm 1 with negative powers read
    as conjugate transposes (Proposition 2).  M[0] is P_c.
    """
    L = len(M) - 1
    c = coefficients(alpha, L)          # c[L + n] = c_n
    Q = np.exp(1j * np.pi * alpha) * P + c[L] * M[0]
    for n in range(1, L + 1):
        Q = Q + c[L + n] * M[n] + c[L - n] * M[n].conj().T
    return Q


def term_matrix(M: list[np.ndarray]) -> np.ndarray:
    """The 2L+1 real-coefficient terms of the online combination, one per row:
    [P_c, M_1, .., M_L, M_1^H, .., M_L^H], each flattened row-major -> [(2L+1), N*N]."""
    L = len(M) - 1
    N = M[0].shape[0]
    T = np.empty((2 * L + 1, N * N), dtype=M[0].dtype)
    T[0] = M[0].reshape(-1)
    for n in range(1, L + 1):
        T[n] = M[n].reshape(-1)
        T[L + n] = M[n].conj().T.reshape(-1)
    return T


def fgfrft_combine_many(P: np.ndarray, T: np.ndarray, alphas) -> np.ndarray:
    """Q(alpha_a) for a batch of orders (Algorithm 1's online combination, Proposition 2).

    The real coefficients [c_0, c_1..c_L, c_{-1}..c_{-L}] of every order form the rows of C,
    and C T (one matrix product over the terms of :func:`term_matrix`) is the sum
    c_0 P_c + sum_n (c_n M_n + c_{-n} M_n^H) for all orders at once; e^{j pi alpha} P is added
    per order.  Returns complex128 [n_alpha, N, N].  With the row-sampled terms of
    :func:`sampled_term_rows` and P[R, :] in place of P it returns the rows R instead,
    [n_alpha, |R|, N].
    """
    alphas = np.atleast_1d(np.asarray(alphas, dtype=np.float64))
    K = T.shape[0]
    L = (K - 1) // 2
    C = np.empty((alphas.size, K))
    for a, al in enumerate(alphas):
        c = coefficients(al, L)                 # c[L + n] = c_n
        C[a, 0] = c[L]
        C[a, 1:L + 1] = c[L + 1:]
        C[a, L + 1:] = c[L - 1::-1]
    S = (C @ T).reshape((alphas.size,) + P.shape)
    Q = np.empty((alphas.size,) + P.shape, dtype=np.complex128)
    for a, al in enumerate(alphas):
        Q[a] = S[a] + np.exp(1j * np.pi * al) * P
    return Q


def fgfrft_operator(F: np.ndarray, alpha: float, L: int, tau: float = TAU_SNAP,
                    decomposition=None, stack=None) -> np.ndarray:
    """Q_L^alpha by Algorithm 1 (offline split + powers, online combination).

    Integer orders return F^alpha (Definition 1 / Algorithm 1); negative
    integer powers are conjugate-transposed positive powers.
    ``stack`` may pass a precomputed (P, M) pair.
    """
    F = np.asarray(F)
    if float(alpha).is_integer():
        m = int(alpha)
        Fm = np.linalg.matrix_power(F.astype(np.complex128), abs(m))
        return Fm if m >= 0 else Fm.conj().T
    if stack is None:
        P, Pc, _ = split_projectors(F, tau, decomposition)
        M = power_stack(F, Pc, L)
    else:
        P, M = stack
    return fgfrft_combine(P, M, alpha)


def fgfrft_operator_standard(F: np.ndarray, alpha: float, L: int) -> np.ndarray:
    """Standard truncated form sum_{n=-L}^{L} c_n F^n with no -1 split (Remark after Def. 1)."""
    n = F.shape[0]
    return fgfrft_combine(np.zeros((n, n)), power_stack(F, np.eye(n), L), alpha)


def fgfrft_operator_eigen(F: np.ndarray, alpha: float, L: int, tau: float = TAU_SNAP,
                          decomposition=None) -> np.ndarray:
    """Q_L^alpha through the eigenbasis (Proposition 1 truncated at |n| <= L).

    Q = Z diag(q) Z^H, q_k = e^{j pi alpha} on I_{-1}, else sum_n c_n e^{j n theta_k}.
    An independent route to the same operator as :func:`fgfrft_operator`.
    """
    Z, theta, m1 = decomposition if decomposition is not None else spectral_decomposition(F, tau)
    c = coefficients(alpha, L)
    n = np.arange(-L, L + 1)
    q = np.exp(1j * np.outer(theta, n)) @ c
    q[m1] = np.exp(1j * np.pi * alpha)
    return (Z * q[None, :]) @ Z.conj().T


# ----------------------------------------------------------------------------
# Proposition 4: order derivative; Definition 2: apply; gradients of a loss
# ----------------------------------------------------------------------------
def dQ_dalpha(P: np.ndarray, M: list[np.ndarray], alpha: float) -> np.ndarray:
    """dQ/dalpha = j pi e^{j pi alpha} P + sum_n c_n'(alpha) F^n P_c (Proposition 4)."""
    L = len(M) - 1
    d = coefficient_derivatives(alpha, L)
    D = 1j * np.pi * np.exp(1j * np.pi * alpha) * P + d[L] * M[0]
    for n in range(1, L + 1):
        D = D + d[L + n] * M[n] + d[L - n] * M[n].conj().T
    return D


def dQ_dalpha_eigen(F: np.ndarray, alpha: float, L: int, tau: float = TAU_SNAP,
                    decomposition=None) -> np.ndarray:
    """dQ/dalpha through the eigenbasis: Z diag(g) Z^H with g_k = j pi e^{j pi alpha} on I_{-1},
    else sum_n c_n'(alpha) e^{j n theta_k}."""
    Z, theta, m1 = decomposition if decomposition is not None else spectral_decomposition(F, tau)
    d = coefficient_derivatives(alpha, L)
    n = np.arange(-L, L + 1)
    g = np.exp(1j * np.outer(theta, n)) @ d
    g[m1] = 1j * np.pi * np.exp(1j * np.pi * alpha)
    return (Z * g[None, :]) @ Z.conj().T


def apply(Q: np.ndarray, X: np.ndarray) -> np.ndarray:
    """FGFRFT of graph signals, x~ = Q x (Definition 2); X holds one signal per column."""
    return Q @ X


def grad(P: np.ndarray, M: list[np.ndarray], alphas, X, GY, x_real: bool | None = None):
    """Gradients of a real loss l(Y), Y[a] = Q(alpha_a) X[a].

    GY[a] = dl/dRe Y[a] + j dl/dIm Y[a] (the convention of complex autograd).
    dl/dalpha_a = Re <GY[a] X[a]^H, dQ/dalpha>  with <A, B> = sum conj(A) B,
    dl/dX[a]    = Q(alpha_a)^H GY[a]  (real part for a real X).
    Returns (dalpha [n_alpha], dX like X).
    """
    X = np.asarray(X)
    if x_real is None:
        x_real = np.isrealobj(X)
    dal = np.empty(len(alphas))
    dX = np.empty(X.shape, dtype=np.float64 if x_real else np.complex128)
    for a, al in enumerate(alphas):
        Q = fgfrft_combine(P, M, al)
        D = dQ_dalpha(P, M, al)
        GQ = GY[a] @ X[a].conj().T
        dal[a] = float(np.real(np.sum(GQ.conj() * D)))
        g = Q.conj().T @ GY[a]
        dX[a] = g.real if x_real else g
    return dal, dX


# ----------------------------------------------------------------------------
# Sec. III-D: truncation error, bounds; Sec. IV-A: metrics and predictions
# ----------------------------------------------------------------------------
def truncation_residual(theta, alpha: float, L: int) -> np.ndarray:
    """R_L(theta) = e^{j alpha theta} - sum_{n=-L}^{L} c_n(alpha) e^{j n theta}."""
    theta = np.atleast_1d(np.asarray(theta, dtype=np.float64))
    c = coefficients(alpha, L)
    n = np.arange(-L, L + 1)
    return np.exp(1j * alpha * theta) - np.exp(1j * np.outer(theta, n)) @ c


def pointwise_bound(theta, alpha: float, L: int) -> np.ndarray:
    """Theorem 1: |sin(pi alpha)| / (pi cos(theta/2)) * (1/(L+1-alpha) + 1/(L+1+alpha)), L > |alpha|."""
    theta = np.asarray(theta, dtype=np.float64)
    return (np.abs(np.sin(np.pi * alpha)) / (np.pi * np.cos(theta / 2.0))
            * (1.0 / (L + 1 - alpha) + 1.0 / (L + 1 + alpha)))


def frobenius_error_exact(theta, in_minus1, alpha: float, L: int) -> float:
    """Theorem 2 identity: ||F^alpha - Q||_F = sqrt(sum_{k not in I_{-1}} |R_L(theta_k)|^2)."""
    th = np.asarray(theta)[~np.asarray(in_minus1)]
    return float(np.sqrt(np.sum(np.abs(truncation_residual(th, alpha, L)) ** 2)))


def frobenius_bound_tight(theta, in_minus1, alpha: float, L: int) -> float:
    """Theorem 2, first bound (with sum over 1/cos^2(theta_k/2))."""
    th = np.asarray(theta)[~np.asarray(in_minus1)]
    pre = 2 * (L + 1) * abs(np.sin(np.pi * alpha)) / (np.pi * ((L + 1) ** 2 - alpha ** 2))
    return float(pre * np.sqrt(np.sum(1.0 / np.cos(th / 2.0) ** 2)))


def frobenius_bound_simplified(theta, in_minus1, alpha: float, L: int) -> float:
    """Theorem 2, second bound (with sqrt(N - r_{-1}) / cos_{c,min})."""
    th = np.asarray(theta)[~np.asarray(in_minus1)]
    ccmin = float(np.min(np.abs(np.cos(th / 2.0))))
    pre = 2 * (L + 1) * np.sqrt(th.size) * abs(np.sin(np.pi * alpha))
    return float(pre / (np.pi * ccmin * ((L + 1) ** 2 - alpha ** 2)))


def worst_case_nmse_bound(theta, in_minus1, alpha: float, L: int) -> float:
    """Sec. IV-A worst-case NMSE bound; 0 when r_{-1} = N."""
    in_minus1 = np.asarray(in_minus1)
    N = in_minus1.size
    th = np.asarray(theta)[~in_minus1]
    if th.size == 0:
        return 0.0
    ccmin = float(np.min(np.abs(np.cos(th / 2.0))))
    return float(4 * (L + 1) ** 2 * np.sin(np.pi * alpha) ** 2
                 / (np.pi ** 2 * ((L + 1) ** 2 - alpha ** 2) ** 2) * th.size / (N * ccmin ** 2))


def parseval_tail(alpha: float, L: int) -> float:
    """sum_{|n|>L} c_n(alpha)^2 = 1 - sum_{|n|<=L} c_n^2 (Parseval: the full sum is 1)."""
    c = coefficients(alpha, L)
    return float(1.0 - np.sum(c * c))


def parseval_nmse_prediction(alpha: float, L: int, N: int, r_minus1: int = 0) -> float:
    """Typical-case NMSE ~ (N - r_{-1})/N * sum_{|n|>L} c_n^2 (Sec. IV-A)."""
    return (N - r_minus1) / N * parseval_tail(alpha, L)


def error_metrics(E: np.ndarray) -> dict:
    """MSE = ||E||_F^2/N^2, MAE = sum|E_ij|/N^2, NMSE = ||E||_F^2/N (Sec. IV-A)."""
    N = E.shape[0]
    f2 = float(np.sum(np.abs(E) ** 2))
    return dict(MSE=f2 / N ** 2, MAE=float(np.sum(np.abs(E))) / N ** 2, NMSE=f2 / N)


def block_errors(Q: np.ndarray, Fa: np.ndarray, P: np.ndarray) -> dict:
    """E_total, E_{-1} = ||P (Q - F^a) P||_F and E_c = ||P_c (Q - F^a) P_c||_F (Sec. IV-F)."""
    E = Q - Fa
    Pc = np.eye(P.shape[0]) - P
    return dict(E_total=float(np.linalg.norm(E)), E_m1=float(np.linalg.norm(P @ E @ P)),
                E_c=float(np.linalg.norm(Pc @ E @ Pc)))


# ----------------------------------------------------------------------------
# Large N: sampled rows of Q without the full power stack
# ----------------------------------------------------------------------------
def sampled_rows(F: np.ndarray, P: np.ndarray, alphas, L: int, rows) -> np.ndarray:
    """Rows R of Q_L^alpha for each alpha, in O(L N^2 |R|).

    Since P_c commutes with F, (M_n)[R, :] = P_c[R, :] F^n (row recurrence)
    and (M_n^H)[R, :] = ((M_n)[:, R])^H with (M_n)[:, R] = F^n P_c[:, R]
    (column recurrence).  Returns complex128 [n_alpha, |R|, N].
    """
    rows = np.asarray(rows)
    N = F.shape[0]
    Pc = np.eye(N) - P
    rr = [Pc[rows, :].astype(np.complex128)]
    cc = [Pc[:, rows].astype(np.complex128)]
    for _ in range(L):
        rr.append(rr[-1] @ F)
        cc.append(F @ cc[-1])
    out = np.empty((len(alphas), rows.size, N), dtype=np.complex128)
    for a, al in enumerate(alphas):
        c = coefficients(al, L)
        acc = np.exp(1j * np.pi * al) * P[rows, :] + c[L] * rr[0]
        for n in range(1, L + 1):
            acc = acc + c[L + n] * rr[n] + c[L - n] * cc[n].conj().T
        out[a] = acc
    return out


def sampled_term_rows(F: np.ndarray, P: np.ndarray, L: int, rows) -> np.ndarray:
    """Rows R of the 2L+1 terms of :func:`term_matrix`, [P_c, M_1..M_L, M_1^H..M_L^H][R, :],
    flattened per term -> [(2L+1), |R| N], by the row and column recurrences of
    :func:`sampled_rows` ((M_n)[R, :] = P_c[R, :] F^n, (M_n^H)[R, :] = (F^n P_c[:, R])^H), so that
    ``fgfrft_combine_many(P[rows, :], T, alphas)`` gives the rows R of Q for many orders at once."""
    rows = np.asarray(rows)
    N = F.shape[0]
    Pc = np.eye(N) - P
    r = Pc[rows, :].astype(np.result_type(F, Pc))
    c = Pc[:, rows].astype(np.result_type(F, Pc))
    T = np.empty((2 * L + 1, rows.size * N), dtype=r.dtype)
    T[0] = r.reshape(-1)
    for n in range(1, L + 1):
        r = r @ F
        c = F @ c
        T[n] = r.reshape(-1)
        T[L + n] = c.conj().T.reshape(-1)
    return T


class Plan:
    """Offline stage of Algorithm 1 held for repeated online queries.

    ``route`` is "schur" (complex Schur, any unitary F) or "symmetric"
    (eigh of the symmetric part, real orthogonal F, large N).
    """

    def __init__(self, F: np.ndarray, L: int, tau: float = TAU_SNAP, route: str = "schur"):
        self.F = np.asarray(F)
        self.L = int(L)
        self.N = self.F.shape[0]
        if route == "schur":
            self.decomposition = spectral_decomposition(self.F, tau)
            self.P, self.Pc, self.r_minus1 = split_projectors(self.F, tau, self.decomposition)
        elif route == "symmetric":
            self.decomposition = None
            self.P, self.Pc, self.r_minus1, self.next_cos = projectors_symmetric_route(self.F)
        else:
            raise ValueError(route)
        if np.isrealobj(self.F):
            self.P = self.P.real.copy()
            self.Pc = self.Pc.real.copy()
        self.M = power_stack(self.F, self.Pc, self.L)

    def operator(self, alpha: float) -> np.ndarray:
        return fgfrft_operator(self.F, alpha, self.L, stack=(self.P, self.M))

    def combine(self, alpha: float) -> np.ndarray:
        return fgfrft_combine(self.P, self.M, alpha)
