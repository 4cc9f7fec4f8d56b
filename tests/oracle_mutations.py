"""Plausible mistakes planted in the CPU oracle, to check that the pins catch each of them.

Each entry replaces one oracle routine by a variant with a single slip (a dropped term, a
wrong sign or index, a missing conjugate, a transposed operand).  ``apply(name)`` installs
it in both the module and the package namespace, in this process only; the mutation test
runs the pin suite in a child process with the variable FGFRFT_ORACLE_MUTATION set, and the
test configuration installs the named mutation before collection.  Nothing here touches the
GPU library.
"""
from __future__ import annotations

import numpy as np


def _coefficients_index_flip(alpha, L):
    n = np.arange(-L, L + 1, dtype=np.float64)
    x = alpha + n                                   # slip: c_n(alpha) = sinc(alpha + n)
    out = np.ones_like(x)
    nz = x != 0.0
    out[nz] = np.sin(np.pi * x[nz]) / (np.pi * x[nz])
    return out


def _coefficients_unnormalised(alpha, L):
    n = np.arange(-L, L + 1, dtype=np.float64)
    x = alpha - n
    out = np.ones_like(x)
    nz = x != 0.0
    out[nz] = np.sin(np.pi * x[nz]) / x[nz]         # slip: the 1/pi of the sinc dropped
    return out


def _derivatives_sign(alpha, L):
    from oracle import fgfrft as m
    return -_ORIG["coefficient_derivatives"](alpha, L)  # slip: sign of dc_n/dalpha


def _combine(variant):
    def f(P, M, alpha):
        from oracle import fgfrft as m
        L = len(M) - 1
        c = m.coefficients(alpha, L)
        ph = np.exp(-1j * np.pi * alpha) if variant == "phase_sign" else np.exp(1j * np.pi * alpha)
        Q = (0.0 if variant == "drop_P" else ph) * P
        Q = Q + c[L] * (np.eye(P.shape[0]) if variant == "c0_identity" else M[0])
        for n in range(1, L + 1):
            neg = M[n] if variant == "no_adjoint" else (M[n].T if variant == "transpose_only" else M[n].conj().T)
            Q = Q + c[L + n] * M[n] + c[L - n] * neg
        return Q
    return f


def _power_stack_off_by_one(F, Pc, L):
    M = [np.array(Pc, dtype=np.result_type(F, Pc))]
    for _ in range(L):
        M.append(F @ M[-1])
    return [M[0]] + [F @ m_ for m_ in M[1:]]        # slip: M_n = F^{n+1} P_c for n >= 1


def _split_projectors_transpose(F, tau=1e-6, decomposition=None):
    from oracle import fgfrft as m
    Z, theta, m1 = decomposition if decomposition is not None else m.spectral_decomposition(F, tau)
    W = Z[:, m1]
    P = W @ W.T                                     # slip: transpose instead of conjugate transpose
    return P, np.eye(F.shape[0]) - P, int(m1.sum())


def _spectral_snap_minus_pi(F, tau=1e-6):
    Z, theta, m1 = _ORIG["spectral_decomposition"](F, tau)
    theta = theta.copy()
    theta[m1] = -np.pi                              # slip: the -1 phase on the other branch end
    return Z, theta, m1


def _dQ_drop_P(P, M, alpha):
    from oracle import fgfrft as m
    L = len(M) - 1
    d = m.coefficient_derivatives(alpha, L)
    D = d[L] * M[0]                                 # slip: the j pi e^{j pi alpha} P term dropped
    for n in range(1, L + 1):
        D = D + d[L + n] * M[n] + d[L - n] * M[n].conj().T
    return D


def _grad_no_conj(P, M, alphas, X, GY, x_real=None):
    from oracle import fgfrft as m
    X = np.asarray(X)
    if x_real is None:
        x_real = np.isrealobj(X)
    dal = np.empty(len(alphas))
    dX = np.empty(X.shape, dtype=np.float64 if x_real else np.complex128)
    for a, al in enumerate(alphas):
        Q = m.fgfrft_combine(P, M, al)
        D = m.dQ_dalpha(P, M, al)
        GQ = GY[a] @ X[a].T                         # slip: X^T instead of X^H
        dal[a] = float(np.real(np.sum(GQ.conj() * D)))
        g = Q.T @ GY[a]                             # slip: Q^T instead of Q^H
        dX[a] = g.real if x_real else g
    return dal, dX


def _residual_sign(theta, alpha, L):
    from oracle import fgfrft as m
    theta = np.atleast_1d(np.asarray(theta, dtype=np.float64))
    c = m.coefficients(alpha, L)
    n = np.arange(-L, L + 1)
    return np.exp(1j * alpha * theta) - np.exp(-1j * np.outer(theta, n)) @ c   # slip: e^{-j n theta}


def _exact_conj(F, alpha, decomposition=None):
    from oracle import fgfrft as m
    Z, theta, _ = decomposition if decomposition is not None else m.spectral_decomposition(F)
    return (Z * np.exp(-1j * alpha * theta)[None, :]) @ Z.conj().T   # slip: e^{-j alpha theta}


def _standard_with_split(F, alpha, L):
    from oracle import fgfrft as m
    return m.fgfrft_operator(F, alpha, L)           # slip: the -1 eigenspace still split off


def _standard_stack_from_Pc(F, alpha, L):
    from oracle import fgfrft as m
    n = F.shape[0]
    _, Pc, _ = m.split_projectors(F)
    return m.fgfrft_combine(np.zeros((n, n)), m.power_stack(F, Pc, L), alpha)   # slip: M_0 = P_c, not I


def _sampled_rows(variant):
    def f(F, P, alphas, L, rows):
        from oracle import fgfrft as m
        rows = np.asarray(rows)
        N = F.shape[0]
        Pc = np.eye(N) - P
        rr = [Pc[rows, :].astype(np.complex128)]
        cc = [Pc[:, rows].astype(np.complex128)]
        step = F.conj().T if variant == "inverse_rows" else F
        for _ in range(L):
            rr.append(rr[-1] @ step)                # slip (inverse_rows): rows of F^{-n} P_c
            cc.append(F @ cc[-1])
        out = np.empty((len(alphas), rows.size, N), dtype=np.complex128)
        for a, al in enumerate(alphas):
            c = m.coefficients(al, L)
            acc = np.exp(1j * np.pi * al) * P[rows, :] + c[L] * rr[0]
            for n in range(1, L + 1):
                neg = cc[n].T if variant == "no_conj" else cc[n].conj().T   # slip (no_conj): plain transpose
                acc = acc + c[L + n] * rr[n] + c[L - n] * neg
            out[a] = acc
        return out
    return f


def _symmetric_route_plus1(F, cos_tol=1e-10):
    F = np.asarray(F, dtype=np.float64)
    w, V = np.linalg.eigh(0.5 * (F + F.T))
    m1 = w >= 1.0 - cos_tol                         # slip: the +1 eigenspace instead of -1
    W = V[:, m1]
    P = W @ W.T
    nxt = float(w[~m1].min()) if (~m1).any() else float("nan")
    return P, np.eye(F.shape[0]) - P, int(m1.sum()), nxt


def _metrics_nmse_per_entry(E):
    N = E.shape[0]
    f2 = float(np.sum(np.abs(E) ** 2))
    return dict(MSE=f2 / N ** 2, MAE=float(np.sum(np.abs(E))) / N ** 2, NMSE=f2 / N ** 2)   # slip: NMSE over N^2


def _pointwise_bound_no_pi(theta, alpha, L):
    theta = np.asarray(theta, dtype=np.float64)
    return (np.abs(np.sin(np.pi * alpha)) / np.cos(theta / 2.0)        # slip: the 1/pi dropped
            * (1.0 / (L + 1 - alpha) + 1.0 / (L + 1 + alpha)))


def _frobenius_tight_prefactor(theta, in_minus1, alpha, L):
    th = np.asarray(theta)[~np.asarray(in_minus1)]
    pre = 2 * (L + 1) * abs(np.sin(np.pi * alpha)) / (np.pi * ((L + 1) ** 2 + alpha ** 2))   # slip: + alpha^2
    return float(pre * np.sqrt(np.sum(1.0 / np.cos(th / 2.0) ** 2)))


def _worst_case_nmse_no_N(theta, in_minus1, alpha, L):
    in_minus1 = np.asarray(in_minus1)
    th = np.asarray(theta)[~in_minus1]
    if th.size == 0:
        return 0.0
    ccmin = float(np.min(np.abs(np.cos(th / 2.0))))
    return float(4 * (L + 1) ** 2 * np.sin(np.pi * alpha) ** 2
                 / (np.pi ** 2 * ((L + 1) ** 2 - alpha ** 2) ** 2) * th.size / ccmin ** 2)   # slip: not over N


def _frobenius_tight_keeps_minus1(theta, in_minus1, alpha, L):
    th = np.asarray(theta)                          # slip: the -1 phases left in the sum
    pre = 2 * (L + 1) * abs(np.sin(np.pi * alpha)) / (np.pi * ((L + 1) ** 2 - alpha ** 2))
    return float(pre * np.sqrt(np.sum(1.0 / np.cos(th / 2.0) ** 2)))


def _frobenius_simplified_full_N(theta, in_minus1, alpha, L):
    in_minus1 = np.asarray(in_minus1)
    th = np.asarray(theta)[~in_minus1]
    ccmin = float(np.min(np.abs(np.cos(th / 2.0))))
    pre = 2 * (L + 1) * np.sqrt(in_minus1.size) * abs(np.sin(np.pi * alpha))   # slip: sqrt(N), not sqrt(N - r)
    return float(pre / (np.pi * ccmin * ((L + 1) ** 2 - alpha ** 2)))


def _worst_case_nmse_full_N(theta, in_minus1, alpha, L):
    in_minus1 = np.asarray(in_minus1)
    N = in_minus1.size
    th = np.asarray(theta)[~in_minus1]
    if th.size == 0:
        return 0.0
    ccmin = float(np.min(np.abs(np.cos(th / 2.0))))
    return float(4 * (L + 1) ** 2 * np.sin(np.pi * alpha) ** 2
                 / (np.pi ** 2 * ((L + 1) ** 2 - alpha ** 2) ** 2) * N / (N * ccmin ** 2))   # slip: N for N - r


def _term_matrix(variant):
    def f(M):
        L = len(M) - 1
        N = M[0].shape[0]
        T = np.empty((2 * L + 1, N * N), dtype=M[0].dtype)
        T[0] = M[0].reshape(-1)
        for n in range(1, L + 1):
            T[n] = M[n].reshape(-1)
            T[L + n] = (M[n].T if variant == "transpose_only" else M[n]).reshape(-1)   # slip: no conjugate / no adjoint
        return T
    return f


def _combine_many_coefficients_unreversed(P, T, alphas):
    from oracle import fgfrft as m
    alphas = np.atleast_1d(np.asarray(alphas, dtype=np.float64))
    K = T.shape[0]
    L = (K - 1) // 2
    N = P.shape[0]
    C = np.empty((alphas.size, K))
    for a, al in enumerate(alphas):
        c = m.coefficients(al, L)
        C[a, 0] = c[L]
        C[a, 1:L + 1] = c[L + 1:]
        C[a, L + 1:] = c[:L]                        # slip: c_{-L}..c_{-1} against M_1^H..M_L^H
    S = (C @ T).reshape(alphas.size, N, N)
    return np.stack([S[a] + np.exp(1j * np.pi * al) * P for a, al in enumerate(alphas)])


def _sampled_term_rows(variant):
    def f(F, P, L, rows):
        rows = np.asarray(rows)
        N = F.shape[0]
        Pc = np.eye(N) - P
        r = Pc[rows, :].astype(np.result_type(F, Pc))
        c = Pc[:, rows].astype(np.result_type(F, Pc))
        step = F.conj().T if variant == "inverse_rows" else F
        T = np.empty((2 * L + 1, rows.size * N), dtype=r.dtype)
        T[0] = r.reshape(-1)
        for n in range(1, L + 1):
            r = r @ step                                # slip (inverse_rows): rows of F^{-n} P_c
            c = F @ c
            T[n] = r.reshape(-1)
            T[L + n] = (c.T if variant == "no_conj" else c.conj().T).reshape(-1)   # slip (no_conj)
        return T
    return f


def _exact_grad_no_theta(F, alpha, decomposition=None):
    from oracle import fgfrft as m
    Z, theta, _ = decomposition if decomposition is not None else m.spectral_decomposition(F)
    return (Z * (1j * np.exp(1j * alpha * theta))[None, :]) @ Z.conj().T   # slip: the factor theta dropped


def _dQ_eigen_P_sign(F, alpha, L, tau=1e-6, decomposition=None):
    from oracle import fgfrft as m
    Z, theta, m1 = decomposition if decomposition is not None else m.spectral_decomposition(F, tau)
    d = m.coefficient_derivatives(alpha, L)
    n = np.arange(-L, L + 1)
    g = np.exp(1j * np.outer(theta, n)) @ d
    g[m1] = -1j * np.pi * np.exp(1j * np.pi * alpha)   # slip: sign of the -1 eigenspace term
    return (Z * g[None, :]) @ Z.conj().T


def _operator_eigen_conj_phase(F, alpha, L, tau=1e-6, decomposition=None):
    from oracle import fgfrft as m
    Z, theta, m1 = decomposition if decomposition is not None else m.spectral_decomposition(F, tau)
    c = m.coefficients(alpha, L)
    n = np.arange(-L, L + 1)
    q = np.exp(-1j * np.outer(theta, n)) @ c           # slip: e^{-j n theta}
    q[m1] = np.exp(1j * np.pi * alpha)
    return (Z * q[None, :]) @ Z.conj().T


def _parseval_tail_short(alpha, L):
    from oracle import fgfrft as m
    c = m.coefficients(alpha, L)[1:-1]                 # slip: the n = +-L terms left in the tail
    return float(1.0 - np.sum(c * c))


def _parseval_prediction_full_N(alpha, L, N, r_minus1=0):
    from oracle import fgfrft as m
    return m.parseval_tail(alpha, L)                   # slip: the (N - r_{-1}) / N factor dropped


def _block_errors_c_whole(Q, Fa, P):
    E = Q - Fa
    return dict(E_total=float(np.linalg.norm(E)), E_m1=float(np.linalg.norm(P @ E @ P)),
                E_c=float(np.linalg.norm(E)))          # slip: P_c dropped from the complementary block


def _apply_transpose(Q, X):
    return Q.T @ X                                     # slip: Q^T x


def _unitarity_no_conj(F):
    n = F.shape[0]
    return float(np.max(np.abs(F.T @ F - np.eye(n))))  # slip: F^T F


def _derivatives_taylor_sign(alpha, L):
    n = np.arange(-L, L + 1, dtype=np.float64)
    x = alpha - n
    out = np.empty_like(x)
    small = np.abs(x) < 1e-4
    xs = x[small]
    out[small] = (np.pi ** 2) * xs / 3.0               # slip: sign of the series near integers
    xb = x[~small]
    out[~small] = (np.cos(np.pi * xb) - np.sin(np.pi * xb) / (np.pi * xb)) / xb
    return out


def _residual_short_sum(theta, alpha, L):
    from oracle import fgfrft as m
    theta = np.atleast_1d(np.asarray(theta, dtype=np.float64))
    c = m.coefficients(alpha, L)[:-1]                  # slip: the sum stops at n = L - 1
    n = np.arange(-L, L)
    return np.exp(1j * alpha * theta) - np.exp(1j * np.outer(theta, n)) @ c


def _frobenius_exact_keeps_minus1(theta, in_minus1, alpha, L):
    from oracle import fgfrft as m
    th = np.asarray(theta)                             # slip: I_{-1} left in the sum
    return float(np.sqrt(np.sum(np.abs(m.truncation_residual(th, alpha, L)) ** 2)))


def _operator_integer_no_adjoint(F, alpha, L, tau=1e-6, decomposition=None, stack=None):
    from oracle import fgfrft as m
    F = np.asarray(F)
    if float(alpha).is_integer():
        Fm = np.linalg.matrix_power(F.astype(np.complex128), abs(int(alpha)))
        return Fm                                      # slip: F^{-m} returned as F^m
    return _ORIG["fgfrft_operator"](F, alpha, L, tau, decomposition, stack)


def _grad_variant(variant):
    def f(P, M, alphas, X, GY, x_real=None):
        from oracle import fgfrft as m
        X = np.asarray(X)
        if x_real is None:
            x_real = np.isrealobj(X)
        dal = np.empty(len(alphas))
        dX = np.empty(X.shape, dtype=np.float64 if x_real else np.complex128)
        for a, al in enumerate(alphas):
            Q = m.fgfrft_combine(P, M, al)
            D = m.dQ_dalpha(P, M, al)
            GQ = GY[a] @ X[a].conj().T
            if variant == "inner_no_conj":
                dal[a] = float(np.real(np.sum(GQ * D)))          # slip: <A, B> without conj(A)
            else:
                dal[a] = float(np.real(np.sum(GQ.conj() * D)))
            g = Q @ GY[a] if variant == "dX_with_Q" else Q.conj().T @ GY[a]   # slip (dX_with_Q): Q, not Q^H
            dX[a] = g.real if x_real else g
        return dal, dX
    return f


def _pointwise_bound_no_abs(theta, alpha, L):
    theta = np.asarray(theta, dtype=np.float64)
    return (np.sin(np.pi * alpha) / (np.pi * np.cos(theta / 2.0))      # slip: |sin(pi alpha)| lost
            * (1.0 / (L + 1 - alpha) + 1.0 / (L + 1 + alpha)))


def _frobenius_simplified_ccmax(theta, in_minus1, alpha, L):
    th = np.asarray(theta)[~np.asarray(in_minus1)]
    cc = float(np.max(np.abs(np.cos(th / 2.0))))       # slip: the largest cos(theta/2), not the smallest
    pre = 2 * (L + 1) * np.sqrt(th.size) * abs(np.sin(np.pi * alpha))
    return float(pre / (np.pi * cc * ((L + 1) ** 2 - alpha ** 2)))


def _coefficients_integer_zero(alpha, L):
    n = np.arange(-L, L + 1, dtype=np.float64)
    x = alpha - n
    out = np.zeros_like(x)                              # slip: c_n(n) = 0 instead of 1
    nz = x != 0.0
    out[nz] = np.sin(np.pi * x[nz]) / (np.pi * x[nz])
    return out


def _power_stack_no_Pc(F, Pc, L):
    M = [np.array(Pc, dtype=np.result_type(F, Pc))]
    Fn = np.eye(F.shape[0], dtype=np.result_type(F, Pc))
    for _ in range(L):
        Fn = F @ Fn
        M.append(Fn)                                    # slip: M_n = F^n, P_c dropped
    return M


def _spectral_theta_conj(F, tau=1e-6):
    Z, theta, m1 = _ORIG["spectral_decomposition"](F, tau)
    theta = -theta                                       # slip: phases of the conjugate eigenvalues
    theta[m1] = np.pi
    return Z, theta, m1


def _combine_many_phase_sign(P, T, alphas):
    from oracle import fgfrft as m
    alphas = np.atleast_1d(np.asarray(alphas, dtype=np.float64))
    Q = _ORIG["fgfrft_combine_many"](P, T, alphas)
    for a, al in enumerate(alphas):                     # slip: e^{-j pi alpha} P
        Q[a] += (np.exp(-1j * np.pi * al) - np.exp(1j * np.pi * al)) * P
    return Q


MUTATIONS = {
    "coefficients_index_flip": ("coefficients", _coefficients_index_flip),
    "coefficients_unnormalised": ("coefficients", _coefficients_unnormalised),
    "derivatives_sign": ("coefficient_derivatives", _derivatives_sign),
    "combine_drop_P": ("fgfrft_combine", _combine("drop_P")),
    "combine_phase_sign": ("fgfrft_combine", _combine("phase_sign")),
    "combine_c0_identity": ("fgfrft_combine", _combine("c0_identity")),
    "combine_no_adjoint": ("fgfrft_combine", _combine("no_adjoint")),
    "combine_transpose_only": ("fgfrft_combine", _combine("transpose_only")),
    "power_stack_off_by_one": ("power_stack", _power_stack_off_by_one),
    "projector_transpose": ("split_projectors", _split_projectors_transpose),
    "snap_minus_pi": ("spectral_decomposition", _spectral_snap_minus_pi),
    "dQ_drop_P": ("dQ_dalpha", _dQ_drop_P),
    "grad_no_conj": ("grad", _grad_no_conj),
    "residual_sign": ("truncation_residual", _residual_sign),
    "exact_conj": ("gfrft_exact", _exact_conj),
    "standard_with_split": ("fgfrft_operator_standard", _standard_with_split),
    "standard_stack_from_Pc": ("fgfrft_operator_standard", _standard_stack_from_Pc),
    "sampled_rows_no_conj": ("sampled_rows", _sampled_rows("no_conj")),
    "sampled_rows_inverse_rows": ("sampled_rows", _sampled_rows("inverse_rows")),
    "symmetric_route_plus1": ("projectors_symmetric_route", _symmetric_route_plus1),
    "metrics_nmse_per_entry": ("error_metrics", _metrics_nmse_per_entry),
    "pointwise_bound_no_pi": ("pointwise_bound", _pointwise_bound_no_pi),
    "frobenius_tight_prefactor": ("frobenius_bound_tight", _frobenius_tight_prefactor),
    "worst_case_nmse_no_N": ("worst_case_nmse_bound", _worst_case_nmse_no_N),
    "frobenius_tight_keeps_minus1": ("frobenius_bound_tight", _frobenius_tight_keeps_minus1),
    "frobenius_simplified_full_N": ("frobenius_bound_simplified", _frobenius_simplified_full_N),
    "worst_case_nmse_full_N": ("worst_case_nmse_bound", _worst_case_nmse_full_N),
    "term_matrix_no_adjoint": ("term_matrix", _term_matrix("no_adjoint")),
    "term_matrix_transpose_only": ("term_matrix", _term_matrix("transpose_only")),
    "combine_many_coefficients_unreversed": ("fgfrft_combine_many", _combine_many_coefficients_unreversed),
    "sampled_term_rows_no_conj": ("sampled_term_rows", _sampled_term_rows("no_conj")),
    "sampled_term_rows_inverse_rows": ("sampled_term_rows", _sampled_term_rows("inverse_rows")),
    "exact_grad_no_theta": ("gfrft_exact_grad", _exact_grad_no_theta),
    "dQ_eigen_P_sign": ("dQ_dalpha_eigen", _dQ_eigen_P_sign),
    "operator_eigen_conj_phase": ("fgfrft_operator_eigen", _operator_eigen_conj_phase),
    "parseval_tail_short": ("parseval_tail", _parseval_tail_short),
    "parseval_prediction_full_N": ("parseval_nmse_prediction", _parseval_prediction_full_N),
    "block_errors_c_whole": ("block_errors", _block_errors_c_whole),
    "apply_transpose": ("apply", _apply_transpose),
    "unitarity_no_conj": ("unitarity_defect", _unitarity_no_conj),
    "derivatives_taylor_sign": ("coefficient_derivatives", _derivatives_taylor_sign),
    "residual_short_sum": ("truncation_residual", _residual_short_sum),
    "frobenius_exact_keeps_minus1": ("frobenius_error_exact", _frobenius_exact_keeps_minus1),
    "operator_integer_no_adjoint": ("fgfrft_operator", _operator_integer_no_adjoint),
    "grad_inner_no_conj": ("grad", _grad_variant("inner_no_conj")),
    "grad_dX_with_Q": ("grad", _grad_variant("dX_with_Q")),
    "pointwise_bound_no_abs": ("pointwise_bound", _pointwise_bound_no_abs),
    "frobenius_simplified_ccmax": ("frobenius_bound_simplified", _frobenius_simplified_ccmax),
    "coefficients_integer_zero": ("coefficients", _coefficients_integer_zero),
    "power_stack_no_Pc": ("power_stack", _power_stack_no_Pc),
    "spectral_theta_conj": ("spectral_decomposition", _spectral_theta_conj),
    "combine_many_phase_sign": ("fgfrft_combine_many", _combine_many_phase_sign),
}

_ORIG: dict = {}


def apply(name: str) -> None:
    import oracle
    from oracle import fgfrft as m
    target, fn = MUTATIONS[name]
    _ORIG[target] = getattr(m, target)
    setattr(m, target, fn)
    setattr(oracle, target, fn)
