"""Pins of the CPU oracle against values fixed by the paper or by mathematics.

None of these re-types the oracle's own formula: each compares it with a
quadrature, a closed form, a printed table value, an exact identity from
the paper, or brute force.  A dropped term, a wrong sign, a transposed
operand or a mis-indexed coefficient in the oracle fails at least one.
"""
import json
import os

import numpy as np
import pytest
from scipy import integrate

import oracle as O
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _quad_coeff(alpha, n):
    """c_n(alpha) = (1/2pi) int_{-pi}^{pi} e^{j(alpha-n)theta} dtheta by quadrature (Sec. III-A)."""
    re = integrate.quad(lambda t: np.cos((alpha - n) * t), -np.pi, np.pi, limit=200)[0]
    im = integrate.quad(lambda t: np.sin((alpha - n) * t), -np.pi, np.pi, limit=200)[0]
    return complex(re, im) / (2 * np.pi)


def _random_unitary(n, seed):
    return synth.haar_unitary(n, np.random.default_rng(seed))


def _real_orthogonal_with_minus1(n, r, seed, margin=0.3):
    """Real orthogonal matrix: r eigenvalues at -1, conjugate pairs elsewhere kept
    at least ``margin`` away from +-pi."""
    rng = np.random.default_rng(seed)
    rest = n - r
    pairs = rest // 2
    ph = rng.uniform(0.05, np.pi - margin, size=pairs)
    blocks = synth.rotation_blocks(ph)
    d = np.zeros((n, n))
    d[: 2 * pairs, : 2 * pairs] = blocks
    k = 2 * pairs
    if rest % 2:
        d[k, k] = 1.0
        k += 1
    for i in range(k, n):
        d[i, i] = -1.0
    g = rng.standard_normal((n, n))
    v, rr = np.linalg.qr(g)
    v = v * np.sign(np.diag(rr))[None, :]
    return v @ d @ v.T


# ----------------------------------------------------------------------------
# coefficients (Sec. III-A) and their derivatives (Prop. 4)
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("alpha", [0.55, -1.37, 0.0, 1.0, -2.0, 0.5, 1e-7, 2.9999])
def test_coefficients_match_quadrature(alpha):
    L = 12
    c = O.coefficients(alpha, L)
    for k, n in enumerate(range(-L, L + 1)):
        q = _quad_coeff(alpha, n)
        assert abs(q.imag) < 1e-12
        assert abs(c[k] - q.real) < 1e-12, (alpha, n, c[k], q)


def test_integer_order_coefficients_are_kronecker():
    """Remark (integer order): c_n(m) = delta_{n,m}."""
    for m in range(-3, 4):
        c = O.coefficients(float(m), 5)
        e = np.zeros(11)
        e[5 + m] = 1.0
        assert np.max(np.abs(c - e)) < 1e-15


@pytest.mark.parametrize("alpha", [0.55, -1.37, 0.3, 1.0, 2e-5, -0.99995])
def test_coefficient_derivatives_match_quadrature_fd(alpha):
    L = 6
    d = O.coefficient_derivatives(alpha, L)
    h = 1e-5
    for k, n in enumerate(range(-L, L + 1)):
        fd = (_quad_coeff(alpha + h, n).real - _quad_coeff(alpha - h, n).real) / (2 * h)
        assert abs(d[k] - fd) < 1e-8, (alpha, n, d[k], fd)


# ----------------------------------------------------------------------------
# exact GFRFT (O1) against closed forms
# ----------------------------------------------------------------------------
def test_rotation_closed_form():
    """R(phi)^alpha = R(alpha phi) for |phi| < pi (principal branch)."""
    phis = [0.3, -1.1, 2.9, -3.0, 1.7]
    F = synth.rotation_blocks(phis)
    for alpha in (0.37, -1.6, 1.9):
        Fa = O.gfrft_exact(F, alpha)
        assert np.max(np.abs(Fa.imag)) < 1e-12
        ref = synth.rotation_blocks([alpha * p for p in phis])
        assert np.max(np.abs(Fa.real - ref)) < 1e-12


def _dft_projectors(F):
    """Spectral projectors of the unitary DFT from F^4 = I (no eigensolver):
    P_m = 1/4 sum_{k=0}^{3} (conj(lambda_m) F)^k for lambda in {1, -j, -1, j}."""
    n = F.shape[0]
    lams = [1.0, -1j, -1.0, 1j]
    thetas = [0.0, -np.pi / 2, np.pi, np.pi / 2]
    F2 = F @ F
    F3 = F2 @ F
    Ps = []
    for lam in lams:
        b = np.conj(lam)
        Ps.append((np.eye(n) + b * F + b ** 2 * F2 + b ** 3 * F3) / 4.0)
    return Ps, thetas


def test_dft_multiplicities_and_exact_gfrft():
    N = 256
    F = synth.dft_matrix(N)
    Ps, thetas = _dft_projectors(F)
    mult = [round(np.trace(P).real) for P in Ps]
    assert mult == [65, 64, 64, 63]
    dec = O.spectral_decomposition(F)
    assert int(dec[2].sum()) == 64
    for alpha in (0.55, -1.3):
        closed = sum(np.exp(1j * alpha * t) * P for P, t in zip(Ps, thetas))
        assert _rel(O.gfrft_exact(F, alpha, dec), closed) < 1e-12


@pytest.mark.parametrize("L", [3, 10, 32])
def test_dft_fgfrft_closed_form(L):
    """Q = sum_m q_m P_m with q = e^{j pi alpha} on the -1 block, sum_n c_n e^{j n theta_m} else."""
    N = 64
    F = synth.dft_matrix(N)
    Ps, thetas = _dft_projectors(F)
    plan = O.Plan(F, L)
    assert plan.r_minus1 == N // 4
    for alpha in (0.55, -1.3, 1.99):
        qs = []
        for t in thetas:
            if t == np.pi:
                qs.append(np.exp(1j * np.pi * alpha))
            else:
                qs.append(sum(_quad_coeff(alpha, n).real * np.exp(1j * n * t) for n in range(-L, L + 1)))
        closed = sum(q * P for q, P in zip(qs, Ps))
        assert _rel(plan.combine(alpha), closed) < 1e-12
        assert _rel(O.fgfrft_operator_eigen(F, alpha, L), closed) < 1e-12


def test_minus_identity_is_exact_for_every_L():
    """r_{-1} = N (F = -I): Q = e^{j pi alpha} I for every L (Sec. III-D)."""
    F = -np.eye(6)
    for L in (0, 1, 5):
        for alpha in (0.3, -1.7):
            Q = O.fgfrft_operator(F, alpha, L)
            assert np.max(np.abs(Q - np.exp(1j * np.pi * alpha) * np.eye(6))) < 1e-14


# ----------------------------------------------------------------------------
# FGFRFT (O2) structure
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("maker", ["haar", "orth"])
def test_integer_orders_equal_matrix_powers(maker):
    F = _random_unitary(12, 3) if maker == "haar" else _real_orthogonal_with_minus1(12, 3, 4)
    plan = O.Plan(F, 6)
    for m in range(-3, 4):
        ref = np.linalg.matrix_power(F, abs(m)).astype(complex)
        ref = ref if m >= 0 else ref.conj().T
        assert np.max(np.abs(plan.combine(float(m)) - ref)) < 1e-13, m
        # the operator's integer short cut gives the same matrix as the online combination
        assert np.max(np.abs(O.fgfrft_operator(F, float(m), 6) - plan.combine(float(m)))) < 1e-13, m
    # and order -1 inverts F (a library inverse, no adjoint involved)
    assert np.max(np.abs(O.fgfrft_operator(F, -1.0, 6) - np.linalg.inv(F))) < 1e-12


def test_two_routes_agree():
    """Algorithm 1 (powers) vs eigenbasis route (Prop. 1 truncated)."""
    for F in (_random_unitary(40, 1), _real_orthogonal_with_minus1(40, 5, 2), synth.dft_matrix(32)):
        plan = O.Plan(F, 9)
        for alpha in (0.55, -1.21, 1.999):
            assert _rel(plan.combine(alpha), O.fgfrft_operator_eigen(F, alpha, 9, decomposition=plan.decomposition)) < 1e-12


def test_adjoint_symmetry():
    """Proposition 3: Q^{-alpha} = (Q^alpha)^H."""
    F = _real_orthogonal_with_minus1(30, 4, 7)
    plan = O.Plan(F, 8)
    for alpha in (0.55, 1.3, -0.2):
        assert np.max(np.abs(plan.combine(-alpha) - plan.combine(alpha).conj().T)) < 1e-14


def test_rotation_fgfrft_closed_form():
    """For R(phi): Q = [[Re q, -Im q], [Im q, Re q]] with q = sum_n c_n e^{j n phi}."""
    phi = 2.2
    F = synth.rotation_blocks([phi])
    L = 7
    for alpha in (0.4, -1.3):
        q = sum(_quad_coeff(alpha, n).real * np.exp(1j * n * phi) for n in range(-L, L + 1))
        ref = np.array([[q.real, -q.imag], [q.imag, q.real]])
        Q = O.fgfrft_operator(F, alpha, L)
        assert np.max(np.abs(Q - ref)) < 1e-13


def test_real_F_gives_real_stack_and_imaginary_part_sin_P():
    """Real F: Im Q = sin(pi alpha) P (the only complex term is e^{j pi alpha} P)."""
    F = _real_orthogonal_with_minus1(20, 3, 9)
    plan = O.Plan(F, 5)
    assert plan.r_minus1 == 3
    for alpha in (0.3, -1.4):
        Q = plan.combine(alpha)
        assert np.max(np.abs(Q.imag - np.sin(np.pi * alpha) * plan.P)) < 1e-14
        # P is an orthogonal projector of rank 3 and commutes with F
        assert np.max(np.abs(plan.P @ plan.P - plan.P)) < 1e-13
        assert abs(np.trace(plan.P) - 3) < 1e-12
        assert np.max(np.abs(F @ plan.P - plan.P @ F)) < 1e-13


# ----------------------------------------------------------------------------
# error analysis (Thm 1, Thm 2, Props 5-7)
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("L", [10, 20, 32, 48, 64])
def test_pointwise_bound_theorem1(L):
    theta = np.linspace(-np.pi + 1e-3, np.pi - 1e-3, 801)
    for alpha in np.linspace(-2, 2, 17):
        if float(alpha).is_integer():
            continue
        R = np.abs(O.truncation_residual(theta, alpha, L))
        assert np.all(R <= O.pointwise_bound(theta, alpha, L) * (1 + 1e-12) + 1e-15)


def test_theorem1_bound_is_twice_the_leading_order_residual():
    """The bound's size, not only its validity.  c_n = (-1)^n sin(pi alpha) / (pi (alpha - n)), so each
    tail of R_L is a sum of (-e^{j theta})^n / (n -+ alpha) over n > L.  To leading order in 1/L that is
    a geometric tail, its first term over 1 + e^{j theta}: modulus 1 / (2 cos(theta/2) (L+1 -+ alpha)).
    Two tails in phase make half of Theorem 1's bound.  So sup_theta |R_L| / bound tends to 1/2 from
    above, with an O(1/L) excess."""
    theta = np.linspace(-np.pi + 1e-3, np.pi - 1e-3, 4001)
    for L in (10, 20, 32, 48, 64):
        for alpha in (-1.75, -0.5, 0.25, 0.55, 1.3):
            ratio = np.max(np.abs(O.truncation_residual(theta, alpha, L)) / O.pointwise_bound(theta, alpha, L))
            assert 0.5 < ratio < 0.5 + 0.3 / L, (L, alpha, ratio)


def test_theorem2_bounds_follow_from_theorem1():
    """Theorem 2's first bound is the root-sum-square of Theorem 1's pointwise bound over the
    eigenphases outside the -1 eigenspace; the worst-case NMSE bound is the simplified Frobenius
    bound squared over N (NMSE = ||E||_F^2 / N)."""
    F = _random_unitary(40, 12)
    _, theta, m1 = O.spectral_decomposition(F)
    for alpha, L in ((0.55, 10), (-1.37, 24)):
        rss = np.sqrt(np.sum(O.pointwise_bound(theta[~m1], alpha, L) ** 2))
        assert abs(O.frobenius_bound_tight(theta, m1, alpha, L) - rss) <= 1e-13 * rss
        bs = O.frobenius_bound_simplified(theta, m1, alpha, L)
        assert abs(O.worst_case_nmse_bound(theta, m1, alpha, L) - bs ** 2 / 40) <= 1e-13 * bs ** 2


def test_residual_limit_at_minus_one_is_cos():
    """Remark (obstruction): the series at theta = pi tends to cos(pi alpha), so R_L(pi) -> j sin(pi alpha)."""
    for alpha in (0.55, -1.3):
        r = O.truncation_residual(np.pi, alpha, 4000)[0]
        assert abs(r - 1j * np.sin(np.pi * alpha)) < 2e-4


def test_frobenius_identity_theorem2():
    F = _random_unitary(48, 11)
    plan = O.Plan(F, 10)
    Z, theta, m1 = plan.decomposition
    for alpha in (0.55, -1.37, 0.15):
        E = O.gfrft_exact(F, alpha, plan.decomposition) - plan.combine(alpha)
        ex = O.frobenius_error_exact(theta, m1, alpha, 10)
        assert abs(np.linalg.norm(E) - ex) < 1e-12 * max(1, ex)
        assert ex <= O.frobenius_bound_tight(theta, m1, alpha, 10) + 1e-14
        assert O.frobenius_bound_tight(theta, m1, alpha, 10) <= O.frobenius_bound_simplified(theta, m1, alpha, 10) + 1e-12
        assert np.linalg.norm(E) ** 2 / 48 <= O.worst_case_nmse_bound(theta, m1, alpha, 10) + 1e-15


def test_minus1_split_removes_block_error():
    """With the split the -1 block of F^alpha is reproduced exactly (Sec. III-B)."""
    F = _real_orthogonal_with_minus1(24, 6, 5)
    plan = O.Plan(F, 10)
    Fa = O.gfrft_exact(F, 0.55, plan.decomposition)
    be = O.block_errors(plan.combine(0.55), Fa, plan.P)
    assert be["E_m1"] < 1e-13
    assert abs(be["E_total"] - be["E_c"]) < 1e-12


def test_table6_standard_form_minus1_block():
    g = json.load(open(os.path.join(GOLD, "table6_lambda_minus1.json")))
    N, r, alpha = 120, g["r_minus1"], g["alpha"]
    rng = np.random.default_rng(123)
    phases = np.concatenate([np.full(r, np.pi), rng.uniform(-0.9 * np.pi, 0.9 * np.pi, N - r)])
    F = synth.prescribed_spectrum_unitary(phases, rng)
    plan = O.Plan(F, 20)
    assert plan.r_minus1 == r
    for row in g["rows"]:
        L = row["L"]
        Fa = O.gfrft_exact(F, alpha, plan.decomposition)
        std = O.block_errors(O.fgfrft_operator_standard(F, alpha, L), Fa, plan.P)
        prop = O.block_errors(O.fgfrft_combine(plan.P, plan.M[: L + 1], alpha), Fa, plan.P)
        assert round(std["E_m1"], g["digits"]) == pytest.approx(row["standard_E_m1"], abs=1.5 * 10 ** -g["digits"])
        assert prop["E_m1"] < 100 * row["proposed_E_m1_order"]
        assert abs(prop["E_total"] - prop["E_c"]) < 1e-12
        # Q and F^alpha are functions of F and commute with P, so the error has no cross blocks:
        # ||E||^2 = ||P E P||^2 + ||P_c E P_c||^2 (Sec. IV-F's split of the error is exhaustive)
        assert abs(std["E_total"] ** 2 - std["E_m1"] ** 2 - std["E_c"] ** 2) <= 1e-9 * std["E_total"] ** 2
        # Table VI shape: the standard form's error is dominated by its -1 block
        assert std["E_total"] > std["E_m1"] > prop["E_total"]


def test_props_5_6_7_on_random_unitaries():
    for seed in range(3):
        F = _random_unitary(24, 100 + seed)
        plan = O.Plan(F, 6)
        rng = np.random.default_rng(seed)
        for alpha, beta in ((0.55, 0.3), (-1.2, 0.7), (0.9, -0.45)):
            eps = lambda g: np.linalg.norm(O.gfrft_exact(F, g, plan.decomposition) - plan.combine(g))
            Qa = plan.combine(alpha)
            e = eps(alpha)
            assert np.linalg.norm(Qa.conj().T @ Qa - np.eye(24)) <= 2 * e + e * e + 1e-12
            x = rng.standard_normal(24) + 1j * rng.standard_normal(24)
            xh = Qa.conj().T @ (Qa @ x)
            assert np.linalg.norm(xh - x) <= (2 * e + e * e) * np.linalg.norm(x) + 1e-12
            Xi = Qa @ plan.combine(beta) - plan.combine(alpha + beta)
            assert np.linalg.norm(Xi) <= eps(alpha + beta) + e + eps(beta) + e * eps(beta) + 1e-12


# ----------------------------------------------------------------------------
# statistical pins against the printed tables (Sec. IV-A/C)
# ----------------------------------------------------------------------------
def test_parseval_tail_sum_rule():
    """sum over all n of c_n^2 is 1 (Parseval for |e^{j alpha theta}| = 1): brute-force long sum."""
    for alpha in (0.55, 0.15, -1.3):
        L = 200000
        c = O.coefficients(alpha, L)
        tail_est = 2 * np.sin(np.pi * alpha) ** 2 / (np.pi ** 2 * L)
        assert abs(np.sum(c * c) - (1 - tail_est)) < 1e-9
        assert abs(O.parseval_tail(alpha, 10) - np.sum(c * c) + np.sum(O.coefficients(alpha, 10) ** 2)) < 2e-5


def test_alpha_ratio_sec4c():
    g = json.load(open(os.path.join(GOLD, "sec4c_alpha_ratio.json")))
    ratio = O.parseval_tail(0.15, 10) / O.parseval_tail(0.55, 10)
    assert abs(ratio - g["ratio"]) < g["abs_tol"]


def test_parseval_prediction_counts_only_the_complementary_spectrum():
    """Sec. IV-A's typical-case NMSE, (N - r_-1)/N times the Parseval tail, on spectra where it is a
    quadrature: r_-1 phases at pi (reproduced exactly by the split) and the other N - r_-1 at the
    midpoints of N - r_-1 equal cells of (-pi, pi], so (1/N) sum_k |R_L(theta_k)|^2 is a midpoint
    rule for (N - r_-1)/N times the mean of |R_L|^2, which Parseval's identity makes the tail sum.
    The NMSE comes from the matrices (Algorithm 1 against the exact GFRFT)."""
    for N, r, L, alpha in ((256, 128, 10, 0.55), (200, 50, 8, -0.7)):
        M = N - r
        phases = np.concatenate([np.full(r, np.pi), -np.pi + 2 * np.pi * (np.arange(M) + 0.5) / M])
        F = synth.prescribed_spectrum_unitary(phases, np.random.default_rng(7))
        plan = O.Plan(F, L)
        assert plan.r_minus1 == r
        nmse = O.error_metrics(plan.combine(alpha) - O.gfrft_exact(F, alpha, plan.decomposition))["NMSE"]
        pred = O.parseval_nmse_prediction(alpha, L, N, r)
        assert abs(nmse / pred - 1) < 0.05, (N, r, nmse, pred)
    # every eigenvalue -1: the split reproduces F^alpha, nothing is predicted
    assert O.parseval_nmse_prediction(0.55, 10, 64, 64) == 0.0


# ----------------------------------------------------------------------------
# gradients (Prop. 4) against finite differences; the large-N helpers
# ----------------------------------------------------------------------------
def test_order_gradient_matches_finite_differences():
    F = _real_orthogonal_with_minus1(16, 2, 21)
    plan = O.Plan(F, 8)
    rng = np.random.default_rng(0)
    alphas = np.array([0.55, -1.3, 0.0, 1.0])
    X = rng.standard_normal((4, 16, 3))
    T = rng.standard_normal((4, 16, 3)) + 1j * rng.standard_normal((4, 16, 3))

    def loss(a, idx, Xa):
        Y = plan.combine(a) @ Xa
        return float(np.sum(np.abs(Y - T[idx]) ** 2))

    GY = np.stack([2 * (plan.combine(a) @ X[i] - T[i]) for i, a in enumerate(alphas)])
    dal, dX = O.grad(plan.P, plan.M, alphas, X, GY)
    h = 1e-3
    for i, a in enumerate(alphas):
        fd = (loss(a + h, i, X[i]) - loss(a - h, i, X[i])) / (2 * h)
        assert abs(dal[i] - fd) < 1e-5 * max(1.0, abs(fd)), (a, dal[i], fd)
        for (p, q) in ((0, 0), (5, 2), (15, 1)):
            Xp = X[i].copy(); Xp[p, q] += h
            Xm = X[i].copy(); Xm[p, q] -= h
            fdx = (loss(a, i, Xp) - loss(a, i, Xm)) / (2 * h)
            assert abs(dX[i][p, q] - fdx) < 1e-7 * max(1.0, abs(fdx))


def test_order_derivative_two_routes():
    # a Haar F (no -1 eigenvalue) and an F with a 6-dimensional -1 eigenspace, where the
    # j pi e^{j pi alpha} P term of Proposition 4 is present in both routes
    for F in (_random_unitary(20, 8), _real_orthogonal_with_minus1(24, 6, 5)):
        plan = O.Plan(F, 9)
        for alpha in (0.55, -1.7, 1.0):
            a = O.dQ_dalpha(plan.P, plan.M, alpha)
            b = O.dQ_dalpha_eigen(F, alpha, 9, decomposition=plan.decomposition)
            assert _rel(a, b) < 1e-12


def test_sampled_rows_match_full_operator():
    F = _real_orthogonal_with_minus1(50, 1, 31)
    plan = O.Plan(F, 7)
    rows = np.array([0, 7, 49, 23])
    al = [0.55, -1.9, 2.0]
    S = O.sampled_rows(F, plan.P, al, 7, rows)
    for a, alpha in enumerate(al):
        assert np.max(np.abs(S[a] - plan.combine(alpha)[rows])) < 1e-13
    # complex F: the negative powers' rows are conjugate transposes of columns (Proposition 2)
    Fc = synth.haar_unitary(36, np.random.default_rng(32))
    plan = O.Plan(Fc, 6)
    rows = np.array([1, 35, 17])
    S = O.sampled_rows(Fc, plan.P, al, 6, rows)
    for a, alpha in enumerate(al):
        assert np.max(np.abs(S[a] - plan.combine(alpha)[rows])) < 1e-12


def test_symmetric_route_projector_matches_schur_route():
    F = _real_orthogonal_with_minus1(40, 2, 41)
    P1, _, r1 = O.split_projectors(F)
    P2, _, r2, nxt = O.projectors_symmetric_route(F)
    assert r1 == r2 == 2
    assert np.max(np.abs(P1 - P2)) < 1e-9
    assert nxt > -1 + 1e-3


def test_unitarity_defect_closed_form():
    """max |F^H F - I| is 0 up to rounding for a unitary F, and (1+e)^2 - 1 for diag(1, 1+e)."""
    assert O.unitarity_defect(synth.haar_unitary(30, np.random.default_rng(3))) < 1e-13
    for e in (1e-3, -0.25):
        assert abs(O.unitarity_defect(np.diag([1.0, 1.0 + e])) - abs((1.0 + e) ** 2 - 1.0)) < 1e-15


def test_exact_gfrft_order_derivative_against_finite_differences():
    """dF^alpha/dalpha against central differences of F^alpha (h = 1e-5, error O(h^2))."""
    F = synth.haar_unitary(20, np.random.default_rng(8))
    dec = O.spectral_decomposition(F)
    h = 1e-5
    for alpha in (0.3, -1.45):
        fd = (O.gfrft_exact(F, alpha + h, dec) - O.gfrft_exact(F, alpha - h, dec)) / (2 * h)
        assert _rel(O.gfrft_exact_grad(F, alpha, dec), fd) < 1e-8


def test_apply_at_integer_order_is_the_graph_fourier_transform():
    """Definition 2 at alpha = 1 (the operator is F exactly) and alpha = 0 (the identity)."""
    F = _real_orthogonal_with_minus1(24, 3, 5)
    plan = O.Plan(F, 6)
    X = np.random.default_rng(9).standard_normal((24, 4))
    assert np.max(np.abs(O.apply(plan.combine(1.0), X) - F @ X)) < 1e-13
    assert np.max(np.abs(O.apply(plan.combine(0.0), X) - X)) < 1e-13


def test_degenerate_sizes():
    for f in (np.array([[1.0]]), np.array([[-1.0]]), np.array([[0.0, 1.0], [1.0, 0.0]])):
        plan = O.Plan(f, 3)
        for alpha in (0.5, -1.25):
            Q = plan.combine(alpha)
            E = O.gfrft_exact(f, alpha, plan.decomposition) - Q
            _, theta, m1 = plan.decomposition
            assert abs(np.linalg.norm(E) - O.frobenius_error_exact(theta, m1, alpha, 3)) < 1e-13


def test_table4_accuracy_columns_on_a_haar_draw():
    """Table IV's accuracy columns (L = 10, alpha = 0.5) against a Haar draw at N = 1000.

    The eigenphases of a Haar matrix are CUE-distributed: uniform one-point density and rigid,
    so NMSE = (1/N) sum_k |R_L(theta_k)|^2 sits close to its expectation for every draw, and the
    printed column is flat in N.  MSE = NMSE / N and MAE ~ sqrt(NMSE / N) (MAE sqrt(N) is flat
    in the table too).  The test compares the draw with the column means (NMSE and MAE sqrt(N))."""
    g = json.load(open(os.path.join(GOLD, "table4_online.json")))
    L, alpha, N = g["L"], g["alpha"], 1000
    nmse_printed = np.mean([r["NMSE"] for r in g["rows"]])
    mae_printed = np.mean([r["MAE"] * np.sqrt(r["N"]) for r in g["rows"]])
    for r in g["rows"]:   # the table's own MSE column is NMSE / N
        assert abs(r["MSE"] * r["N"] - r["NMSE"]) <= 0.01 * r["NMSE"]
    F = synth.haar_unitary(N, np.random.default_rng(4))
    dec = O.spectral_decomposition(F)
    E = O.fgfrft_operator_eigen(F, alpha, L, decomposition=dec) - O.gfrft_exact(F, alpha, dec)
    m = O.error_metrics(E)
    assert abs(m["MSE"] * N - m["NMSE"]) <= 1e-12
    # the printed column sits ~3% above the uniform-phase expectation (one random matrix per size)
    assert abs(m["NMSE"] - nmse_printed) <= g["rel_tol"] * nmse_printed, (m["NMSE"], nmse_printed)
    assert abs(m["MAE"] * np.sqrt(N) - mae_printed) <= g["rel_tol"] * mae_printed, (m["MAE"], mae_printed)
    # and the expectation sum_{|n| > L} c_n^2 itself (L - 1 or L + 1 would be ~10% off)
    assert abs(m["NMSE"] - O.parseval_tail(alpha, L)) <= 0.03 * O.parseval_tail(alpha, L)


# ----------------------------------------------------------------------------
# the batched online combination (Algorithm 1 for many orders as one product)
# ----------------------------------------------------------------------------
def test_batched_combination_dft_closed_form():
    """C T over the term matrix, plus e^{j pi alpha} P, equals the DFT's closed form
    Q = sum_m q_m P_m (projectors from F^4 = I, coefficients by quadrature) for every order."""
    N, L = 64, 10
    F = synth.dft_matrix(N)
    Ps, thetas = _dft_projectors(F)
    plan = O.Plan(F, L)
    alphas = [0.55, -1.3, 1.99, 0.0, 1.0]
    Qs = O.fgfrft_combine_many(plan.P, O.term_matrix(plan.M), alphas)
    for a, alpha in enumerate(alphas):
        qs = []
        for t in thetas:
            if t == np.pi:
                qs.append(np.exp(1j * np.pi * alpha))
            else:
                qs.append(sum(_quad_coeff(alpha, n).real * np.exp(1j * n * t) for n in range(-L, L + 1)))
        closed = sum(q * P for q, P in zip(qs, Ps))
        assert _rel(Qs[a], closed) < 1e-12, alpha


def test_batched_sampled_rows_dft_closed_form():
    """Rows R of Q for many orders from the row-sampled terms (one product C T_R plus e^{j pi alpha} P[R, :])
    equal the rows of the DFT's closed form sum_m q_m P_m (complex F, 16 eigenvalues at -1)."""
    N, L = 64, 10
    F = synth.dft_matrix(N)
    Ps, thetas = _dft_projectors(F)
    plan = O.Plan(F, L)
    rows = np.array([0, 5, 63, 31])
    alphas = [0.55, -1.3, 1.99, 0.0]
    Qr = O.fgfrft_combine_many(plan.P[rows, :], O.sampled_term_rows(F, plan.P, L, rows), alphas)
    assert Qr.shape == (len(alphas), rows.size, N)
    for a, alpha in enumerate(alphas):
        qs = []
        for t in thetas:
            if t == np.pi:
                qs.append(np.exp(1j * np.pi * alpha))
            else:
                qs.append(sum(_quad_coeff(alpha, n).real * np.exp(1j * n * t) for n in range(-L, L + 1)))
        closed = sum(q * P for q, P in zip(qs, Ps))
        assert _rel(Qr[a], closed[rows]) < 1e-12, alpha


def test_batched_sampled_rows_integer_orders_are_power_rows():
    """Real orthogonal F with two eigenvalues at -1: integer orders give the rows of F^m, negative
    ones the rows of (F^|m|)^T."""
    F = _real_orthogonal_with_minus1(30, 2, 23)
    plan = O.Plan(F, 5)
    rows = np.array([29, 0, 11])
    ms = [-4, -1, 0, 3]
    Qr = O.fgfrft_combine_many(plan.P[rows, :], O.sampled_term_rows(F, plan.P, 5, rows), [float(m) for m in ms])
    for a, m in enumerate(ms):
        ref = np.linalg.matrix_power(F, abs(m))
        ref = ref if m >= 0 else ref.T
        assert np.max(np.abs(Qr[a] - ref[rows])) < 1e-13, m


def test_batched_combination_integer_orders_are_powers():
    """Real orthogonal F with three eigenvalues at -1: integer orders give F^m, negative ones (F^|m|)^T."""
    F = _real_orthogonal_with_minus1(14, 3, 21)
    plan = O.Plan(F, 6)
    assert plan.r_minus1 == 3
    ms = [-3, -1, 0, 2, 5]
    Qs = O.fgfrft_combine_many(plan.P, O.term_matrix(plan.M), [float(m) for m in ms])
    for a, m in enumerate(ms):
        ref = np.linalg.matrix_power(F, abs(m))
        ref = ref if m >= 0 else ref.T
        assert np.max(np.abs(Qs[a] - ref)) < 1e-13, m


# ----------------------------------------------------------------------------
# Theorem 2 and the worst-case NMSE bound with a nonempty -1 eigenspace
# ----------------------------------------------------------------------------
def _dft_phase_multiset(N):
    """Eigenphases of the unitary DFT, N divisible by 4, from the multiplicities N/4+1, N/4, N/4, N/4-1
    of the eigenvalues 1, -j, -1, j (traces of the projectors built from F^4 = I, checked below)."""
    q = N // 4
    return {0.0: q + 1, -np.pi / 2: q, np.pi: q, np.pi / 2: q - 1}


def test_theorem2_bounds_with_minus1_eigenspace_on_dft():
    """DFT, N = 64 (r_{-1} = 16).  Theorem 2's first bound is the root-sum-square of Theorem 1 over the
    48 phases outside I_{-1} (17 at 0, 16 at -pi/2, 15 at pi/2); the simplified bound is sqrt(N - r_{-1})
    times Theorem 1 at the worst remaining phase (cos_{c,min} = cos(pi/4)); the worst-case NMSE bound
    is that squared over N.  The -1 phases must be left out: at theta = pi Theorem 1 is infinite."""
    N = 64
    F = synth.dft_matrix(N)
    Ps, thetas = _dft_projectors(F)
    mult = _dft_phase_multiset(N)
    assert [round(np.trace(P).real) for P in Ps] == [mult[t] for t in thetas]
    _, theta, m1 = O.spectral_decomposition(F)
    assert int(m1.sum()) == mult[np.pi] == 16
    for alpha, L in ((0.55, 10), (-1.37, 24), (1.9, 32)):
        b = {t: float(O.pointwise_bound(np.array([t]), alpha, L)[0]) for t in mult if t != np.pi}
        rss = np.sqrt(sum(mult[t] * b[t] ** 2 for t in b))
        tight = O.frobenius_bound_tight(theta, m1, alpha, L)
        assert abs(tight - rss) <= 1e-12 * rss, (alpha, L, tight, rss)
        simp = O.frobenius_bound_simplified(theta, m1, alpha, L)
        want = np.sqrt(N - 16) * b[np.pi / 2]
        assert abs(simp - want) <= 1e-12 * want, (alpha, L, simp, want)
        wc = O.worst_case_nmse_bound(theta, m1, alpha, L)
        assert abs(wc - want ** 2 / N) <= 1e-12 * want ** 2 / N
        # the identity side: ||F^alpha - Q||_F from the closed-form projectors
        plan = O.Plan(F, L)
        Fa = sum(np.exp(1j * alpha * t) * P for P, t in zip(Ps, thetas))
        Qc = plan.combine(alpha)
        ex = O.frobenius_error_exact(theta, m1, alpha, L)
        assert abs(np.linalg.norm(Fa - Qc) - ex) <= 1e-10 * max(ex, 1e-12)
        assert ex <= tight <= simp
        assert np.linalg.norm(Fa - Qc) ** 2 / N <= wc


def test_bounds_vanish_when_every_eigenvalue_is_minus_one():
    """F = -I: I_{-1} is everything, the split reproduces F^alpha exactly and each bound is 0."""
    F = -np.eye(8)
    _, theta, m1 = O.spectral_decomposition(F)
    assert m1.all()
    for alpha, L in ((0.55, 10), (-1.3, 4)):
        assert O.worst_case_nmse_bound(theta, m1, alpha, L) == 0.0
        assert O.frobenius_bound_tight(theta, m1, alpha, L) == 0.0
        assert O.frobenius_error_exact(theta, m1, alpha, L) == 0.0


def test_order_gradient_at_minus_alpha_is_the_adjoint_term():
    """Proposition 3 differentiated: Q(-a) = Q(a)^H for all a gives dQ/da(-a) = -(dQ/da(a))^H, so the
    order gradient of Y = Q(-a) M for the upstream G equals minus that of Y = Q(a) G for the upstream
    M (the identity that lets a filter Q^{-a} diag(h) Q^{a} take one order gradient over both signal
    blocks).  Checked on the oracle's operators for a Haar unitary F and one with a -1 eigenspace."""
    rng = np.random.default_rng(17)
    N, L, B = 24, 7, 4
    for F in (synth.haar_unitary(N, rng), synth.dft_matrix(N)):
        plan = O.Plan(F, L)
        alphas = np.array([0.37, -1.21, 1.9])
        Mx = rng.standard_normal((3, N, B)) + 1j * rng.standard_normal((3, N, B))
        G = rng.standard_normal((3, N, B)) + 1j * rng.standard_normal((3, N, B))
        g_minus, _ = O.grad(plan.P, plan.M, -alphas, Mx, G, x_real=False)
        g_plus, _ = O.grad(plan.P, plan.M, alphas, G, Mx, x_real=False)
        assert np.max(np.abs(g_minus + g_plus)) <= 1e-10 * np.max(np.abs(g_plus))
        # and pointwise on the operators themselves
        for a in alphas:
            Dm = O.dQ_dalpha(plan.P, plan.M, -a)
            Dp = O.dQ_dalpha(plan.P, plan.M, a)
            assert np.max(np.abs(Dm + Dp.conj().T)) <= 1e-10 * np.max(np.abs(Dp))


# the slowest pin last: a mutated oracle that an earlier pin already fails stops before it
@pytest.mark.slow
def test_table3_nmse_on_haar_random():
    g = json.load(open(os.path.join(GOLD, "table3_nmse.json")))
    F = _random_unitary(g["N"], 2000)
    dec = O.spectral_decomposition(F)
    Z, theta, m1 = dec
    for row in g["rows"]:
        # NMSE through the matrix route for the first L, the Thm-2 identity for the rest
        nmse = O.frobenius_error_exact(theta, m1, g["alpha"], row["L"]) ** 2 / g["N"]
        assert abs(nmse / row["NMSE"] - 1) < g["rel_tol"], (row, nmse)
        pred = O.parseval_nmse_prediction(g["alpha"], row["L"], g["N"], int(m1.sum()))
        assert abs(pred / row["NMSE"] - 1) < g["rel_tol"]
    L = g["rows"][0]["L"]
    plan_P, plan_Pc, _ = O.split_projectors(F, decomposition=dec)
    Q = O.fgfrft_combine(plan_P, O.power_stack(F, plan_Pc, L), g["alpha"])
    nmse_m = O.error_metrics(Q - O.gfrft_exact(F, g["alpha"], dec))["NMSE"]
    assert abs(nmse_m / g["rows"][0]["NMSE"] - 1) < g["rel_tol"]
