"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed forms on
matrices with prescribed singular values, numpy's LAPACK SVD, exact rational
arithmetic, explicit matrix powers, identities the paper states, and printed values.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from workloads import gen

RNG_CASES = [(24, 40), (40, 24), (16, 16), (1, 9), (9, 1)]


def _spectral(rows, cols, seed, sigma=None):
    r = min(rows, cols)
    if sigma is None:
        sigma = 0.05 + gen.uniform_np(seed, 5, r)
    U = gen.haar_np(rows, r, seed, 1)
    V = gen.haar_np(cols, r, seed, 2)
    return (U * sigma) @ V.T, U, np.asarray(sigma), V


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("shape", RNG_CASES)
@pytest.mark.parametrize("basis", ["gram", "complement"])
@pytest.mark.parametrize("norm", ["frobenius", "gram_frobenius", "none"])
def test_closed_form_prescribed_spectrum(shape, basis, norm):
    """Y = U diag(f(sigma~)) V^T for M = U diag(sigma) V^T (the SVD argument of Sec. 1)."""
    M, U, s, V = _spectral(*shape, seed=3)
    if norm == "none":
        M, s = M * 0.9, s * 0.9  # keep sigma in (0, 1)
    exps = [0, 1, 2, 4, 8]
    c = [0.7, -1.3, 2.1, -0.4, 0.9]
    Y = O.ifnso(M, exps, c, basis, norm)
    Yc = O.closed_form(U, s, V, exps, c, basis, norm)
    assert Y.shape == M.shape
    assert _rel(Y, Yc) < 1e-12


def test_closed_form_rank_deficient():
    M, U, s, V = _spectral(20, 30, seed=4)
    s = s.copy()
    s[5:] = 0.0
    M = (U * s) @ V.T
    for basis in ("gram", "complement"):
        Y = O.ifnso(M, [0, 1, 4], [1.5, -0.7, 0.3], basis, "frobenius")
        assert _rel(Y, O.closed_form(U, s, V, [0, 1, 4], [1.5, -0.7, 0.3], basis, "frobenius")) < 1e-12


def test_svd_polar_gaussian():
    """Gaussian input: the oracle equals U f(s~) V^T built from numpy's SVD."""
    M = gen.gaussian_np(32, 48, seed=0)
    U, s, Vt = np.linalg.svd(M, full_matrices=False)
    exps, c = [0, 1, 2, 4, 8, 16], O.gform_ls_fit([0, 1, 2, 4, 8, 16])
    Y = O.ifnso(M, exps, c)
    assert _rel(Y, O.closed_form(U, s, Vt.T, exps, c)) < 1e-12
    # polar factor distance identity: ||Y - U V^T||^2 = sum (f - 1)^2
    st = s / np.linalg.norm(s)
    f = O.singular_value_map(st, exps, c)
    d2 = np.linalg.norm(Y - U @ Vt) ** 2
    assert abs(d2 - np.sum((f - 1) ** 2)) < 1e-10 * max(1.0, d2)
    e2 = O.orth_error(Y) ** 2
    assert abs(e2 - np.sum((f * f - 1) ** 2)) < 1e-10 * max(1.0, e2)


def test_identity_preservation_gram_sum_one():
    """Constraint 'y -> 1 as x -> 1' (Sec. 2.1): with orthonormal rows and no normalisation,
    Y = (sum c) Q, so Y = Q iff sum c = 1."""
    Q = gen.haar_np(40, 24, 9, 1).T  # 24 x 40, orthonormal rows
    c = O.gform_ls_fit([0, 1, 2, 4, 8, 16])
    assert abs(c.sum() - 1) < 1e-12
    Y = O.ifnso(Q, [0, 1, 2, 4, 8, 16], c, "gram", "none")
    assert np.max(np.abs(Y - Q)) < 1e-9
    Y2 = O.ifnso(Q, [0, 1, 2], [1.0, 0.5, 0.25], "gram", "none")
    assert np.max(np.abs(Y2 - 1.75 * Q)) < 1e-12


def test_identity_preservation_complement():
    """Complement basis: (I - QQ^T) = 0 so every term but the first vanishes."""
    Q = gen.haar_np(40, 24, 9, 1).T
    w = O.tform_ls_fit(14)
    exps, c = O.paper_coeffs_to_terms(w)
    Y = O.ifnso(Q, exps, c, "complement", "none")
    assert np.max(np.abs(Y - Q)) < 1e-9
    # also on a tall input (returned in M's orientation)
    Y = O.ifnso(Q.T, exps, c, "complement", "none")
    assert np.max(np.abs(Y - Q.T)) < 1e-9


def test_single_row_is_normalised_vector():
    x = gen.gaussian_np(1, 37, seed=2)
    c = [0.25, 0.5, 0.25]
    Y = O.ifnso(x, [0, 1, 2], c)
    assert np.max(np.abs(Y - x / np.linalg.norm(x))) < 1e-15
    Yt = O.ifnso(x.T, [0, 1, 2], c)
    assert np.max(np.abs(Yt - x.T / np.linalg.norm(x))) < 1e-15


@pytest.mark.parametrize("norm", ["frobenius", "gram_frobenius"])
def test_scaling_invariance(norm):
    M = gen.gaussian_np(20, 33, seed=5)
    for basis in ("gram", "complement"):
        Y1 = O.ifnso(M, [0, 1, 2, 4], [1.2, -0.3, 0.5, 0.1], basis, norm)
        Y2 = O.ifnso(M * 37.5, [0, 1, 2, 4], [1.2, -0.3, 0.5, 0.1], basis, norm)
        assert _rel(Y2, Y1) < 1e-13


def test_zero_input_gives_zero():
    Z = np.zeros((8, 12))
    for norm in O.NORMS:
        assert np.all(O.ifnso(Z, [0, 1], [2.0, -1.0], "gram", norm) == 0)
    assert np.all(O.classical_ns(Z, 3, (3.4445, -4.775, 2.0315)) == 0)
    assert np.all(O.paper_form(Z, [1.0, 2.0]) == 0)


def test_ns_one_step_is_gram_polynomial(golden_dir):
    abc = json.load(open(os.path.join(golden_dir, "paper_constants.json")))["muon_abc"]["value"]
    M = gen.gaussian_np(24, 50, seed=6)
    Y1 = O.classical_ns(M, 1, abc)
    Y2 = O.ifnso(M, [0, 1, 2], abc, "gram", "frobenius")
    assert _rel(Y1, Y2) < 1e-14


@pytest.mark.parametrize("abc", [(1.5, -0.5, 0.0), (3.4445, -4.7750, 2.0315)])
def test_ns_iterates_scalar_map(abc):
    """N steps act on each singular value as the N-fold scalar map (Eq. (N_fold))."""
    M, U, s, V = _spectral(18, 30, seed=8)
    st = s / np.linalg.norm(s)
    a, b, c = abc
    x = st.copy()
    for _ in range(5):
        x = a * x + b * x ** 3 + c * x ** 5
    Y = O.classical_ns(M, 5, abc)
    assert _rel(Y, (U * x) @ V.T) < 1e-12


def _frac_matmul(A, B):
    return [[sum((A[i][k] * B[k][j] for k in range(len(B))), Fraction(0)) for j in range(len(B[0]))]
            for i in range(len(A))]


def _frac_T(A):
    return [list(r) for r in zip(*A)]


@pytest.mark.parametrize("ints,rows,cols,fro", [
    ([1, 2, 3, 4, 5, 3], 2, 3, 8),
    ([5, 3, 5, 2, -3, 5, 1, -3, -3, -4, 2, 2, 3, 2, 4], 3, 5, 13),
])
def test_rational_brute_force(ints, rows, cols, fro):
    """Exact rational arithmetic on tiny matrices whose Frobenius norm is an integer."""
    A = [[Fraction(ints[i * cols + j]) for j in range(cols)] for i in range(rows)]
    X0 = [[a / fro for a in r] for r in A]
    abc = [Fraction(34445, 10000), Fraction(-4775, 1000), Fraction(20315, 10000)]
    X = X0
    for _ in range(3):
        G = _frac_matmul(X, _frac_T(X))
        GX = _frac_matmul(G, X)
        GGX = _frac_matmul(G, GX)
        X = [[abc[0] * X[i][j] + abc[1] * GX[i][j] + abc[2] * GGX[i][j] for j in range(cols)] for i in range(rows)]
    exact = np.array([[float(v) for v in r] for r in X])
    Mf = np.array(ints, dtype=np.float64).reshape(rows, cols)
    assert _rel(O.classical_ns(Mf, 3, [float(v) for v in abc]), exact) < 1e-13
    assert _rel(O.classical_ns(Mf.T, 3, [float(v) for v in abc]), exact.T) < 1e-13
    # IFNSO polynomial with exponents {0, 1, 2, 4} and rational coefficients
    cs = [Fraction(3, 2), Fraction(-1, 3), Fraction(5, 4), Fraction(-7, 5)]
    G = _frac_matmul(X0, _frac_T(X0))
    G2 = _frac_matmul(G, G)
    G4 = _frac_matmul(G2, G2)
    eye = [[Fraction(int(i == j)) for j in range(rows)] for i in range(rows)]
    P = [[cs[0] * eye[i][j] + cs[1] * G[i][j] + cs[2] * G2[i][j] + cs[3] * G4[i][j] for j in range(rows)]
         for i in range(rows)]
    Y = np.array([[float(v) for v in r] for r in _frac_matmul(P, X0)])
    assert _rel(O.ifnso(Mf, [0, 1, 2, 4], [float(c) for c in cs]), Y) < 1e-13
    # complement basis, no normalisation beyond X0: B = I - X0 X0^T
    Bc = [[eye[i][j] - G[i][j] for j in range(rows)] for i in range(rows)]
    Bc2 = _frac_matmul(Bc, Bc)
    P = [[cs[0] * eye[i][j] + cs[1] * Bc[i][j] + cs[2] * Bc2[i][j] for j in range(rows)] for i in range(rows)]
    Y = np.array([[float(v) for v in r] for r in _frac_matmul(P, X0)])
    assert _rel(O.ifnso(Mf, [0, 1, 2], [float(c) for c in cs[:3]], "complement"), Y) < 1e-13


def test_unrolled_polynomial_matches_iterations():
    """Eq. (polynomial_unify)/(old_unified_formula): N quintic steps equal one odd polynomial
    of degree 5^N in x_0, evaluated with consecutive powers of X0 X0^T."""
    a, b, c = 3.4445, -4.7750, 2.0315
    step = np.array([0, a, 0, b, 0, c])
    p = np.array([0.0, 1.0])
    for _ in range(2):
        p = _compose(step, p)
    assert len(p) - 1 == 25
    M = gen.gaussian_np(6, 9, seed=12)
    X0 = M / np.linalg.norm(M)
    G = X0 @ X0.T
    Y = np.zeros_like(X0)
    Gn = np.eye(6)
    for n in range(13):  # coefficient of x^(2n+1)
        Y += p[2 * n + 1] * (Gn @ X0)
        Gn = Gn @ G
    assert _rel(Y, O.classical_ns(M, 2, (a, b, c))) < 1e-12


def _compose(outer, inner):
    """coefficients of outer(inner(x))."""
    from numpy.polynomial import polynomial as Pn
    res = np.array([0.0])
    pw = np.array([1.0])
    for k, ck in enumerate(outer):
        if k:
            pw = Pn.polymul(pw, inner)
        res = Pn.polyadd(res, ck * pw)
    return res


def test_paper_form_spectral_equals_squaring_route():
    """The paper's form through the eigendecomposition of A A^T and through repeated squaring of
    the complement basis (two independent routes) agree; and on a prescribed spectrum both equal
    U diag(sigma~ (1 + sum_l w_l (1 - sigma~^2)^(2^(l-1)))) V^T with sigma~ = sigma / ||sigma^2||^(1/2)."""
    M = gen.gaussian_np(30, 70, seed=13)
    w = O.tform_ls_fit(10)
    exps, c = O.paper_coeffs_to_terms(w)
    Y1 = O.paper_form(M, w)
    Y2 = O.ifnso(M, exps, c, "complement", "gram_frobenius")
    assert _rel(Y1, Y2) < 1e-11
    assert _rel(O.paper_form(M.T, w), Y1.T) < 1e-14
    sigma = np.linspace(0.05, 2.0, 12)
    U = gen.haar_np(12, 12, 31, 1)
    V = gen.haar_np(40, 12, 31, 2)
    st = sigma / np.sqrt(np.sqrt(np.sum(sigma ** 4)))
    f = st * (1.0 + sum(wl * (1.0 - st ** 2) ** (2 ** l) for l, wl in enumerate(w)))
    assert _rel(O.paper_form((U * sigma) @ V.T, w), (U * f) @ V.T) < 1e-11


def test_tl_recursion_is_explicit_power():
    """T_l = T_{l-1}^2 equals (I - XX^T)^(2^(l-1)) computed by plain repeated products."""
    M = gen.gaussian_np(12, 20, seed=14)
    parts = O.ifnso_parts(M, [0, 1, 2, 4, 8, 16, 32], [1] * 7, "complement", "gram_frobenius")
    T1 = parts["B"]
    for e in (2, 4, 8, 16, 32):
        assert _rel(parts["powers"][e], np.linalg.matrix_power(T1, e)) < 1e-12
    A = M
    T0 = A @ A.T
    assert _rel(T1, np.eye(12) - T0 / np.linalg.norm(T0)) < 1e-14


# ---------------------------------------------------------------------------------------------
# scalar analysis of the term family (Sec. 2.2-2.3)
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("l", [1, 2, 3, 5, 8])
def test_term_gradient_and_extreme_point(l):
    x = np.linspace(0.01, 0.99, 57)
    h = 1e-6
    fl = lambda t: t * (1 - t * t) ** (2 ** (l - 1))
    fd = (fl(x + h) - fl(x - h)) / (2 * h)
    assert np.max(np.abs(fd - O.tform_term_grad(x, l))) < 1e-6
    xs, ys, ys_approx = O.tform_extreme_point(l)
    grid = np.linspace(0, 1, 2_000_001)
    i = np.argmax(fl(grid))
    assert abs(grid[i] - xs) < 1e-6
    assert abs(fl(xs) - ys) < 1e-14
    assert abs(O.tform_term_grad(np.array([xs]), l)[0]) < 1e-12
    assert abs(ys_approx / ys - 1) < 0.25 / 2 ** l + 1e-3  # e^(-1/2) limit


def test_peak_constraint_exact_vs_approx():
    L = 14
    w = O.tform_ls_fit(L)
    xs = 1 / math.sqrt(2 ** L + 1)
    wx = O.tform_full_w(w[:-1], L, exact=True)
    assert abs(O.tform_f(np.array([xs]), wx)[0] - 1) < 1e-12
    # the printed approximation misses the constraint (reading of Eq. (b_approximation))
    fa = O.tform_f(np.array([xs]), w)[0]
    assert 1.02 < fa < 1.2


def test_ls_fit_is_stationary_under_quadrature():
    """The Beta-integral closed form is checked by an independent quadrature: any small
    move of a free coefficient increases the expected loss."""
    L = 8
    w = O.tform_ls_fit(L)
    base = O.tform_expected_loss(w)
    for i in range(L - 1):
        for d in (1e-3, -1e-3):
            head = w[:-1].copy()
            head[i] += d
            assert O.tform_expected_loss(O.tform_full_w(head, L)) > base


def test_gform_fit_constrained_optimum():
    exps = [0, 1, 2, 4, 8, 16]
    c = O.gform_ls_fit(exps)
    assert abs(c.sum() - 1) < 1e-12
    base = O.gform_expected_loss(exps, c)
    for i in range(1, len(c)):
        for d in (1e-3, -1e-3):
            c2 = c.copy()
            c2[i] += d
            c2[0] -= d  # stay on sum = 1
            assert O.gform_expected_loss(exps, c2) > base


def test_first_reach_one_matches_paper(golden_dir):
    ref = json.load(open(os.path.join(golden_dir, "paper_constants.json")))["first_reach_one_x"]["value"]
    w = O.tform_ls_fit(14)
    x = O.first_reach_one(w)
    assert 0.5 * ref < x < 2.0 * ref  # loose: the paper's fitted w is unpublished


@pytest.mark.slow
def test_adam_replica_approaches_ls_optimum():
    L = 14
    w_ls = O.tform_ls_fit(L)
    w_adam = O.tform_adam_fit(L, iters=20000)
    la, ll = O.tform_expected_loss(w_adam), O.tform_expected_loss(w_ls)
    assert ll <= la < 5.0 * ll


def test_flop_model_reproduces_table1(golden_dir):
    rows = json.load(open(os.path.join(golden_dir, "table1.json")))["rows"]
    for r in rows:
        h, w = r["h"], r["w"]
        if r["method"] == "ifnso":
            model = O.flops_ifnso(h, w, 14)
            tol = 0.005
        elif r["method"] == "original_ns":
            model = O.flops_ns(h, w, 8, 2)
            tol = 0.007
        else:
            model = O.flops_ns(h, w, 5, 3)
            tol = 0.007
        assert abs(model / r["flops"] - 1) < tol, r


def test_orth_error_of_polar_factor_is_zero():
    Q = gen.haar_np(30, 12, 21, 1)
    assert O.orth_error(Q) < 1e-13
    assert O.orth_error(Q.T) < 1e-13
    assert abs(O.orth_error(2 * Q.T) - 3 * math.sqrt(12)) < 1e-12


def test_generator_streams():
    """The counter generator is deterministic, stream-separated and offset-consistent."""
    u = gen.uniform_np(5, 2, 1000)
    assert np.all((u >= 0) & (u < 1))
    assert np.array_equal(u[100:200], gen.uniform_np(5, 2, 100, offset=100))
    assert not np.array_equal(u, gen.uniform_np(5, 3, 1000))
    z = gen.normal_np(0, 0, 200000)
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1) < 0.01
    # SplitMix64 reference output for state 0 -> first word after one GAMMA increment
    assert int(gen.mix64_np(np.array([gen.GAMMA], dtype=np.uint64))[0]) == 0xE220A8397B1DCDAF


def test_bf16_rounding_is_nearest_even():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -8 + 2 ** -30, -1.0 - 2 ** -8, 3.14159])
    r = gen.round_to_bf16_np(x)
    assert r[0] == 1.0
    assert r[1] == 1.0  # tie -> even
    assert r[2] == 1.0 + 4 * 2 ** -8  # tie -> even (up)
    assert r[3] == 1.0 + 2 ** -7  # above tie
    assert r[4] == -1.0
    assert abs(r[5] - 3.140625) < 1e-15
