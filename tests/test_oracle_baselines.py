"""Pins of the baseline iterations' oracle (Cesista's quintics, CANS, Gelfand scaling, step
schedules) against things other than itself: numpy's polynomial-from-roots routine, a
closed-form cubic minimax derived by hand, a linear-programming minimax on a fine grid,
brute-force evaluation, closed forms on prescribed spectra and explicit matrix powers."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import baselines as BL
from workloads import configs, gen


def _spectral(rows, cols, seed, sigma):
    r = min(rows, cols)
    U = gen.haar_np(rows, r, seed, 1)
    V = gen.haar_np(cols, r, seed, 2)
    return (U * sigma) @ V.T, U, np.asarray(sigma, dtype=np.float64), V


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# ---------------------------------------------------------------------------------------------
# Cesista's reparameterisation
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("gamma,r,u", [(2.0, 0.3, 0.1), (1.7, 0.05, 0.4), (3.1, 0.6, -0.2)])
def test_cesista_expansion_matches_root_product(gamma, r, u):
    """a x + b x^3 + c x^5 = gamma prod_i (x - f_i) + x, with the product expanded by numpy
    from the five roots; every root f_i is a fixed point of the map."""
    f = np.array([-(1 + r), -(1 - u), 0.0, 1 - u, 1 + r])
    poly = np.poly(f)  # monic, highest power first
    x = np.linspace(-1.6, 1.6, 41)
    want = gamma * np.polyval(poly, x) + x
    got = BL.compose_scalar(x, [BL.cesista_to_abc(gamma, r, u)])
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
    assert np.max(np.abs(BL.compose_scalar(f, [BL.cesista_to_abc(gamma, r, u)]) - f)) <= 1e-13


def test_muon_quintic_round_trip():
    """Muon's quintic has a real (gamma, r, u) form, and mapping back reproduces it."""
    g, r, u = BL.abc_to_cesista(*configs.MUON_ABC)
    assert g == configs.MUON_ABC[2] and 0.0 < u < r < 1.0
    assert np.allclose(BL.cesista_to_abc(g, r, u), configs.MUON_ABC, rtol=1e-13, atol=0)
    with pytest.raises(ValueError):
        BL.abc_to_cesista(*configs.CUBIC_ABC)


def test_cesista_gradient_matches_central_differences():
    params = [(2.05, 0.32, 0.12), (2.0, 0.3, 0.15), (1.9, 0.1, 0.05)]
    L, g = BL.cesista_objective_grad(params)
    assert abs(L - BL.cesista_objective([BL.cesista_to_abc(*p) for p in params])) <= 1e-15
    th = np.array(params)
    for i in range(th.shape[0]):
        for j in range(3):
            e = np.zeros_like(th)
            e[i, j] = 1e-6
            fd = (BL.cesista_objective_grad(th + e)[0] - BL.cesista_objective_grad(th - e)[0]) / 2e-6
            assert abs(fd - g[i, j]) <= 1e-7 * max(1.0, abs(g[i, j]))


def test_cesista_fit_is_stationary_and_stored():
    """The stored schedule is a stationary point of the stated objective (the paper prints no
    fitted values, so the values themselves are parity unpinned) and beats five Muon steps."""
    params, sched = BL.cesista_fit()
    assert len(sched) == 5
    L, g = BL.cesista_objective_grad(params)
    assert np.abs(g).max() <= 1e-8
    assert L < 0.05 * BL.cesista_objective([configs.MUON_ABC] * 5)
    for p, abc in zip(params, sched):
        assert np.allclose(BL.abc_to_cesista(*abc), p, rtol=1e-9, atol=1e-12)
    stored, q = configs.load_schedule("cesista_ns5")
    assert q == 0 and np.allclose(stored, sched, rtol=1e-7, atol=1e-10)


# ---------------------------------------------------------------------------------------------
# CANS: minimax odd polynomials
# ---------------------------------------------------------------------------------------------
def _cubic_minimax_closed_form(lo, hi):
    """Degree-3 odd minimax of 1 on [lo, hi], derived by hand from the alternation conditions
    e(lo) = E, e(x*) = -E, e(hi) = E with e = 1 - (alpha x + beta x^3) and p'(x*) = 0:
    alpha = -beta (lo^2 + lo hi + hi^2), x*^2 = (lo^2 + lo hi + hi^2) / 3,
    -beta = 2 / (lo hi (lo + hi) + 2 x*^3), E = 1 + beta lo hi (lo + hi)."""
    q = lo * lo + lo * hi + hi * hi
    xs = math.sqrt(q / 3.0)
    nb = 2.0 / (lo * hi * (lo + hi) + 2.0 * xs ** 3)
    return (nb * q, -nb), 1.0 - nb * lo * hi * (lo + hi)


@pytest.mark.parametrize("lo,hi", [(1e-3, 1.0), (0.05, 1.0), (0.3, 1.7), (0.9, 1.1)])
def test_cubic_minimax_closed_form(lo, hi):
    (a, b, c), E = BL.minimax_odd(lo, hi, 3)
    (a0, b0), E0 = _cubic_minimax_closed_form(lo, hi)
    assert c == 0.0
    assert abs(a - a0) <= 1e-12 * abs(a0) and abs(b - b0) <= 1e-12 * abs(b0) and abs(E - E0) <= 1e-12


def _lp_minimax(lo, hi, degree, n=20001):
    from scipy.optimize import linprog
    x = np.geomspace(lo, hi, n)
    d = (degree + 1) // 2
    P = x[:, None] ** (2 * np.arange(d) + 1)[None, :]
    A = np.vstack([np.hstack([-P, -np.ones((n, 1))]), np.hstack([P, -np.ones((n, 1))])])
    b = np.concatenate([-np.ones(n), np.ones(n)])
    r = linprog(np.r_[np.zeros(d), 1.0], A_ub=A, b_ub=b, bounds=[(None, None)] * (d + 1), method="highs")
    assert r.success
    return r.x[:d], r.x[d]


@pytest.mark.parametrize("lo,hi", [(1e-3, 1.0), (0.05, 1.0), (0.3, 1.7), (0.9, 1.1)])
@pytest.mark.parametrize("degree", [3, 5])
def test_minimax_equioscillates_and_matches_lp(lo, hi, degree):
    """Chebyshev alternation: |1 - p| reaches E at d + 1 points with alternating signs and
    nowhere exceeds it; a linear program over a fine grid finds the same polynomial."""
    abc, E = BL.minimax_odd(lo, hi, degree)
    x = np.geomspace(lo, hi, 400001)
    err = 1.0 - BL.compose_scalar(x, [abc])
    assert abs(np.max(np.abs(err)) - E) <= 1e-12
    # alternation: sign changes between the extremes of the error curve
    ext = x[np.r_[0, np.where(np.diff(np.sign(np.diff(err))) != 0)[0] + 1, len(x) - 1]]
    ev = 1.0 - BL.compose_scalar(ext, [abc])
    assert len(ev) == (degree + 1) // 2 + 1
    assert np.all(np.abs(np.abs(ev) - E) <= 1e-9) and np.all(ev[:-1] * ev[1:] < 0)
    c_lp, E_lp = _lp_minimax(lo, hi, degree)
    assert E_lp <= E + 1e-12 and E - E_lp <= 1e-6
    d = (degree + 1) // 2
    assert np.allclose(abc[:d], c_lp, rtol=1e-4, atol=1e-6)


def test_cans_schedule_maps_interval_brute_force():
    """Every step sends its interval into the next one, and the composed map on [delta, 1]
    stays within [1 - E, 1 + E] of the last step, reaching both ends."""
    sched, iv = BL.cans_schedule(5, 1e-3, 5)
    x = np.geomspace(1e-3, 1.0 * 1.02, 200001)
    for k, abc in enumerate(sched):
        y = BL.compose_scalar(x, [abc])
        lo, hi = iv[k + 1]
        assert y.min() >= lo - 1e-10 and y.max() <= hi + 1e-10
        assert abs(y.min() - lo) <= 1e-7 and abs(y.max() - hi) <= 1e-7
        # the next step is built for [lo, 1.02 hi]
        x = np.geomspace(lo, hi * 1.02, 200001)
    # without the margin the same construction chains the plain intervals
    s0, iv0 = BL.cans_schedule(2, 1e-3, 5, margin=0.0)
    assert np.allclose(s0[0], BL.minimax_odd(1e-3, 1.0, 5)[0], rtol=1e-14, atol=0)
    assert np.allclose(s0[1], BL.minimax_odd(*iv0[1], 5)[0], rtol=1e-14, atol=0)
    stored, q = configs.load_schedule("cans_ns5_q2")
    assert q == 2 and np.allclose(stored, sched, rtol=1e-12, atol=0)


# ---------------------------------------------------------------------------------------------
# Gelfand scaling and the matrix iteration
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("q", [1, 2, 3])
def test_gelfand_scale_closed_form_and_bound(q):
    sigma = np.array([1.3, 0.9, 0.5, 0.2, 0.01])
    M, U, s, V = _spectral(5, 11, seed=21, sigma=sigma)
    want = float(np.sum(s ** (4 * q))) ** (1.0 / (4 * q))
    got = BL.gelfand_scale(M, q)
    assert abs(got - want) <= 1e-13 * want
    assert got >= s.max()
    if q > 1:
        assert got < BL.gelfand_scale(M, q - 1)
    # rank one: the bound is attained
    v = gen.gaussian_np(1, 7, 5, 0, 1.0)
    assert abs(BL.gelfand_scale(v, q) - np.linalg.norm(v)) <= 1e-14 * np.linalg.norm(v)


def test_gelfand_q1_is_gram_frobenius():
    A = gen.gaussian_np(6, 13, 8, 0, 1.0)
    assert abs(BL.gelfand_scale(A, 1) - O.normalise(A, "gram_frobenius")[1]) <= 1e-14 * BL.gelfand_scale(A, 1)


@pytest.mark.parametrize("q", [0, 1, 2])
@pytest.mark.parametrize("shape", [(9, 20), (20, 9)])
def test_ns_schedule_closed_form(q, shape):
    """On M = U diag(sigma) V^T the iteration acts on singular values only:
    Y = U diag(phi(sigma / s)) V^T with phi the composed scalar map."""
    sched, _ = BL.cans_schedule(4, 1e-2, 5)
    sigma = 10.0 ** np.linspace(-1.5, 0.3, min(shape))
    M, U, s, V = _spectral(*shape, seed=31, sigma=sigma)
    scale = math.sqrt(float(np.sum(s * s))) if q == 0 else float(np.sum(s ** (4 * q))) ** (1.0 / (4 * q))
    want = (U * BL.compose_scalar(s / scale, sched)) @ V.T
    assert _rel(BL.ns_schedule(M, sched, q), want) <= 1e-12


def test_ns_schedule_constant_is_classical_ns():
    M = gen.gaussian_np(12, 30, 4, 0, 1.0)
    assert _rel(BL.ns_schedule(M, [configs.MUON_ABC] * 3), O.classical_ns(M, 3, configs.MUON_ABC)) <= 1e-14
    assert not BL.ns_schedule(np.zeros((3, 5)), [configs.MUON_ABC], 2).any()


def test_stored_reference_schedules():
    s, q = configs.load_schedule("muon_ns5")
    assert q == 0 and np.array_equal(np.array(s), np.array([configs.MUON_ABC] * 5))
    s, q = configs.load_schedule("original_ns8")
    assert q == 0 and np.array_equal(np.array(s), np.array([configs.CUBIC_ABC] * 8))
