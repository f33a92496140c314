"""Pins of the FP64 oracle against what the paper and mathematics fix.

Each test ties one part of the oracle to something other than its own code:
values printed in the paper, closed forms, a dense Liouvillian assembled from
operator definitions, quadrature of the spectral density, exact limits and
invariants.  All CPU-only.
"""

import os
from math import comb

import numpy as np
import pytest
from scipy import integrate
from scipy.linalg import expm

import dense_heom
import heom_inputs as hi

HERE = os.path.dirname(os.path.abspath(__file__))
TWO_PI_C = 2.0 * np.pi * 2.99792458e-5


def _golden_counts():
    rows = []
    with open(os.path.join(HERE, "golden", "ado_counts.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                W, D, n, _src = line.split()
                rows.append((int(W), int(D), int(n)))
    return rows


def _fmo_paper_h():
    return np.loadtxt(os.path.join(HERE, "golden", "fmo_paper_hamiltonian.txt"))


# ---------------------------------------------------------------- counts ----

@pytest.mark.parametrize("W,D,n", _golden_counts())
def test_ado_count_paper_values(orc, W, D, n):
    # eq. Nmatrices; 12271512 is printed in "Convergence analysis".
    assert orc.count(W, D) == n


@pytest.mark.parametrize("W,D", [(1, 0), (1, 7), (2, 3), (5, 3), (4, 4), (7, 2), (14, 4),
                                 (24, 4), (28, 5), (96, 3)])
def test_ado_count_binomial(orc, W, D):
    assert orc.count(W, D) == comb(W + D, W)


def test_workload_counts(orc):
    # Hierarchy sizes of the named workloads: dimer, FMO-like, 24-site, 48-site.
    for prob, n in ((hi.dimer(), 10), (hi.fmo_like(), 3060), (hi.aggregate24(), 20475),
                    (hi.aggregate48(), 156849)):
        W = sum(b["matsubara"] + 1 for b in prob["baths"])
        assert orc.count(W, prob["depth"]) == n == comb(W + prob["depth"], W)


# ---------------------------------------------------------------- tables ----

@pytest.mark.parametrize("W,D", [(1, 4), (2, 3), (3, 3), (5, 3), (4, 4), (6, 2), (7, 2)])
def test_tables_brute_force(orc, W, D):
    tup, plus, minus, level = orc.tables(W, D)
    ref = dense_heom.enumerate_tuples(W, D)
    assert [tuple(t) for t in tup] == ref
    index = {t: u for u, t in enumerate(ref)}
    for u, t in enumerate(ref):
        assert level[u] == sum(t)
        for l in range(W):
            tp = list(t)
            tp[l] += 1
            assert plus[u, l] == (index[tuple(tp)] if sum(t) < D else -1)
            tm = list(t)
            tm[l] -= 1
            assert minus[u, l] == (index[tuple(tm)] if t[l] > 0 else -1)


@pytest.mark.parametrize("W,D", [(14, 4), (24, 3), (9, 5)])
def test_table_invariants(orc, W, D):
    tup, plus, minus, level = orc.tables(W, D)
    n = len(tup)
    assert n == comb(W + D, W)
    # level-1 ADO e_l sits at index 1 + l
    for l in range(W):
        e = np.zeros(W, np.uint8)
        e[l] = 1
        assert np.array_equal(tup[1 + l], e)
    u = np.arange(n)
    for l in range(W):
        ok = plus[:, l] >= 0
        assert np.array_equal(minus[plus[ok, l], l], u[ok])
        assert np.all(level[plus[ok, l]] == level[ok] + 1)
        assert np.all(ok == (level < D))
        okm = minus[:, l] >= 0
        assert np.array_equal(plus[minus[okm, l], l], u[okm])
        assert np.all(okm == (tup[:, l] > 0))
    # levels non-decreasing, descending lexicographic inside a level
    assert np.all(np.diff(level) >= 0)
    for a in range(n - 1):
        if level[a] == level[a + 1]:
            assert tuple(tup[a]) > tuple(tup[a + 1])


# ---------------------------------------------------------- coefficients ----

def _corr_quadrature(lam_cm, tau, T, t):
    """C(t) = (1/pi) int_0^inf J(w) [coth(beta w/2) cos wt - i sin wt] dw with
    the Drude-Lorentz density of eq. spectral_density_DL at Omega = 0,
    J(w) = 2 lambda nu w / (w^2 + nu^2)."""
    lam = lam_cm * TWO_PI_C
    nu = 1.0 / tau
    beta = 1.0 / (0.6950348004 * T * TWO_PI_C)

    def jre(w):
        if w == 0.0:
            return 4.0 * lam / (beta * nu)  # limit of J(w) coth(beta w / 2)
        return 2.0 * lam * nu * w / (w * w + nu * nu) / np.tanh(beta * w / 2.0)

    def jim(w):
        return 2.0 * lam * nu * w / (w * w + nu * nu)

    re = integrate.quad(jre, 0.0, np.inf, weight="cos", wvar=t, limlst=200)[0] / np.pi
    im = -integrate.quad(jim, 0.0, np.inf, weight="sin", wvar=t, limlst=200)[0] / np.pi
    return re, im


@pytest.mark.parametrize("lam,tau,T", [(35.0, 50.0, 300.0), (50.0, 100.0, 277.0),
                                       (20.0, 30.0, 77.0)])
def test_correlation_matches_spectral_density(orc, lam, tau, T):
    M = 20000
    g, c, lamnu, delta = orc.bath_coefficients(lam, tau, T, M)
    for t in (5.0, 20.0, 60.0):
        re_q, im_q = _corr_quadrature(lam, tau, T, t)
        re_s = np.sum(c * np.exp(-g * t))
        # scale: the k = 0 weight (Re C(t) can nearly cancel at low T)
        assert abs(re_s - re_q) <= 5e-6 * max(abs(re_q), abs(c[0]))
        # imaginary part: the lambda*nu V^o term carries -lambda nu e^{-nu t}
        assert abs(-lamnu * np.exp(-g[0] * t) - im_q) <= 1e-6 * abs(im_q)


def test_terminator_sum_rule(orc):
    # sum_{k>=0} c_k / gamma_k = 2 lambda / (beta nu): the correction term of
    # eq. HEOM vanishes as M -> infinity, and falls like 1/M.
    prev = None
    for M in (0, 1, 10, 100, 1000, 10000):
        _, _, _, d = orc.bath_coefficients(35.0, 50.0, 300.0, M)
        assert d > 0.0
        if prev is not None:
            assert d < prev
        prev = d
    _, _, _, d0 = orc.bath_coefficients(35.0, 50.0, 300.0, 0)
    _, _, _, d_big = orc.bath_coefficients(35.0, 50.0, 300.0, 20000)
    assert d_big < 1e-4 * d0


def test_first_matsubara_frequency(orc):
    # gamma(b,1) = 2 pi / (beta hbar); beta hbar = 25.4608 fs at 300 K
    g, _, _, _ = orc.bath_coefficients(35.0, 50.0, 300.0, 3)
    beta = 1.0 / (0.6950348004 * 300.0 * TWO_PI_C)
    assert abs(beta - 25.4608) < 1e-3
    assert np.allclose(g[1:], 2 * np.pi * np.arange(1, 4) / beta, rtol=1e-14)
    assert g[0] == pytest.approx(1.0 / 50.0, rel=1e-15)


# ---------------------------------------------------------- Pade modes ----

def _bose_pade(x, K, orc):
    xi, eta = orc.pade_poles(K)
    return 1.0 / x + 0.5 + sum(2.0 * e * x / (x * x + z * z) for z, e in zip(xi, eta))


def test_pade_k1_closed_form(orc):
    # Lambda is [[0, 1/sqrt(15)], [1/sqrt(15), 0]] and Lambda' = [0]: xi = 2 sqrt(15),
    # eta = K^2 + 3K/2 = 5/2.  1/x + 1/2 + 5x/(x^2 + 60) then matches the Taylor
    # series of 1/(1 - e^-x) = 1/x + 1/2 + x/12 - x^3/720 + ... through x^3.
    xi, eta = orc.pade_poles(1)
    assert xi[0] == pytest.approx(2.0 * np.sqrt(15.0), rel=1e-14)
    assert eta[0] == pytest.approx(2.5, rel=1e-14)
    x = 1e-2
    err = _bose_pade(np.array([x]), 1, orc)[0] - 1.0 / (-np.expm1(-x))
    assert abs(err) < 1e-11   # the next term is O(x^5)


def test_pade_poles_match_eigvalsh(orc):
    # an independent eigensolver on the same two matrices
    for K in (2, 3, 5, 8, 16):
        def lam(n, shift):
            m = np.arange(1, n)
            off = 1.0 / np.sqrt((2.0 * m + shift) * (2.0 * m + shift + 2.0))
            return np.diag(off, 1) + np.diag(off, -1)
        ev = np.sort(np.linalg.eigvalsh(lam(2 * K, 1)))[::-1][:K]
        evp = np.sort(np.linalg.eigvalsh(lam(2 * K - 1, 3)))[::-1][:K - 1]
        xi, eta = orc.pade_poles(K)
        assert np.allclose(xi, 2.0 / ev, rtol=1e-12, atol=0)
        zeta = 2.0 / evp
        ref = np.array([(K * K + 1.5 * K) * np.prod(zeta**2 - x**2) /
                        np.prod([xi[j]**2 - x**2 for j in range(K) if j != i])
                        for i, x in enumerate(xi)])
        assert np.allclose(eta, ref, rtol=1e-10, atol=0)


def test_pade_reproduces_bose_function(orc):
    # the [K-1/K] approximant converges fast on |x| < 2 pi (Hu, Xu and Yan)
    x = np.linspace(-6.0, 6.0, 241)
    x = x[np.abs(x) > 1e-9]
    exact = 1.0 / (-np.expm1(-x))
    errs = [np.max(np.abs(_bose_pade(x, K, orc) - exact)) for K in (1, 2, 3, 4, 6)]
    assert errs[0] < 3e-2 and errs[1] < 3e-4 and errs[2] < 1e-6 and errs[3] < 1e-9
    assert errs[4] < 1e-13
    assert all(a > b for a, b in zip(errs[:4], errs[1:4]))


def test_pade_first_poles_tend_to_matsubara(orc):
    # the lowest poles become the Matsubara frequencies 2 pi j with unit weight
    xi, eta = orc.pade_poles(20)
    assert np.allclose(xi[:5], 2 * np.pi * np.arange(1, 6), rtol=1e-12)
    assert np.allclose(eta[:5], 1.0, rtol=1e-12)
    assert np.all(eta > 0) and np.all(np.diff(xi) > 0)


@pytest.mark.parametrize("T", [300.0, 77.0, 30.0])
def test_pade_sum_rule_and_cot(orc, T):
    # with c(b,0) in its Pade form, sum_k c_k / gamma_k = 2 lambda / (beta nu)
    # for every K, so the correction coefficient vanishes; c(b,0) tends to
    # lambda nu cot(beta nu / 2)
    lam, tau = 35.0, 50.0
    beta = 1.0 / (0.6950348004 * T * TWO_PI_C)
    l, nu = lam * TWO_PI_C, 1.0 / tau
    for K in (0, 1, 2, 4, 8):
        g, c, lamnu, d = orc.bath_coefficients(lam, tau, T, K, pade=True)
        assert abs(d) <= 1e-13 * (2 * l / (beta * nu))
        assert g[0] == nu and lamnu == pytest.approx(l * nu, rel=1e-15)
    g, c, _, _ = orc.bath_coefficients(lam, tau, T, 12, pade=True)
    assert c[0] == pytest.approx(l * nu / np.tan(beta * nu / 2), rel=1e-11)


@pytest.mark.parametrize("lam,tau,T", [(35.0, 50.0, 300.0), (20.0, 30.0, 77.0),
                                       (50.0, 100.0, 30.0)])
def test_pade_correlation_matches_spectral_density(orc, lam, tau, T):
    g, c, lamnu, _ = orc.bath_coefficients(lam, tau, T, 40, pade=True)
    for t in (5.0, 20.0, 60.0):
        re_q, _ = _corr_quadrature(lam, tau, T, t)
        assert abs(np.sum(c * np.exp(-g * t)) - re_q) <= 5e-6 * max(abs(re_q), abs(c[0]))
    # at 30 K four poles already beat four Matsubara terms at short times
    if T == 30.0:
        re_q, _ = _corr_quadrature(lam, tau, T, 5.0)
        gp, cp, _, _ = orc.bath_coefficients(lam, tau, T, 4, pade=True)
        gm, cm, _, _ = orc.bath_coefficients(lam, tau, T, 4)
        assert abs(np.sum(cp * np.exp(-gp * 5.0)) - re_q) < abs(np.sum(cm * np.exp(-gm * 5.0)) - re_q)


def test_pade_pure_dephasing_cumulant(orc):
    # the exactly solvable dephasing limit (see the Matsubara test below) with
    # Pade modes: the hierarchy reproduces the cumulant of its own expansion
    eps, lam, tau, T, K = 100.0, 20.0, 50.0, 77.0, 2
    prob = {"H": np.diag([0.0, eps]), "temperature_K": T, "depth": 10, "flags": hi.FLAG_PADE,
            "baths": [{"state": 1, "lambda_cm": lam, "tau_fs": tau, "matsubara": K}]}
    W, n = orc.sizes(prob)
    g, c, lamnu, delta = orc.bath_coefficients(lam, tau, T, K, pade=True)
    ct = c.astype(complex)
    ct[0] -= 1j * lamnu
    s = orc.initial_state(prob, n, np.full((2, 2), 0.5, complex))
    t = 0.0
    for _ in range(4):
        s, _ = orc.propagate(prob, s, 0.25, 200, 200)
        t += 50.0
        gt = np.sum(ct / g**2 * (g * t - 1 + np.exp(-g * t))) + delta * t
        ref = 0.5 * np.exp(-1j * eps * TWO_PI_C * t - gt)
        assert abs(s[0][1, 0] - ref) < 1e-8


# ------------------------------------------------------------------- RHS ----

def _small_problems():
    yield hi.dimer()
    yield hi.random_problem(3, 3, M=1, D=2)
    yield hi.random_problem(4, 3, n_baths=2, M=2, D=2, complex_h=True)
    p = hi.random_problem(5, 2, n_baths=2, M=0, D=4)
    p["flags"] = hi.FLAG_NO_RESCALE
    yield p


@pytest.mark.parametrize("prob", list(_small_problems()))
def test_rhs_matches_dense_liouvillian(orc, prob):
    rescale = not (prob["flags"] & hi.FLAG_NO_RESCALE)
    L, tups = dense_heom.liouvillian(prob, orc, rescale=rescale)
    N = prob["H"].shape[0]
    x = hi.random_state(11, len(tups), N)
    f = orc.rhs(prob, x)
    ref = (L @ x.reshape(-1)).reshape(x.shape)
    assert np.max(np.abs(f - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_rhs_flags_match_dense(orc):
    prob = hi.random_problem(6, 3, M=1, D=2)
    N = 3
    for flags, kw in ((hi.FLAG_NO_TERMINATOR, {"terminator": False}),
                      (hi.FLAG_STANDARD_GAUGE, {"gauge": -1.0}),
                      (hi.FLAG_ADD_REORG, {"add_reorg": True}),
                      (hi.FLAG_ADD_REORG | hi.FLAG_NO_TERMINATOR,
                       {"add_reorg": True, "terminator": False})):
        p = dict(prob, flags=flags)
        L, tups = dense_heom.liouvillian(p, orc, **kw)
        x = hi.random_state(12, len(tups), N)
        f = orc.rhs(p, x)
        ref = (L @ x.reshape(-1)).reshape(x.shape)
        assert np.max(np.abs(f - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_rhs_range_matches_full(orc):
    prob = hi.random_problem(7, 3, M=1, D=3)
    W, n = orc.sizes(prob)
    x = hi.random_state(13, n, 3)
    full = orc.rhs(prob, x)
    part = orc.rhs(prob, x, 5, 17)
    assert np.array_equal(part[5:17], full[5:17])
    assert not np.any(part[:5]) and not np.any(part[17:])


# ----------------------------------------------------------- propagation ----

def test_rk4_matches_exact_polynomial_and_expm(orc):
    prob = hi.dimer()
    L, tups = dense_heom.liouvillian(prob, orc)
    n = len(tups)
    y0 = np.zeros(n * 4, np.complex128)
    y0[0] = 1.0
    R = dense_heom.rk4_matrix(L, 1.0)
    ref = np.linalg.matrix_power(R, 1000) @ y0
    y, rec = orc.propagate(prob, y0.reshape(n, 2, 2), 1.0, 1000, 1)
    assert np.max(np.abs(y.reshape(-1) - ref)) < 1e-13
    ex = expm(L * 1000.0) @ y0
    assert np.max(np.abs(y.reshape(-1) - ex)) < 1e-12
    # smoke value of the dimer at 1 ps (dense expm, not from the paper)
    assert abs(ex[0].real - 0.6154393558) < 1e-10
    assert abs(rec[-1][0] - ex[0].real) < 1e-12


def test_rk4_fourth_order(orc):
    prob = hi.random_problem(8, 2, M=1, D=2)
    L, tups = dense_heom.liouvillian(prob, orc)
    n = len(tups)
    y0 = np.zeros((n, 2, 2), np.complex128)
    y0[0] = [[0.7, 0.2 + 0.1j], [0.2 - 0.1j, 0.3]]
    T = 240.0
    ex = expm(L * T) @ y0.reshape(-1)
    errs = []
    for dt in (4.0, 2.0, 1.0):  # max |eigenvalue| ~ 0.5/fs: dt = 8 is unstable
        y, _ = orc.propagate(prob, y0, dt, int(T / dt), 1000)
        errs.append(np.max(np.abs(y.reshape(-1) - ex)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 12.0 < r1 < 20.0 and 12.0 < r2 < 20.0


def test_lambda_zero_dimer_closed_form(orc):
    # Unitary limit: lambda = 0 makes every bath weight vanish, so sigma_0
    # follows -i[H, rho]; two-level Rabi formula.
    prob = hi.dimer()
    for b in prob["baths"]:
        b["lambda_cm"] = 0.0
    # dt = 0.25 fs so that the RK4 truncation error (~dt^4) is ~1e-10 at 1 ps
    _, rec = orc.run(dict(prob, dt_fs=0.25, n_steps=4000, record_every=4))
    t = np.arange(len(rec)) * 1.0
    d, J = 100.0, 50.0
    Om = np.sqrt(d * d + 4 * J * J) * TWO_PI_C
    P1 = 1.0 - 4 * J * J / (d * d + 4 * J * J) * np.sin(Om * t / 2.0) ** 2
    assert np.max(np.abs(rec[:, 0] - P1)) < 3e-10


def test_lambda_zero_fmo_unitary(orc):
    H = _fmo_paper_h()
    prob = {"H": H, "baths": [{"state": m, "lambda_cm": 0.0, "tau_fs": 50.0, "matsubara": 1}
                              for m in range(7)],
            "temperature_K": 300.0, "depth": 2, "flags": 0}
    W, n = orc.sizes(prob)
    rho0 = hi.population_rho0(7)
    y, rec = orc.propagate(prob, orc.initial_state(prob, n, rho0), 0.5, 400, 100)
    w, v = np.linalg.eigh(H * TWO_PI_C)
    U = v @ np.diag(np.exp(-1j * w * 200.0)) @ v.conj().T
    ref = U @ rho0 @ U.conj().T
    # dt = 0.5 fs at |E| ~ 2.4 rad/fs: RK4 phase error is the limit here
    assert np.max(np.abs(y[0] - ref)) < 2e-5


def test_pure_dephasing_cumulant(orc):
    # Exactly solvable limit: H and the coupling V = |1><1| commute, so the
    # coherence is rho_10(t) = rho_10(0) exp(-i eps t - g(t)) with the
    # cumulant g(t) of the bath correlation sum_k c~_k exp(-gamma_k t), where
    # c~_0 = lambda nu (cot(beta nu/2) - i); the correction term adds Delta t.
    eps, lam, tau, T, M = 100.0, 20.0, 50.0, 300.0, 1
    prob = {"H": np.diag([0.0, eps]), "temperature_K": T, "depth": 12, "flags": 0,
            "baths": [{"state": 1, "lambda_cm": lam, "tau_fs": tau, "matsubara": M}]}
    W, n = orc.sizes(prob)
    g, c, lamnu, delta = orc.bath_coefficients(lam, tau, T, M)
    ct = c.astype(complex)
    ct[0] -= 1j * lamnu
    s = orc.initial_state(prob, n, np.full((2, 2), 0.5, complex))
    t = 0.0
    for _ in range(5):
        s, _ = orc.propagate(prob, s, 0.5, 100, 100)
        t += 50.0
        gt = np.sum(ct / g**2 * (g * t - 1 + np.exp(-g * t))) + delta * t
        ref = 0.5 * np.exp(-1j * eps * TWO_PI_C * t - gt)
        assert abs(s[0][1, 0] - ref) < 1e-9
        assert abs(s[0][0, 1] - np.conj(ref)) < 1e-9


# ------------------------------------------------------------ invariants ----

def test_trace_and_hermiticity_preserved(orc):
    prob = hi.fmo_like(n_steps=40)
    prob["depth"] = 2
    W, n = orc.sizes(prob)
    y, rec = orc.run(prob)
    assert np.max(np.abs(rec[:, 7] - 1.0)) < 1e-13   # Re Tr
    assert np.max(np.abs(rec[:, 8])) < 1e-13         # Im Tr
    assert np.max(rec[:, 9]) < 1e-13                 # |rho - rho^dagger|
    herm = np.max(np.abs(y - np.conj(np.transpose(y, (0, 2, 1)))))
    assert herm < 1e-13 * max(1.0, np.max(np.abs(y)))


def test_absorption_trace_zero(orc):
    runs = hi.fmo_like_absorption(n_steps=30)
    for r in runs:
        r["depth"] = 2
        _, rec = orc.run(r)
        assert np.max(np.abs(rec[:, 2:4])) < 1e-14


def test_rescaling_and_sign_gauge_leave_rho_unchanged(orc):
    prob = hi.random_problem(9, 3, M=1, D=3)
    W, n = orc.sizes(prob)
    rho0 = hi.population_rho0(3, 1)
    base, _ = orc.propagate(prob, orc.initial_state(prob, n, rho0), 1.0, 200, 200)
    for flags in (hi.FLAG_NO_RESCALE, hi.FLAG_STANDARD_GAUGE):
        p = dict(prob, flags=flags)
        y, _ = orc.propagate(p, orc.initial_state(p, n, rho0), 1.0, 200, 200)
        assert np.max(np.abs(y[0] - base[0])) < 1e-13


# --------------------------------------------------------------- spectra ----

def test_spectrum_trapezoid_closed_form(orc):
    # P(t) = exp(-i e t): the trapezoid sum is a geometric series.
    dt, n_t, e_cm = 1.0, 1001, 37.0
    t = np.arange(n_t) * dt
    P = np.exp(-1j * e_cm * TWO_PI_C * t)
    w = np.linspace(-300.0, 300.0, 61)
    S = orc.spectrum(P[None, :], dt, w)
    r = np.exp(1j * (w - e_cm) * TWO_PI_C * dt)
    with np.errstate(divide="ignore", invalid="ignore"):
        geo = np.where(np.abs(r - 1) > 1e-15, (1 - r**n_t) / (1 - r), n_t)
    ref = ((geo - 0.5 * (1 + r ** (n_t - 1))) * dt).real
    assert np.max(np.abs(S - ref)) < 1e-9 * np.max(np.abs(ref))


def _fluor_spectra(orc, lam, tau, D, sigma0_only=False):
    H = np.array([[12000.0]])
    dip = np.array([[1.0, 0.0, 0.0]])
    baths = [{"state": 0, "lambda_cm": lam, "tau_fs": tau, "matsubara": 0}]
    relax, emis = hi.fluorescence_runs(H, dip, baths, 300.0, D, 1.0, 5000, 3000)
    st, P = orc.fluorescence(relax, emis[:1])
    if sigma0_only:
        st[1:] = 0.0
        Y = orc.emission_start(st, emis[0]["observable"]["mu"][1:])
        _, rec = orc.propagate(emis[0], Y, 1.0, 3000, 1, emis[0]["observable"])
        P = (rec[:, 0] + 1j * rec[:, 1])[None]
    _, rec = orc.run(hi.absorption_runs(H, dip, baths, 300.0, D, 1.0, 3000)[0])
    w = np.arange(-800.0, 800.0, 1.0)
    Sf = orc.spectrum(P, 1.0, w)
    Sa = orc.spectrum((rec[:, 0] + 1j * rec[:, 1])[None], 1.0, w)
    mean = lambda S: np.sum(w * S) / np.sum(S)
    return mean(Sa), mean(Sf)


@pytest.mark.parametrize("lam", [20.0, 35.0])
def test_fluorescence_stokes_shift_monomer(orc, lam):
    # One excited state with a slow Drude-Lorentz bath: the first moments of
    # absorption and emission differ by the Stokes shift 2 lambda.  Applying
    # the dipole to sigma_0 alone (dropping the thermal ADOs) loses it.
    ma, mf = _fluor_spectra(orc, lam, 500.0, 16)
    assert abs((ma - mf) - 2 * lam) <= 0.02 * 2 * lam
    ma0, mf0 = _fluor_spectra(orc, lam, 500.0, 16, sigma0_only=True)
    assert abs(ma0 - mf0) <= 0.05 * 2 * lam


def test_fluorescence_lambda_zero_closed_form(orc):
    # lambda = 0: the Boltzmann state is stationary and the emission
    # correlation is sum_k p_k (phi_k . mu)^2 R(z_k)^n, the thermal weights
    # of the excitons times their RK4-amplified phases.
    rng = np.random.default_rng(3)
    H = hi.fmo_like_hamiltonian(rng, 3)
    dip = hi.unit_vectors(rng, 3)
    baths = [{"state": s, "lambda_cm": 0.0, "tau_fs": 50.0, "matsubara": 0} for s in range(3)]
    relax, emis = hi.fluorescence_runs(H, dip, baths, 300.0, 1, 1.0, 50, 200)
    st, P = orc.fluorescence(relax, emis)
    assert np.max(np.abs(st[0] - hi.boltzmann_rho(H, 300.0))) < 1e-13
    wref = np.mean(np.diag(H))
    e, v = np.linalg.eigh(H)
    p = np.exp(-(e - e.min()) / (0.6950348004 * 300.0))
    p /= p.sum()
    z = -1j * (e - wref) * TWO_PI_C * 1.0
    R = 1 + z + z**2 / 2 + z**3 / 6 + z**4 / 24
    n = np.arange(P.shape[1])
    for k, r in enumerate(emis):
        amp = p * (v.T @ r["observable"]["mu"][1:]) ** 2
        ref = (amp[None, :] * R[None, :] ** n[:, None]).sum(axis=1)
        assert np.max(np.abs(P[k] - ref)) < 1e-12


def test_absorption_stays_in_the_coherence_block(orc):
    # the closure behind the coherence-block form: with the ground state
    # uncoupled, a full absorption run keeps every ADO zero outside its
    # (e, g) column (exactly: the other entries never receive a contribution)
    rng = np.random.default_rng(21)
    H = hi.fmo_like_hamiltonian(rng, 4)
    d = hi.unit_vectors(rng, 4)
    baths = [{"state": s, "lambda_cm": 35.0, "tau_fs": 50.0, "matsubara": 1} for s in range(4)]
    run = hi.absorption_runs(H, d, baths, 300.0, 3, 1.0, 100)[1]
    st, _ = orc.run(run)
    mask = np.zeros(st.shape[1:], bool)
    mask[1:, 0] = True
    assert np.max(np.abs(st[:, mask])) > 1e-3
    assert np.max(np.abs(st[:, ~mask])) == 0.0


def _cd_correlation(orc, H, R, d, T=300.0, D=3, steps=200):
    """Full (N+1)-state oracle runs: start m_p^+ |g><g|, observe mu_p."""
    baths = [{"state": s, "lambda_cm": 35.0, "tau_fs": 50.0, "matsubara": 0}
             for s in range(H.shape[0])]
    runs = hi.absorption_runs(H, d, baths, T, D, 1.0, steps)
    m = orc.cd_vectors(R, d)
    P = []
    for p, r in enumerate(runs):
        rho0 = np.zeros_like(r["rho0"])
        rho0[1:, 0] = m[p]
        _, rec = orc.run(dict(r, rho0=rho0))
        P.append(rec[:, 0] + 1j * rec[:, 1])
    return np.stack(P)


def test_cd_conservative_and_origin_independent(orc):
    # eq. CDdipoleoperator: sum_p m_p . mu_p = sum_a (R_a x d_a) . d_a = 0, so
    # the averaged CD correlation starts at 0 (the spectrum integrates to 0);
    # shifting every R_a by one vector c adds sum_ab c . (d_a x d_b) G_ab(t),
    # which vanishes because the block propagator is symmetric in the sites
    rng = np.random.default_rng(9)
    R = hi.aggregate_geometry(rng, 3)
    d = hi.unit_vectors(rng, 3)
    H = hi.dipole_couplings(R, d) + np.diag(rng.normal(12400.0, 100.0, 3))
    m = orc.cd_vectors(R, d)
    assert np.allclose(m[:, 0], np.cross(R[0], d[0]), rtol=0, atol=1e-14)
    P = _cd_correlation(orc, H, R, d)
    scale = np.max(np.abs(P))
    assert abs(P[:, 0].sum()) <= 1e-13 * scale
    P2 = _cd_correlation(orc, H, R + np.array([3.0, -7.0, 11.0]), d)
    assert np.max(np.abs(P.sum(axis=0) - P2.sum(axis=0))) <= 1e-11 * scale


def test_dipole_correlation_lambda_zero(orc):
    # lambda = 0: P_p(t) = sum_e |e_p . D_e|^2 exp(-i eps_e t) over excitons.
    runs = hi.fmo_like_absorption(n_steps=200)
    for r in runs:
        r["depth"] = 1
        for b in r["baths"]:
            b["lambda_cm"] = 0.0
        _, rec = orc.run(r)
        mu = r["observable"]["mu"]
        assert abs(rec[0, 0] - np.sum(mu**2)) < 1e-15
        Hc = r["H"] * TWO_PI_C
        w, v = np.linalg.eigh(Hc[1:, 1:])
        amp = (v.T @ mu[1:]) ** 2
        # every ADO but sigma_0 stays exactly zero, so RK4 advances each
        # exciton component by its stability polynomial R(z), z = -i eps dt
        z = -1j * w * r["dt_fs"]
        R = 1 + z + z**2 / 2 + z**3 / 6 + z**4 / 24
        n = np.arange(len(rec))
        P = (amp[None, :] * R[None, :] ** n[:, None]).sum(axis=1)
        assert np.max(np.abs(rec[:, 0] + 1j * rec[:, 1] - P)) < 1e-12
        # and R^n tracks the exact exp(-i eps t) to the RK4 truncation error
        Pex = (amp[None, :] * np.exp(-1j * np.outer(n * r["dt_fs"], w))).sum(axis=1)
        assert np.max(np.abs(P - Pex)) < 1e-5


# ------------------------------------------------- records, CD, c_k < 0 ----

def test_record_known_residual_trace_and_polarisation(orc):
    # the observables of sigma_0 on a state with known values: populations,
    # trace, max_ij |rho_ij - conj(rho_ji)| and P = sum_a mu_a rho[a][g]
    prob = hi.dimer()
    rho = np.array([[0.6, 0.3 + 0.1j], [0.5 - 0.2j, 0.4 + 0.05j]])
    W, n = orc.sizes(prob)
    _, rec = orc.propagate(prob, orc.initial_state(prob, n, rho), 1.0, 0, 1)
    # (0,1): 0.3+0.1i - (0.5+0.2i) = -0.2-0.1i, |.| = sqrt(0.05); (1,1): 0.1i
    assert np.array_equal(rec[0, :4], [0.6, 0.4, 1.0, 0.05])
    assert abs(rec[0, 4] - 0.22360679774997896) < 1e-16
    obs = {"kind": "dipole", "mu": np.array([2.0, -1.5]), "ground": 1}
    _, rec = orc.propagate(prob, orc.initial_state(prob, n, rho), 1.0, 0, 1, obs)
    # 2 (0.3+0.1i) - 1.5 (0.4+0.05i) = 0 + 0.125i
    assert abs(rec[0, 0] - 0.0) < 1e-15 and abs(rec[0, 1] - 0.125) < 1e-15
    assert np.array_equal(rec[0, 2:4], [1.0, 0.05])


def test_cd_vectors_literal_orientation(orc):
    # eq. CDdipoleoperator: m_p = (R_a x d_a) . e_p; x cross y = z, y cross z = x,
    # z cross x = y, and a dipole along R gives nothing
    R = np.array([[1.0, 0, 0], [0, 2.0, 0], [0, 0, 3.0], [4.0, 0, 0]])
    d = np.array([[0, 1.0, 0], [0, 0, 1.0], [1.0, 0, 0], [2.0, 0, 0]])
    m = orc.cd_vectors(R, d)
    assert m.shape == (3, 4)
    assert np.array_equal(m, [[0, 2, 0, 0], [0, 0, 3, 0], [1, 0, 0, 0]])


def test_cd_correlation_lambda_zero_closed_form(orc):
    # lambda = 0: the run started from m_p^+|g><g| and observed with d_p gives
    # P_p(n dt) = sum_e (d_p . phi_e)(m_p . phi_e) R(-i eps_e dt)^n, R the RK4
    # stability polynomial; m and d enter in different roles, so exchanging
    # them in the start vector or the observable changes the result's sign
    rng = np.random.default_rng(31)
    R = hi.aggregate_geometry(rng, 3)
    d = hi.unit_vectors(rng, 3)
    H = hi.dipole_couplings(R, d) + np.diag(rng.normal(12400.0, 100.0, 3))
    baths = [{"state": s, "lambda_cm": 0.0, "tau_fs": 50.0, "matsubara": 0} for s in range(3)]
    runs = hi.absorption_runs(H, d, baths, 300.0, 1, 1.0, 150)
    m = orc.cd_vectors(R, d)
    for p, r in enumerate(runs):
        rho0 = np.zeros_like(r["rho0"])
        rho0[1:, 0] = m[p]
        _, rec = orc.run(dict(r, rho0=rho0))
        w, v = np.linalg.eigh(r["H"][1:, 1:] * TWO_PI_C)
        amp = (v.T @ d[:, p]) * (v.T @ m[p])
        z = -1j * w * r["dt_fs"]
        Rz = 1 + z + z**2 / 2 + z**3 / 6 + z**4 / 24
        n = np.arange(len(rec))
        ref = (amp[None, :] * Rz[None, :] ** n[:, None]).sum(axis=1)
        assert np.max(np.abs(rec[:, 0] + 1j * rec[:, 1] - ref)) < 1e-12 * max(1.0, np.abs(amp).sum())


def _low_t_bath():
    # 10 K, nu^-1 = 20 fs: the first Matsubara rate 2 pi k_B T / hbar
    # (0.0082 / fs) lies below nu (0.05 / fs), so c_1 < 0
    return {"lambda_cm": 20.0, "tau_fs": 20.0, "matsubara": 1}, 10.0


def test_negative_weight_bath_dense_liouvillian(orc):
    b, T = _low_t_bath()
    g, c, _, _ = orc.bath_coefficients(b["lambda_cm"], b["tau_fs"], T, b["matsubara"])
    assert c[1] < 0 < c[0] and g[1] < g[0]
    prob = hi.random_problem(17, 3, M=1, D=2)
    prob["temperature_K"] = T
    prob["baths"] = [dict(b, state=s) for s in range(3)]
    for flags in (0, hi.FLAG_NO_RESCALE):
        p = dict(prob, flags=flags)
        L, tups = dense_heom.liouvillian(p, orc, rescale=not flags)
        x = hi.random_state(18, len(tups), 3)
        f = orc.rhs(p, x)
        ref = (L @ x.reshape(-1)).reshape(x.shape)
        assert np.max(np.abs(f - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_negative_weight_bath_rescaling_invariance(orc):
    # sigma_0 must not depend on the |c|-rescaling when some c_k < 0
    b, T = _low_t_bath()
    prob = hi.random_problem(19, 3, M=1, D=3)
    prob["temperature_K"] = T
    prob["baths"] = [dict(b, state=s) for s in range(3)]
    W, n = orc.sizes(prob)
    rho0 = hi.population_rho0(3, 2)
    base, _ = orc.propagate(prob, orc.initial_state(prob, n, rho0), 1.0, 200, 200)
    p = dict(prob, flags=hi.FLAG_NO_RESCALE)
    y, _ = orc.propagate(p, orc.initial_state(p, n, rho0), 1.0, 200, 200)
    assert np.max(np.abs(base[0])) > 0.1
    assert np.max(np.abs(y[0] - base[0])) < 1e-13


def test_negative_weight_bath_pure_dephasing_cumulant(orc):
    # the second-cumulant closed form of the pure-dephasing test with a bath
    # whose Matsubara weight is negative
    b, T = _low_t_bath()
    eps = 100.0
    prob = {"H": np.diag([0.0, eps]), "temperature_K": T, "depth": 12, "flags": 0,
            "baths": [dict(b, state=1)]}
    W, n = orc.sizes(prob)
    g, c, lamnu, delta = orc.bath_coefficients(b["lambda_cm"], b["tau_fs"], T, b["matsubara"])
    ct = c.astype(complex)
    ct[0] -= 1j * lamnu
    s = orc.initial_state(prob, n, np.full((2, 2), 0.5, complex))
    t = 0.0
    for _ in range(4):
        s, _ = orc.propagate(prob, s, 0.5, 100, 100)
        t += 50.0
        gt = np.sum(ct / g**2 * (g * t - 1 + np.exp(-g * t))) + delta * t
        ref = 0.5 * np.exp(-1j * eps * TWO_PI_C * t - gt)
        assert abs(s[0][1, 0] - ref) < 1e-9
