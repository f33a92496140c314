"""Host-side checks of the C ABI (no GPU): the library loads, exports every
entry point the header declares, and heom_plan validates and sizes problems."""

import ctypes
import os
import re
from math import comb

import numpy as np
import pytest

import heom_inputs as hi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "heom.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(heom_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def heom():
    import paper_1803_03498_amd as heom
    heom.load()
    return heom


def test_exports_every_declared_symbol(heom):
    from paper_1803_03498_amd import _abi
    lib = heom.load()
    names = _header_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
        assert name in _abi.SIGNATURES, name


def test_status_strings(heom):
    lib = heom.load()
    assert lib.heom_status_string(0) == b"HEOM_OK"
    assert lib.heom_status_string(-6) == b"HEOM_E_UNSTABLE"


@pytest.mark.parametrize("prob,n", [(hi.dimer(), 10), (hi.fmo_like(), 3060),
                                    (hi.aggregate24(), 20475), (hi.aggregate48(), 156849)])
def test_plan_sizes(heom, prob, n):
    for prec, e in ((heom.FP64, 16), (heom.FP32_MIXED, 8)):
        info = heom.plan(prob, prec)
        W = sum(b["matsubara"] + 1 for b in prob["baths"])
        D = prob["depth"]
        N = prob["H"].shape[0]
        assert info["n_ado"] == n == comb(W + D, W)
        assert info["n_modes"] == W
        assert info["n_plus_edges"] == W * comb(W + D - 1, W)
        assert info["sigma0_bytes"] == N * N * 16
        assert info["rest_bytes"] == (n - 1) * N * N * e
        assert info["work_bytes"] >= 3 * (info["sigma0_bytes"] + info["rest_bytes"])
        assert info["tables_bytes"] >= n * W * 9


def _bad(prob, **kw):
    p = dict(prob)
    p.update(kw)
    return p


def test_plan_validation(heom):
    from paper_1803_03498_amd._abi import HeomError
    d = hi.dimer()
    bad_bath = [dict(d["baths"][0], state=5), d["baths"][1]]
    cases = [
        (_bad(d, temperature_K=0.0), -1),
        (_bad(d, temperature_K=float("nan")), -1),
        (_bad(d, depth=-1), -1),
        (_bad(d, baths=bad_bath), -1),
        (_bad(d, baths=[dict(d["baths"][0], tau_fs=0.0)]), -1),
        (_bad(d, baths=[dict(d["baths"][0], lambda_cm=-1.0)]), -1),
        (_bad(d, H=np.array([[0.0, 1.0], [2.0, 0.0]])), -1),       # not Hermitian
        (_bad(d, H=np.array([[0.0, np.inf], [np.inf, 0.0]])), -1),
        (_bad(d, flags=1 << 8), -1),
        (_bad(d, H=np.zeros((65, 65)), baths=[]), -2),              # N > 64
        (_bad(d, depth=300), -2),
        (_bad(hi.fmo_like(), depth=40), -2),                        # n_ado >= 2^31
    ]
    for prob, code in cases:
        with pytest.raises(HeomError) as ei:
            heom.plan(prob)
        assert ei.value.status == code, prob
    lib = heom.load()
    assert lib.heom_last_error()  # message kept


def test_plan_rejects_matsubara_rate_equal_nu(heom):
    from paper_1803_03498_amd._abi import HeomError
    # gamma_1 = 2 pi k_B T / hbar equals nu for tau = 1/gamma_1
    beta = 1.0 / (0.6950348004 * 300.0 * 2 * np.pi * 2.99792458e-5)
    tau = beta / (2 * np.pi)
    p = _bad(hi.dimer(), baths=[{"state": 0, "lambda_cm": 35.0, "tau_fs": tau, "matsubara": 1}])
    with pytest.raises(HeomError):
        heom.plan(p)


def test_record_helpers(heom):
    lib = heom.load()
    assert lib.heom_record_doubles(7, 0) == 10
    assert lib.heom_record_doubles(7, 1) == 4
    assert lib.heom_record_count(1000, 1) == 1001
    assert lib.heom_record_count(1000, 10) == 101
    assert lib.heom_record_count(0, 3) == 1


def test_edge_sizes(heom):
    # no baths: a single ADO; depth 0: a single ADO
    p = {"H": np.array([[1.0]]), "baths": [], "temperature_K": 300.0, "depth": 3, "flags": 0}
    assert heom.plan(p)["n_ado"] == 1
    assert heom.plan(_bad(hi.dimer(), depth=0))["n_ado"] == 1


def test_spectrum_closed_form_and_oracle(heom, orc):
    # P(t) = exp(-i e t): trapezoid sum is a geometric series; and the library
    # agrees with the oracle's spectrum on random dipole correlations.
    two_pi_c = 2.0 * np.pi * 2.99792458e-5
    dt, n_t, e_cm = 1.0, 801, -23.0
    t = np.arange(n_t) * dt
    P = np.exp(-1j * e_cm * two_pi_c * t)
    w = np.linspace(-400.0, 400.0, 81)
    S = heom.spectrum(P[None, :], dt, w)
    r = np.exp(1j * (w - e_cm) * two_pi_c * dt)
    with np.errstate(divide="ignore", invalid="ignore"):
        geo = np.where(np.abs(r - 1) > 1e-15, (1 - r**n_t) / (1 - r), n_t)
    ref = ((geo - 0.5 * (1 + r ** (n_t - 1))) * dt).real
    assert np.max(np.abs(S - ref)) < 1e-9 * np.max(np.abs(ref))
    rng = np.random.default_rng(5)
    Pr = rng.normal(size=(3, 300)) + 1j * rng.normal(size=(3, 300))
    assert np.allclose(heom.spectrum(Pr, 2.0, w), orc.spectrum(Pr, 2.0, w), rtol=1e-12, atol=1e-12)


def test_bulk_kernel_choice(heom):
    # matrix cores for real H with N >= 16 (FP64 up to 48 states), FMA otherwise
    assert heom.plan(hi.aggregate48(), heom.FP32_MIXED)["bulk_kernel"] == 1
    assert heom.plan(hi.aggregate48(), heom.FP64)["bulk_kernel"] == 1
    assert heom.plan(hi.aggregate24(), heom.FP32_MIXED)["bulk_kernel"] == 1
    assert heom.plan(hi.fmo_like(), heom.FP32_MIXED)["bulk_kernel"] == 0
    big = _bad(hi.dimer(), H=np.eye(64), baths=[])
    assert heom.plan(big, heom.FP32_MIXED)["bulk_kernel"] == 1
    assert heom.plan(big, heom.FP64)["bulk_kernel"] == 0
    cplx = _bad(hi.aggregate24(), H=hi.aggregate24()["H"] * (1 + 0j))
    cplx["H"][0, 1] += 1j
    cplx["H"][1, 0] -= 1j
    assert heom.plan(cplx, heom.FP32_MIXED)["bulk_kernel"] == 0


def test_fp32_herm_plan(heom):
    # Hermitian-packed storage: N^2 reals per ADO, matrix-core path only
    from paper_1803_03498_amd._abi import HeomError
    for prob in (hi.aggregate24(), hi.aggregate48()):
        info = heom.plan(prob, heom.FP32_HERM)
        N = prob["H"].shape[0]
        assert info["elem_bytes"] == 4
        assert info["rest_bytes"] == (info["n_ado"] - 1) * N * N * 4
        assert info["sigma0_bytes"] == N * N * 16
        assert info["bulk_kernel"] == 1
    big = _bad(hi.dimer(), H=np.eye(64), baths=[])
    assert heom.plan(big, heom.FP32_HERM)["elem_bytes"] == 4
    cplx = _bad(hi.aggregate24(), H=hi.aggregate24()["H"] * (1 + 0j))
    cplx["H"][0, 1] += 1j
    cplx["H"][1, 0] -= 1j
    for prob in (hi.fmo_like(), hi.dimer(), cplx):
        with pytest.raises(HeomError) as ei:
            heom.plan(prob, heom.FP32_HERM)
        assert ei.value.status == -1


def test_pack_hermitian_layout(heom):
    rng = np.random.default_rng(11)
    x = rng.normal(size=(4, 6, 6)) + 1j * rng.normal(size=(4, 6, 6))
    x = (x + np.conj(np.swapaxes(x, 1, 2))) / 2
    P = heom.pack_hermitian(x)
    assert P.shape == x.shape and P.dtype == np.float64
    for i in range(6):
        for j in range(6):
            want = x[:, i, j].real if i <= j else x[:, j, i].imag
            assert np.array_equal(P[:, i, j], want)
    assert np.array_equal(heom.unpack_hermitian(P), x)


@pytest.mark.parametrize("pade", [False, True])
def test_problem_coefficients_match_oracle(heom, orc, pade):
    # host-only coefficients of the library (its own Pade eigensolver) against the oracle
    for T, M in ((300.0, 0), (300.0, 1), (77.0, 2), (30.0, 4), (30.0, 12)):
        baths = [{"state": 0, "lambda_cm": 35.0, "tau_fs": 50.0, "matsubara": M},
                 {"state": 1, "lambda_cm": 20.0, "tau_fs": 100.0, "matsubara": M},
                 {"state": 1, "lambda_cm": 50.0, "tau_fs": 30.0, "matsubara": M}]
        prob = {"H": np.diag([0.0, 100.0, 200.0]), "baths": baths, "temperature_K": T,
                "depth": 2, "flags": hi.FLAG_PADE if pade else 0}
        g, c, ln, ds = heom.problem_coefficients(prob)
        off, delta = 0, np.zeros(3)
        for b in baths:
            rg, rc, rln, rd = orc.bath_coefficients(b["lambda_cm"], b["tau_fs"], T, M, pade=pade)
            assert np.allclose(g[off:off + M + 1], rg, rtol=1e-13, atol=0)
            assert np.allclose(c[off:off + M + 1], rc, rtol=1e-12, atol=0)
            assert ln[off] == pytest.approx(rln, rel=1e-14)
            off += M + 1
            delta[b["state"]] += rd
        scale = np.max(np.abs(c))
        assert np.allclose(ds, delta, rtol=1e-10, atol=1e-12 * scale)


def test_pade_validation(heom):
    from paper_1803_03498_amd._abi import HeomError
    p = {"H": np.eye(2), "temperature_K": 300.0, "depth": 2, "flags": hi.FLAG_PADE,
         "baths": [{"state": 0, "lambda_cm": 35.0, "tau_fs": 50.0, "matsubara": 65}]}
    with pytest.raises(HeomError) as ei:
        heom.plan(p)
    assert ei.value.status == -2
    p["baths"][0]["matsubara"] = 64
    assert heom.plan(p)["n_modes"] == 65


def test_block_work_bytes(heom):
    # three copies of n_ado x N x 3 complex128, the records and a status word
    info = heom._info_struct(heom.plan(hi.fmo_like()))
    n = 3060 * 7 * 3 * 16
    copy = (n + 255) // 256 * 256
    rec = (1001 * 6 * 8 + 255) // 256 * 256
    assert heom.load().heom_block_work_bytes(ctypes.byref(info), 1000, 1) == 256 + 3 * copy + rec


def test_cd_vectors_match_oracle(heom, orc):
    rng = np.random.default_rng(4)
    R = rng.normal(size=(9, 3)) * 10
    d = rng.normal(size=(9, 3))
    assert np.allclose(heom.cd_vectors(R, d), orc.cd_vectors(R, d), rtol=1e-15, atol=1e-14)


def test_cd_vectors_literal_orientation(heom):
    # eq. CDdipoleoperator: m_p = (R_a x d_a) . e_p, with x cross y = z etc.
    R = np.array([[1.0, 0, 0], [0, 2.0, 0], [0, 0, 3.0], [4.0, 0, 0]])
    d = np.array([[0, 1.0, 0], [0, 0, 1.0], [1.0, 0, 0], [2.0, 0, 0]])
    assert np.array_equal(heom.cd_vectors(R, d), [[0, 2, 0, 0], [0, 0, 3, 0], [1, 0, 0, 0]])
