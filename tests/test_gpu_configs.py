"""Parity of whole propagations at the sizes the benchmark times, and the
degenerate cases of the method, on the GPU against the FP64 oracle.

* 24-site aggregate (20475 ADOs of 24x24, depth 4): the oracle's first 10
  RK4 steps (tests/golden/aggregate24_prefix_*.txt, written by
  make_oracle_golden.py from the oracle alone) against the GPU in FP64 and
  FP32-mixed; then the full 1000 steps of FP32-mixed against the GPU FP64 run.
* 48-site aggregate (156849 ADOs of 48x48, 96 modes, depth 3): the oracle's
  first 2 steps (aggregate48_prefix_*.txt); the full 500 steps of FP32-mixed
  against the GPU FP64 run.
* lambda = 0 (every bath weight zero: unitary sigma_0), no baths (W = 0),
  depth 0 (sigma_0 alone with the correction term), and a bath whose first
  Matsubara weight is negative (10 K), on both kernel families.

Tolerances: populations 1e-12 (FP64) and 1e-5 (FP32-mixed) absolute.  Sampled
ADO elements (row 0 and the diagonal of ADOs from every level): FP64 within
1e-11 of the ADO's largest sampled element, FP32-mixed within 1e-4 of it: an
FP32 stage rounds every stored element once (relative 6e-8), 40 stages in 10
steps give ~2.4e-6, and the couplings mix ADOs of comparable scale; 1e-4 leaves
room for cancellation inside an element.
"""

import os

import numpy as np
import pytest

import heom_inputs as hi

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def heom():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1803_03498_amd as heom
    heom.load()
    return heom


def _case(*args):
    print("CASE", *args, flush=True)


def _prefix(name):
    rec = np.loadtxt(os.path.join(HERE, "golden", name + "_prefix_records.txt"))
    ados = np.loadtxt(os.path.join(HERE, "golden", name + "_prefix_ados.txt"))
    return rec, ados


def _ado(st, u):
    """Host complex128 copy of ADO u of a device state (u >= 1)."""
    return st[1][u - 1].cpu().numpy().astype(np.complex128)


def _ado_errors(st, ados):
    """Largest |gpu - oracle| per sampled ADO and that ADO's largest element."""
    errs = {}
    for u in np.unique(ados[:, 0]).astype(int):
        sel = ados[ados[:, 0] == u]
        ref = sel[:, 3] + 1j * sel[:, 4]
        k = sel[:, 2].astype(int)
        a = _ado(st, u)
        got = np.where(sel[:, 1] == 0, a[0, k], a[k, k])
        errs[u] = (float(np.max(np.abs(got - ref))), float(np.max(np.abs(ref))))
    return errs


def _check_prefix(heom, name, prob, steps, precision):
    rec_ref, ados = _prefix(name)
    assert len(rec_ref) == steps + 1
    N = prob["H"].shape[0]
    h = heom.Hierarchy(prob, precision)
    st = h.new_state(prob["rho0"])
    rec = h.propagate(st, prob["dt_fs"], steps, 1, prob["observable"], hermitian=True)
    pop_tol = 1e-12 if precision == 0 else 1e-5
    assert np.max(np.abs(rec[:, :N] - rec_ref[:, 1:N + 1])) <= pop_tol
    assert np.max(np.abs(rec[:, N] - 1.0)) <= 1e-12
    rel = 1e-11 if precision == 0 else 1e-4
    worst = 0.0
    for u, (err, scale) in _ado_errors(st, ados).items():
        assert err <= rel * scale + 1e-300, (u, err, scale)
        worst = max(worst, err / max(scale, 1e-300))
    print("  worst ADO relative error %.3e" % worst, flush=True)


@pytest.mark.parametrize("precision", [0, 1])
def test_aggregate24_oracle_prefix(heom, precision):
    _case("aggregate24 10-step oracle prefix", precision)
    _check_prefix(heom, "aggregate24", hi.aggregate24(), 10, precision)


@pytest.mark.parametrize("precision", [0, 1])
def test_aggregate48_oracle_prefix(heom, precision):
    _case("aggregate48 2-step oracle prefix", precision)
    _check_prefix(heom, "aggregate48", hi.aggregate48(), 2, precision)


@pytest.mark.parametrize("name,steps", [("aggregate24", 1000), ("aggregate48", 500)])
def test_aggregate_fp32_full_run_tracks_fp64(heom, name, steps):
    _case(name, "full run FP32-mixed vs FP64", steps)
    prob = getattr(hi, name)(n_steps=steps)
    N = prob["H"].shape[0]
    recs = []
    for precision in (0, 1):
        h = heom.Hierarchy(prob, precision)
        st = h.new_state(prob["rho0"])
        recs.append(h.propagate(st, prob["dt_fs"], steps, prob["record_every"],
                                prob["observable"], hermitian=True))
        del st, h
    err = np.max(np.abs(recs[1][:, :N] - recs[0][:, :N]))
    print("  max population difference %.3e" % err, flush=True)
    assert err <= 1e-5
    assert np.max(np.abs(recs[1][:, N] - 1.0)) <= 1e-12
    # the populations have moved: the comparison is not between two idle runs
    assert np.max(np.abs(recs[0][-1, :N] - recs[0][0, :N])) > 1e-2


# ------------------------------------------------------- degenerate cases ----

def _edge_problems():
    # N = 16 takes the matrix-core kernels, N <= 5 the FMA kernel
    lam0 = hi.random_problem(31, 16, M=0, D=2)
    for b in lam0["baths"]:
        b["lambda_cm"] = 0.0
    lam0_small = hi.random_problem(32, 4, M=1, D=3)
    for b in lam0_small["baths"]:
        b["lambda_cm"] = 0.0
    nobath = dict(hi.random_problem(33, 16, M=0, D=3), baths=[])
    nobath_small = dict(hi.random_problem(34, 5, M=0, D=3), baths=[])
    depth0 = hi.random_problem(35, 16, M=1, D=0)
    depth0_small = hi.random_problem(36, 3, M=1, D=0)
    cold = hi.random_problem(37, 16, n_baths=8, M=1, D=2, T=10.0)
    cold_small = hi.random_problem(38, 4, M=1, D=3, T=10.0)
    for p in (cold, cold_small):
        for b in p["baths"]:
            b["tau_fs"] = 20.0  # first Matsubara rate below nu: c_1 < 0
    return [("lambda0_N16", lam0), ("lambda0_N4", lam0_small), ("nobath_N16", nobath),
            ("nobath_N5", nobath_small), ("depth0_N16", depth0), ("depth0_N3", depth0_small),
            ("negative_c_N16", cold), ("negative_c_N4", cold_small)]


_ORACLE_RUNS = {}


@pytest.mark.parametrize("name,prob", _edge_problems(), ids=[n for n, _ in _edge_problems()])
@pytest.mark.parametrize("precision", [0, 1])
def test_degenerate_cases_match_oracle(heom, orc, name, prob, precision):
    _case("edge", name, precision)
    N = prob["H"].shape[0]
    if name.startswith("negative_c"):
        g, c, _, _ = orc.bath_coefficients(20.0, 20.0, 10.0, 1)
        assert c[1] < 0
    # dt = 0.2 fs: with lambda = 0 the rescaled "+" weights sqrt(n + 1) (|c| taken
    # as 1) enter the step-size guard although those couplings never act
    run = dict(prob, dt_fs=0.2, n_steps=250, record_every=5, rho0=hi.population_rho0(N, N - 1),
               observable={"kind": "population"})
    if name not in _ORACLE_RUNS:
        _ORACLE_RUNS[name] = orc.run(run)[1]
    rec_ref = _ORACLE_RUNS[name]
    h = heom.Hierarchy(run, precision)
    st = h.new_state(run["rho0"])
    rec = h.propagate(st, run["dt_fs"], run["n_steps"], run["record_every"], run["observable"],
                      hermitian=True)
    tol = 1e-12 if precision == 0 else 1e-5
    assert np.max(np.abs(rec[:, :N] - rec_ref[:, :N])) <= tol
    assert np.max(np.abs(rec[:, N] - 1.0)) <= 1e-12
    assert np.max(np.abs(rec_ref[-1, :N] - rec_ref[0, :N])) > 1e-3  # something happened
