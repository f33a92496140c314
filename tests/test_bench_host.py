"""Host-side checks of the benchmark's bookkeeping (no GPU): the table bytes
it reports next to the roofline, the serving leg's error summary and the
oracle's timing entry used by the serving leg's CPU baseline."""

import os
import sys

import numpy as np
import pytest

import heom_inputs as hi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("W,D", [(6, 3), (14, 4), (4, 1), (5, 0)])
def test_table_bytes_count_the_oracle_tables(orc, W, D):
    # n_low (the ADOs u >= 1 below the top level, the ones with "+" links)
    # counted from the oracle's own enumeration, against the closed form
    # the benchmark uses
    _, plus, _, lev = orc.tables(W, D)
    n = len(lev)
    n_low = int(np.sum((lev >= 1) & (lev <= D - 1)))
    assert np.all(plus[lev == D] == -1)  # the top level has no "+" links
    Dm = max(D, 1)
    for fp64, wb in ((False, 8), (True, 16)):
        want = (n - 1) * (Dm * (8 + 4 + wb) + 8) + n_low * W * 12
        assert bench._table_bytes_per_launch("k_stage_persist", n, W, D, fp64) == want
    assert (bench._table_bytes_per_launch("k_bulk_mfma", n, W, D, True)
            == bench._table_bytes_per_launch("k_stage_small", n, W, D, True) + (n - 1))


def _serve_req(rid, kind, N):
    run = {"H": np.zeros((N, N)), "dt_fs": 1.0, "record_every": 2}
    return {"id": rid, "kind": kind, "runs": [run] * (1 if kind == "population" else 3)}


def test_serve_accuracy_summary():
    import paper_1803_03498_amd as heom
    rng = np.random.default_rng(3)
    N, n_rec = 4, 51
    pop = rng.standard_normal((1, n_rec, N + 3))
    pop[..., N] = 1.0
    pop[..., N + 2] = 0.0
    t = np.arange(n_rec) * 2.0
    P = np.exp(-t / 40.0) * np.exp(1j * 0.01 * t)
    ab = np.zeros((3, n_rec, 4))
    ab[:, :, 0], ab[:, :, 1] = P.real, P.imag
    reqs = [_serve_req(0, "population", N), _serve_req(1, "absorption", N)]
    ref = {0: pop, 1: ab}
    out = bench._serve_accuracy(heom, reqs, {0: pop.copy(), 1: ab.copy()}, ref)
    assert out["requests_compared"] == 2
    for k in ("max_population_error", "max_trace_drift", "max_hermiticity_residual",
              "max_dipole_response_error", "max_spectrum_rel_error"):
        assert out[k] == 0.0, k
    got_pop = pop.copy()
    got_pop[0, 7, 2] += 3e-6
    got_pop[0, 9, N] += 2e-7
    got_pop[0, 4, N + 2] = 5e-8
    got_ab = ab.copy()
    got_ab[1, 10, 0] += 1e-5
    out = bench._serve_accuracy(heom, reqs, {0: got_pop, 1: got_ab}, ref)
    assert out["max_population_error"] == pytest.approx(3e-6, rel=1e-9)
    assert out["max_trace_drift"] == pytest.approx(2e-7, rel=1e-6)
    assert out["max_hermiticity_residual"] == 5e-8
    assert out["max_dipole_response_error"] == pytest.approx(1e-5, rel=1e-9)
    # one record of one direction moved by 1e-5 against |S| of order
    # sum_p sum_n |P| dt: a small, positive relative error
    assert 0.0 < out["max_spectrum_rel_error"] < 1e-5
    # a request missing on either side is not compared
    out = bench._serve_accuracy(heom, reqs, {0: pop}, ref)
    assert out["requests_compared"] == 1 and out["absorption_requests"] == 0


def test_oracle_step_timing_leaves_state_and_counts_work(orc):
    prob = hi.dimer()
    _, n = orc.sizes(prob)
    N = prob["H"].shape[0]
    rng = np.random.default_rng(5)
    x = rng.standard_normal((n, N, N)) + 1j * rng.standard_normal((n, N, N))
    keep = x.copy()
    full = orc.time_step_sample(prob, x, 1.0, 0, n, 1, 3)
    half = orc.time_step_sample(prob, x, 1.0, 0, n, 2, 3)
    assert full > 0.0 and half > 0.0
    assert np.array_equal(x, keep)
    with pytest.raises(ValueError):
        orc.time_step_sample(prob, x, 1.0, 0, n, 0, 1)


def test_oracle_request_seconds_small_request():
    r = hi.serving_mix(n_requests=4, seed=512, n_steps=1000)[0]
    sec, stride = bench._oracle_request_seconds((r["runs"], 1000, 0.5))
    assert stride == 1  # a small request is timed over all of its ADOs
    assert sec > 0.0


def test_serve_cpu_baseline_summary():
    # requests/s of P cores each running whole requests one after another:
    # P / mean request time, over the first n requests only
    cpu = {"seconds": [10.0, 30.0, 20.0, 1000.0], "steps_timed": [1, 1, 5, 1],
           "procs": 4, "budget_s": 1.5, "wall_s": 3.0}
    out = bench._serve_cpu_baseline(cpu, 3)
    assert out["value"] == pytest.approx(4 / 20.0)
    assert out["cores"] == 4 and out["unit"] == "req/s" and out["kind"] == "oracle"
    assert out["p50_request_s_one_core"] == pytest.approx(20.0)
    assert "first 3 requests" in out["sample"]
    # asking for more requests than were timed uses those that were
    assert bench._serve_cpu_baseline(cpu, 10)["value"] == pytest.approx(4 / 265.0)


def test_cpu_baseline_dimer():
    out = bench.cpu_baseline(hi.dimer(), 0.2)
    assert out["value"] > 0.0 and out["cores"] == 1 and out["kind"] == "oracle"
    assert "every ADO of dimer" in out["sample"]
