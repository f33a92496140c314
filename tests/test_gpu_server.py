"""Serving loop on the GPU: results are the same alone and in the mix, agree
with the oracle, and failures stay with their request."""

import numpy as np
import pytest

import heom_inputs as hi

pytestmark = pytest.mark.gpu

ARENA = 2 << 30


@pytest.fixture(scope="module")
def heom():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1803_03498_amd as heom
    heom.load()
    return heom


def _case(*args):
    print("CASE", *args, flush=True)


def _small_mix(n, n_steps, seed=512):
    """Requests of the serving mix, trimmed to small hierarchies."""
    reqs = []
    for r in hi.serving_mix(n_requests=n, seed=seed, n_steps=n_steps):
        for run in r["runs"]:
            run["depth"] = min(run["depth"], 3)
        reqs.append(r)
    return reqs


def _alone(heom, runs, precision):
    out = []
    for run in runs:
        h = heom.Hierarchy(run, precision)
        st = h.new_state(run["rho0"])
        herm = run["observable"]["kind"] == "population"
        out.append(h.propagate(st, run["dt_fs"], run["n_steps"], run["record_every"],
                               run["observable"], hermitian=herm))
    return np.stack(out)


@pytest.mark.parametrize("precision", [0, 1])
def test_alone_vs_mix_bit_identical(heom, precision):
    # every request served alone and in the mix: the same records bit for
    # bit; and against heom_propagate of the same runs (another kernel for
    # FP32 Hermitian runs) within the precision's tolerance
    _case("alone vs mix", precision)
    reqs = _small_mix(14, 40)
    srv = heom.Server(ARENA, max_active=8)
    tickets = [srv.submit(r["runs"], precision) for r in reqs]
    results = [srv.wait(t, 120.0) for t in tickets]
    srv.close()
    tol = 1e-12 if precision == 0 else 1e-5
    for r, res in zip(reqs, results):
        assert res["status"] == 0, (r["id"], res["status"])
        assert res["t_submit"] <= res["t_admit"] <= res["t_finish"]
        one = heom.Server(ARENA, max_active=1)
        alone = one.wait(one.submit(r["runs"], precision), 120.0)
        one.close()
        assert alone["status"] == 0
        assert np.array_equal(res["records"], alone["records"]), r["id"]
        ref = _alone(heom, r["runs"], precision)
        assert np.max(np.abs(res["records"] - ref)) <= tol, r["id"]


def test_mix_matches_oracle(heom, orc):
    _case("mix vs oracle")
    reqs = [r for r in _small_mix(40, 30) if r["N"] <= 6][:4]
    assert reqs
    srv = heom.Server(ARENA, max_active=4)
    tickets = [srv.submit(r["runs"], heom.FP64) for r in reqs]
    for r, t in zip(reqs, tickets):
        res = srv.wait(t, 120.0)
        assert res["status"] == 0
        for k, run in enumerate(r["runs"]):
            _, rec = orc.run(run)
            assert np.max(np.abs(res["records"][k] - rec)) <= 1e-12
    srv.close()


def test_submit_validation_and_nomem(heom):
    from paper_1803_03498_amd._abi import HeomError
    srv = heom.Server(64 << 20, max_active=2)
    big = hi.aggregate24(n_steps=5)
    with pytest.raises(HeomError) as ei:
        srv.submit([big], heom.FP32_MIXED)
    assert ei.value.status == -3   # can never fit a 64 MiB arena
    bad = dict(hi.dimer(n_steps=5), temperature_K=-1.0)
    with pytest.raises(HeomError) as ei:
        srv.submit([bad], heom.FP64)
    assert ei.value.status == -1
    unstable = dict(hi.dimer(n_steps=5), dt_fs=500.0)
    with pytest.raises(HeomError) as ei:
        srv.submit([unstable], heom.FP64)
    assert ei.value.status == -6
    srv.close()


def test_numeric_failure_is_isolated(heom):
    _case("numeric isolation")
    reqs = _small_mix(6, 20)
    poisoned = [dict(run) for run in reqs[2]["runs"]]
    for run in poisoned:
        run["rho0"] = np.full_like(run["rho0"], np.inf)
    srv = heom.Server(ARENA, max_active=8)
    tickets = []
    for i, r in enumerate(reqs):
        tickets.append(srv.submit(poisoned if i == 2 else r["runs"], heom.FP32_MIXED))
    results = [srv.wait(t, 120.0) for t in tickets]
    srv.close()
    assert results[2]["status"] == -5
    for i, (r, res) in enumerate(zip(reqs, results)):
        if i == 2:
            continue
        assert res["status"] == 0
        one = heom.Server(ARENA, max_active=1)
        alone = one.wait(one.submit(r["runs"], heom.FP32_MIXED), 120.0)
        one.close()
        assert np.array_equal(res["records"], alone["records"])


def test_cancel_and_queueing(heom):
    _case("cancel and queueing")
    reqs = _small_mix(6, 30)
    long_run = [dict(run, n_steps=200000) for run in hi.fmo_like_absorption(n_steps=10)[:1]]
    srv = heom.Server(ARENA, max_active=2)
    t_long = srv.submit(long_run, heom.FP32_MIXED)
    tickets = [srv.submit(r["runs"], heom.FP32_MIXED) for r in reqs]
    srv.cancel(t_long)
    res_long = srv.wait(t_long, 120.0)
    assert res_long["status"] == -8
    results = [srv.wait(t, 120.0) for t in tickets]
    assert all(res["status"] == 0 for res in results)
    # FIFO admission with two slots
    admits = [res["t_admit"] for res in results]
    assert admits == sorted(admits)
    for t in tickets:
        srv.release(t)
    srv.close()
