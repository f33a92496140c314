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


# ------------------------------------------------ coherence-block requests ----

def _absorption(seed, N, D, M, n_steps=60):
    rng = np.random.default_rng(seed)
    H = hi.fmo_like_hamiltonian(rng, N)
    dip = hi.unit_vectors(rng, N)
    baths = [{"state": s, "lambda_cm": 35.0, "tau_fs": 50.0, "matsubara": M} for s in range(N)]
    return hi.absorption_runs(H, dip, baths, 300.0, D, 1.0, n_steps)


def _block_problem(run):
    return {"H": np.asarray(run["H"])[1:, 1:], "temperature_K": run["temperature_K"],
            "depth": run["depth"], "flags": run.get("flags", 0),
            "baths": [dict(b, state=b["state"] - 1) for b in run["baths"]]}


@pytest.mark.parametrize("precision", [0, 1])
def test_block_form_requests(heom, orc, precision):
    # eligible absorption requests run in the coherence-block form (FP64 for
    # either request precision): the same records as heom_propagate_block bit
    # for bit, a zero trace, and the oracle's full-matrix correlations
    for seed, N, D, M in [(21, 3, 3, 1), (22, 6, 2, 1), (23, 12, 3, 0)]:
        _case("block request", precision, seed, N, D, M)
        runs = _absorption(seed, N, D, M)
        srv = heom.Server(ARENA, max_active=4)
        tb = srv.submit(runs, precision)
        tf = srv.submit(runs, precision, form=1)
        rb, rf = srv.wait(tb, 120.0), srv.wait(tf, 120.0)
        srv.close()
        assert rb["status"] == 0 and rf["status"] == 0
        assert rb["form"] == 2 and rf["form"] == 1
        assert np.all(rb["records"][:, :, 2:] == 0.0)
        P = rb["records"][:, :, 0] + 1j * rb["records"][:, :, 1]
        mu3 = np.stack([r["observable"]["mu"][1:] for r in runs])
        h = heom.Hierarchy(_block_problem(runs[0]), precision)
        P_direct = h.propagate_block(h.block_state(mu3), 1.0, runs[0]["n_steps"], 1, mu3).T
        assert np.array_equal(P, P_direct)
        P_full = rf["records"][:, :, 0] + 1j * rf["records"][:, :, 1]
        tol = 1e-12 if precision == 0 else 1e-5
        assert np.max(np.abs(P - P_full)) <= tol * max(1.0, np.max(np.abs(P)))
        if N <= 6:
            recs = [orc.run(r)[1] for r in runs]
            P_ref = np.stack([rec[:, 0] + 1j * rec[:, 1] for rec in recs])
            assert np.max(np.abs(P - P_ref)) <= 1e-12 * max(1.0, np.max(np.abs(P_ref)))


def test_block_form_eligibility(heom):
    # requests the block form cannot run stay on full matrices, with the same
    # correlations as heom_propagate
    runs = _absorption(31, 4, 3, 1, n_steps=40)
    bath_on_g = [dict(r, baths=r["baths"] + [{"state": 0, "lambda_cm": 20.0, "tau_fs": 80.0,
                                              "matsubara": 0}]) for r in runs]
    coupled = []
    for r in runs:
        H = np.array(r["H"])
        H[0, 2] = H[2, 0] = 15.0
        coupled.append(dict(r, H=H))
    diag_g = []
    for r in runs:
        rho0 = np.array(r["rho0"])
        rho0[0, 0] = 0.25
        diag_g.append(dict(r, rho0=rho0))
    unrotated = []
    for r in runs:
        H = np.array(r["H"])
        H[1:, 1:] += 5000.0 * np.eye(4)  # 0.94 rad per 1-fs step
        unrotated.append(dict(r, H=H))
    four = runs + [runs[0]]
    cases = [("eligible", runs, 2), ("bath on ground", bath_on_g, 1), ("ground coupled", coupled, 1),
             ("ground population", diag_g, 1), ("unrotated frame", unrotated, 1),
             ("four runs", four, 1)]
    srv = heom.Server(ARENA, max_active=8)
    tickets = [srv.submit(c, heom.FP64) for _, c, _ in cases]
    for (name, c, form), t in zip(cases, tickets):
        _case("eligibility", name)
        res = srv.wait(t, 120.0)
        assert res["status"] == 0, name
        assert res["form"] == form, name
        ref = _alone(heom, c, heom.FP64)
        assert np.max(np.abs(res["records"] - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref))), name
    srv.close()


# ------------------------------------------ matrix-core groups in the mix ----

def _population(seed, N, D, M, n_steps=20):
    rng = np.random.default_rng(seed)
    H = hi.fmo_like_hamiltonian(rng, N)
    baths = [{"state": s, "lambda_cm": 35.0, "tau_fs": 50.0, "matsubara": M} for s in range(N)]
    return [{"H": H, "baths": baths, "temperature_K": 300.0, "depth": D, "flags": 0,
             "dt_fs": 1.0, "n_steps": n_steps, "record_every": 1,
             "rho0": hi.population_rho0(N, N // 2), "observable": {"kind": "population"}}]


@pytest.mark.parametrize("precision", [0, 1])
def test_matrix_core_sizes_in_the_mix(heom, orc, precision):
    # N = 16, 17, 24, 33 (one, two and three 16-row blocks, ragged) beside
    # small FMA-path requests; in FP32 the 4845- and 7140-ADO runs get
    # launches of their own.  Mix and alone agree bit for bit, and
    # heom_propagate within the precision's tolerance; the FP64 mix matches
    # the oracle at 1e-12.
    specs = [(41, 16, 2, 0), (42, 17, 3, 0), (43, 24, 2, 0), (44, 33, 3, 0), (45, 16, 4, 0),
             (46, 5, 3, 1), (47, 9, 2, 1), (48, 3, 4, 1)]
    reqs = [_population(*s) for s in specs]
    srv = heom.Server(ARENA, max_active=8)
    tickets = [srv.submit(r, precision) for r in reqs]
    results = [srv.wait(t, 120.0) for t in tickets]
    srv.close()
    tol = 1e-12 if precision == 0 else 1e-5
    for s, r, res in zip(specs, reqs, results):
        _case("matrix-core mix", precision, s)
        assert res["status"] == 0
        one = heom.Server(ARENA, max_active=1)
        alone = one.wait(one.submit(r, precision), 120.0)
        one.close()
        assert np.array_equal(res["records"], alone["records"]), s
        ref = _alone(heom, r, precision)
        assert np.max(np.abs(res["records"] - ref)) <= tol, s
        assert np.max(np.abs(ref[0, -1, :s[1]] - ref[0, 0, :s[1]])) > 1e-4  # populations moved
        if precision == 0 and orc.sizes(r[0])[1] * s[1] ** 2 <= 2_000_000:
            # the FP64 mix against the oracle (all but the 7140-ADO N = 33 run,
            # which the oracle would take a minute for)
            _, rec_ref = orc.run(r[0])
            assert np.max(np.abs(res["records"][0] - rec_ref)) <= 1e-12, s


@pytest.mark.parametrize("precision", [0, 1])
def test_persistent_fma_requests_in_the_mix(heom, precision):
    # runs with N <= 16 and at least 32768 ADOs get launches of their own on
    # the persistent FMA kernel (the 74613- and 38760-ADO runs here) beside
    # batched small requests: mix and alone bit for bit, heom_propagate
    # within the precision's tolerance
    specs = [(81, 8, 6, 1), (82, 7, 6, 1), (83, 5, 3, 1), (84, 4, 2, 0)]
    reqs = []
    for s in specs:
        r = _population(*s, n_steps=12)
        r[0]["dt_fs"] = 0.5
        reqs.append(r)
    srv = heom.Server(ARENA, max_active=8)
    tickets = [srv.submit(r, precision) for r in reqs]
    results = [srv.wait(t, 120.0) for t in tickets]
    srv.close()
    tol = 1e-12 if precision == 0 else 1e-5
    for s, r, res in zip(specs, reqs, results):
        _case("persistent FMA mix", precision, s)
        assert res["status"] == 0
        one = heom.Server(ARENA, max_active=1)
        alone = one.wait(one.submit(r, precision), 120.0)
        one.close()
        assert np.array_equal(res["records"], alone["records"]), s
        ref = _alone(heom, r, precision)
        assert np.max(np.abs(res["records"] - ref)) <= tol, s


def test_request_log(heom, tmp_path):
    # one JSON line per finished request, with the form, sizes and timings
    import json
    path = tmp_path / "requests.jsonl"
    runs_b = _absorption(41, 4, 3, 1, n_steps=30)
    runs_f = _population(42, 5, 3, 1, n_steps=30)
    srv = heom.Server(ARENA, max_active=4)
    srv.set_log(path)
    tb, tf = srv.submit(runs_b, heom.FP32_MIXED), srv.submit(runs_f, heom.FP32_MIXED)
    rb, rf = srv.wait(tb, 120.0), srv.wait(tf, 120.0)
    srv.set_log(None)
    srv.close()
    lines = [json.loads(x) for x in path.read_text().splitlines()]
    by = {x["ticket"]: x for x in lines}
    assert set(by) == {tb, tf}
    assert by[tb]["form"] == "block" and by[tf]["form"] == "full"
    assert by[tb]["runs"] == 3 and by[tf]["runs"] == 1 and by[tf]["n_states"] == 5
    for t, res in ((tb, rb), (tf, rf)):
        x = by[t]
        assert x["status"] == 0 and x["n_steps"] == 30
        assert abs(x["latency_ms"] - 1e3 * (res["t_finish"] - res["t_submit"])) < 1e-2
        assert abs(x["queue_ms"] + x["service_ms"] - x["latency_ms"]) < 1e-2
