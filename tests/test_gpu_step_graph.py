"""heom_propagate replays a captured HIP graph of one RK4 step from the
second step on (runs of at least 8 steps, timing off).  The same
propagation with timing on launches every stage directly: records and final
state must agree bit for bit, on every replay of the graph, with the
program's own GPU work and synchronisations between the calls."""

import numpy as np
import pytest

import heom_inputs as hi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def heom():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1803_03498_amd as heom
    heom.load()
    return heom


def _case(*args):
    print("CASE", *args, flush=True)


def _cases():
    fmo = hi.fmo_like(n_steps=40)
    absn = hi.fmo_like_absorption(n_steps=40)[0]
    pop = lambda p, N: dict(p, dt_fs=0.5, n_steps=24, record_every=3,
                            rho0=hi.population_rho0(N, N // 2), observable={"kind": "population"})
    return [
        ("fmo_like FMA fp32", fmo, 1, True),
        ("fmo_like FMA fp64", fmo, 0, True),
        ("absorption FMA fp32 non-Hermitian", absn, 1, False),
        ("N=12 persistent fp32", pop(hi.random_problem(91, 12, M=1, D=2), 12), 1, True),
        ("N=20 MFMA fp64", pop(hi.random_problem(92, 20, M=0, D=2), 20), 0, True),
        ("N=8 D=6 persistent FMA fp32", pop(hi.random_problem(93, 8, M=1, D=6), 8), 1, True),
        ("aggregate24 packed fp32", dict(hi.aggregate24(n_steps=10), record_every=1), 2, True),
    ]


def _run(heom, run, precision, herm, timing):
    lib = heom.load()
    h = heom.Hierarchy(run, precision)
    st = h.new_state(run["rho0"])
    lib.heom_timing_enable(1 if timing else 0)
    try:
        rec = h.propagate(st, run["dt_fs"], run["n_steps"], run["record_every"],
                          run["observable"], hermitian=herm)
    finally:
        lib.heom_timing_enable(0)
        lib.heom_timing_read(None, None, None, 1)
    s0, rest = h.get_state(st)
    return rec, s0, rest


@pytest.mark.parametrize("name,run,precision,herm", _cases(), ids=[c[0] for c in _cases()])
def test_step_graph_matches_direct_launches(heom, name, run, precision, herm):
    import torch
    _case("step graph", name)
    assert run["n_steps"] >= 8
    direct = _run(heom, run, precision, herm, timing=True)
    assert np.all(np.isfinite(direct[0]))
    for rep in range(3):
        # the program's own work between the replays
        x = torch.randn(512, 512, device="cuda")
        (x @ x).sum().item()
        torch.cuda.synchronize()
        graphed = _run(heom, run, precision, herm, timing=False)
        assert all(np.array_equal(a, b) for a, b in zip(direct, graphed)), (name, rep)
