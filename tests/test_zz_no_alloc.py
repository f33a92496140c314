"""heom_propagate_noalloc (workspace in the library's static device scratch)
against heom_propagate with a caller workspace: the same kernels on the same
inputs, so records and final states must agree bit for bit.  Two calls in a
row, the second on a smaller problem, so a stale scratch would show."""

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


def _run_both(heom, prob, precision, observable=None, hermitian=True):
    print("CASE noalloc", prob.get("name", "?"), precision, prob["H"].shape[0], flush=True)
    h = heom.Hierarchy(prob, precision)
    obs = observable or prob["observable"]
    a = h.new_state(prob["rho0"])
    rec_a = h.propagate(a, prob["dt_fs"], prob["n_steps"], prob["record_every"], obs,
                        hermitian=hermitian)
    b = h.new_state(prob["rho0"])
    rec_b = h.propagate_noalloc(b, prob["dt_fs"], prob["n_steps"], prob["record_every"], obs,
                                hermitian=hermitian)
    assert rec_a.shape == rec_b.shape
    assert np.array_equal(rec_a, rec_b)
    assert np.array_equal(h.state_to_numpy(a), h.state_to_numpy(b))
    assert np.all(np.isfinite(rec_a))
    return rec_b


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_matches_propagate_two_calls(heom, precision):
    big = dict(hi.fmo_like(n_steps=40), record_every=4)      # 3060 ADOs of 7x7
    small = dict(hi.dimer(n_steps=30), record_every=1)        # 10 ADOs of 2x2
    r1 = _run_both(heom, big, precision)
    r2 = _run_both(heom, small, precision)
    assert r1.shape[1] == 7 + 3 and r2.shape[1] == 2 + 3
    assert abs(r2[0, 0] - 1.0) < 1e-15   # the second call recorded its own start


def test_noalloc_dipole_observable(heom):
    run = hi.fmo_like_absorption(n_steps=30)[1]
    run["depth"] = 2
    _run_both(heom, run, 1, hermitian=False)


def test_noalloc_refuses_oversized_workspace(heom):
    prob = hi.aggregate24(n_steps=2)                          # 94 MB per FP32 stage copy
    h = heom.Hierarchy(prob, 1)
    st = h.new_state(prob["rho0"])
    with pytest.raises(heom.HeomError) as e:
        h.propagate_noalloc(st, 1.0, 2, 1)
    assert e.value.status == -3 and "static scratch" in str(e.value)
