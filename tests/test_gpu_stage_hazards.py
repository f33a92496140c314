"""Stage hazards and launch-shape independence of the RK4 stage kernels.

* Poison: before a propagation every byte of its workspace (the three RK4
  stage copies, the control block and the records) is set to 0xFF, a NaN in
  FP32 and in FP64.  A stage that read a copy before an earlier stage of the
  same step wrote it would carry the NaNs (or other values) into the result:
  records and final state must equal, bit for bit, those of the run with a
  zeroed workspace.
* Launch shape: the same propagation with the persistent kernel held to a
  few workers (each walks many more tiles, in another order) and the FMA
  kernel to one ADO per workgroup gives the same records and state bit for
  bit: no result depends on which workgroup computes which element.

Cases cover every stage kernel: FMA (FP32 and FP64, Hermitian and not,
complex H), the persistent FMA kernel (FP32, FP64 non-Hermitian), MFMA
(FP64, FP32 non-Hermitian), the persistent MFMA kernel (one, two and three
16-row blocks), the Hermitian-packed kernel and the coherence-block form.
"""

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
    fmo = hi.fmo_like(n_steps=6)
    absn = hi.fmo_like_absorption(n_steps=6)[0]
    agg24 = hi.aggregate24(n_steps=3)
    r16 = hi.random_problem(61, 16, M=0, D=3)
    r20 = hi.random_problem(62, 20, M=0, D=2)
    r33 = hi.random_problem(63, 33, M=0, D=2)
    r12 = hi.random_problem(64, 12, M=1, D=2)
    r9c = hi.random_problem(65, 9, M=1, D=2, complex_h=True)
    r8 = hi.random_problem(67, 8, M=1, D=6)     # 74613 ADOs: persistent FMA kernel
    r7 = hi.random_problem(68, 7, M=1, D=6)     # 38760 ADOs
    r18c = hi.random_problem(66, 18, M=0, D=2, complex_h=True)
    pop = lambda p, N: dict(p, dt_fs=0.5, n_steps=5, record_every=1,
                            rho0=hi.population_rho0(N, N // 2), observable={"kind": "population"})
    # (name, run, precision, hermitian)
    return [
        ("fmo_like FMA fp32", fmo, 1, True),
        ("fmo_like FMA fp64", fmo, 0, True),
        ("absorption FMA fp32 non-Hermitian", absn, 1, False),
        ("absorption FMA fp64 non-Hermitian", absn, 0, False),
        ("N=9 complex H FMA fp32", pop(r9c, 9), 1, True),
        ("N=18 complex H FMA fp64", pop(r18c, 18), 0, True),
        ("N=8 D=6 persistent FMA fp32", pop(r8, 8), 1, True),
        ("N=7 D=6 persistent FMA fp64 non-Hermitian", pop(r7, 7), 0, False),
        ("N=16 MFMA fp64", pop(r16, 16), 0, True),
        ("N=20 MFMA fp32 non-Hermitian", pop(r20, 20), 1, False),
        ("N=12 persistent fp32", pop(r12, 12), 1, True),
        ("aggregate24 persistent fp32", agg24, 1, True),
        ("N=33 persistent fp32", pop(r33, 33), 1, True),
        ("aggregate24 packed fp32", agg24, 2, True),
    ]


def _run(heom, run, precision, herm, fill):
    import torch
    h = heom.Hierarchy(run, precision)
    st = h.new_state(run["rho0"])
    obs = run["observable"]
    kind = 0 if obs["kind"] == "population" else 1
    work = h.workspace(run["n_steps"], run["record_every"], kind)
    work.fill_(fill)
    torch.cuda.synchronize()
    rec = h.propagate(st, run["dt_fs"], run["n_steps"], run["record_every"], obs,
                      hermitian=herm, work=work)
    s0, rest = h.get_state(st)
    return rec, s0, rest


def _same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("name,run,precision,herm", _cases(), ids=[c[0] for c in _cases()])
def test_poisoned_workspace_and_launch_shape(heom, name, run, precision, herm):
    _case("hazards", name)
    ref = _run(heom, run, precision, herm, 0)
    assert np.all(np.isfinite(ref[0]))
    poisoned = _run(heom, run, precision, herm, 255)
    assert _same(ref, poisoned), name
    try:
        heom.set_launch_shape(max_workgroups=3, max_ados_per_tile=1)
        shaped = _run(heom, run, precision, herm, 255)
    finally:
        heom.set_launch_shape(0, 0)
    assert _same(ref, shaped), name


def test_block_form_poisoned_workspace(heom):
    import torch
    _case("hazards block form")
    runs = hi.fmo_like_absorption(n_steps=20)
    prob = {"H": np.asarray(runs[0]["H"])[1:, 1:], "temperature_K": runs[0]["temperature_K"],
            "depth": runs[0]["depth"], "flags": 0,
            "baths": [dict(b, state=b["state"] - 1) for b in runs[0]["baths"]]}
    mu3 = np.stack([r["observable"]["mu"][1:] for r in runs])
    h = heom.Hierarchy(prob, heom.FP64)
    out = []
    for fill in (0, 255):
        info = h.info
        work = torch.full((1 << 26,), fill, dtype=torch.uint8, device="cuda")
        y = h.block_state(mu3)
        P = h.propagate_block(y, 1.0, 20, 1, mu3, work=work)
        out.append((P, y.cpu().numpy()))
        del info
    assert np.all(np.isfinite(out[0][0]))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
