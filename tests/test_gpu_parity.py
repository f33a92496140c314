"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances: integer tables bit-exact; FP64 right-hand side within 1e-12 of the
largest output element; FP64 propagation within 1e-12 absolute on
populations; FP32-mixed propagation within 1e-5 absolute on populations.
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


def _print_case(*args):
    print("CASE", *args, flush=True)


def _modes_problem(W, D, N=3):
    """W single-mode baths spread over N states (for table checks)."""
    H = np.diag(np.arange(N, dtype=float) * 30.0)
    baths = [{"state": l % N, "lambda_cm": 20.0, "tau_fs": 60.0, "matsubara": 0} for l in range(W)]
    return {"H": H, "baths": baths, "temperature_K": 300.0, "depth": D, "flags": 0}


# ---------------------------------------------------------------- tables ----

@pytest.mark.parametrize("W,D", [(1, 5), (2, 3), (5, 3), (14, 4), (24, 4), (28, 5), (96, 3),
                                 (7, 6), (3, 0)])
def test_tables_bit_exact(heom, orc, W, D):
    _print_case("tables", W, D)
    h = heom.Hierarchy(_modes_problem(W, D))
    t, p, m, lev = h.tables()
    rt, rp, rm, rlev = orc.tables(W, D)
    assert h.n_ado == len(rt)
    assert np.array_equal(t, rt)
    assert np.array_equal(p, rp)
    assert np.array_equal(m, rm)
    assert np.array_equal(lev.astype(np.int32), rlev)


def test_coefficients_match_oracle(heom, orc):
    for prob in (hi.dimer(), hi.fmo_like(), hi.aggregate24(), hi.random_problem(1, 4, M=3, D=1),
                 hi.fmo_like_pade(30.0, 3, 3)):
        h = heom.Hierarchy(prob)
        g, c, ln, ds = h.coefficients()
        off = 0
        pade = bool(prob.get("flags", 0) & hi.FLAG_PADE)
        for b in prob["baths"]:
            rg, rc, rln, rd = orc.bath_coefficients(b["lambda_cm"], b["tau_fs"],
                                                    prob["temperature_K"], b["matsubara"], pade)
            K = b["matsubara"] + 1
            assert np.allclose(g[off:off + K], rg, rtol=1e-15, atol=0)
            assert np.allclose(c[off:off + K], rc, rtol=1e-14, atol=0)
            assert ln[off] == pytest.approx(rln, rel=1e-15)
            off += K


# ------------------------------------------------------------------- RHS ----

RHS_CASES = [
    # (seed, N, n_baths, M, D, extra)
    (1, 1, 1, 1, 3, {}),
    (2, 2, 2, 0, 4, {}),
    (3, 3, 3, 1, 3, {}),
    (4, 5, 5, 1, 2, {}),
    (5, 7, 7, 1, 2, {}),
    (6, 8, 4, 2, 2, {}),
    (7, 12, 12, 0, 2, {}),
    (8, 16, 16, 0, 2, {}),
    (9, 17, 17, 0, 2, {}),
    (10, 24, 24, 0, 1, {}),
    (11, 31, 8, 1, 2, {}),
    (12, 40, 40, 0, 1, {}),
    (13, 48, 48, 0, 1, {}),
    (14, 64, 64, 0, 1, {}),
    (15, 6, 3, 1, 3, {"complex_h": True}),
    (16, 5, 5, 1, 2, {"flags": 1}),
    (17, 5, 5, 1, 2, {"flags": 2}),
    (18, 5, 5, 1, 2, {"flags": 4}),
    (19, 5, 5, 1, 2, {"flags": 8}),
    (20, 4, 6, 1, 2, {}),       # several baths on one state
    # matrix-core path corner cases: an odd number of bulk tiles (two ADOs
    # per FP32 workgroup leave one half idle), three modes per state (more
    # "+" modes than are loaded ahead), depth 5 (more "-" links than are
    # staged as rows)
    (21, 40, 39, 0, 1, {}),
    (22, 44, 17, 1, 2, {}),
    (23, 40, 10, 2, 2, {}),
    (24, 20, 3, 1, 5, {}),
    (25, 40, 3, 1, 5, {}),
    (26, 14, 14, 1, 3, {}),     # the serving mix's largest N on the FMA path
    # Pade modes (only the coefficients differ): FMA and matrix-core paths
    (27, 5, 5, 2, 2, {"flags": 16}),
    (28, 7, 7, 3, 3, {"flags": 16}),
    (29, 24, 24, 1, 2, {"flags": 16}),
]
FP32_CASES = RHS_CASES[:14] + RHS_CASES[20:]


def _rhs_problem(seed, N, nb, M, D, extra):
    p = hi.random_problem(seed, N, n_baths=nb, M=M, D=D, complex_h=extra.get("complex_h", False))
    p["flags"] = extra.get("flags", 0)
    return p


@pytest.mark.parametrize("case", RHS_CASES, ids=[f"N{c[1]}_B{c[2]}_M{c[3]}_D{c[4]}_{c[0]}"
                                                 for c in RHS_CASES])
@pytest.mark.parametrize("herm", [False, True])
def test_rhs_fp64(heom, orc, case, herm):
    seed, N, nb, M, D, extra = case
    _print_case("rhs fp64", case, herm)
    prob = _rhs_problem(seed, N, nb, M, D, extra)
    h = heom.Hierarchy(prob, heom.FP64)
    x = hi.random_state(100 + seed, h.n_ado, N, hermitian=herm)
    ref = orc.rhs(prob, x)
    out = h.new_state()
    h.rhs(h.state_from_numpy(x), out, hermitian=herm)
    got = h.state_to_numpy(out)
    err = np.max(np.abs(got - ref))
    assert err <= 1e-12 * np.max(np.abs(ref)), err


@pytest.mark.parametrize("case", FP32_CASES, ids=[f"N{c[1]}_B{c[2]}_M{c[3]}_D{c[4]}_{c[0]}"
                                                  for c in FP32_CASES])
@pytest.mark.parametrize("herm", [True, False])
def test_rhs_fp32_mixed(heom, orc, case, herm):
    seed, N, nb, M, D, extra = case
    _print_case("rhs fp32", case, herm)
    prob = _rhs_problem(seed, N, nb, M, D, extra)
    h = heom.Hierarchy(prob, heom.FP32_MIXED)
    x = hi.random_state(200 + seed, h.n_ado, N, hermitian=herm)
    x[1:] = x[1:].astype(np.complex64)  # the oracle sees the same FP32 inputs
    ref = orc.rhs(prob, x)
    out = h.new_state()
    h.rhs(h.state_from_numpy(x), out, hermitian=herm)
    got = h.state_to_numpy(out)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(got[0] - ref[0])) <= 1e-6 * scale  # sigma_0 row: FP64 arithmetic
    assert np.max(np.abs(got - ref)) <= 1e-5 * scale


# Hermitian-packed FP32 storage: real H, N >= 16 (the matrix-core path)
PK_CASES = [c for c in RHS_CASES if c[1] >= 16 and not c[5].get("complex_h")]


@pytest.mark.parametrize("case", PK_CASES, ids=[f"N{c[1]}_B{c[2]}_M{c[3]}_D{c[4]}_{c[0]}"
                                                for c in PK_CASES])
def test_rhs_fp32_herm(heom, orc, case):
    seed, N, nb, M, D, extra = case
    _print_case("rhs fp32 packed", case)
    prob = _rhs_problem(seed, N, nb, M, D, extra)
    h = heom.Hierarchy(prob, heom.FP32_HERM)
    x = hi.random_state(300 + seed, h.n_ado, N, hermitian=True)
    # the oracle sees the same FP32 inputs
    x[1:] = heom.unpack_hermitian(heom.pack_hermitian(x[1:]).astype(np.float32))
    ref = orc.rhs(prob, x)
    out = h.new_state()
    assert out[1].dtype.itemsize == 4
    h.rhs(h.state_from_numpy(x), out, hermitian=True)
    got = h.state_to_numpy(out)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(got[0] - ref[0])) <= 1e-6 * scale
    assert np.max(np.abs(got - ref)) <= 1e-5 * scale


@pytest.mark.parametrize("case", [c for c in PK_CASES if c[0] in (8, 11, 22, 24, 25)],
                         ids=lambda c: f"N{c[1]}_D{c[4]}_{c[0]}")
def test_propagate_fp32_herm_matches_fp32_mixed(heom, case):
    # propagation keeps complex copies of the lower levels for the "-" rows;
    # the packed run must track the complex FP32 run on every ADO
    seed, N, nb, M, D, extra = case
    _print_case("propagate fp32 packed vs complex", case)
    prob = _rhs_problem(seed, N, nb, M, D, extra)
    finals = []
    for prec in (heom.FP32_MIXED, heom.FP32_HERM):
        h = heom.Hierarchy(prob, prec)
        x = hi.random_state(400 + seed, h.n_ado, N, hermitian=True, scale=0.05)
        x[0] = np.eye(N) / N
        x[1:] = heom.unpack_hermitian(heom.pack_hermitian(x[1:]).astype(np.float32))
        st = h.state_from_numpy(x)
        rec = h.propagate(st, 0.25, 12, 3, hermitian=True)
        assert np.all(np.isfinite(rec))
        finals.append(h.state_to_numpy(st))
    scale = np.max(np.abs(finals[0]))
    assert np.max(np.abs(finals[0] - finals[1])) <= 1e-5 * scale


def test_fp32_herm_rejections(heom):
    from paper_1803_03498_amd._abi import HeomError
    prob = hi.aggregate24(n_steps=4)
    h = heom.Hierarchy(prob, heom.FP32_HERM)
    st = h.new_state(prob["rho0"])
    out = h.new_state()
    with pytest.raises(HeomError):
        h.rhs(st, out, hermitian=False)
    with pytest.raises(HeomError):
        h.propagate(st, 1.0, 2, 1, hermitian=False)
    srv = heom.Server(1 << 28, 2)
    with pytest.raises(HeomError, match="server takes"):
        srv.submit(hi.serving_mix(1, seed=3)[0]["runs"], precision=heom.FP32_HERM)


# ----------------------------------------------------------- propagation ----

def test_propagate_fp64_dimer_full(heom, orc):
    _print_case("dimer fp64 1000 steps")
    prob = hi.dimer()
    y_ref, rec_ref = orc.run(prob)
    h = heom.Hierarchy(prob, heom.FP64)
    st = h.new_state(prob["rho0"])
    rec = h.propagate(st, prob["dt_fs"], prob["n_steps"], prob["record_every"],
                      prob["observable"], hermitian=True)
    assert rec.shape == rec_ref.shape
    assert np.max(np.abs(rec[:, :2] - rec_ref[:, :2])) <= 1e-12
    assert abs(rec[-1, 0] - 0.6154393558) < 1e-9
    assert np.max(np.abs(h.state_to_numpy(st) - y_ref)) <= 1e-12


@pytest.mark.parametrize("seed,N,M,D,herm", [(31, 3, 1, 3, True), (32, 5, 0, 3, False),
                                             (33, 8, 1, 2, True), (34, 17, 0, 2, True),
                                             (35, 24, 0, 1, False)])
def test_propagate_fp64_random(heom, orc, seed, N, M, D, herm):
    _print_case("propagate fp64", seed, N, M, D, herm)
    prob = hi.random_problem(seed, N, M=M, D=D)
    W, n = orc.sizes(prob)
    x0 = np.zeros((n, N, N), np.complex128)
    x0[0] = hi.population_rho0(N, 1 % N)
    if not herm:
        x0[0, 0, N - 1] = 0.3 + 0.1j
    y_ref, rec_ref = orc.propagate(prob, x0, 1.0, 40, 4)
    h = heom.Hierarchy(prob, heom.FP64)
    st = h.state_from_numpy(x0)
    rec = h.propagate(st, 1.0, 40, 4, hermitian=herm)
    assert np.max(np.abs(rec[:, :N] - rec_ref[:, :N])) <= 1e-12
    assert np.max(np.abs(h.state_to_numpy(st) - y_ref)) <= 1e-12 * max(1.0, np.max(np.abs(y_ref)))


def test_propagate_fp32_dimer(heom, orc):
    _print_case("dimer fp32 1000 steps")
    prob = hi.dimer()
    _, rec_ref = orc.run(prob)
    h = heom.Hierarchy(prob, heom.FP32_MIXED)
    st = h.new_state(prob["rho0"])
    rec = h.propagate(st, prob["dt_fs"], prob["n_steps"], prob["record_every"], hermitian=True)
    assert np.max(np.abs(rec[:, :2] - rec_ref[:, :2])) <= 1e-5


def test_dipole_record_and_trace(heom, orc):
    _print_case("dipole record")
    runs = hi.fmo_like_absorption(n_steps=60)
    r = runs[0]
    r["depth"] = 2
    _, rec_ref = orc.run(r)
    h = heom.Hierarchy(r, heom.FP64)
    st = h.new_state(r["rho0"])
    rec = h.propagate(st, r["dt_fs"], r["n_steps"], 1, r["observable"], hermitian=False)
    assert np.max(np.abs(rec - rec_ref)) <= 1e-12


def test_checkpoint_resume_bit_identical(heom):
    _print_case("checkpoint")
    prob = hi.random_problem(41, 6, M=1, D=3)
    for prec in (heom.FP64, heom.FP32_MIXED):
        h = heom.Hierarchy(prob, prec)
        a = h.new_state(hi.population_rho0(6))
        h.propagate(a, 1.0, 30, 30, hermitian=True)
        b = h.new_state(hi.population_rho0(6))
        h.propagate(b, 1.0, 12, 12, hermitian=True)
        s0, rest = h.get_state(b)
        c = h.new_state()
        h.set_state(c, s0, rest)
        h.propagate(c, 1.0, 18, 18, hermitian=True)
        assert np.array_equal(h.state_to_numpy(a), h.state_to_numpy(c))


def test_unstable_step_rejected(heom):
    from paper_1803_03498_amd._abi import HeomError
    h = heom.Hierarchy(hi.dimer())
    st = h.new_state(hi.population_rho0(2))
    with pytest.raises(HeomError) as ei:
        h.propagate(st, 200.0, 2, 1)
    assert ei.value.status == -6


def test_invariants_fp32(heom):
    _print_case("invariants")
    prob = hi.fmo_like(n_steps=200)
    h = heom.Hierarchy(prob, heom.FP32_MIXED)
    st = h.new_state(prob["rho0"])
    rec = h.propagate(st, 1.0, 200, 1, hermitian=True)
    assert np.max(np.abs(rec[:, 7] - 1.0)) < 1e-12   # trace conserved in FP64
    assert np.max(np.abs(rec[:, 8])) < 1e-12
    assert np.max(rec[:, 9]) < 1e-12                 # Hermitian sigma_0
