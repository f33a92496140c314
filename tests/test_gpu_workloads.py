"""Parity on the named workloads at their real sizes.

* FMO-like (3060 ADOs): full 2000-step FP64 and FP32-mixed runs against the
  oracle's stored records (tests/golden, written by make_oracle_golden.py).
* FMO-like linear absorption (3 directions, 1 ps): dipole correlation and the
  spectrum within 1e-4 relative.
* 24-site (20475 ADOs) and 48-site (156849 ADOs) aggregates: the right-hand
  side in the launch configurations the benchmark times (FP64, FP32-mixed and
  Hermitian-packed FP32), compared with the
  oracle on sampled ADOs from every level (the oracle evaluates them one by
  one; every other ADO is zero except the neighbours of the sampled ones).
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


def _golden(name):
    return np.loadtxt(os.path.join(HERE, "golden", name))


# ------------------------------------------------------------- FMO-like ----

@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 1e-5)])
def test_fmo_like_full_run(heom, precision, tol):
    _case("fmo_like 2000 steps", precision)
    prob = hi.fmo_like()
    ref = _golden("fmo_like_fp64_records.txt")
    h = heom.Hierarchy(prob, precision)
    st = h.new_state(prob["rho0"])
    rec = h.propagate(st, prob["dt_fs"], prob["n_steps"], 1, prob["observable"], hermitian=True)
    got = rec[ref[:, 0].astype(int)]
    assert np.max(np.abs(got[:, :7] - ref[:, 1:8])) <= tol
    assert np.max(np.abs(got[:, 7] - 1.0)) <= 1e-12   # FP64 trace
    assert np.max(got[:, 9]) <= 1e-12                  # Hermitian sigma_0


def test_fmo_like_absorption_spectrum(heom, orc):
    _case("fmo_like absorption")
    runs = hi.fmo_like_absorption()
    ref = _golden("fmo_like_absorption_P.txt")
    P_ref = np.stack([ref[:, 1 + 2 * p] + 1j * ref[:, 2 + 2 * p] for p in range(3)])
    w = np.arange(-1000.0, 1001.0, 1.0)
    S_ref = orc.spectrum(P_ref, 1.0, w)
    for precision, p_tol in ((0, 1e-12), (1, 1e-5)):
        P = []
        for r in runs:
            h = heom.Hierarchy(r, precision)
            st = h.new_state(r["rho0"])
            rec = h.propagate(st, r["dt_fs"], r["n_steps"], 1, r["observable"], hermitian=False)
            P.append(rec[:, 0] + 1j * rec[:, 1])
            assert np.max(np.abs(rec[:, 2:4])) <= 1e-12  # trace stays 0
        P = np.stack(P)
        assert np.max(np.abs(P - P_ref)) <= p_tol
        S = heom.spectrum(P, 1.0, w)
        rel = np.max(np.abs(S - S_ref)) / np.max(np.abs(S_ref))
        assert rel <= (1e-12 if precision == 0 else 1e-4), rel


# ------------------------------------ low temperature, Pade expansion ----

@pytest.mark.parametrize("T,poles,steps,dt", [(77.0, 1, 200, 1.0), (30.0, 3, 100, 0.5)])
@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 1e-5)])
def test_fmo_like_pade_low_temperature(heom, orc, T, poles, steps, dt, precision, tol):
    # the paper's working settings (D, K) = (3, 2) at 77 K and (3, 4) at 30 K
    _case("fmo_like pade", T, poles, precision)
    prob = hi.fmo_like_pade(T, 3, poles, n_steps=steps, dt_fs=dt)
    _, rec_ref = orc.run(prob)
    h = heom.Hierarchy(prob, precision)
    st = h.new_state(prob["rho0"])
    rec = h.propagate(st, dt, steps, 1, prob["observable"], hermitian=True)
    assert np.max(np.abs(rec[:, :7] - rec_ref[:, :7])) <= tol
    assert np.max(np.abs(rec[:, 7] - 1.0)) <= 1e-12


# ------------------------------------------ absorption, coherence block ----

def _block_problem(run):
    """The excited-state problem of a ground + excited absorption run."""
    return {"H": np.asarray(run["H"])[1:, 1:], "temperature_K": run["temperature_K"],
            "depth": run["depth"], "flags": run.get("flags", 0),
            "baths": [dict(b, state=b["state"] - 1) for b in run["baths"]]}


def test_block_form_refuses_unrotated_frame(heom):
    # excited energies ~12300 cm^-1 above a ground state at 0 (no rotating
    # frame): the column keeps that offset, 2.3 rad per 1-fs step
    run = hi.fmo_like_absorption(n_steps=10)[0]
    prob = _block_problem(run)
    prob["H"] = prob["H"] + 12300.0 * np.eye(7)
    mu3 = np.stack([r["observable"]["mu"][1:] for r in hi.fmo_like_absorption(n_steps=10)])
    h = heom.Hierarchy(prob, heom.FP64)
    with pytest.raises(heom.HeomError) as e:
        h.propagate_block(h.block_state(mu3), 1.0, 10, 1, mu3)
    assert e.value.status == -6
    # the same block in the rotating frame is accepted
    h2 = heom.Hierarchy(_block_problem(run), heom.FP64)
    P = h2.propagate_block(h2.block_state(mu3), 1.0, 10, 1, mu3)
    assert np.all(np.isfinite(P))


def test_fmo_like_absorption_block_form(heom, orc):
    # the three directions of the FMO-like absorption run in one block
    # propagation against the oracle's stored full-matrix correlations
    _case("fmo_like absorption block form")
    runs = hi.fmo_like_absorption()
    ref = _golden("fmo_like_absorption_P.txt")
    P_ref = np.stack([ref[:, 1 + 2 * p] + 1j * ref[:, 2 + 2 * p] for p in range(3)])
    mu3 = np.stack([r["observable"]["mu"][1:] for r in runs])
    h = heom.Hierarchy(_block_problem(runs[0]), heom.FP64)
    P = h.propagate_block(h.block_state(mu3), runs[0]["dt_fs"], runs[0]["n_steps"], 1, mu3).T
    assert np.max(np.abs(P - P_ref)) <= 1e-12
    w = np.arange(-1000.0, 1001.0, 1.0)
    S_ref = orc.spectrum(P_ref, 1.0, w)
    assert np.max(np.abs(heom.spectrum(P, 1.0, w) - S_ref)) <= 1e-12 * np.max(np.abs(S_ref))


@pytest.mark.parametrize("seed,N,M,D", [(1, 2, 0, 4), (2, 3, 1, 3), (3, 5, 1, 2), (4, 4, 2, 2)])
@pytest.mark.parametrize("cross", [False, True])
def test_absorption_block_form_random(heom, orc, seed, N, M, D, cross):
    # against full (N+1)-state oracle runs; cross: observed with another
    # vector per direction (the form of a circular-dichroism correlation)
    _case("absorption block form", seed, N, M, D, cross)
    rng = np.random.default_rng(seed)
    H = hi.fmo_like_hamiltonian(rng, N)
    dip = hi.unit_vectors(rng, N)
    baths = [{"state": s, "lambda_cm": 35.0, "tau_fs": 50.0, "matsubara": M} for s in range(N)]
    runs = hi.absorption_runs(H, dip, baths, 300.0, D, 1.0, 150)
    mu3 = np.stack([r["observable"]["mu"][1:] for r in runs])
    obs3 = rng.normal(size=(3, N)) if cross else mu3
    P_ref = []
    for p, r in enumerate(runs):
        r = dict(r, observable=dict(r["observable"], mu=np.concatenate([[0.0], obs3[p]])))
        _, rec = orc.run(r)
        P_ref.append(rec[:, 0] + 1j * rec[:, 1])
    P_ref = np.stack(P_ref)
    # the block path is FP64 whatever precision the hierarchy was built for
    for prec in (heom.FP64, heom.FP32_MIXED):
        h = heom.Hierarchy(_block_problem(runs[0]), prec)
        P = h.propagate_block(h.block_state(mu3), 1.0, 150, 1, obs3).T
        assert np.max(np.abs(P - P_ref)) <= 1e-12 * max(1.0, np.max(np.abs(P_ref)))


def test_cd_block_form(heom, orc):
    # circular dichroism: the block run started from the rotational vectors
    # m_p and observed with the dipoles, against full-matrix oracle runs
    _case("cd block form")
    rng = np.random.default_rng(12)
    R = hi.aggregate_geometry(rng, 5)
    d = hi.unit_vectors(rng, 5)
    H = hi.dipole_couplings(R, d) + np.diag(rng.normal(12400.0, 100.0, 5))
    baths = [{"state": s, "lambda_cm": 35.0, "tau_fs": 50.0, "matsubara": 1} for s in range(5)]
    runs = hi.absorption_runs(H, d, baths, 300.0, 3, 1.0, 200)
    m = heom.cd_vectors(R, d)
    P_ref = []
    for p, r in enumerate(runs):
        rho0 = np.zeros_like(r["rho0"])
        rho0[1:, 0] = m[p]
        _, rec = orc.run(dict(r, rho0=rho0))
        P_ref.append(rec[:, 0] + 1j * rec[:, 1])
    P_ref = np.stack(P_ref)
    mu3 = np.stack([r["observable"]["mu"][1:] for r in runs])
    h = heom.Hierarchy(_block_problem(runs[0]), heom.FP64)
    P = h.propagate_block(h.block_state(m), 1.0, 200, 1, mu3).T
    assert np.max(np.abs(P - P_ref)) <= 1e-12 * np.max(np.abs(P_ref))


# ------------------------------------------------ static fluorescence ----

def _gpu_fluorescence(heom, relax, emis, prec_exc, prec_full):
    he = heom.Hierarchy(relax, prec_exc)
    st = he.new_state(relax["rho0"])
    he.propagate(st, relax["dt_fs"], relax["n_steps"], relax["record_every"], hermitian=True)
    P = []
    for r in emis:
        hf = heom.Hierarchy(r, prec_full)
        y = hf.new_state()
        heom.emission_start(he, st, hf, y, r["observable"]["mu"][1:])
        rec = hf.propagate(y, r["dt_fs"], r["n_steps"], r["record_every"], r["observable"],
                           hermitian=False)
        P.append(rec[:, 0] + 1j * rec[:, 1])
    return he.state_to_numpy(st), np.stack(P)


@pytest.mark.parametrize("N,M,D", [(2, 0, 4), (3, 1, 3), (7, 1, 3)])
@pytest.mark.parametrize("precs,tol", [((0, 0), 1e-12), ((1, 1), 1e-5), ((0, 1), 1e-5)])
def test_fluorescence_pipeline(heom, orc, N, M, D, precs, tol):
    _case("fluorescence", N, M, D, precs)
    rng = np.random.default_rng(40 + N)
    H = hi.fmo_like_hamiltonian(rng, N)
    dip = hi.unit_vectors(rng, N)
    baths = [{"state": s, "lambda_cm": 35.0, "tau_fs": 50.0, "matsubara": M} for s in range(N)]
    relax, emis = hi.fluorescence_runs(H, dip, baths, 300.0, D, 1.0, 300, 200)
    st_ref, P_ref = orc.fluorescence(relax, emis)
    st, P = _gpu_fluorescence(heom, relax, emis, *precs)
    scale = np.max(np.abs(P_ref))
    assert np.max(np.abs(P - P_ref)) <= tol * scale
    if precs == (0, 0):
        assert np.max(np.abs(st - st_ref)) <= 1e-12


def test_emission_start_rejects_mismatch(heom):
    from paper_1803_03498_amd._abi import HeomError
    rng = np.random.default_rng(1)
    H = hi.fmo_like_hamiltonian(rng, 3)
    baths = [{"state": s, "lambda_cm": 35.0, "tau_fs": 50.0, "matsubara": 0} for s in range(3)]
    relax, emis = hi.fluorescence_runs(H, hi.unit_vectors(rng, 3), baths, 300.0, 2, 1.0, 1, 1)
    he = heom.Hierarchy(relax)
    st = he.new_state(relax["rho0"])
    bad = dict(emis[0], depth=3)
    hf = heom.Hierarchy(bad)
    with pytest.raises(HeomError):
        heom.emission_start(he, st, hf, hf.new_state(), np.ones(3))
    with pytest.raises(HeomError):
        heom.emission_start(he, st, he, he.new_state(), np.ones(3))


# ----------------------------------------------- aggregates, full size ----

def _level_ranges(W, D, width):
    """A block of `width` ADOs at the start of every level >= 1 and at the end."""
    from math import comb
    starts = [comb(W + L - 1, W) for L in range(1, D + 1)]
    n = comb(W + D, W)
    out = [(s, min(s + width, n)) for s in starts]
    out.append((n - width, n))
    return out


def _sampled_rhs(heom, orc, prob, precision, width, seed):
    import torch
    N = prob["H"].shape[0]
    W, n = orc.sizes(prob)
    _, plus, minus, _ = orc.tables(W, prob["depth"])
    ranges = _level_ranges(W, prob["depth"], width)
    sample = np.unique(np.concatenate([np.arange(a, b) for a, b in ranges]))
    nb = np.concatenate([plus[sample].ravel(), minus[sample].ravel()])
    need = np.unique(np.concatenate([sample, nb[nb >= 0], [0]]))
    rng = np.random.default_rng(seed)
    vals = rng.normal(size=(len(need), N, N)) + 1j * rng.normal(size=(len(need), N, N))
    vals = (vals + np.conj(np.transpose(vals, (0, 2, 1)))) / 2  # Hermitian ADOs
    if precision == heom.FP32_HERM:
        vals[need > 0] = heom.unpack_hermitian(heom.pack_hermitian(vals[need > 0]).astype(np.float32))
    else:
        vals[need > 0] = vals[need > 0].astype(np.complex128 if precision == 0 else np.complex64)
    # oracle input: zero except the needed ADOs (pages of the rest stay untouched)
    x = np.zeros((n, N, N), np.complex128)
    x[need] = vals
    h = heom.Hierarchy(prob, precision)
    s0, rest = h.new_state(vals[0])
    idx = torch.as_tensor(need[need > 0] - 1, device="cuda")
    src = vals[need > 0]
    if precision == heom.FP32_HERM:
        src = heom.pack_hermitian(src)
    rest.index_copy_(0, idx, torch.as_tensor(src).to(rest.dtype).cuda())
    out = h.new_state()
    h.rhs((s0, rest), out, hermitian=True)
    torch.cuda.synchronize()
    del rest
    got_rest = out[1][torch.as_tensor(sample - 1, device="cuda")].cpu().numpy()
    if precision == heom.FP32_HERM:
        got_rest = heom.unpack_hermitian(got_rest)
    ref = np.zeros((len(sample), N, N), np.complex128)
    pos = {u: k for k, u in enumerate(sample)}
    for a, b in ranges:
        f = orc.rhs(prob, x, a, b)
        for u in range(a, b):
            ref[pos[u]] = f[u]
        del f
    return got_rest, ref


@pytest.mark.parametrize("precision,tol", [(1, 1e-5), (0, 1e-12), (2, 1e-5)])
def test_aggregate24_rhs_sampled(heom, orc, precision, tol):
    _case("aggregate24 sampled rhs", precision)
    got, ref = _sampled_rhs(heom, orc, hi.aggregate24(), precision, 40, 24)
    assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref))


@pytest.mark.parametrize("precision,tol", [(1, 1e-5), (0, 1e-12), (2, 1e-5)])
def test_aggregate48_rhs_sampled(heom, orc, precision, tol):
    _case("aggregate48 sampled rhs", precision)
    got, ref = _sampled_rhs(heom, orc, hi.aggregate48(), precision, 12, 48)
    assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref))


def test_aggregate24_fp32_tracks_fp64(heom):
    _case("aggregate24 fp32 and fp32 packed vs fp64 100 steps")
    prob = hi.aggregate24(n_steps=100)
    recs = []
    for precision in (0, 1, 2):
        h = heom.Hierarchy(prob, precision)
        st = h.new_state(prob["rho0"])
        recs.append(h.propagate(st, 1.0, 100, 10, hermitian=True))
        del st, h
    assert np.max(np.abs(recs[0][:, :24] - recs[1][:, :24])) <= 1e-5
    # Hermitian-packed storage: the same FP32 arithmetic on half the bytes
    assert np.max(np.abs(recs[0][:, :24] - recs[2][:, :24])) <= 1e-5
    assert np.max(np.abs(recs[2][:, 24] - 1.0)) <= 1e-12   # FP64 trace
