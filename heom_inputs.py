"""Seeded synthetic inputs for HEOM runs.

Shared by the test suite, the benchmark and the smoke check: both the GPU
library and the oracle consume the problems built here.  This module holds none
of the HEOM arithmetic (no bath coefficients, no hierarchy, no right-hand side);
it only draws Hamiltonians, baths, dipoles, initial states and arrival times.

Workload shapes follow the paper's light-harvesting examples (Frenkel-exciton
Hamiltonian, eq. h-ex; one Drude-Lorentz bath per site, eq.
spectral_density_DL; FMO parameters of Table 1: lambda = 35 cm^-1,
nu^-1 = 50 fs) and the workload functions below.  Every array is
drawn from ``numpy.random.default_rng(seed)`` in the order written below.

A problem is a dict::

    {"H": (N, N) float or complex array in cm^-1,
     "baths": [{"state": s, "lambda_cm": .., "tau_fs": .., "matsubara": M}, ...],
     "temperature_K": T, "depth": D, "flags": 0}

and a run adds ``dt_fs``, ``n_steps``, ``record_every``, ``rho0`` (N, N complex)
and ``observable`` ({"kind": "population"} or {"kind": "dipole", "mu": (N,),
"ground": 0}).
"""

from __future__ import annotations

import numpy as np

# Transition-dipole coupling prefactor: 1 Debye^2 / (4 pi eps0 1 Angstrom^3)
# expressed in cm^-1.
DIPOLE_CM = 5034.12

# Test-only switches understood by both implementations.
FLAG_NO_RESCALE = 1
FLAG_NO_TERMINATOR = 2
FLAG_ADD_REORG = 4
FLAG_STANDARD_GAUGE = 8
FLAG_PADE = 16


def _baths(n_sites, lam, tau, M, first_state=0):
    return [{"state": first_state + m, "lambda_cm": float(lam), "tau_fs": float(tau),
             "matsubara": int(M)} for m in range(n_sites)]


def population_rho0(N, state=0):
    rho = np.zeros((N, N), dtype=np.complex128)
    rho[state, state] = 1.0
    return rho


def unit_vectors(rng, n):
    """n directions uniform on the sphere (normalised Gaussian triples)."""
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def fmo_like_hamiltonian(rng, n, lo=12000.0, hi=12600.0, sd=60.0):
    """Energies U[lo, hi]; upper-triangle couplings N(0, sd^2), row-major."""
    e = rng.uniform(lo, hi, n)
    iu = np.triu_indices(n, 1)
    J = rng.normal(0.0, sd, len(iu[0]))
    H = np.diag(e)
    H[iu] = J
    H[(iu[1], iu[0])] = J
    return H


def aggregate_geometry(rng, n, dmin=5.0, dmax=25.0):
    """Chain growth of n sites: each new site hangs off a random earlier site at
    a uniform direction and a distance U[dmin, dmax] (Angstrom); placements
    closer than dmin to any site are redrawn."""
    pos = [np.zeros(3)]
    while len(pos) < n:
        parent = pos[int(rng.integers(0, len(pos)))]
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        cand = parent + rng.uniform(dmin, dmax) * d
        if min(np.linalg.norm(cand - p) for p in pos) >= dmin:
            pos.append(cand)
    return np.array(pos)


def dipole_couplings(pos, dip):
    """Point-dipole couplings J_mn in cm^-1 (positions in Angstrom, dipoles in
    Debye)."""
    n = len(pos)
    J = np.zeros((n, n))
    for m in range(n):
        for k in range(m + 1, n):
            r = pos[k] - pos[m]
            d = np.linalg.norm(r)
            rh = r / d
            v = DIPOLE_CM * (dip[m] @ dip[k] - 3.0 * (dip[m] @ rh) * (dip[k] @ rh)) / d**3
            J[m, k] = J[k, m] = v
    return J


def aggregate_hamiltonian(rng, n, mean, sd):
    e = rng.normal(mean, sd, n)
    pos = aggregate_geometry(rng, n)
    dip = unit_vectors(rng, n)
    H = dipole_couplings(pos, dip) + np.diag(e)
    return H, pos, dip


def with_ground_state(H_sites, omega_ref):
    """(N+1)-state Hamiltonian: ground state 0 at energy 0, excited block in a
    frame rotating at omega_ref (cm^-1)."""
    n = H_sites.shape[0]
    H = np.zeros((n + 1, n + 1))
    H[1:, 1:] = H_sites - omega_ref * np.eye(n)
    return H


def absorption_runs(H_sites, dip, baths_sites, T, depth, dt, n_steps, record_every=1):
    """Three dipole-correlation runs (directions x, y, z) in the rotating frame
    at the mean site energy: sigma_0(0) = mu_p^+ |g><g|, all other ADOs 0, and
    P_p(t) = sum_a (e_p . d_a) sigma_0[a][g]."""
    n = H_sites.shape[0]
    wref = float(np.mean(np.diag(H_sites)))
    H = with_ground_state(H_sites, wref)
    baths = [dict(b, state=b["state"] + 1) for b in baths_sites]
    runs = []
    for p in range(3):
        mu = np.zeros(n + 1)
        mu[1:] = dip[:, p]
        rho0 = np.zeros((n + 1, n + 1), dtype=np.complex128)
        rho0[1:, 0] = mu[1:]
        runs.append({"H": H, "baths": baths, "temperature_K": T, "depth": depth, "flags": 0,
                     "dt_fs": dt, "n_steps": n_steps, "record_every": record_every,
                     "rho0": rho0, "omega_ref_cm": wref,
                     "observable": {"kind": "dipole", "mu": mu, "ground": 0}})
    return runs


def boltzmann_rho(H_sites, T):
    """exp(-H/(k_B T)) / Tr (eq. rho_Boltzmann), H in cm^-1 (input preparation)."""
    kT = 0.6950348004 * T
    w, v = np.linalg.eigh(H_sites)
    p = np.exp(-(w - w.min()) / kT)
    p /= p.sum()
    return (v * p) @ v.T


def fluorescence_runs(H_sites, dip, baths_sites, T, depth, dt, n_relax, n_steps, record_every=1):
    """Static fluorescence (section "Static Fluorescence Spectra"): a
    population run of the excited states from the Boltzmann state for
    n_relax steps (the long-time propagation route to the thermal state
    sigma_u(inf)), then three dipole-correlation runs (x, y, z) of the
    (N+1)-state system started from sigma_u(inf) mu_p^+ (all ADOs) in the
    frame rotating at the mean site energy."""
    n = H_sites.shape[0]
    wref = float(np.mean(np.diag(H_sites)))
    relax = {"H": H_sites - wref * np.eye(n), "baths": [dict(b) for b in baths_sites],
             "temperature_K": T, "depth": depth, "flags": 0, "dt_fs": dt, "n_steps": n_relax,
             "record_every": n_relax if n_relax > 0 else 1, "rho0": boltzmann_rho(H_sites, T),
             "observable": {"kind": "population"}}
    emis = absorption_runs(H_sites, dip, baths_sites, T, depth, dt, n_steps, record_every)
    for r in emis:
        r["rho0"] = None  # the start is sigma_u(inf) mu_p^+, built from the relaxed state
    return relax, emis


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

def dimer(n_steps=1000):
    """2 sites, E = {0, 100}, J = 50 cm^-1; lambda = 35 cm^-1, nu^-1 = 50 fs,
    300 K, no Matsubara term, depth 3 (10 ADOs); dt = 1 fs; rho = |1><1|."""
    H = np.array([[0.0, 50.0], [50.0, 100.0]])
    return {"name": "dimer", "H": H, "baths": _baths(2, 35.0, 50.0, 0), "temperature_K": 300.0,
            "depth": 3, "flags": 0, "dt_fs": 1.0, "n_steps": n_steps, "record_every": 1,
            "rho0": population_rho0(2), "observable": {"kind": "population"}}


def fmo_like(n_steps=2000, seed=7):
    """7 sites, energies U[12000, 12600], couplings N(0, 60^2); lambda = 35,
    nu^-1 = 50 fs, 300 K, one Matsubara term, depth 4 (3060 ADOs); dt = 1 fs."""
    rng = np.random.default_rng(seed)
    H = fmo_like_hamiltonian(rng, 7)
    return {"name": "fmo_like", "H": H, "baths": _baths(7, 35.0, 50.0, 1), "temperature_K": 300.0,
            "depth": 4, "flags": 0, "dt_fs": 1.0, "n_steps": n_steps, "record_every": 1,
            "rho0": population_rho0(7), "observable": {"kind": "population"}}


def fmo_like_pade(T=77.0, depth=3, poles=1, n_steps=200, dt_fs=1.0, seed=7):
    """The fmo_like system at temperature T with the Pade expansion of the
    paper's low-temperature settings: (D, K) = (3, 2) at 77 K and (3, 4) at
    30 K, K counting the k = 0 mode, i.e. K - 1 Pade poles per bath."""
    rng = np.random.default_rng(seed)
    H = fmo_like_hamiltonian(rng, 7)
    return {"name": "fmo_like_pade", "H": H, "baths": _baths(7, 35.0, 50.0, poles),
            "temperature_K": T, "depth": depth, "flags": FLAG_PADE, "dt_fs": dt_fs,
            "n_steps": n_steps, "record_every": 1, "rho0": population_rho0(7),
            "observable": {"kind": "population"}}


def fmo_like_absorption(n_steps=1000, seed=7, dipole_seed=70):
    """The fmo_like system plus a ground state (N = 8), three dipole
    directions, rotating frame; 1 ps at dt = 1 fs."""
    H_sites = fmo_like(seed=seed)["H"]
    dip = unit_vectors(np.random.default_rng(dipole_seed), 7)
    runs = absorption_runs(H_sites, dip, _baths(7, 35.0, 50.0, 1), 300.0, 4, 1.0, n_steps)
    for r in runs:
        r["name"] = "fmo_like_absorption"
    return runs


def aggregate24(n_steps=1000, seed=24):
    """24 sites, energies N(12400, 150^2), point-dipole couplings; lambda = 50,
    nu^-1 = 100 fs, 277 K, no Matsubara term (W = 24), depth 4 (20475 ADOs)."""
    rng = np.random.default_rng(seed)
    H, pos, dip = aggregate_hamiltonian(rng, 24, 12400.0, 150.0)
    return {"name": "aggregate24", "H": H, "baths": _baths(24, 50.0, 100.0, 0),
            "temperature_K": 277.0, "depth": 4, "flags": 0, "dt_fs": 1.0, "n_steps": n_steps,
            "record_every": 10, "rho0": population_rho0(24), "observable": {"kind": "population"},
            "positions": pos, "dipoles": dip}


def aggregate48(n_steps=500, seed=48):
    """48 sites, energies N(12400, 200^2), point-dipole couplings; lambda = 35,
    nu^-1 = 50 fs, 300 K, one Matsubara term (W = 96), depth 3 (156849 ADOs)."""
    rng = np.random.default_rng(seed)
    H, pos, dip = aggregate_hamiltonian(rng, 48, 12400.0, 200.0)
    return {"name": "aggregate48", "H": H, "baths": _baths(48, 35.0, 50.0, 1),
            "temperature_K": 300.0, "depth": 3, "flags": 0, "dt_fs": 1.0, "n_steps": n_steps,
            "record_every": 10, "rho0": population_rho0(48), "observable": {"kind": "population"},
            "positions": pos, "dipoles": dip}


def serving_mix(n_requests=512, seed=512, n_steps=1000):
    """Independent propagation requests: N ~ U{2..14}, D ~ U{2..5},
    M ~ U{0, 1}, kind ~ U{population, absorption}; FMO-like Hamiltonian plus
    static Gaussian disorder (sd 50 cm^-1) on the site energies; lambda = 35,
    nu^-1 = 50 fs, 300 K; 1 ps at dt = 1 fs.  ``gap`` is a unit-rate
    exponential inter-arrival time (Poisson arrivals once scaled by a rate).
    An absorption request carries three runs (x, y, z)."""
    rng = np.random.default_rng(seed)
    reqs = []
    for r in range(n_requests):
        N = int(rng.integers(2, 15))
        D = int(rng.integers(2, 6))
        M = int(rng.integers(0, 2))
        kind = "absorption" if rng.integers(0, 2) else "population"
        H = fmo_like_hamiltonian(rng, N)
        H[np.diag_indices(N)] += rng.normal(0.0, 50.0, N)
        gap = float(rng.exponential(1.0))
        baths = _baths(N, 35.0, 50.0, M)
        if kind == "absorption":
            dip = unit_vectors(rng, N)
            runs = absorption_runs(H, dip, baths, 300.0, D, 1.0, n_steps)
        else:
            runs = [{"H": H, "baths": baths, "temperature_K": 300.0, "depth": D, "flags": 0,
                     "dt_fs": 1.0, "n_steps": n_steps, "record_every": 1,
                     "rho0": population_rho0(N), "observable": {"kind": "population"}}]
        reqs.append({"id": r, "kind": kind, "N": N, "depth": D, "matsubara": M, "gap": gap,
                     "runs": runs})
    return reqs


def random_problem(seed, N, n_baths=None, M=1, D=2, T=300.0, complex_h=False, hermitian_h=True):
    """Small random problem for parity tests: random Hermitian H (cm^-1, scale
    ~100), baths on random states with random lambda and tau."""
    rng = np.random.default_rng(seed)
    A = rng.normal(0.0, 80.0, (N, N))
    if complex_h:
        A = A + 1j * rng.normal(0.0, 80.0, (N, N))
    H = (A + A.conj().T) / 2 if hermitian_h else A
    H = H + np.diag(rng.uniform(-200.0, 200.0, N))
    nb = N if n_baths is None else n_baths
    states = rng.permutation(N)[:nb] if nb <= N else rng.integers(0, N, nb)
    baths = [{"state": int(s), "lambda_cm": float(rng.uniform(10.0, 80.0)),
              "tau_fs": float(rng.uniform(30.0, 150.0)), "matsubara": int(M)} for s in states]
    return {"H": H, "baths": baths, "temperature_K": float(T), "depth": int(D), "flags": 0}


def random_state(seed, n_ado, N, hermitian=False, scale=1.0):
    """Random ADO array [n_ado][N][N] complex128 (optionally each ADO
    Hermitian)."""
    rng = np.random.default_rng(seed)
    s = rng.normal(size=(n_ado, N, N)) + 1j * rng.normal(size=(n_ado, N, N))
    if hermitian:
        s = (s + np.conj(np.transpose(s, (0, 2, 1)))) / 2
    return scale * s
