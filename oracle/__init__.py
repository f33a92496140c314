"""HEOM oracle — TEST INFRASTRUCTURE ONLY.

Python access to ``heom_oracle.cpp``: a plain, slow, single-threaded FP64 HEOM
right-hand side with textbook RK4, written from the equations of the paper
(section "HEOM formalism", eq. HEOM and the definitions that follow it).  Only
the test suite, the smoke check and the benchmark's CPU-baseline leg may import
this package; the GPU library never does, and the two share no code.

Build with :func:`build` (plain ``g++``); ``__graft_entry__.build()`` calls it.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "heom_oracle.cpp")
_LIB = os.path.join(_HERE, "liborc.so")

KIND_POPULATION = 0
KIND_DIPOLE = 1


def build(force=True):
    """Compile the oracle with g++ (-O2, no fast-math, strict IEEE FP64)."""
    if force or not os.path.exists(_LIB):
        cmd = ["g++", "-std=c++17", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fPIC",
               "-shared", "-o", _LIB + ".tmp", _SRC]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Problem(ctypes.Structure):
    _fields_ = [
        ("n_states", ctypes.c_int32),
        ("h_re", ctypes.POINTER(ctypes.c_double)),
        ("h_im", ctypes.POINTER(ctypes.c_double)),
        ("n_baths", ctypes.c_int32),
        ("bath_state", ctypes.POINTER(ctypes.c_int32)),
        ("bath_lambda_cm", ctypes.POINTER(ctypes.c_double)),
        ("bath_tau_fs", ctypes.POINTER(ctypes.c_double)),
        ("bath_matsubara", ctypes.POINTER(ctypes.c_int32)),
        ("temperature_K", ctypes.c_double),
        ("depth", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        d, i32, i64 = ctypes.c_double, ctypes.c_int32, ctypes.c_int64
        L.orc_count.argtypes = [i32, i32, P(i64)]
        L.orc_tables.argtypes = [i32, i32, i64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_void_p, P(i64)]
        L.orc_bath_coefficients.argtypes = [d, d, d, i32, P(d), P(d), P(d), P(d)]
        L.orc_bath_coefficients_pade.argtypes = [d, d, d, i32, P(d), P(d), P(d), P(d)]
        L.orc_pade_poles.argtypes = [i32, P(d), P(d)]
        L.orc_model_sizes.argtypes = [P(_Problem), P(i32), P(i64)]
        L.orc_rhs.argtypes = [P(_Problem), ctypes.c_void_p, ctypes.c_void_p, i64, i64]
        L.orc_time_step_sample.argtypes = [P(_Problem), ctypes.c_void_p, d, i64, i64, i64, i32,
                                           P(d)]
        L.orc_propagate.argtypes = [P(_Problem), ctypes.c_void_p, d, i64, i32, i32,
                                    ctypes.c_void_p, i32, ctypes.c_void_p]
        L.orc_spectrum.argtypes = [ctypes.c_void_p, i32, i64, d, ctypes.c_void_p, i64,
                                   ctypes.c_void_p]
        for f in ("orc_count", "orc_tables", "orc_bath_coefficients",
                  "orc_bath_coefficients_pade", "orc_pade_poles", "orc_model_sizes",
                  "orc_rhs", "orc_propagate", "orc_spectrum"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class _Packed:
    """Keeps the numpy buffers behind an _Problem alive."""

    def __init__(self, prob):
        H = np.asarray(prob["H"])
        self.N = H.shape[0]
        self.h_re = np.ascontiguousarray(H.real, dtype=np.float64)
        self.h_im = np.ascontiguousarray(H.imag, dtype=np.float64) if np.iscomplexobj(H) else None
        baths = prob["baths"]
        self.bs = np.array([b["state"] for b in baths], dtype=np.int32)
        self.bl = np.array([b["lambda_cm"] for b in baths], dtype=np.float64)
        self.bt = np.array([b["tau_fs"] for b in baths], dtype=np.float64)
        self.bm = np.array([b["matsubara"] for b in baths], dtype=np.int32)
        P32 = ctypes.POINTER(ctypes.c_int32)
        self.s = _Problem(self.N, _dptr(self.h_re),
                          _dptr(self.h_im) if self.h_im is not None else None,
                          len(baths), self.bs.ctypes.data_as(P32), _dptr(self.bl), _dptr(self.bt),
                          self.bm.ctypes.data_as(P32), float(prob["temperature_K"]),
                          int(prob["depth"]), int(prob.get("flags", 0)))


def count(W, D):
    n = ctypes.c_int64()
    if lib().orc_count(W, D, ctypes.byref(n)):
        raise ValueError("orc_count failed")
    return n.value


def tables(W, D):
    """(tuples uint8 [n][W], plus int32 [n][W], minus int32 [n][W], level int32 [n])."""
    n = count(W, D)
    t = np.zeros((n, max(W, 1)), np.uint8)
    p = np.zeros((n, max(W, 1)), np.int32)
    m = np.zeros((n, max(W, 1)), np.int32)
    lev = np.zeros(n, np.int32)
    got = ctypes.c_int64()
    rc = lib().orc_tables(W, D, n, t.ctypes.data, p.ctypes.data, m.ctypes.data, lev.ctypes.data,
                          ctypes.byref(got))
    if rc:
        raise ValueError("orc_tables failed: %d" % rc)
    return t[:, :W], p[:, :W], m[:, :W], lev


def bath_coefficients(lambda_cm, tau_fs, T, M, pade=False):
    """(gamma[M+1] 1/fs, c[M+1] rad/fs^2, lambda*nu, Delta) in hbar = 1 units;
    M Matsubara terms, or M Pade poles with pade=True."""
    g = np.zeros(M + 1)
    c = np.zeros(M + 1)
    ln = ctypes.c_double()
    dl = ctypes.c_double()
    f = lib().orc_bath_coefficients_pade if pade else lib().orc_bath_coefficients
    if f(lambda_cm, tau_fs, T, M, _dptr(g), _dptr(c), ctypes.byref(ln), ctypes.byref(dl)):
        raise ValueError("bad bath")
    return g, c, ln.value, dl.value


def pade_poles(K):
    """(xi[K], eta[K]): Pade poles and residues of the Bose function."""
    xi, eta = np.zeros(K), np.zeros(K)
    if lib().orc_pade_poles(K, _dptr(xi), _dptr(eta)):
        raise ValueError("K < 1")
    return xi, eta


def sizes(prob):
    pk = _Packed(prob)
    W = ctypes.c_int32()
    n = ctypes.c_int64()
    if lib().orc_model_sizes(ctypes.byref(pk.s), ctypes.byref(W), ctypes.byref(n)):
        raise ValueError("invalid problem")
    return W.value, n.value


def rhs(prob, state, u_begin=0, u_end=-1):
    """One evaluation of eq. (HEOM); state is complex128 [n_ado][N][N]."""
    pk = _Packed(prob)
    x = np.ascontiguousarray(state, dtype=np.complex128)
    out = np.zeros(x.shape, np.complex128)  # calloc: untouched pages stay unmapped
    if lib().orc_rhs(ctypes.byref(pk.s), x.ctypes.data, out.ctypes.data, u_begin, u_end):
        raise ValueError("invalid problem")
    return out


def time_step_sample(prob, state, dt_fs, u_begin=0, u_end=-1, stride=1, repeats=1):
    """Seconds of one RK4 step's work for the ADOs u_begin, u_begin + stride,
    ... below u_end, the smallest of `repeats` timings (timing only: the
    model is built outside the timed region; see orc_time_step_sample)."""
    pk = _Packed(prob)
    x = np.ascontiguousarray(state, dtype=np.complex128)
    sec = ctypes.c_double()
    if lib().orc_time_step_sample(ctypes.byref(pk.s), x.ctypes.data, float(dt_fs), int(u_begin),
                                  int(u_end), int(stride), int(repeats), ctypes.byref(sec)):
        raise ValueError("invalid problem or out of memory")
    return sec.value


def record_size(N, kind):
    return N + 3 if kind == KIND_POPULATION else 4


def propagate(prob, state, dt_fs, n_steps, record_every=1, observable=None, inplace=False):
    """Textbook RK4.  Returns (final state, records [n_rec][record_size]).
    With ``inplace`` a C-contiguous complex128 ``state`` is advanced in place
    (no copy: large hierarchies need every gigabyte)."""
    pk = _Packed(prob)
    if inplace:
        x = state
        if x.dtype != np.complex128 or not x.flags["C_CONTIGUOUS"]:
            raise ValueError("inplace propagation needs a C-contiguous complex128 array")
    else:
        x = np.array(state, dtype=np.complex128, order="C", copy=True)
    obs = observable or {"kind": "population"}
    kind = KIND_POPULATION if obs["kind"] == "population" else KIND_DIPOLE
    mu = np.ascontiguousarray(obs.get("mu", np.zeros(pk.N)), dtype=np.float64)
    ground = int(obs.get("ground", 0))
    n_rec = n_steps // record_every + 1
    rec = np.zeros((n_rec, record_size(pk.N, kind)))
    rc = lib().orc_propagate(ctypes.byref(pk.s), x.ctypes.data, float(dt_fs), int(n_steps),
                             int(record_every), kind, mu.ctypes.data, ground, rec.ctypes.data)
    if rc:
        raise ValueError("invalid problem")
    return x, rec


def initial_state(prob, n_ado, rho0):
    N = np.asarray(prob["H"]).shape[0]
    s = np.zeros((n_ado, N, N), np.complex128)
    s[0] = rho0
    return s


def emission_start(state, mu):
    """Start of a fluorescence run (section "Static Fluorescence Spectra": the
    dipole operator acts on every ADO): for the thermalised excited-state
    hierarchy `state` [n][N][N], the (N+1)-state ADOs Y_u = sigma_u mu^+,
    i.e. Y_u[1 + a][0] = sum_b sigma_u[a][b] mu[b], ground state at index 0."""
    state = np.asarray(state, np.complex128)
    n, N, _ = state.shape
    Y = np.zeros((n, N + 1, N + 1), np.complex128)
    Y[:, 1:, 0] = state @ np.asarray(mu, np.float64)
    return Y


def cd_vectors(R, d):
    """Excitation vectors of circular dichroism (eq. CDdipoleoperator):
    m[p][a] = (R_a x d_a) . e_p."""
    return np.cross(np.asarray(R, np.float64), np.asarray(d, np.float64)).T.copy()


def fluorescence(relax, emis):
    """Oracle fluorescence pipeline: relax the excited-state hierarchy from
    its Boltzmann start, then propagate sigma_u(inf) mu_p^+ for each
    direction.  Returns (thermal state, P [n_dir][n_t] complex)."""
    W, n = sizes(relax)
    s0 = initial_state(relax, n, relax["rho0"])
    st, _ = propagate(relax, s0, relax["dt_fs"], relax["n_steps"], relax["record_every"])
    P = []
    for r in emis:
        Y = emission_start(st, r["observable"]["mu"][1:])
        _, rec = propagate(r, Y, r["dt_fs"], r["n_steps"], r["record_every"], r["observable"])
        P.append(rec[:, 0] + 1j * rec[:, 1])
    return st, np.stack(P)


def run(run_spec, n_steps=None):
    """Propagate a run dict (see heom_inputs); returns (final state, records)."""
    W, n = sizes(run_spec)
    s0 = initial_state(run_spec, n, run_spec["rho0"])
    steps = run_spec["n_steps"] if n_steps is None else n_steps
    return propagate(run_spec, s0, run_spec["dt_fs"], steps, run_spec["record_every"],
                     run_spec["observable"])


def spectrum(P, dt_fs, omega_cm):
    """Trapezoid-rule linear absorption, P complex [n_dir][n_t]."""
    P = np.ascontiguousarray(np.atleast_2d(P), dtype=np.complex128)
    w = np.ascontiguousarray(omega_cm, dtype=np.float64)
    S = np.zeros(len(w))
    if lib().orc_spectrum(P.ctypes.data, P.shape[0], P.shape[1], float(dt_fs), w.ctypes.data,
                          len(w), S.ctypes.data):
        raise ValueError("bad spectrum input")
    return S
