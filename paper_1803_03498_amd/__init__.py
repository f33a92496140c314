"""MI355X (gfx950) HEOM library: Python binding of the C ABI in include/heom.h.

The right-hand side of the hierarchical equations of motion (Kramer et al.,
arXiv:1803.03498, section "HEOM formalism", eq. HEOM) and its classic RK4
integration run in hand-written HIP kernels inside ``libheom.so``.  This module
only marshals arguments: PyTorch provides device memory and the stream, and
every step of the computation happens in the library.  There is no CPU
fallback: without the built library (or without a gfx950 GPU) the calls raise.
"""

from __future__ import annotations

import ctypes

import numpy as np

from . import _abi
from ._abi import FP32_HERM, FP32_MIXED, FP64, OBS_DIPOLE, OBS_POPULATION, HeomError, check, load

__all__ = ["FP64", "FP32_MIXED", "FP32_HERM", "problem_coefficients", "emission_start", "cd_vectors", "pack_hermitian", "unpack_hermitian", "OBS_POPULATION", "OBS_DIPOLE", "HeomError", "Problem", "plan",
           "Hierarchy", "Server", "spectrum", "load"]


def _torch():
    import torch
    return torch


def _stream_handle(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Problem:
    """A problem dict (see heom_inputs) packed into a heom_problem struct."""

    def __init__(self, prob, precision=FP64):
        H = np.asarray(prob["H"])
        self.N = int(H.shape[0])
        self._h_re = np.ascontiguousarray(H.real, dtype=np.float64)
        self._h_im = (np.ascontiguousarray(H.imag, dtype=np.float64)
                      if np.iscomplexobj(H) else None)
        baths = prob["baths"]
        self._baths = (_abi.HeomBath * max(1, len(baths)))()
        for k, b in enumerate(baths):
            self._baths[k] = _abi.HeomBath(int(b["state"]), int(b["matsubara"]),
                                           float(b["lambda_cm"]), float(b["tau_fs"]))
        dp = ctypes.POINTER(ctypes.c_double)
        self.struct = _abi.HeomProblem(
            self.N, len(baths), self._h_re.ctypes.data_as(dp),
            self._h_im.ctypes.data_as(dp) if self._h_im is not None else None,
            self._baths, float(prob["temperature_K"]), int(prob["depth"]), int(precision),
            int(prob.get("flags", 0)))
        self.precision = int(precision)


def plan(prob, precision=FP64):
    """heom_plan: sizes of a problem as a dict (host only, no GPU needed)."""
    p = prob if isinstance(prob, Problem) else Problem(prob, precision)
    info = _abi.HeomInfo()
    check(load().heom_plan(ctypes.byref(p.struct), ctypes.byref(info)))
    return {f: getattr(info, f) for f, _ in _abi.HeomInfo._fields_}


def problem_coefficients(prob):
    """heom_problem_coefficients: (gamma [W], c [W], lambda*nu [W], Delta [N]) of a
    problem, on the host (no GPU needed)."""
    p = prob if isinstance(prob, Problem) else Problem(prob)
    info = plan(p)
    W, N = max(int(info["n_modes"]), 1), int(info["n_states"])
    g, c, ln, ds = np.zeros(W), np.zeros(W), np.zeros(W), np.zeros(N)
    check(load().heom_problem_coefficients(ctypes.byref(p.struct), g.ctypes.data, c.ctypes.data,
                                           ln.ctypes.data, ds.ctypes.data))
    n = int(info["n_modes"])
    return g[:n], c[:n], ln[:n], ds


def spectrum(P, dt_fs, omega_cm):
    """heom_spectrum: linear absorption from P [n_dir, n_t] (complex)."""
    P = np.ascontiguousarray(np.atleast_2d(P), dtype=np.complex128)
    w = np.ascontiguousarray(omega_cm, dtype=np.float64)
    S = np.zeros(len(w))
    check(load().heom_spectrum(P.ctypes.data, P.shape[0], P.shape[1], float(dt_fs), w.ctypes.data,
                               len(w), S.ctypes.data))
    return S


def _info_struct(d):
    info = _abi.HeomInfo()
    for f, _ in _abi.HeomInfo._fields_:
        setattr(info, f, d[f])
    return info


def pack_hermitian(x):
    """Hermitian matrices [..., N, N] -> the packed real layout of the
    FP32_HERM storage: P[i][j] = Re x[i][j] (i <= j), Im x[j][i] (i > j)."""
    x = np.asarray(x)
    upper = np.triu(np.ones(x.shape[-2:], bool))
    return np.where(upper, x.real, np.swapaxes(x.imag, -1, -2))


def unpack_hermitian(p):
    """Inverse of pack_hermitian: complex128 [..., N, N]."""
    p = np.asarray(p, np.float64)
    pt = np.swapaxes(p, -1, -2)
    i, j = np.indices(p.shape[-2:])
    re = np.where(i <= j, p, pt)
    im = np.where(i < j, pt, np.where(i > j, -p, 0.0))
    return re + 1j * im


class Hierarchy:
    """A hierarchy built on the current GPU (heom_build_hierarchy)."""

    def __init__(self, prob, precision=FP64, stream=None):
        torch = _torch()
        self.problem = Problem(prob, precision)
        self.precision = int(precision)
        self.info = plan(self.problem)
        self.N = self.problem.N
        self.n_ado = int(self.info["n_ado"])
        self.W = int(self.info["n_modes"])
        self.tables_dev = torch.empty(self.info["tables_bytes"], dtype=torch.uint8, device="cuda")
        h = ctypes.c_void_p()
        check(load().heom_build_hierarchy(ctypes.byref(self.problem.struct),
                                          ctypes.c_void_p(self.tables_dev.data_ptr()),
                                          self.info["tables_bytes"], _stream_handle(stream),
                                          ctypes.byref(h)))
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                load().heom_destroy(h)
            except Exception:
                pass
            self.handle = None

    # -------------------------------------------------------------- state --
    @property
    def rest_dtype(self):
        torch = _torch()
        return {FP64: torch.complex128, FP32_MIXED: torch.complex64}.get(self.precision,
                                                                         torch.float32)

    @property
    def _host_rest_dtype(self):
        return {FP64: np.complex128, FP32_MIXED: np.complex64}.get(self.precision, np.float32)

    def new_state(self, rho0=None):
        """(sigma0 complex128 [N,N], rest [n_ado-1,N,N]) on the GPU, zeroed;
        sigma0 set to rho0 if given."""
        torch = _torch()
        s0 = torch.zeros((self.N, self.N), dtype=torch.complex128, device="cuda")
        rest = torch.zeros((max(self.n_ado - 1, 0), self.N, self.N), dtype=self.rest_dtype,
                           device="cuda")
        if rho0 is not None:
            s0.copy_(torch.as_tensor(np.asarray(rho0, dtype=np.complex128)))
        return s0, rest

    def state_from_numpy(self, full):
        """Device state from a numpy complex array [n_ado, N, N]."""
        torch = _torch()
        full = np.asarray(full)
        s0 = torch.as_tensor(np.ascontiguousarray(full[0], dtype=np.complex128)).cuda()
        rest = full[1:] if self.precision != FP32_HERM else pack_hermitian(full[1:])
        rest = torch.as_tensor(np.ascontiguousarray(rest, dtype=self._host_rest_dtype)).cuda()
        return s0, rest

    def state_to_numpy(self, state):
        """Host complex128 [n_ado, N, N] of a device state."""
        s0, rest = state
        out = np.zeros((1 + rest.shape[0],) + tuple(s0.shape), np.complex128)
        out[0] = s0.cpu().numpy()
        r = rest.cpu().numpy()
        out[1:] = unpack_hermitian(r) if self.precision == FP32_HERM else r
        return out

    @staticmethod
    def _st(state):
        s0, rest = state
        return _abi.HeomState(s0.data_ptr(), rest.data_ptr() if rest.numel() else None)

    # ---------------------------------------------------------------- calls --
    def tables(self):
        """(tuples uint8 [n][W], plus int32 [n][W], minus int32 [n][W], level uint8 [n])."""
        n, W = self.n_ado, max(self.W, 1)
        t = np.zeros((n, W), np.uint8)
        p = np.zeros((n, W), np.int32)
        m = np.zeros((n, W), np.int32)
        lev = np.zeros(n, np.uint8)
        check(load().heom_copy_tables(self.handle, t.ctypes.data, p.ctypes.data, m.ctypes.data,
                                      lev.ctypes.data, _stream_handle()))
        return t[:, :self.W], p[:, :self.W], m[:, :self.W], lev

    def coefficients(self):
        W, N = max(self.W, 1), self.N
        g, c, ln, ds = np.zeros(W), np.zeros(W), np.zeros(W), np.zeros(N)
        check(load().heom_coefficients(self.handle, g.ctypes.data, c.ctypes.data, ln.ctypes.data,
                                       ds.ctypes.data))
        return g[:self.W], c[:self.W], ln[:self.W], ds

    def rhs(self, state_in, state_out, hermitian=False, stream=None):
        check(load().heom_rhs(self.handle, self._st(state_in), self._st(state_out),
                              1 if hermitian else 0, _stream_handle(stream)))

    def work_bytes(self, n_steps, record_every, kind):
        info = _info_struct(self.info)
        return load().heom_propagate_work_bytes(ctypes.byref(info), n_steps, record_every, kind)

    def workspace(self, n_steps, record_every, kind):
        torch = _torch()
        return torch.empty(self.work_bytes(n_steps, record_every, kind), dtype=torch.uint8,
                           device="cuda")

    def propagate(self, state, dt_fs, n_steps, record_every=1, observable=None, hermitian=False,
                  work=None, stream=None, want_records=True):
        """heom_propagate; returns the records [n_rec, record_doubles] (numpy)."""
        obs = observable or {"kind": "population"}
        kind = OBS_POPULATION if obs["kind"] == "population" else OBS_DIPOLE
        mu = np.ascontiguousarray(obs.get("mu", np.zeros(self.N)), dtype=np.float64)
        o = _abi.HeomObservable(kind, int(obs.get("ground", 0)),
                                mu.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        if work is None:
            work = self.workspace(n_steps, record_every, kind)
        n_rec = load().heom_record_count(n_steps, record_every)
        rd = load().heom_record_doubles(self.N, kind)
        rec = np.zeros((n_rec, rd)) if want_records else None
        check(load().heom_propagate(self.handle, self._st(state), ctypes.c_void_p(work.data_ptr()),
                                    work.numel(), float(dt_fs), int(n_steps), int(record_every),
                                    ctypes.byref(o), 1 if hermitian else 0,
                                    rec.ctypes.data if rec is not None else None,
                                    _stream_handle(stream)))
        return rec

    def propagate_noalloc(self, state, dt_fs, n_steps, record_every=1, observable=None,
                          hermitian=False, stream=None):
        """heom_propagate_noalloc (workspace in the library's static device
        scratch); returns the records [n_rec, record_doubles] (numpy)."""
        obs = observable or {"kind": "population"}
        kind = OBS_POPULATION if obs["kind"] == "population" else OBS_DIPOLE
        mu = np.ascontiguousarray(obs.get("mu", np.zeros(self.N)), dtype=np.float64)
        o = _abi.HeomObservable(kind, int(obs.get("ground", 0)),
                                mu.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        n_rec = load().heom_record_count(n_steps, record_every)
        rec = np.zeros((n_rec, load().heom_record_doubles(self.N, kind)))
        check(load().heom_propagate_noalloc(self.handle, self._st(state), float(dt_fs),
                                            int(n_steps), int(record_every), ctypes.byref(o),
                                            1 if hermitian else 0, rec.ctypes.data,
                                            _stream_handle(stream)))
        return rec

    def block_state(self, mu3):
        """Start of a coherence-block absorption run: complex128 [n_ado, N, 3]
        on the GPU with Y_0[a][p] = mu3[p][a], every other ADO zero."""
        torch = _torch()
        y = torch.zeros((self.n_ado, self.N, 3), dtype=torch.complex128, device="cuda")
        y[0] = torch.as_tensor(np.asarray(mu3, np.float64).T.astype(np.complex128))
        return y

    def propagate_block(self, y, dt_fs, n_steps, record_every, obs, stream=None, work=None):
        """heom_propagate_block; returns the correlations P [n_rec, 3] (complex)."""
        torch = _torch()
        o = np.ascontiguousarray(obs, dtype=np.float64)
        if o.shape != (3, self.N):
            raise ValueError("obs must be [3][N]")
        info = _info_struct(self.info)
        nb = load().heom_block_work_bytes(ctypes.byref(info), int(n_steps), int(record_every))
        if work is None:
            work = torch.empty(nb, dtype=torch.uint8, device="cuda")
        if work.numel() < nb:
            raise ValueError("block workspace smaller than heom_block_work_bytes")
        n_rec = load().heom_record_count(n_steps, record_every)
        rec = np.zeros((n_rec, 6))
        check(load().heom_propagate_block(self.handle, ctypes.c_void_p(y.data_ptr()),
                                          ctypes.c_void_p(work.data_ptr()), work.numel(), float(dt_fs),
                                          int(n_steps), int(record_every), o.ctypes.data,
                                          rec.ctypes.data, _stream_handle(stream)))
        return rec[:, 0::2] + 1j * rec[:, 1::2]

    def get_state(self, state):
        s0, rest = state
        h0 = np.zeros((self.N, self.N), np.complex128)
        hr = np.zeros(tuple(rest.shape), self._host_rest_dtype)
        check(load().heom_get_state(self.handle, self._st(state), h0.ctypes.data,
                                    hr.ctypes.data if hr.size else None, _stream_handle()))
        return h0, hr

    def set_state(self, state, host_sigma0, host_rest):
        h0 = np.ascontiguousarray(host_sigma0, dtype=np.complex128)
        hr = np.ascontiguousarray(host_rest, dtype=self._host_rest_dtype)
        check(load().heom_set_state(self.handle, self._st(state), h0.ctypes.data,
                                    hr.ctypes.data if hr.size else None, _stream_handle()))


def set_launch_shape(max_workgroups=0, max_ados_per_tile=0):
    """heom_set_launch_shape: cap the persistent kernel's workers and the FMA
    kernel's ADOs per workgroup (0 = the library's choice)."""
    check(load().heom_set_launch_shape(int(max_workgroups), int(max_ados_per_tile)))


def cd_vectors(R, d):
    """heom_cd_vectors: m [3][N], m[p][a] = (R_a x d_a) . e_p (host only)."""
    R = np.ascontiguousarray(R, dtype=np.float64)
    d = np.ascontiguousarray(d, dtype=np.float64)
    n = R.shape[0]
    if R.shape != (n, 3) or d.shape != (n, 3):
        raise ValueError("R and d must be [N][3]")
    m = np.zeros((3, n))
    check(load().heom_cd_vectors(R.ctypes.data, d.ctypes.data, n, m.ctypes.data))
    return m


def emission_start(h_exc, state_exc, h_full, state_full, mu, stream=None):
    """heom_emission_start: Y_u = sigma_u(inf) mu^+ of every ADO of the
    thermalised N-state hierarchy, embedded into the (N+1)-state state_full."""
    m = np.ascontiguousarray(mu, dtype=np.float64)
    if m.shape != (h_exc.N,):
        raise ValueError("mu must have N entries")
    check(load().heom_emission_start(h_exc.handle, Hierarchy._st(state_exc), h_full.handle,
                                     Hierarchy._st(state_full), m.ctypes.data,
                                     _stream_handle(stream)))


class Server:
    """Continuous-batching server (heom_server_create / heom_submit / heom_poll).

    The arena is one caller-owned device buffer; the library sub-allocates
    tables, states, workspaces and records of admitted requests from it."""

    def __init__(self, arena_bytes, max_active, stream=None):
        torch = _torch()
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device="cuda")
        self._stream = stream
        h = ctypes.c_void_p()
        check(load().heom_server_create(ctypes.c_void_p(self.arena.data_ptr()), int(arena_bytes),
                                        int(max_active), _stream_handle(stream), ctypes.byref(h)))
        self.handle = h
        self._keep = {}

    def submit(self, runs, precision=FP32_MIXED, hermitian=None, form=0):
        """Submit runs (list of run dicts sharing one problem, see heom_inputs)
        as one request; returns its ticket.  form: 0 = the server may use the
        coherence-block form for eligible dipole runs, 1 = full matrices."""
        r0 = runs[0]
        prob = Problem(r0, precision)
        N = prob.N
        kind = OBS_POPULATION if r0["observable"]["kind"] == "population" else OBS_DIPOLE
        rho0 = np.ascontiguousarray(np.stack([np.asarray(r["rho0"], np.complex128) for r in runs]))
        mu = np.ascontiguousarray(np.stack([np.asarray(r["observable"].get("mu", np.zeros(N)),
                                                       np.float64) for r in runs]))
        if hermitian is None:
            hermitian = kind == OBS_POPULATION
        dp = ctypes.POINTER(ctypes.c_double)
        req = _abi.HeomRequest(prob.struct, len(runs), int(r0["record_every"]), int(r0["n_steps"]),
                               float(r0["dt_fs"]), rho0.ctypes.data_as(dp),
                               _abi.HeomObservable(kind, int(r0["observable"].get("ground", 0)),
                                                   mu.ctypes.data_as(dp)),
                               1 if hermitian else 0, int(form))
        t = ctypes.c_uint64()
        check(load().heom_submit(self.handle, ctypes.byref(req), ctypes.byref(t)))
        self._keep[t.value] = len(runs)
        return t.value

    def _result(self, ticket, res, status):
        n_runs = self._keep.get(ticket, 1)
        out = {"status": status, "t_submit": res.t_submit_s, "t_admit": res.t_admit_s,
               "t_finish": res.t_finish_s, "form": res.form, "records": None}
        if status == _abi.HEOM_OK and res.records:
            n = n_runs * res.n_records * res.record_doubles
            arr = np.ctypeslib.as_array(res.records, shape=(n,)).copy()
            out["records"] = arr.reshape(n_runs, res.n_records, res.record_doubles)
        return out

    def poll(self, ticket):
        res = _abi.HeomResult()
        st = load().heom_poll(self.handle, ticket, ctypes.byref(res))
        if st == -7:
            check(st)
        return self._result(ticket, res, st)

    def wait(self, ticket, timeout_s=-1.0):
        res = _abi.HeomResult()
        st = load().heom_wait(self.handle, ticket, float(timeout_s), ctypes.byref(res))
        if st == -7:
            check(st)
        return self._result(ticket, res, st)

    def cancel(self, ticket):
        check(load().heom_cancel(self.handle, ticket))

    def release(self, ticket):
        check(load().heom_release(self.handle, ticket))
        self._keep.pop(ticket, None)

    def set_log(self, path):
        """heom_server_set_log: one JSON line per finished request appended to
        `path` (None stops the log)."""
        check(load().heom_server_set_log(self.handle, None if path is None else str(path).encode()))

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            load().heom_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
