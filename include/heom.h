/*
 * heom.h — C ABI of the MI355X (gfx950) HEOM library.
 *
 * The library evaluates the hierarchical equations of motion (eq. HEOM of the
 * section "HEOM formalism" of Kramer et al., "Efficient calculation of open
 * quantum system dynamics and time-resolved spectroscopy with Distributed
 * Memory HEOM (DM-HEOM)", arXiv:1803.03498) for a Frenkel-exciton Hamiltonian
 * (eq. h-ex) coupled to Drude-Lorentz baths (eq. spectral_density_DL with
 * Omega = 0) expanded in Matsubara terms, and integrates them with classic
 * RK4 (four right-hand-side evaluations per step, section "Distributed memory
 * HEOM implementation").
 *
 * Conventions used throughout:
 *   - Units at the boundary: energies in cm^-1, times in fs, temperature in K.
 *     Internally hbar = 1 and energies are angular frequencies in rad/fs.
 *   - A hierarchy member ("ADO") sigma_u is an N x N complex matrix, row-major,
 *     real and imaginary parts interleaved.  u = 0 is the reduced density
 *     matrix rho = sigma_0.  ADOs are numbered by level |n| = 0..D and, inside a
 *     level, by descending lexicographic order of the index tuple n.
 *   - Mode l of the tuple is bath b, Matsubara term k: l = (sum of (1 + M_b')
 *     over baths b' < b) + k, 0-based (the paper's l = (b-1)K + k + 1 when
 *     every bath has K = 1 + M modes).
 *   - Device memory is always owned by the caller: every call that needs
 *     device memory takes a pointer and a size obtained from heom_plan (or the
 *     size helpers below).  The library never allocates device memory.
 *   - Streams are hipStream_t values passed as void* (NULL = default stream).
 *     Work is enqueued on that stream; calls documented as synchronous wait
 *     for the stream before returning.
 *   - Every call returns a heom_status.  On failure heom_last_error() returns a
 *     thread-local message.  No C++ exception crosses the ABI.
 */
#ifndef HEOM_H
#define HEOM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t heom_status;

enum {
    HEOM_OK = 0,
    HEOM_PENDING = 1,         /* heom_poll: the request has not finished      */
    HEOM_E_INVAL = -1,        /* invalid argument or problem                  */
    HEOM_E_RANGE = -2,        /* sizes overflow (n_ado >= 2^31, N > 64, ...)  */
    HEOM_E_NOMEM = -3,        /* caller buffer too small / can never fit      */
    HEOM_E_DEVICE = -4,       /* HIP runtime error or no gfx950 device        */
    HEOM_E_NUMERIC = -5,      /* NaN/Inf seen by an FP64 observable reduction */
    HEOM_E_UNSTABLE = -6,     /* dt times the rate bound leaves RK4's region  */
    HEOM_E_NOTFOUND = -7,     /* unknown ticket                               */
    HEOM_E_CANCELLED = -8     /* request cancelled before it finished         */
};

/* Precision of the hierarchy state. */
enum {
    HEOM_FP64 = 0,        /* every ADO complex128                                   */
    HEOM_FP32_MIXED = 1,  /* sigma_0 complex128 with FP64 RK4 and FP64 observables; */
                          /* ADOs u >= 1 complex64 with FP32 arithmetic             */
    HEOM_FP32_HERM = 2    /* as HEOM_FP32_MIXED for Hermitian ADOs (population runs,
                             hermitian = 1 only), each ADO u >= 1 stored packed as one
                             real FP32 N x N matrix P: P[i][j] = Re sigma[i][j] for
                             i <= j and P[i][j] = Im sigma[j][i] for i > j, half the
                             bytes of complex64.  Needs the matrix-core path (real H,
                             16 <= N <= 64); not accepted by heom_submit.           */
};

/* Switches (heom_problem.flags).  Both the library and the oracle honour them. */
enum {
    HEOM_FLAG_NO_RESCALE = 1u,     /* plain couplings i V^x and n theta instead of the
                                      rescaled ones (substitution of section "HEOM
                                      formalism") */
    HEOM_FLAG_NO_TERMINATOR = 2u,  /* drop the third line of eq. HEOM                  */
    HEOM_FLAG_ADD_REORG = 4u,      /* add lambda_b to H[s_b][s_b] (eq. h-ex)           */
    HEOM_FLAG_STANDARD_GAUGE = 8u, /* flip the sign of both coupling lines             */
    HEOM_FLAG_PADE = 16u           /* Pade expansion of the Bose function (section "HEOM
                                      formalism", the replacement of the Matsubara
                                      expansion): each bath's n_matsubara counts Pade
                                      poles K (1 + K modes, K <= 64), gamma(b,k) and
                                      c(b,k) take their Pade forms.  The correction
                                      coefficient Delta then vanishes up to rounding. */
};

/* Observables recorded from sigma_0 (FP64). */
enum {
    HEOM_OBS_POPULATION = 0, /* record = [Re rho_mm (m < N), Re Tr, Im Tr, max|rho - rho^+|] */
    HEOM_OBS_DIPOLE = 1      /* record = [Re P, Im P, Re Tr, Im Tr], P = sum_a mu_a rho[a][g]
                                (polarisation of eq. polarization with mu^+ of eq.
                                mu_plusp, section "Optical spectra") */
};

/* One Drude-Lorentz bath (eq. spectral_density_DL, Omega = 0) coupled to the
 * projector |state><state| (section "Frenkel exciton model"). */
typedef struct {
    int32_t state;        /* 0 <= state < n_states                        */
    int32_t n_matsubara;  /* M >= 0: the bath contributes 1 + M modes (M Matsubara
                             terms, or M Pade poles with HEOM_FLAG_PADE)  */
    double lambda_cm;     /* reorganisation energy lambda >= 0, cm^-1     */
    double tau_fs;        /* nu^-1 > 0, fs                                */
} heom_bath;

typedef struct {
    int32_t n_states;       /* N, 1..64                                         */
    int32_t n_baths;        /* B >= 0                                           */
    const double* h_re_cm;  /* [N*N] row-major Hermitian H, cm^-1 (required)    */
    const double* h_im_cm;  /* [N*N] or NULL for a real symmetric H             */
    const heom_bath* baths; /* [B]                                              */
    double temperature_K;   /* T > 0                                            */
    int32_t depth;          /* truncation depth D >= 0 (sum of tuple <= D)      */
    int32_t precision;      /* HEOM_FP64, HEOM_FP32_MIXED or HEOM_FP32_HERM     */
    uint32_t flags;         /* HEOM_FLAG_*                                      */
} heom_problem;

/* Sizes of a problem (heom_plan). */
typedef struct {
    int64_t n_ado;          /* C(W + D, W), eq. Nmatrices                 */
    int64_t n_plus_edges;   /* number of valid "+" links                  */
    int32_t n_states;       /* N                                          */
    int32_t n_modes;        /* W = sum over baths of (1 + M_b)            */
    int32_t depth;          /* D                                          */
    int32_t elem_bytes;     /* bytes per element of ADOs u >= 1 (16/8/4)  */
    size_t tables_bytes;    /* device bytes for heom_build_hierarchy      */
    size_t sigma0_bytes;    /* N*N*16                                     */
    size_t rest_bytes;      /* (n_ado - 1) * N*N * elem_bytes             */
    size_t work_bytes;      /* device workspace of heom_propagate without
                               records (three RK4 stage copies + control) */
    int32_t bulk_kernel;    /* stage kernel of ADOs u >= 1: 1 = matrix-core
                               commutator (real H, N >= 16), 0 = FMA       */
    int32_t reserved;
} heom_info;

/* A hierarchy state: sigma_0 (complex128 [N][N]) and ADOs 1..n_ado-1
 * (complex128, complex64 or packed real FP32 [n_ado-1][N][N] by precision).  Both device
 * pointers, 256-byte aligned, caller-owned.  In HEOM_FP64, rest may equal
 * sigma0 + N*N complex elements (one contiguous array). */
typedef struct {
    void* sigma0;
    void* rest;
} heom_state;

typedef struct {
    int32_t kind;        /* HEOM_OBS_*                                         */
    int32_t ground;      /* HEOM_OBS_DIPOLE: index g of the ground state       */
    const double* mu;    /* HEOM_OBS_DIPOLE: host [N] projected dipoles e_p.d_a */
} heom_observable;

typedef struct heom_hierarchy heom_hierarchy;

/* Message of the last failed call on this thread ("" if none). */
const char* heom_last_error(void);
/* Static name of a status code. */
const char* heom_status_string(heom_status s);

/* Host only (no device call): validate a problem and report its sizes.
 * Validation (HEOM_E_INVAL): N in 1..64, D >= 0, B >= 0, bath states in
 * [0, N), lambda >= 0, tau > 0, M >= 0, T > 0, finite inputs, H Hermitian to
 * 1e-12 relative, no Matsubara rate equal to nu.  HEOM_E_RANGE if
 * n_ado >= 2^31 or W > 255 or D > 255. */
heom_status heom_plan(const heom_problem* problem, heom_info* info);

/* Bytes per record and records produced by a propagation (step 0 plus every
 * record_every-th step). */
int32_t heom_record_doubles(int32_t n_states, int32_t kind);
int64_t heom_record_count(int64_t n_steps, int32_t record_every);
/* Device workspace for heom_propagate: info->work_bytes plus the records. */
size_t heom_propagate_work_bytes(const heom_info* info, int64_t n_steps, int32_t record_every,
                                 int32_t kind);

/* Build the hierarchy on the device: bath coefficients (host FP64, section
 * "HEOM formalism": gamma(b,k), c(b,k), the correction coefficient of the third
 * line, rescaled coupling weights), then on the GPU the tuple enumeration of
 * eq. Nmatrices, the +/- link tables ("computed in a first step") and the
 * per-ADO damping sum_l n_l gamma_l.  tables_dev must hold info.tables_bytes
 * bytes and stay valid until heom_destroy.  Asynchronous on `stream`; the
 * problem struct may be freed on return.  *out receives a handle. */
heom_status heom_build_hierarchy(const heom_problem* problem, void* tables_dev,
                                 size_t tables_bytes, void* stream, heom_hierarchy** out);

/* Synchronous: copy the tables to host buffers (any may be NULL):
 * tuples uint8 [n_ado][W], plus/minus int32 [n_ado][W] (-1 = absent link),
 * level uint8 [n_ado]. */
heom_status heom_copy_tables(const heom_hierarchy* h, uint8_t* tuples, int32_t* plus,
                             int32_t* minus, uint8_t* level, void* stream);

/* Host copy of the per-mode coefficients (FP64, hbar = 1): gamma [W] (1/fs),
 * c [W] (rad/fs^2), lambda*nu [W] (0 for k > 0), and delta [N] (the correction
 * coefficient summed per state, 1/fs).  Any pointer may be NULL. */
heom_status heom_coefficients(const heom_hierarchy* h, double* gamma, double* c, double* lamnu,
                              double* delta_state);

/* The same coefficients straight from a problem, on the host (no GPU, no
 * hierarchy): validates the problem as heom_plan does; the arrays hold W
 * (n_modes of heom_plan) and N entries.  Any pointer may be NULL. */
heom_status heom_problem_coefficients(const heom_problem* problem, double* gamma, double* c,
                                      double* lamnu, double* delta_state);

/* One evaluation out = f(in) of eq. HEOM (with the rescaled couplings unless
 * HEOM_FLAG_NO_RESCALE) over every ADO.  in and out must not overlap.
 * Asynchronous.  hermitian != 0 asserts that every ADO of `in` is Hermitian:
 * the kernels then read the column s of a neighbour as the conjugate of its
 * row s (otherwise the result is undefined). */
heom_status heom_rhs(const heom_hierarchy* h, heom_state in, heom_state out, int32_t hermitian,
                     void* stream);

/* Advance `io` by n_steps classic RK4 steps of dt_fs:
 *   Y2 = y + dt/2 f(y), Y3 = y + dt/2 f(Y2), Y4 = y + dt f(Y3),
 *   y' = (-y + Y2 + 2 Y3 + Y4)/3 + dt/6 f(Y4),
 * the textbook step rewritten so that each stage reads one ADO array with its
 * neighbours and writes the next.  work_dev (heom_propagate_work_bytes) holds
 * the three stage copies, the records and a status word.  Observables of
 * sigma_0 are reduced in FP64 at step 0 and every record_every steps.
 * hermitian: as for heom_rhs, for the initial state (it is preserved).
 * Synchronous: returns after the stream has finished; if host_out != NULL
 * the records are copied to host_out [n_rec][heom_record_doubles].
 * HEOM_E_UNSTABLE if dt exceeds the RK4 bound for the problem's rates;
 * HEOM_E_NUMERIC if a recorded observable was not finite.  Runs of 8 steps
 * or more launch the first step directly and replay a HIP graph of one step
 * (captured on a private stream) for the rest, unless kernel timing is on
 * (heom_timing_enable); the results are the same either way, bit for bit. */
heom_status heom_propagate(const heom_hierarchy* h, heom_state io, void* work_dev,
                           size_t work_bytes, double dt_fs, int64_t n_steps, int32_t record_every,
                           const heom_observable* obs, int32_t hermitian, double* host_out,
                           void* stream);

/* heom_propagate for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the workspace is the library's static device scratch, one 64 MiB array per
 * GPU held until the process ends, instead of a caller buffer.  Same
 * arguments, results and errors as heom_propagate otherwise; the step counter,
 * status word and records in the scratch are rewritten at every call.
 * HEOM_E_NOMEM if heom_propagate_work_bytes exceeds 64 MiB (three stage copies
 * of the state plus the records).  Allocates nothing (no hipMalloc/hipFree,
 * no events).  All calls on one GPU share its scratch: calls that overlap on
 * one GPU (from several threads or streams) race and must be serialised by
 * the caller; a call is complete when it returns (it synchronises). */
heom_status heom_propagate_noalloc(const heom_hierarchy* h, heom_state io, double dt_fs,
                                   int64_t n_steps, int32_t record_every,
                                   const heom_observable* obs, int32_t hermitian,
                                   double* host_out, void* stream);

/* Checkpoint / resume of a state: synchronous device <-> host copies of
 * sigma_0 (complex128 [N][N]) and the ADOs u >= 1 (element type by precision). */
heom_status heom_get_state(const heom_hierarchy* h, heom_state s, void* host_sigma0,
                           void* host_rest, void* stream);
heom_status heom_set_state(const heom_hierarchy* h, heom_state s, const void* host_sigma0,
                           const void* host_rest, void* stream);

/* Linear absorption in the coherence-block form (section "Linear absorption
 * spectra" with the ground state uncoupled): for the hierarchy `h` of the N
 * excited states alone (in the frame where the ground energy is 0), each
 * ADO keeps only its column g, for three directions at once: `state` is
 * complex128 [n_ado][N][3], Y_u[a][p] = sigma_u^{(p)}[a][g] (start:
 * Y_0[a][p] = mu_p[a], every other ADO 0).  Classic RK4 in FP64 (the
 * arrays are 3N complex per ADO instead of 3 (N+1)^2).  Records, every
 * record_every steps from step 0, the correlations
 * P_p = sum_a obs[p][a] Y_0[a][p] as [n_rec][6] (Re P_x, Im P_x, ..., Im P_z):
 * obs = mu gives the absorption correlation of eq. polarization; another
 * dipole-like vector per direction (e.g. the magnetic term of circular
 * dichroism) gives the corresponding cross correlation.  `work_dev` holds
 * heom_block_work_bytes; obs is a host pointer [3][N].  Synchronous.
 * HEOM_E_UNSTABLE as for heom_propagate, with the mean of diag(H) added to
 * the rate bound (a single column keeps it), and also when that mean times
 * dt exceeds 0.5 rad: give the excited block in a frame rotating near the
 * excited energies (subtract their mean).  HEOM_E_NUMERIC as for
 * heom_propagate. */
size_t heom_block_work_bytes(const heom_info* info, int64_t n_steps, int32_t record_every);
heom_status heom_propagate_block(const heom_hierarchy* h, void* state, void* work_dev,
                                 size_t work_bytes, double dt_fs, int64_t n_steps,
                                 int32_t record_every, const double* obs, double* host_out,
                                 void* stream);

/* Host only: the excitation vectors of circular dichroism (eq.
 * CDdipoleoperator, section "Circular dichroism spectra"):
 *   m[p][a] = (R_a x d_a) . e_p,  p = x, y, z,
 * for pigment centres R [N][3] and transition dipoles d [N][3] (any
 * consistent units).  A coherence-block run started from m (Y_0[a][p] =
 * m[p][a]) and observed with the dipoles (obs[p][a] = d_a . e_p) gives the
 * rotationally averaged CD correlation through heom_spectrum. */
heom_status heom_cd_vectors(const double* R, const double* d, int32_t n_sites, double* m);

/* Start of a static fluorescence run (section "Static Fluorescence
 * Spectra"): the dipole operator acts on every ADO of the thermalised
 * hierarchy.  `exc` describes the N excited states alone (its state
 * `exc_state` holds sigma_u(inf), e.g. after a long population run from the
 * Boltzmann state); `full` the same baths on N + 1 states with the ground
 * state at index 0 and site a at index 1 + a (equal mode count and depth, so
 * equal ADO numbering).  Writes into `full_state`, for every ADO u,
 *   Y_u[1 + a][0] = sum_b sigma_u(inf)[a][b] mu[b],   all other elements 0,
 * i.e. sigma_u(inf) mu^+ restricted to the (e, g) block.  Propagating Y with
 * the dipole observable (mu on indices 1..N, ground 0, hermitian = 0) gives
 * the emission correlation whose heom_spectrum is the fluorescence of
 * direction mu.  mu: host pointer, N doubles (e_p . d_a).  Both hierarchies
 * on the current device; exc in HEOM_FP64 or HEOM_FP32_MIXED, full in
 * either (elements converted).  Enqueued on `stream` (not synchronised).
 * HEOM_E_INVAL on a mismatch (N, W, D) or a packed precision. */
heom_status heom_emission_start(const heom_hierarchy* exc, heom_state exc_state,
                                const heom_hierarchy* full, heom_state full_state,
                                const double* mu, void* stream);

/* Host only: linear absorption spectrum from dipole-correlation records
 * (eq. lin_abs_mukamel on a finite window, section "Linear absorption
 * spectra"):  S(w_k) = Re sum_p sum_n c_n exp(i w_k t_n) P_p(t_n) dt,
 * trapezoid weights c_0 = c_last = 1/2, t_n = n * dt_fs.  P is interleaved
 * complex [n_dir][n_t] (the Re P, Im P columns of the records); omega_cm
 * [n_omega] in cm^-1 (relative to the rotating frame, if one was used);
 * S [n_omega] is written.  FP64. */
heom_status heom_spectrum(const double* P, int32_t n_dir, int64_t n_t, double dt_fs,
                          const double* omega_cm, int64_t n_omega, double* S);

/* Release a handle (does not touch caller memory). */
heom_status heom_destroy(heom_hierarchy* h);

/* Kernel timing, for benchmarks (process-wide, off by default).  While
 * enabled, heom_propagate brackets every launch of the bulk RK4 stage kernel
 * (ADOs u >= 1) with a pair of HIP events recorded on the caller's stream and,
 * after its final synchronisation, adds their elapsed times.  heom_timing_read
 * returns the accumulated milliseconds, the number of launches and the
 * algorithmic bytes those launches move (per RK4 step: 13 passes over the
 * ADO array, i.e. 2/3/3/5 passes for stages 1..4; neighbour reads counted
 * once), and optionally resets the counters. */
heom_status heom_timing_enable(int32_t enable);
/* Launch-shape override, for tests and tuning (process-wide; 0 = the
 * library's choice).  max_workgroups caps the number of workers of the
 * persistent stage kernel; max_ados_per_tile caps the ADOs one workgroup of
 * the FMA stage kernel takes (applied when a propagation or a server request
 * binds its workspace).  Every element is computed by the same arithmetic in
 * any shape, so results do not change, bit for bit.  Negative values:
 * HEOM_E_INVAL. */
heom_status heom_set_launch_shape(int32_t max_workgroups, int32_t max_ados_per_tile);
heom_status heom_timing_read(double* bulk_ms, int64_t* bulk_launches, double* bulk_bytes,
                             int32_t reset);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching of independent propagations.                  */
/* ------------------------------------------------------------------------ */

typedef struct heom_server heom_server;

/* A propagation request: a problem, its step count and observable, and n_runs
 * initial states that share the problem (e.g. three dipole directions of a
 * linear-absorption run).  rho0 is host complex128 [n_runs][N][N]; every other
 * ADO starts at zero.  obs.mu is [n_runs][N] for HEOM_OBS_DIPOLE. */
typedef struct {
    heom_problem problem;
    int32_t n_runs;         /* 1..8                                   */
    int32_t record_every;   /* >= 1                                   */
    int64_t n_steps;        /* >= 1                                   */
    double dt_fs;
    const double* rho0;     /* host complex128 [n_runs][N][N]         */
    heom_observable obs;    /* mu: [n_runs][N] for dipole runs        */
    int32_t hermitian;      /* the initial state is Hermitian         */
    int32_t form;           /* HEOM_FORM_*: how the server may run it  */
} heom_request;

/* heom_request.form.  AUTO lets the server run an eligible dipole request in
 * the coherence-block form (as heom_propagate_block, FP64): at most three
 * runs, the ground state `obs.ground` without a bath and without coupling in
 * H, each initial state zero outside column `ground` (rows != ground), and a
 * step that passes the block form's step check.  Its records keep the
 * layout of the full form: [Re P, Im P, Re Tr, Im Tr] with Tr = 0 exactly.
 * FULL always propagates the full density matrices in the request's
 * precision. */
enum { HEOM_FORM_AUTO = 0, HEOM_FORM_FULL = 1, HEOM_FORM_BLOCK = 2 /* reported only */ };

typedef struct {
    heom_status status;     /* HEOM_OK, HEOM_PENDING or an error       */
    int64_t n_records;      /* per run                                 */
    int32_t record_doubles; /* doubles per record                      */
    const double* records;  /* [n_runs][n_records][record_doubles], owned by
                               the server until heom_release          */
    double t_submit_s;      /* host monotonic clock, seconds           */
    double t_admit_s;
    double t_finish_s;
    int32_t form;           /* HEOM_FORM_FULL or HEOM_FORM_BLOCK: the form
                               the server chose at submission            */
} heom_result;

/* Create a server on one device stream.  arena_dev/arena_bytes is caller-owned
 * device memory that the server sub-allocates for tables, states, workspaces
 * and records of admitted requests; max_active bounds the requests resident
 * at once.  A scheduler thread owns the stream until heom_server_destroy. */
heom_status heom_server_create(void* arena_dev, size_t arena_bytes, int32_t max_active,
                               void* stream, heom_server** out);
/* Thread-safe.  Copies the request; HEOM_E_NOMEM if it can never fit the
 * arena, HEOM_E_INVAL / HEOM_E_RANGE as heom_plan. */
heom_status heom_submit(heom_server* s, const heom_request* req, uint64_t* ticket);
/* Thread-safe.  HEOM_PENDING until the request finished; then its status. */
heom_status heom_poll(heom_server* s, uint64_t ticket, heom_result* out);
/* Thread-safe: block until the request finished (timeout_s < 0: no limit). */
heom_status heom_wait(heom_server* s, uint64_t ticket, double timeout_s, heom_result* out);
/* Thread-safe: cancel a queued or running request. */
heom_status heom_cancel(heom_server* s, uint64_t ticket);
/* Thread-safe: free the result of a finished request. */
heom_status heom_release(heom_server* s, uint64_t ticket);
/* Thread-safe: append one JSON object per finished request, one per line,
 * to the file at `path` (created if absent); NULL stops the log.  Fields:
 * ticket, status, form ("full" / "block"), runs, n_states, n_ado, n_steps,
 * queue_ms (admission - submission), service_ms (finish - admission),
 * latency_ms, ado_updates (n_ado * n_steps * runs).  HEOM_E_INVAL if the
 * file cannot be opened. */
heom_status heom_server_set_log(heom_server* s, const char* path);
/* Stop the scheduler (running requests are cancelled) and free the server. */
heom_status heom_server_destroy(heom_server* s);

#ifdef __cplusplus
}
#endif

#endif /* HEOM_H */
