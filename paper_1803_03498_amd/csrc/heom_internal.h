// Internal descriptors shared by the host runtime and the gfx950 kernels.
// Not part of the C ABI (include/heom.h).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstddef>
#include <cstdint>
#include <string>

namespace heom {

constexpr int kMaxStates = 64;
// Size of the library's static device scratch (heom_propagate_noalloc).
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kBlock = 256;
// Threads of an FMA-path stage workgroup: FP32 256; FP64 64 (its registers
// allow fewer waves per SIMD, and smaller workgroups fill them better),
// except for N^2 <= 64, where 64 threads would hold a single ADO with idle
// lanes and 256 hold several.  The kernel loops over its tile's elements with
// the launch's block size, so any of these is correct for any tile.
constexpr int kFmaMaxBlock = 256;
__host__ __device__ constexpr int fma_block(int tsize, int N) {
    return (tsize == 4 || N * N <= 64) ? 256 : 64;
}

// Device pointers into the caller's tables buffer, plus the scalars the
// kernels need.  Everything here is written once by heom_build_hierarchy.
struct Tables {
    int32_t N, W, D, n_ado;
    int32_t h_complex;            // H has a non-zero imaginary part
    double h_shift;               // the mean of diag(H) taken off h_re, rad/fs
    const double* h_re;           // [N*N] rad/fs, diagonal shifted by -mean(diag)
    const double* h_im;           // [N*N]
    const float* h_re_f32;        // [N*N] h_re rounded to FP32 (FP32 stage kernels)
    const int32_t* mode_site;     // [W]
    const double* mode_gamma;     // [W] 1/fs
    const double* mode_c;         // [W] rad/fs^2 (times the gauge sign)
    const double* mode_lamnu;     // [W] lambda*nu for k = 0 (times the gauge sign)
    const double* plus_coef;      // [W][D+1]: sign * sqrt((n+1)|c_l|)
    const double* minus_coef;     // [W][D+1]: sqrt(n/|c_l|)
    const double* delta_state;    // [N] correction coefficient summed per state
    const int32_t* state_mode_begin;  // [N+1]
    const int32_t* state_modes;       // [W] modes grouped by coupled state
    const int64_t* binom;         // [(D+2)][(W+1)]: C(m+k, k), saturating
    uint8_t* tuples;              // [n_ado][W]
    uint8_t* level;               // [n_ado]
    int32_t* plus;                // [n_ado][W], -1 = absent
    int32_t* minus;               // [n_ado][W], -1 = absent
    int32_t* mlist;               // [n_ado][max(D,1)][2]: active "-" links in mode order,
                                  // [0] = neighbour (-1 = none), [1] = mode | n_l << 8
    int32_t* mlist_site;          // [n_ado][max(D,1)]: state of each "-" link (-1 = none)
    double* mlist_w;              // [n_ado][max(D,1)][2]: sqrt(n_l/|c_l|) * (lambda nu, c_l)
    float* mlist_w32;             // the same rounded to FP32 (FP32 stage kernels)
    double* plus_w;               // [n_ado][W]: sign * sqrt((n_l+1)|c_l|), 0 = absent
    double* damping;              // [n_ado]: sum_l n_l gamma_l
};

// One propagation (or one right-hand-side evaluation) as the kernels see it.
// Array slot 0 is the caller's state; slots 1..3 are RK4 stage copies.
struct Job {
    Tables t;
    void* sig0[4];                // complex128 [N][N]
    void* rest[4];                // [n_ado-1][N][N], complex128 or complex64
    double dt;
    int32_t herm;                 // every ADO is Hermitian
    int32_t tile_begin;           // first bulk tile of this job in a batched launch
    int32_t n_tiles;              // bulk tiles of this job
    int32_t ados_per_tile;
    uint32_t lds_bytes;           // batched launches: LDS of the largest tile (0 = derive)
    int32_t any_complex_h;        // some job of the launch has a complex H
    // Hermitian-packed storage only: complex64 copies [n_low][N][N] of the
    // ADOs 1..n_low (levels 1..D-1, the only "-" neighbours besides sigma_0),
    // so that "-" rows are read contiguously; see StageSpec::mirror_in.
    void* mirror[2];
    int32_t n_low;
    double* records;              // [n_rec_max][rec_doubles]
    const double* mu;             // [N] (dipole observable)
    int64_t* step;                // device step counter
    int32_t* status;              // device status word (1 = non-finite observable)
    int64_t n_rec_max;
    int32_t rec_every, rec_kind, rec_doubles, ground;
};

// What one RK4 stage launch reads and writes:
//   out = w_in * in + sum_m wbase[m] * base[m] + hmul * dt * f(in)
struct StageSpec {
    int32_t in, out;
    int32_t nbase;
    int32_t base[3];
    double wbase[3];
    double w_in;
    double hmul;
    int32_t record_initial;  // record sigma_0 of `in` when the step counter is 0
    int32_t record_after;    // advance the step counter, record the output
    // Hermitian-packed storage: 1 + index into Job::mirror of the copy of
    // `in` to read "-" rows from and of the copy of `out` to write (0 = none;
    // then "-" rows and columns are read from the packed ADOs).
    int32_t mirror_in, mirror_out;
};

// Launch-shape caps (heom_set_launch_shape; 0 = none).
extern std::atomic<int> g_max_workgroups, g_max_ados_per_tile;

// One coherence-block request in a batched launch (device job table).
struct BlockJob {
    Tables t;
    void* y[4];           // complex128 [n_ado][N][3]: the state (0) and stage copies
    double dt;
    int64_t elem_begin;   // first element of this job in the launch
    const double* obs;    // [3][N] observed vectors
    double* rec;          // [n_rec][6]
    int32_t* status;      // set to 1 by a non-finite record
    int64_t* step;        // steps completed, advanced by the record kernel
    int32_t record_every;
};

// Kernel launchers (heom_kernels.hip).  All enqueue on `stream` and return the
// HIP error of the launch.
hipError_t launch_enumerate(const Tables& t, hipStream_t stream);
// Complex64 copy of the packed ADOs 1..n into `mirror` (Hermitian-packed storage).
hipError_t launch_pk_mirror(const void* packed_rest, void* mirror, int N, int n, hipStream_t stream);
// Coherence-block absorption (one RK4 stage over all ADOs, FP64, Y[u][a][p]):
// out = w_in in + sum_m wb[m] base[m] + h f(in).
hipError_t launch_block_stage(const Tables& t, const void* in, void* out, const void* const* base,
                              const double* wb, int nbase, double w_in, double h,
                              hipStream_t stream);
// P_p = sum_a obs[p][a] Y_0[a][p] into rec[0..5] (Re, Im per direction);
// a non-finite value sets *status = 1.
hipError_t launch_block_record(const void* y, const double* obs, int N, double* rec,
                               int32_t* status, hipStream_t stream);
// The same stage over many requests of a device job table; total = the
// last job's elem_begin plus its n_ado * 3 * N.
hipError_t launch_block_stage_batched(const BlockJob* jobs_dev, int n_jobs, int64_t total,
                                      const StageSpec& sp, hipStream_t stream);
// After each step: every job's step counter advances; jobs whose record is
// due write P into rec + 6 * (step / record_every).
hipError_t launch_block_record_batched(const BlockJob* jobs_dev, int n_jobs, hipStream_t stream);
// Fluorescence start: Y_u = sigma_u mu^+ embedded in the (N+1)-state ADOs
// (precisions 0 = complex128, 1 = complex64 for the bulk of each side).
hipError_t launch_emission_start(const void* in_sig0, const void* in_rest, int in_prec,
                                 void* out_sig0, void* out_rest, int out_prec, const double* mu,
                                 int N, int64_t n_ado, hipStream_t stream);
// ev_begin/ev_end (may be null) bracket the bulk-kernel launch.
hipError_t launch_stage(const Job& single, const Job* jobs_dev, int n_jobs, int total_tiles,
                        int precision, const StageSpec& sp, hipStream_t stream,
                        hipEvent_t ev_begin = nullptr, hipEvent_t ev_end = nullptr);
// LDS carve-up of an FMA-path tile of GA ADOs (bytes).
struct FmaLds {
    size_t h, s, mw, pw, mi, pi, lev, st, total;
};

__host__ __device__ inline FmaLds fma_lds(int N, int W, int D, int GA, int tsize) {
    const int Dm = D > 0 ? D : 1;
    const size_t NN = (size_t)N * N;
    FmaLds L{};
    size_t o = 0;
    L.h = o; o += 2 * NN * tsize;
    L.s = o; o += 2 * NN * (size_t)GA * tsize;
    L.mw = o; o += 2 * (size_t)GA * Dm * tsize;                           // "-" weights
    L.pw = o; o += (size_t)GA * W * tsize + (size_t)(GA + N) * tsize;      // "+" weights, damping, delta
    L.mi = o; o += 2 * (size_t)GA * Dm * 4;                                // "-" neighbour and state
    L.pi = o; o += (size_t)GA * W * 4;                                     // "+" neighbour
    L.lev = o; o += (size_t)GA * 4;
    L.st = o; o += (size_t)(N + 1 + W) * 4;                                // per-state mode lists
    L.total = o;
    return L;
}

// LDS of the persistent FMA kernel (k_stage_small) for tiles of GA ADOs:
// launch-wide tables (H, correction coefficients, per-state mode lists and
// mode states), one row buffer and two slots of tile elements and link
// tables, and el > 1 elements per thread a partial-result slot per element
// and thread.  W = 0 for the top-level launch (no "+" links).  Offsets in
// bytes, 16-byte aligned.
struct SmallLds {
    size_t h, delta, begin, rows, comb, part, slot0, slot_bytes, total;
};

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

__host__ __device__ inline SmallLds small_lds(int N, int W, int D, int GA, int tsize, bool herm,
                                              int el) {
    const size_t Dm = D > 0 ? D : 1, NN = (size_t)N * N, G = GA;
    SmallLds L{};
    size_t o = 0;
    L.h = o; o = align16(o + 2 * NN * tsize);
    L.delta = o; o = align16(o + (size_t)N * tsize);
    L.begin = o; o = align16(o + (size_t)(N + 1 + 2 * W) * 4);
    L.rows = o; o = align16(o + 2 * G * (Dm + W) * N * (herm ? 1 : 2) * tsize);
    // Hermitian: the weighted "-" rows of each ADO summed per state [G][N][N]
    L.comb = o; o = align16(o + (herm ? 2 * G * NN * tsize : 0));
    L.part = o; o = align16(o + (el > 1 ? 2 * (size_t)el * 256 * tsize : 0));
    L.slot_bytes = align16((size_t)tsize * (2 * G * NN + 2 * G * Dm + G * W + G) +
                           4 * (2 * G * Dm + G * W));
    L.slot0 = o; o += 2 * L.slot_bytes;
    L.total = o;
    return L;
}

// ADOs per FMA-path tile: fma_block / N^2 threads' worth, reduced to fit 64 KiB of LDS.
int bulk_ados_per_tile(int N, int W, int D, int tsize);
// Device address and size of this device's static scratch array (looked up
// once per device, with that device current; thread-safe).
hipError_t scratch_buffer(void** out, size_t* bytes);
// Name of the kernel whose launch failed in the last launch_stage call on this thread.
const char* last_launch_failure();
// Which bulk kernel a job uses: 0 = FMA path, otherwise 16*nb >= N on the MFMA path.
int bulk_mfma_blocks(int N, bool h_complex, int precision);

}  // namespace heom

#include "heom.h"

namespace heom {
// Host-side accessors of a built hierarchy (heom_host.cpp), for the server.
const Tables& hierarchy_tables(const heom_hierarchy* h);
int hierarchy_precision(const heom_hierarchy* h);
double hierarchy_rate_bound(const heom_hierarchy* h);
Job hierarchy_job(const heom_hierarchy* h);       // job with tables, tiles and sizes set
const heom_info& hierarchy_info(const heom_hierarchy* h);
size_t control_bytes(int N);
// Point a job at a caller state (slot 0) and a propagation workspace of
// heom_propagate_work_bytes bytes (stage copies, control block, records).
Job bind_workspace(const heom_hierarchy* h, heom_state io, char* work, double dt,
                   int64_t n_steps, int record_every, int kind, int ground, int hermitian);
heom_status problem_rate_bound(const heom_problem* p, double* rate);
// The step check of heom_propagate_block (rate bound plus the kept diagonal
// offset, and the offset's phase per step) for the excited-state problem p.
bool block_step_ok(const heom_problem* p, double dt);
double rk4_real_limit();
void set_last_error(const std::string& msg);
void rk4_stage_specs(StageSpec sp[4]);           // the four classic RK4 stages
double monotonic_seconds();
}  // namespace heom
