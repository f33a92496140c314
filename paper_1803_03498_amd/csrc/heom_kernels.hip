// gfx950 kernels of the HEOM library: hierarchy enumeration, +/- link tables,
// the RK4 stage kernels for sigma_0 (FP64) and for the bulk of the ADOs
// (wavefront FMA path).
//
// Equations: section "HEOM formalism" of Kramer et al., arXiv:1803.03498
// (eq. Nmatrices for the hierarchy, eq. HEOM for the right-hand side, the
// superoperator masks that follow it, and the ADO rescaling substitution).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <type_traits>

#include "heom_internal.h"

namespace heom {
namespace {

// --------------------------------------------------------------------------
// Small complex helpers (interleaved re/im, T = float or double).
// --------------------------------------------------------------------------
template <typename T>
struct cpx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cpx<T> cconj(cpx<T> a) {
    return {a.re, -a.im};
}

// (re, im) pairs as clang vector types: one 8- or 16-byte access per element.
typedef float pair_f __attribute__((ext_vector_type(2)));
typedef double pair_d __attribute__((ext_vector_type(2)));
typedef int pair_i __attribute__((ext_vector_type(2)));
template <typename T>
struct vec2;
template <>
struct vec2<float> {
    using type = pair_f;
};
template <>
struct vec2<double> {
    using type = pair_d;
};

// Global-memory views of pointers held in descriptors.  Without the cast the
// compiler cannot prove these generic pointers are global and emits FLAT
// instructions, whose completion is tracked together with LDS traffic.
template <typename T>
using gcptr = const __attribute__((address_space(1))) T*;
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gcptr<T> G(const T* p) {
    return (gcptr<T>)p;
}
template <typename T>
__device__ __forceinline__ gptr<T> G(T* p) {
    return (gptr<T>)p;
}

template <typename T>
__device__ __forceinline__ cpx<T> ld(const void* base, size_t idx) {
    typename vec2<T>::type v = G(reinterpret_cast<const typename vec2<T>::type*>(base))[idx];
    return {v.x, v.y};
}

template <typename T>
__device__ __forceinline__ void st(void* base, size_t idx, cpx<T> a) {
    typename vec2<T>::type v;
    v.x = a.re;
    v.y = a.im;
    G(reinterpret_cast<typename vec2<T>::type*>(base))[idx] = v;
}

// --------------------------------------------------------------------------
// Hierarchy enumeration (eq. Nmatrices): level-major, descending
// lexicographic order inside a level.  binom[m*(W+1)+k] = C(m+k, k).
//   start(L) = #tuples with sum <= L-1 = C(W+L-1, W)
//   rank(n)  = start(|n|) + sum_{i<W-1, R_i>n_i} C(R_i-n_i-1+W-1-i, W-1-i),
//              R_i = |n| - sum_{j<i} n_j  (tuples with a larger n_i come first)
// --------------------------------------------------------------------------
__device__ int64_t rank_with(gcptr<uint8_t> n, int W, gcptr<int64_t> binom, int l, int delta) {
    int L = delta;
    for (int i = 0; i < W; ++i) L += n[i];
    const int ks = W + 1;
    int64_t r = (L == 0) ? 0 : binom[(size_t)(L - 1) * ks + W];
    int R = L;
    for (int i = 0; i < W - 1 && R > 0; ++i) {
        const int ni = n[i] + (i == l ? delta : 0);
        if (R > ni) r += binom[(size_t)(R - ni - 1) * ks + (W - 1 - i)];
        R -= ni;
    }
    return r;
}

__global__ __launch_bounds__(256) void k_enumerate(Tables t) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= t.n_ado) return;
    const int W = t.W, D = t.D;
    const int ks = W + 1;
    gptr<uint8_t> n = G(t.tuples) + (size_t)u * W;
    // level: smallest L with u < C(W+L, W)
    int L = 0;
    while (L < D && (int64_t)u >= G(t.binom)[(size_t)L * ks + W]) ++L;
    int64_t r = u - ((L == 0) ? 0 : G(t.binom)[(size_t)(L - 1) * ks + W]);
    int R = L;
    for (int i = 0; i < W - 1; ++i) {
        int v = R;
        for (; v > 0; --v) {
            const int64_t cnt = G(t.binom)[(size_t)(R - v) * ks + (W - 2 - i)];
            if (r < cnt) break;
            r -= cnt;
        }
        n[i] = (uint8_t)v;
        R -= v;
    }
    if (W > 0) n[W - 1] = (uint8_t)R;
    G(t.level)[u] = (uint8_t)L;
    double damp = 0.0;
    for (int l = 0; l < W; ++l) damp += n[l] * G(t.mode_gamma)[l];
    G(t.damping)[u] = damp;
}

// One thread per (u, l): the "+" link (valid while |n| < D) and the "-" link
// (valid while n_l > 0) of the section "HEOM formalism".
__global__ __launch_bounds__(256) void k_links(Tables t) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int W = t.W;
    if (idx >= (int64_t)t.n_ado * W) return;
    const int u = (int)(idx / W);
    const int l = (int)(idx - (int64_t)u * W);
    const gptr<uint8_t> n = G(t.tuples) + (size_t)u * W;
    const bool up = G(t.level)[u] < t.D;
    G(t.plus)[idx] = up ? (int32_t)rank_with(n, W, G(t.binom), l, +1) : -1;
    G(t.plus_w)[idx] = up ? G(t.plus_coef)[(size_t)l * (t.D + 1) + n[l]] : 0.0;
    G(t.minus)[idx] = (n[l] > 0) ? (int32_t)rank_with(n, W, G(t.binom), l, -1) : -1;
}

// Compact list of the active "-" links of every ADO (n_l > 0; at most D of
// them since |n| <= D), in mode order, padded with -1, with the state and the
// two weights of each link.  The stage kernels read one row of it instead of
// walking the tuple.
__global__ __launch_bounds__(256) void k_minus_list(Tables t) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= t.n_ado) return;
    const int W = t.W, Dm = t.D > 0 ? t.D : 1;
    gptr<pair_i> out = G(reinterpret_cast<pair_i*>(t.mlist)) + (size_t)u * Dm;
    gptr<int32_t> site = G(t.mlist_site) + (size_t)u * Dm;
    gptr<pair_d> wt = G(reinterpret_cast<pair_d*>(t.mlist_w)) + (size_t)u * Dm;
    gptr<pair_f> wt32 = G(reinterpret_cast<pair_f*>(t.mlist_w32)) + (size_t)u * Dm;
    int k = 0;
    for (int l = 0; l < W && k < Dm; ++l) {
        const int nl = G(t.tuples)[(size_t)u * W + l];
        if (nl > 0) {
            pair_i v;
            v.x = G(t.minus)[(size_t)u * W + l];
            v.y = l | (nl << 8);
            const double b = G(t.minus_coef)[(size_t)l * (t.D + 1) + nl];
            pair_d w;
            w.x = b * G(t.mode_lamnu)[l];
            w.y = b * G(t.mode_c)[l];
            site[k] = G(t.mode_site)[l];
            wt[k] = w;
            pair_f w32;
            w32.x = (float)w.x;
            w32.y = (float)w.y;
            wt32[k] = w32;
            out[k++] = v;
        }
    }
    for (; k < Dm; ++k) {
        pair_i v;
        v.x = -1;
        v.y = 0;
        pair_d w;
        w.x = 0.0;
        w.y = 0.0;
        site[k] = -1;
        wt[k] = w;
        pair_f w32;
        w32.x = 0.0f;
        w32.y = 0.0f;
        wt32[k] = w32;
        out[k] = v;
    }
}

// --------------------------------------------------------------------------
// Right-hand side of eq. HEOM for one matrix element (i, j) of ADO u.
// Commutator operands come from LDS (sH: H, sS: sigma_u, both interleaved
// complex, row-major); neighbour elements come from global memory.
//
// Coupling lines for a mode l of state s (V = |s><s|):
//   (V^x A)_ij = ((i==s) - (j==s)) A_ij,  (V^o A)_ij = ((i==s) + (j==s)) A_ij
//   +: i * sign * sqrt((n_l+1)|c_l|) * (V^x sigma_{u+e_l})_ij
//   -: sqrt(n_l/|c_l|) * sign * (i c_l V^x + delta_k0 lambda nu V^o) sigma_{u-e_l}
// Only modes of the states i and j contribute to element (i, j).
// With `herm`, the column s of a neighbour is read as conj(row s).
// --------------------------------------------------------------------------
template <typename T>
struct NbSrc {
    const void* sig0;  // complex128 [N][N] (neighbour index 0)
    const void* rest;  // T [n_ado-1][N][N]
    int N;
};

template <typename T>
__device__ __forceinline__ cpx<T> load_nb(const NbSrc<T>& s, int nb, int r, int c) {
    if (nb == 0) {
        const cpx<double> v = ld<double>(s.sig0, (size_t)r * s.N + c);
        return {(T)v.re, (T)v.im};
    }
    return ld<T>(s.rest, (size_t)(nb - 1) * s.N * s.N + (size_t)r * s.N + c);
}

// Hermitian-packed storage (FP32): ADO u >= 1 is the real N x N array
//   P[i][j] = Re sigma(i, j) for i <= j,   P[i][j] = Im sigma(j, i) for i > j,
// half the bytes of the complex form.  With a = min(r, c), b = max(r, c):
//   sigma(r, c) = (P[a][b], +P[b][a]) above the diagonal, (P[a][b], -P[b][a])
//   below it, (P[a][a], 0) on it.
// Packed value P_nb[r][c] of neighbour nb (index 0: the complex128 sigma_0,
// whose upper triangle is taken).
__device__ __forceinline__ float pk_nb(const NbSrc<float>& s, int nb, int r, int c) {
    if (nb == 0) {
        const cpx<double> v = ld<double>(s.sig0, (size_t)min(r, c) * s.N + max(r, c));
        return (float)(r <= c ? v.re : v.im);
    }
    return G(reinterpret_cast<const float*>(s.rest))[(size_t)(nb - 1) * s.N * s.N + (size_t)r * s.N + c];
}

// Element (r, c) of neighbour nb, from complex (PK false) or packed storage.
template <typename T, bool PK>
__device__ __forceinline__ cpx<T> nb_get(const NbSrc<T>& s, int nb, int r, int c) {
    if constexpr (PK) {
        if (nb == 0) return load_nb<T>(s, 0, r, c);
        const T x = pk_nb(s, nb, min(r, c), max(r, c)), y = pk_nb(s, nb, max(r, c), min(r, c));
        return {x, r < c ? y : (r > c ? -y : (T)0)};
    } else {
        return load_nb<T>(s, nb, r, c);
    }
}

__device__ __forceinline__ int xcd_remap(int b, int nb) {
    // Workgroups are handed to the 8 XCDs round-robin; give each XCD a
    // contiguous range of tiles so neighbouring ADOs share one L2.
    const int per = nb / 8, rem = nb % 8;
    const int x = b % 8, idx = b / 8;
    return x * per + (x < rem ? x : rem) + idx;
}

// As xcd_remap, but the first n_first workgroups (those holding ADOs below
// the top level, which carry the "+" couplings and cost more) keep their
// order and so are spread round-robin over all XCDs instead of loading one.
__device__ __forceinline__ int xcd_remap_low(int b, int nb, int n_first) {
    return b < n_first ? b : n_first + xcd_remap(b - n_first, nb - n_first);
}

// The job a tile belongs to.  Single-job launches read the descriptor from
// the kernel argument; batched launches from the device job table (found by
// binary search over the jobs' first tiles).  Keeping the two apart lets the
// compiler address each descriptor in its own memory space.
template <bool BATCHED>
struct JobOf;
template <>
struct JobOf<false> {
    static __device__ __forceinline__ const Job& get(const Job& single, const Job*, int, int) {
        return single;
    }
};
template <>
struct JobOf<true> {
    static __device__ __forceinline__ const Job& get(const Job&, const Job* jobs, int n_jobs,
                                                     int tile) {
        int lo = 0, hi = n_jobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (jobs[mid].tile_begin <= tile)
                lo = mid;
            else
                hi = mid - 1;
        }
        return jobs[lo];
    }
};

// --------------------------------------------------------------------------
// sigma_0 stage kernel: one workgroup per job, FP64 throughout; reads the
// level-1 ADOs in the bulk precision T.  Also records the observables.
// --------------------------------------------------------------------------
__device__ void record_sigma0(const Job& J, const double* sS, int64_t slot) {
    // sS: interleaved complex128 [N][N] in LDS.  Caller: one thread.
    if (slot < 0 || slot >= J.n_rec_max) return;
    const int N = J.t.N;
    gptr<double> rec = G(J.records) + slot * J.rec_doubles;
    double trr = 0.0, tri = 0.0;
    for (int i = 0; i < N; ++i) {
        trr += sS[2 * (i * N + i)];
        tri += sS[2 * (i * N + i) + 1];
    }
    bool finite = isfinite(trr) && isfinite(tri);
    if (J.rec_kind == 0) {
        double herm = 0.0;
        for (int i = 0; i < N; ++i) {
            rec[i] = sS[2 * (i * N + i)];
            for (int j = 0; j < N; ++j) {
                const double dr = sS[2 * (i * N + j)] - sS[2 * (j * N + i)];
                const double di = sS[2 * (i * N + j) + 1] + sS[2 * (j * N + i) + 1];
                herm = fmax(herm, sqrt(dr * dr + di * di));
            }
        }
        rec[N] = trr;
        rec[N + 1] = tri;
        rec[N + 2] = herm;
        finite = finite && isfinite(herm);
    } else {
        double pr = 0.0, pi = 0.0;
        for (int a = 0; a < N; ++a) {
            pr += G(J.mu)[a] * sS[2 * (a * N + J.ground)];
            pi += G(J.mu)[a] * sS[2 * (a * N + J.ground) + 1];
        }
        rec[0] = pr;
        rec[1] = pi;
        rec[2] = trr;
        rec[3] = tri;
        finite = finite && isfinite(pr) && isfinite(pi);
    }
    if (!finite) *G(J.status) = 1;
}

// LDS plan of the sigma_0 kernel: H and sigma_0 in FP64, per-mode weights,
// per-state tables, and (when they fit) the row s_l (and, for non-Hermitian
// states, the column s_l) of every level-1 ADO e_l.
struct Sigma0Lds {
    size_t h, s, pa, delta, site, begin, modes, rows, cols, total;
    bool rows_in_lds;
};

// cap: the LDS bytes the launch provides (rows are staged only if they fit).
__host__ __device__ inline Sigma0Lds sigma0_lds(int N, int W, int tsize, bool herm, size_t cap) {
    Sigma0Lds L{};
    size_t o = 0;
    const size_t NN = (size_t)N * N;
    L.h = o; o += 16 * NN;
    L.s = o; o += 16 * NN;
    L.pa = o; o += 8 * (size_t)W;
    L.delta = o; o += 8 * (size_t)N;
    L.site = o; o += 4 * (size_t)W;
    L.begin = o; o += 4 * (size_t)(N + 1);
    L.modes = o; o += 4 * (size_t)W;
    o = (o + 15) & ~size_t(15);
    const size_t rows = 2 * (size_t)tsize * W * N;
    L.rows_in_lds = o + rows * (herm ? 1 : 2) <= cap;
    L.rows = o;
    if (L.rows_in_lds) o += rows;
    L.cols = o;
    if (L.rows_in_lds && !herm) o += rows;
    L.total = o;
    return L;
}

// The sigma_0 stage of job `job` by the whole workgroup (any block size):
// the body of k_sigma0, and of the extra workgroups of a bulk launch that
// carries sigma_0 along (lds_cap: the LDS the launch provides).
// HC: the job may have a complex H.  The loops stay rolled: the code also
// runs inside the bulk kernels, whose occupancy its registers would cost.
template <typename T, bool BATCHED, bool HC, bool PK = false>
__device__ void sigma0_stage(const Job& single, const Job* jobs, int job, const StageSpec& sp,
                             unsigned lds_cap, char* smem_s0) {
    const Job& J = BATCHED ? jobs[job] : single;
    const Tables& t = J.t;
    const int N = t.N, NN = N * N, W = t.W, D = t.D;
    const bool herm = J.herm != 0;
    const Sigma0Lds L = sigma0_lds(N, W, (int)sizeof(T), herm, lds_cap);
    double* sH = reinterpret_cast<double*>(smem_s0 + L.h);
    double* sS = reinterpret_cast<double*>(smem_s0 + L.s);
    double* sPa = reinterpret_cast<double*>(smem_s0 + L.pa);
    double* sDelta = reinterpret_cast<double*>(smem_s0 + L.delta);
    int* sSite = reinterpret_cast<int*>(smem_s0 + L.site);
    int* sBegin = reinterpret_cast<int*>(smem_s0 + L.begin);
    int* sModes = reinterpret_cast<int*>(smem_s0 + L.modes);
    T* sRows = reinterpret_cast<T*>(smem_s0 + L.rows);  // [W][N] complex
    T* sCols = reinterpret_cast<T*>(smem_s0 + L.cols);  // [W][N] complex
    const int tid = threadIdx.x;
    const bool hc = HC && t.h_complex != 0;
    const NbSrc<T> nbs{J.sig0[sp.in], J.rest[sp.in], N};
    for (int e = tid; e < NN; e += blockDim.x) {
        sH[2 * e] = G(t.h_re)[e];
        sH[2 * e + 1] = hc ? G(t.h_im)[e] : 0.0;
        const cpx<double> v = ld<double>(J.sig0[sp.in], e);
        sS[2 * e] = v.re;
        sS[2 * e + 1] = v.im;
    }
    for (int l = tid; l < W; l += blockDim.x) {
        sPa[l] = (D > 0) ? G(t.plus_coef)[l * (D + 1)] : 0.0;
        sSite[l] = G(t.mode_site)[l];
        sModes[l] = G(t.state_modes)[l];
    }
    for (int x = tid; x <= N; x += blockDim.x) {
        sBegin[x] = G(t.state_mode_begin)[x];
        if (x < N) sDelta[x] = G(t.delta_state)[x];
    }
    if (D > 0 && L.rows_in_lds) {
        for (int idx = tid; idx < W * N; idx += blockDim.x) {
            const int l = idx / N, c = idx - (idx / N) * N;
            const int site = G(t.mode_site)[l];
            const cpx<T> r = nb_get<T, PK>(nbs, 1 + l, site, c);
            sRows[2 * idx] = r.re;
            sRows[2 * idx + 1] = r.im;
            if (!herm) {
                const cpx<T> v = load_nb<T>(nbs, 1 + l, c, site);
                sCols[2 * idx] = v.re;
                sCols[2 * idx + 1] = v.im;
            }
        }
    }
    __syncthreads();
    if (sp.record_initial && tid == 0 && *G(J.step) == 0) record_sigma0(J, sS, 0);

    const double h = sp.hmul * J.dt;
#pragma unroll 1
    for (int e = tid; e < NN; e += blockDim.x) {
        const int i = e / N, j = e - (e / N) * N;
        // -i [H, sigma_0] (the damping vanishes at u = 0)
        double cr = 0, ci = 0;
        if (hc) {
#pragma unroll 1
            for (int k = 0; k < N; ++k) {
                const double hr = sH[2 * (i * N + k)], hi = sH[2 * (i * N + k) + 1];
                const double xr = sS[2 * (k * N + j)], xi = sS[2 * (k * N + j) + 1];
                const double yr = sS[2 * (i * N + k)], yi = sS[2 * (i * N + k) + 1];
                const double gr = sH[2 * (k * N + j)], gi = sH[2 * (k * N + j) + 1];
                cr += hr * xr - hi * xi - (yr * gr - yi * gi);
                ci += hr * xi + hi * xr - (yr * gi + yi * gr);
            }
        } else {
#pragma unroll 1
            for (int k = 0; k < N; ++k) {
                const double hik = sH[2 * (i * N + k)], hkj = sH[2 * (k * N + j)];
                cr += hik * sS[2 * (k * N + j)] - sS[2 * (i * N + k)] * hkj;
                ci += hik * sS[2 * (k * N + j) + 1] - sS[2 * (i * N + k) + 1] * hkj;
            }
        }
        const double dl = (i != j) ? sDelta[i] + sDelta[j] : 0.0;
        double fr = ci - dl * sS[2 * e], fi = -cr - dl * sS[2 * e + 1];
        // "+" couplings to the level-1 ADOs e_l (index 1 + l), modes of states i and j
        if (D > 0 && i != j) {
            for (int pass = 0; pass < 2; ++pass) {
                const int s = pass == 0 ? i : j;
                for (int m = sBegin[s]; m < sBegin[s + 1]; ++m) {
                    const int l = sModes[m];
                    cpx<T> x;
                    if (L.rows_in_lds) {
                        if (pass == 0) {
                            x = {sRows[2 * (l * N + j)], sRows[2 * (l * N + j) + 1]};
                        } else if (herm) {
                            x = cconj(cpx<T>{sRows[2 * (l * N + i)], sRows[2 * (l * N + i) + 1]});
                        } else {
                            x = {sCols[2 * (l * N + i)], sCols[2 * (l * N + i) + 1]};
                        }
                    } else {
                        x = (herm && pass == 1) ? cconj(nb_get<T, PK>(nbs, 1 + l, s, i))
                                                : nb_get<T, PK>(nbs, 1 + l, i, j);
                    }
                    const double pa = pass == 0 ? sPa[l] : -sPa[l];
                    fr -= pa * (double)x.im;
                    fi += pa * (double)x.re;
                }
            }
        }
        // RK4 stage combination in FP64; out may be a base (stage 4), which
        // only this thread reads at element e.
        double yr = sp.w_in * sS[2 * e], yi = sp.w_in * sS[2 * e + 1];
        for (int m = 0; m < sp.nbase; ++m) {
            const cpx<double> bv = ld<double>(J.sig0[sp.base[m]], e);
            yr += sp.wbase[m] * bv.re;
            yi += sp.wbase[m] * bv.im;
        }
        st<double>(J.sig0[sp.out], e, cpx<double>{yr + h * fr, yi + h * fi});
    }
    if (sp.record_after) {
        // the new sigma_0 back into LDS for the observables
        __threadfence();
        __syncthreads();
        for (int e = tid; e < NN; e += blockDim.x) {
            const cpx<double> v = ld<double>(J.sig0[sp.out], e);
            sS[2 * e] = v.re;
            sS[2 * e + 1] = v.im;
        }
        __syncthreads();
        if (tid == 0) {
            const int64_t step = *G(J.step) + 1;
            *G(J.step) = step;
            if (step % J.rec_every == 0) record_sigma0(J, sS, step / J.rec_every);
        }
    }
}

template <typename T, bool BATCHED, bool PK = false>
__global__ __launch_bounds__(256) void k_sigma0(Job single, const Job* jobs, int n_jobs,
                                                StageSpec sp, unsigned lds_cap) {
    extern __shared__ char smem_s0[];
    (void)n_jobs;
    sigma0_stage<T, BATCHED, true, PK>(single, jobs, blockIdx.x, sp, lds_cap, smem_s0);
}

// H (shifted, rad/fs) in the stage precision: FP32 kernels read the FP32 copy.
template <typename T>
__device__ __forceinline__ T h_entry(const Tables& t, int idx) {
    if constexpr (sizeof(T) == 4)
        return G(t.h_re_f32)[idx];
    else
        return G(t.h_re)[idx];
}

// At most this many "-" links of an ADO are read ahead by the stage kernels
// (the MFMA kernel stages their neighbour rows in LDS); further links read
// global memory where they are used.
constexpr int kPrefRows = 4;

// LDS view of an FMA-path tile of GA ADOs (layout fma_lds).
template <typename T>
struct FmaTile {
    T *sH, *sS, *sMml, *sMmc, *sPa, *sGam, *sDelta;
    int *sMnb, *sMsite, *sPnb, *sLev, *sBegin, *sModes;
    __device__ FmaTile(char* smem, const FmaLds& L, int N, int W, int Dm, int GA) {
        sH = reinterpret_cast<T*>(smem + L.h);     // 2*NN
        sS = reinterpret_cast<T*>(smem + L.s);     // 2*GA*NN
        sMml = reinterpret_cast<T*>(smem + L.mw);  // [GA][Dm]
        sMmc = sMml + GA * Dm;
        sPa = reinterpret_cast<T*>(smem + L.pw);   // [GA][W]
        sGam = sPa + GA * W;                       // [GA]
        sDelta = sGam + GA;                        // [N]
        sMnb = reinterpret_cast<int*>(smem + L.mi);  // [GA][Dm]
        sMsite = sMnb + GA * Dm;
        sPnb = reinterpret_cast<int*>(smem + L.pi);  // [GA][W]
        sLev = reinterpret_cast<int*>(smem + L.lev);
        sBegin = reinterpret_cast<int*>(smem + L.st);  // [N+1]
        sModes = sBegin + N + 1;                       // [W]
    }
};

// The right-hand side at element (i, j) of ADO g of an FMA-path tile (the
// stage combination aside): -i [H, sigma], the damping and correction
// terms, and the coupling lines.  sr, si: the element itself.
//
// The neighbour elements are gathered in batches of KB loads that are all
// issued before the first is used, so a thread keeps several scattered
// loads in flight instead of waiting on each in turn.  With S0 false (no
// level-1 ADO in the tile, so no "-" neighbour is the complex128 sigma_0)
// every load reads the bulk array unconditionally: slots without a
// contributing link read a valid element and are dropped afterwards.
template <typename T, bool S0>
__device__ __forceinline__ void fma_rhs(const FmaTile<T>& V, const NbSrc<T>& nbs, int g, int i,
                                        int j, int N, int W, int D, int Dm, bool herm, bool hc,
                                        T sr, T si, T& fr_out, T& fi_out) {
    const int NN = N * N;
    const T* S = V.sS + 2 * g * NN;
    const T* sH = V.sH;
    T cr = 0, ci = 0;
    if (hc) {
        for (int k = 0; k < N; ++k) {
            const T hr = sH[2 * (i * N + k)], hi = sH[2 * (i * N + k) + 1];
            const T xr = S[2 * (k * N + j)], xi = S[2 * (k * N + j) + 1];
            const T yr = S[2 * (i * N + k)], yi = S[2 * (i * N + k) + 1];
            const T gr = sH[2 * (k * N + j)], gi = sH[2 * (k * N + j) + 1];
            cr += hr * xr - hi * xi - (yr * gr - yi * gi);
            ci += hr * xi + hi * xr - (yr * gi + yi * gr);
        }
    } else {
        for (int k = 0; k < N; ++k) {
            const T hik = sH[2 * (i * N + k)], hkj = sH[2 * (k * N + j)];
            cr += hik * S[2 * (k * N + j)] - S[2 * (i * N + k)] * hkj;
            ci += hik * S[2 * (k * N + j) + 1] - S[2 * (i * N + k) + 1] * hkj;
        }
    }
    const T gm = V.sGam[g] + ((i != j) ? V.sDelta[i] + V.sDelta[j] : (T)0);
    T fr = ci - gm * sr, fi = -cr - gm * si;
    constexpr int KB = sizeof(T) == 4 ? 8 : 4;
    auto nb_elem = [&](int nb, int r, int c) -> cpx<T> {
        if constexpr (S0) return load_nb<T>(nbs, nb, r, c);
        else return ld<T>(nbs.rest, (size_t)(nb - 1) * NN + (size_t)r * N + c);
    };
    // "-" links that touch row or column i, j
    for (int a0 = 0; a0 < Dm; a0 += KB) {
        cpx<T> xs[KB];
#pragma unroll
        for (int q = 0; q < KB; ++q) {
            const int a = a0 + q;
            const int s = a < Dm ? V.sMsite[g * Dm + a] : -1;
            const int nb = a < Dm ? V.sMnb[g * Dm + a] : -1;
            const bool use = s >= 0 && nb >= 0 && (i == s || j == s);
            const bool cj = herm && (j == s) && (i != s);
            if constexpr (S0) {
                xs[q] = cpx<T>{(T)0, (T)0};
                if (use) xs[q] = nb_elem(nb, cj ? s : i, cj ? i : j);
            } else {
                xs[q] = nb_elem(use ? nb : 1, cj ? s : i, cj ? i : j);
            }
        }
#pragma unroll
        for (int q = 0; q < KB; ++q) {
            const int a = a0 + q;
            const int s = a < Dm ? V.sMsite[g * Dm + a] : -1;
            const int nb = a < Dm ? V.sMnb[g * Dm + a] : -1;
            if (!(s >= 0 && nb >= 0 && (i == s || j == s))) continue;
            const cpx<T> x = (herm && (j == s) && (i != s)) ? cconj(xs[q]) : xs[q];
            const T vx = (T)((i == s) - (j == s)), vo = (T)((i == s) + (j == s));
            const T thr = V.sMml[g * Dm + a] * vo, thi = V.sMmc[g * Dm + a] * vx;
            fr += thr * x.re - thi * x.im;
            fi += thr * x.im + thi * x.re;
        }
    }
    // "+" links (never sigma_0): the modes of state i, then those of state j
    if (V.sLev[g] < D && i != j) {
        const int bi = V.sBegin[i], ni = V.sBegin[i + 1] - bi;
        const int bj = V.sBegin[j], n_all = ni + V.sBegin[j + 1] - bj;
        for (int k0 = 0; k0 < n_all; k0 += KB) {
            cpx<T> xs[KB];
#pragma unroll
            for (int q = 0; q < KB; ++q) {
                const int k = min(k0 + q, n_all - 1);
                const bool on_j = k >= ni;
                const int l = V.sModes[on_j ? bj + k - ni : bi + k];
                const bool cj = herm && on_j;
                xs[q] = ld<T>(nbs.rest, (size_t)(V.sPnb[g * W + l] - 1) * NN +
                                            (size_t)(cj ? j : i) * N + (cj ? i : j));
            }
#pragma unroll
            for (int q = 0; q < KB; ++q) {
                const int k = k0 + q;
                if (k >= n_all) continue;
                const bool on_j = k >= ni;
                const int l = V.sModes[on_j ? bj + k - ni : bi + k];
                const cpx<T> x = (herm && on_j) ? cconj(xs[q]) : xs[q];
                const T pa = on_j ? -V.sPa[g * W + l] : V.sPa[g * W + l];
                fr -= pa * x.im;
                fi += pa * x.re;
            }
        }
    }
    fr_out = fr;
    fi_out = fi;
}

// --------------------------------------------------------------------------
// Bulk stage kernel, wavefront-FMA path (batched launches with N < 16 or a
// complex H, and single propagations below the persistent FMA kernel's
// size): a workgroup of fma_block threads takes GA = max(1, fma_block / N^2)
// consecutive ADOs (computed per job by the host; a batched launch uses the
// block size of its largest N, and the element loops stride by the launch's
// block size); every thread owns whole matrix elements.  Each ADO's link
// rows (the compact "-" list with its states and weights, the "+"
// neighbours and weights) are copied to LDS first from the precomputed
// tables; an element's coupling lines then gather one element per
// contributing neighbour (fma_rhs).
// HC: some job of the launch has a complex H (otherwise H is real).
// --------------------------------------------------------------------------
template <typename T, bool BATCHED, bool HC>
__global__ __launch_bounds__(kFmaMaxBlock) __attribute__((amdgpu_waves_per_eu(
    sizeof(T) == 4 ? 8 : 5))) void k_bulk_fma(Job single, const Job* jobs, int n_jobs, StageSpec sp,
                                              int s0_blocks, unsigned lds_total) {
    extern __shared__ char smem_raw[];
    if constexpr (sizeof(T) == 4) {
        if ((int)blockIdx.x < s0_blocks) {
            // the first workgroups carry the sigma_0 stage along
            sigma0_stage<T, BATCHED, HC>(single, jobs, blockIdx.x, sp, lds_total, smem_raw);
            return;
        }
    }
    const int n_first = BATCHED ? 0
                                : min((single.n_low + single.ados_per_tile - 1) / single.ados_per_tile,
                                      (int)gridDim.x - s0_blocks);
    const int b = xcd_remap_low(blockIdx.x - s0_blocks, gridDim.x - s0_blocks, n_first);
    const Job& J = JobOf<BATCHED>::get(single, jobs, n_jobs, b);
    const Tables& t = J.t;
    const int N = t.N, NN = N * N, W = t.W, D = t.D, Dm = D > 0 ? D : 1;
    const int GA = J.ados_per_tile;
    const int u0 = 1 + (b - J.tile_begin) * GA;
    const int n_here = min(GA, t.n_ado - u0);
    const FmaTile<T> V(smem_raw, fma_lds(N, W, D, GA, (int)sizeof(T)), N, W, Dm, GA);
    T* sH = V.sH;
    T* sS = V.sS;
    T *sMml = V.sMml, *sMmc = V.sMmc, *sPa = V.sPa, *sGam = V.sGam, *sDelta = V.sDelta;
    int *sMnb = V.sMnb, *sMsite = V.sMsite, *sPnb = V.sPnb, *sLev = V.sLev;
    int *sBegin = V.sBegin, *sModes = V.sModes;
    const int tid = threadIdx.x;

    // stage H, the tile, the per-ADO link data and the per-state tables
    for (int e = tid; e < NN; e += blockDim.x) {
        sH[2 * e] = h_entry<T>(t, e);
        sH[2 * e + 1] = t.h_complex ? (T)G(t.h_im)[e] : (T)0;
    }
    const size_t base = (size_t)(u0 - 1) * NN;
    const int tot = n_here * NN;
    {
        const void* in = J.rest[sp.in];
        for (int e = tid; e < tot; e += blockDim.x) {
            const cpx<T> v = ld<T>(in, base + e);
            sS[2 * e] = v.re;
            sS[2 * e + 1] = v.im;
        }
    }
    for (int x = tid; x < n_here * Dm; x += blockDim.x) {
        const size_t at = (size_t)u0 * Dm + x;  // row u0 + x / Dm, entry x % Dm
        sMnb[x] = G(reinterpret_cast<const pair_i*>(t.mlist))[at].x;
        sMsite[x] = G(t.mlist_site)[at];
        if constexpr (sizeof(T) == 4) {
            const pair_f w = G(reinterpret_cast<const pair_f*>(t.mlist_w32))[at];
            sMml[x] = w.x;
            sMmc[x] = w.y;
        } else {
            const pair_d w = G(reinterpret_cast<const pair_d*>(t.mlist_w))[at];
            sMml[x] = w.x;
            sMmc[x] = w.y;
        }
    }
    for (int g = tid; g < n_here; g += blockDim.x) {
        sLev[g] = G(t.level)[u0 + g];
        sGam[g] = (T)G(t.damping)[u0 + g];
    }
    // "+" rows: ADOs are stored by level, so a tile whose first ADO is on
    // the top level has none
    if (G(t.level)[u0] < D) {
        for (int x = tid; x < n_here * W; x += blockDim.x) {
            const size_t at = (size_t)u0 * W + x;
            sPnb[x] = G(t.plus)[at];
            sPa[x] = (T)G(t.plus_w)[at];
        }
    }
    for (int x = tid; x <= N; x += blockDim.x) {
        sBegin[x] = G(t.state_mode_begin)[x];
        if (x < N) sDelta[x] = (T)G(t.delta_state)[x];
    }
    for (int l = tid; l < W; l += blockDim.x) sModes[l] = G(t.state_modes)[l];
    // FP32: this thread's first stage-base elements, in flight across the
    // barrier (FP64 keeps the registers for occupancy and loads them late)
    constexpr bool kEarly = sizeof(T) == 4;
    cpx<T> bv0[3];
    const int e0c = min((int)tid, tot - 1);
#pragma unroll
    for (int m = 0; m < 3; ++m)
        if (kEarly && m < sp.nbase) bv0[m] = ld<T>(J.rest[sp.base[m]], base + e0c);
    __syncthreads();

    const NbSrc<T> nbs{J.sig0[sp.in], J.rest[sp.in], N};
    const bool herm = J.herm != 0, hc = HC && t.h_complex != 0;
    const T h = (T)(sp.hmul * J.dt), w_in = (T)sp.w_in;
    const bool s0_tile = sLev[0] <= 1;  // ADOs are stored by level
    for (int e = tid; e < tot; e += blockDim.x) {
        const int g = e / NN;
        const int ij = e - g * NN;
        const int i = ij / N, j = ij - (ij / N) * N;
        const T sr = sS[2 * e], si = sS[2 * e + 1];
        T fr, fi;
        if (s0_tile) fma_rhs<T, true>(V, nbs, g, i, j, N, W, D, Dm, herm, hc, sr, si, fr, fi);
        else fma_rhs<T, false>(V, nbs, g, i, j, N, W, D, Dm, herm, hc, sr, si, fr, fi);
        T yr = w_in * sr + h * fr, yi = w_in * si + h * fi;
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            if (m < sp.nbase) {
                const cpx<T> bv = (kEarly && e == (int)tid) ? bv0[m] : ld<T>(J.rest[sp.base[m]], base + e);
                yr += (T)sp.wbase[m] * bv.re;
                yi += (T)sp.wbase[m] * bv.im;
            }
        }
        st<T>(J.rest[sp.out], base + e, cpx<T>{yr, yi});
    }
}

// --------------------------------------------------------------------------
// Bulk stage kernel, MFMA path (16 <= N <= 64, real H): one ADO per workgroup.
//
// The commutator is a batched GEMM with the shared H: X = H [Re sigma | Im sigma]
// (M = K = N, 2N columns) on 16x16x4 matrix cores, H held in registers as the
// A operand and sigma staged in LDS as separate real and imaginary planes.
// For a Hermitian sigma, sigma H = (H sigma)^dagger, so -i[H, sigma] =
// -i (X - X^dagger) needs only X; otherwise Y = sigma H is a second GEMM.
// The damping, correction and coupling lines are elementwise and are fused
// with the RK4 stage combination in the same pass.
//
// MFMA 16x16x4 operand layout (lane l of a 64-lane wavefront):
//   A[i][k]: l = i + 16 k        B[k][j]: l = j + 16 k
//   D[i][j], f32: l = j + 16 (i / 4), item i % 4
//   D[i][j], f64: l = j + 16 (i % 4), item i / 4
// --------------------------------------------------------------------------
template <typename T>
struct mfma_acc;
template <>
struct mfma_acc<float> {
    typedef float type __attribute__((ext_vector_type(4)));
};
template <>
struct mfma_acc<double> {
    typedef double type __attribute__((ext_vector_type(4)));
};

__device__ __forceinline__ mfma_acc<float>::type mfma16(float a, float b,
                                                        mfma_acc<float>::type c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ mfma_acc<double>::type mfma16(double a, double b,
                                                         mfma_acc<double>::type c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Row (inside a 16x16 tile) of output item r held by `lane`.
template <typename T>
__device__ __forceinline__ int mfma_row(int lane, int r);
template <>
__device__ __forceinline__ int mfma_row<float>(int lane, int r) {
    return 4 * (lane >> 4) + r;
}
template <>
__device__ __forceinline__ int mfma_row<double>(int lane, int r) {
    return 4 * r + (lane >> 4);
}


// LDS carve-up of the MFMA stage kernel (bytes; T-typed arrays first).
template <typename T, int NB, bool HERM>
struct MfmaLds {
    static constexpr int NP = 16 * NB;
    // sigma planes: rows 16 banks apart, so the four rows of an MFMA
    // B-operand read fall in distinct banks
    static constexpr int LS = (NP % 32 == 16) ? NP : NP + 16;
    // X and coupling planes: odd stride, so transposed reads [j][i] hit distinct banks
    static constexpr int LX = NP + 1;
    static constexpr int XPLANE = NP * LX;
    // a sigma plane also holds a coupling plane of stride LX
    static constexpr int PLANE = NP * LS > XPLANE ? NP * LS : XPLANE;
    __host__ __device__ static int n_rows(int D) {
        const int Dm = D > 0 ? D : 1;
        return Dm < kPrefRows ? Dm : kPrefRows;
    }
    // Layout: T planes (sigma, then couplings; X; Y on the general path),
    // prefetched "-" rows (T), "+" neighbour tile addresses (8 bytes each),
    // T: "-" weights, per-state correction, "+" weights; int: per-state mode
    // lists, "-" state and neighbour.  Every block before the addresses is a
    // multiple of 8 bytes.
    __host__ __device__ static size_t t_head(int N, int D) {
        return (size_t)PLANE * (HERM ? 2 : 4) + 2 * (size_t)XPLANE + 2 * (size_t)n_rows(D) * N;
    }
    __host__ __device__ static size_t bytes(int N, int W, int D) {
        const int Dm = D > 0 ? D : 1;
        return sizeof(T) * t_head(N, D) + 8 * (size_t)W + sizeof(T) * (2 * (size_t)Dm + N + W) +
               4 * ((size_t)(N + 1) + W + 2 * (size_t)Dm);
    }
};

// Wave-uniform value into a scalar register.
__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ float uniform(float x) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ __forceinline__ double uniform(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// ADOs per workgroup.  FP32 N <= 48 runs two 6-wave halves in one 12-wave
// workgroup: the waves of a workgroup are spread evenly over the four SIMDs
// of a CU, and 12 waves (3 per SIMD) pack where 6 (2/2/1/1) leave holes.
template <typename T, int NB>
constexpr int mfma_ados_per_wg() {
    return (sizeof(T) == 4 && NB == 3) ? 2 : 1;
}

// Waves per SIMD to ask of the register allocator for N <= 48: two 12-wave
// FP32 workgroups per CU (their LDS fits), two 6-wave FP64 ones; the general
// path holds more values in flight.
template <typename T, int NB, bool HERM>
constexpr int mfma_waves_per_eu() {
    return NB == 3 ? (sizeof(T) == 4 ? (HERM ? 6 : 4) : (HERM ? 3 : 2)) : 1;
}

// Bulk RK4 stage on the matrix cores, one ADO per 128 NB threads (a
// workgroup holds mfma_ados_per_wg of them, each with its own LDS).  Two
// wavefronts per 16-row block of H: wave (mt, half) computes rows
// 16 mt .. 16 mt + 15 of X = H Re(sigma) (half 0) or H Im(sigma) (half 1).
// Thread tid owns column j = tid % NP and rows i = tid / NP + 8 k, k < 2 NB,
// of the padded NP x NP tile.
//
// The coupling terms of the HEOM equation touch only row s and column s of a
// neighbour, s the state of the mode.  On the Hermitian path the workgroup
// forms, for every state s with a link, the row
//   Z[s][c] = sum over "-" links a of state s of (lambda nu_a + i c_a) w_a sigma_{u-e_a}[s][c]
//           + sum over "+" modes l of state s of i w_l sigma_{u+e_l}[s][c],
// and element (i, j), i != j, takes Z[i][j] + conj(Z[j][i]), because column s
// of a Hermitian neighbour is the conjugate of its row s.  The diagonal takes
// the "-" terms 2 lambda nu_a w_a sigma_{u-e_a}[i][i], kept in Z[i][i].  On the
// general path element (i, j) forms its whole coupling sum at (i, j).  Z
// reuses the sigma planes: each thread keeps its sigma elements in registers.
template <typename T, int NB, bool HERM, bool BATCHED, int NBASE>
__global__ __launch_bounds__((128 * NB * mfma_ados_per_wg<T, NB>())) __attribute__((
    amdgpu_waves_per_eu(mfma_waves_per_eu<T, NB, HERM>()))) void k_bulk_mfma(Job single,
                                                                             const Job* jobs,
                                                                             int n_jobs,
                                                                             StageSpec sp,
                                                                             int total_tiles,
                                                                             unsigned lds_stride,
                                                                             int s0_blocks,
                                                                             unsigned lds_total) {
    constexpr int NT = 128 * NB;  // threads per ADO
    constexpr int AW = mfma_ados_per_wg<T, NB>();
    extern __shared__ char smem_raw[];
    if ((int)blockIdx.x < s0_blocks) {
        // the first workgroups carry the sigma_0 stage along (real H on this path)
        sigma0_stage<T, BATCHED, false>(single, jobs, blockIdx.x, sp, lds_total, smem_raw);
        return;
    }
    using L = MfmaLds<T, NB, HERM>;
    constexpr int NP = L::NP, LS = L::LS, LX = L::LX, PLANE = L::PLANE, XPLANE = L::XPLANE;
    constexpr int KS = 4 * NB;      // k-steps of 4
    constexpr int EPT = 2 * NB;     // rows per thread
    constexpr int RS = NT / NP;     // row step (8)
    constexpr int KP = 2;           // "+" modes per state loaded ahead (more are read late)
    constexpr int KX = HERM ? KP : 2 * KP;
    using acc_t = typename mfma_acc<T>::type;
    using C = cpx<T>;

    const int sub = AW > 1 ? uniform((int)threadIdx.x / NT) : 0;  // whole waves per half
    const int tid = (int)threadIdx.x - sub * NT;
    const int lane = tid & 63, wave = tid >> 6;
    const int mt = wave >> 1, half = wave & 1;
    const int n_first = BATCHED ? 0 : min((single.n_low + AW - 1) / AW, (int)gridDim.x - s0_blocks);
    const int tile = xcd_remap_low(blockIdx.x - s0_blocks, gridDim.x - s0_blocks, n_first) * AW + sub;
    // A half without an ADO still takes part in every barrier.
    const bool active = tile < total_tiles;
    const Job& J = JobOf<BATCHED>::get(single, jobs, n_jobs, active ? tile : total_tiles - 1);
    const Tables& t = J.t;
    const int N = t.N, NN = N * N, W = t.W, D = t.D, Dm = D > 0 ? D : 1;
    const int u = active ? 1 + (tile - J.tile_begin) : 1;
    const char* rest_in = reinterpret_cast<const char*>(J.rest[sp.in]);
    const size_t tile_bytes = (size_t)NN * sizeof(C);
    const char* own = rest_in + (size_t)(u - 1) * tile_bytes;
    const NbSrc<T> nbs{J.sig0[sp.in], J.rest[sp.in], N};
    const int n_rows = L::n_rows(D);

    T* sSre = reinterpret_cast<T*>(smem_raw + (size_t)sub * lds_stride);  // sigma (stride LS), then Z (stride LX)
    T* sSim = sSre + PLANE;
    T* sXre = sSim + PLANE;  // stride LX
    T* sXim = sXre + XPLANE;
    T* sYre = sXim + XPLANE;  // general path only
    T* sYim = sYre + PLANE;
    T* sRow = HERM ? sYre : sYim + PLANE;  // n_rows x N complex
    const char** sPptr = reinterpret_cast<const char**>(sRow + 2 * n_rows * N);  // [W]
    T* sMml = reinterpret_cast<T*>(sPptr + W);  // [Dm] "-" weights
    T* sMmc = sMml + Dm;
    T* sDelta = sMmc + Dm;  // [N]
    T* sPa = sDelta + N;    // [W] "+" weights
    int* sBegin = reinterpret_cast<int*>(sPa + W);  // [N+1]
    int* sModes = sBegin + N + 1;                   // [W]
    int* sMsite = sModes + W;                       // [Dm]
    int* sMnb = sMsite + Dm;                        // [Dm]

    const int r0 = tid / NP, j = tid - (tid / NP) * NP;
    const bool jin = active && j < N;  // this thread's column is stored

    // 1. Independent loads: this ADO's tile, its link tables, this wave's block of H.
    // Own elements: clamped, unpredicated loads (they issue together), then
    // zeroed outside the N x N block by a multiply that cannot become a branch.
    C cur[EPT];
    const int jc = min(j, N - 1);
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const int i = r0 + RS * k;
        const T m = (jin && i < N) ? (T)1 : (T)0;
        cur[k] = ld<T>(own, min(i, N - 1) * N + jc);
        cur[k].re *= m;
        cur[k].im *= m;
    }
    T hreg[KS];  // A operand: H[16 mt + lane%16][4 ks + lane/16]
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        // Clamped and unpredicated, so the loads issue together: columns
        // past N meet the zero rows of the padded sigma planes, and rows
        // past N of X are never read.
        const int r = min(16 * mt + (lane & 15), N - 1), c = min(4 * ks + (lane >> 4), N - 1);
        hreg[ks] = h_entry<T>(t, r * N + c);
    }
    const int lev = G(t.level)[u];
    const T gam = (T)G(t.damping)[u];
    const bool has_plus = lev < D;
    // The first kPrefRows "-" links as wave-uniform scalars, read from the
    // tables at a uniform address (scalar loads, no LDS round trip).
    int lsite[kPrefRows];
    T lml[kPrefRows], lmc[kPrefRows];
#pragma unroll
    for (int a = 0; a < kPrefRows; ++a) {
        const size_t at = (size_t)u * Dm + min(a, Dm - 1);
        lsite[a] = a < Dm ? G(t.mlist_site)[at] : -1;
        if constexpr (sizeof(T) == 4) {
            const pair_f w = G(reinterpret_cast<const pair_f*>(t.mlist_w32))[at];
            lml[a] = w.x;
            lmc[a] = w.y;
        } else {
            const pair_d w = G(reinterpret_cast<const pair_d*>(t.mlist_w))[at];
            lml[a] = w.x;
            lmc[a] = w.y;
        }
    }
    // the stage bases of this ADO
    const char* bptr[NBASE];
#pragma unroll
    for (int m = 0; m < NBASE; ++m)
        bptr[m] = reinterpret_cast<const char*>(J.rest[sp.base[m < sp.nbase ? m : 0]]) + (size_t)(u - 1) * tile_bytes;
    for (int a = tid; a < Dm; a += NT) {
        const pair_d w = G(reinterpret_cast<const pair_d*>(t.mlist_w))[(size_t)u * Dm + a];
        sMnb[a] = G(reinterpret_cast<const pair_i*>(t.mlist))[(size_t)u * Dm + a].x;
        sMsite[a] = G(t.mlist_site)[(size_t)u * Dm + a];
        sMml[a] = (T)w.x;
        sMmc[a] = (T)w.y;
    }
    if (has_plus) {
        for (int l = tid; l < W; l += NT) {
            const int nb = G(t.plus)[(size_t)u * W + l];
            sPptr[l] = rest_in + (size_t)(nb - 1) * tile_bytes;
            sPa[l] = (T)G(t.plus_w)[(size_t)u * W + l];
            sModes[l] = G(t.state_modes)[l];
        }
        for (int x = tid; x <= N; x += NT) sBegin[x] = G(t.state_mode_begin)[x];
    }
    for (int x = tid; x < N; x += NT) sDelta[x] = (T)G(t.delta_state)[x];
    // sigma planes, zero outside the N x N block
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const int i = r0 + RS * k;
        sSre[i * LS + j] = cur[k].re;
        sSim[i * LS + j] = cur[k].im;
    }
    __syncthreads();

    // 2. In flight during the matrix cores: the "-" neighbour rows (Hermitian path).
    C pre = {(T)0, (T)0};
    const bool has_pre = HERM && tid < n_rows * N && sMnb[tid / N] >= 0;
    if (has_pre) {
        const int a = tid / N, c = tid - (tid / N) * N;
        pre = load_nb<T>(nbs, sMnb[a], sMsite[a], c);
    }
    // The stage bases: with one base they are in flight through the
    // matrix-core and coupling phases; three would cost registers, so they
    // are read after the couplings.
    C bv[NBASE][EPT];
    if constexpr (NBASE == 1) {
#pragma unroll
        for (int m = 0; m < NBASE; ++m) {
            if (m < sp.nbase) {
#pragma unroll
                for (int k = 0; k < EPT; ++k) {
                    const int i = r0 + RS * k;
                    bv[m][k] = ld<T>(bptr[m], min(i, N - 1) * N + jc);  // unused outside N x N
                }
            }
        }
    }
    // 3. X = H [Re S | Im S]: this wave's 16-row block against every column
    //    block, the NB accumulator chains interleaved so that their LDS reads
    //    and matrix-core latencies overlap.
    {
        const T* plane = half ? sSim : sSre;
        T* out = half ? sXim : sXre;
        acc_t acc[NB];
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) acc[cb] = acc_t{0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            T bval[NB];
#pragma unroll
            for (int cb = 0; cb < NB; ++cb)
                bval[cb] = plane[(4 * ks + (lane >> 4)) * LS + 16 * cb + (lane & 15)];
#pragma unroll
            for (int cb = 0; cb < NB; ++cb) acc[cb] = mfma16(hreg[ks], bval[cb], acc[cb]);
        }
#pragma unroll
        for (int cb = 0; cb < NB; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                out[(16 * mt + mfma_row<T>(lane, r)) * LX + 16 * cb + (lane & 15)] = acc[cb][r];
    }
    if (!HERM) {
        // Y = S H: wave w takes row block w of [Re S; Im S]; H (real
        // symmetric) as the B operand, read per column block.
        const T* plane = wave < NB ? sSre : sSim;
        T* out = wave < NB ? sYre : sYim;
        const int rb = 16 * (wave < NB ? wave : wave - NB);
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) {
            acc_t acc = {0, 0, 0, 0};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                // clamped as for X: rows past N meet zero columns of S,
                // columns past N of Y are never read
                const int kr = min(4 * ks + (lane >> 4), N - 1), hc = min(16 * cb + (lane & 15), N - 1);
                const T hb = h_entry<T>(t, kr * N + hc);
                const T av = plane[(rb + (lane & 15)) * LS + 4 * ks + (lane >> 4)];
                acc = mfma16(av, hb, acc);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
                out[(rb + mfma_row<T>(lane, r)) * LS + 16 * cb + (lane & 15)] = acc[r];
        }
    }
    if (has_pre) {
        sRow[2 * tid] = pre.re;
        sRow[2 * tid + 1] = pre.im;
    }
    __syncthreads();  // sigma planes are free from here on

    // The "+" neighbour values of this thread's elements.
    C xp[EPT][KX];
#pragma unroll
    for (int k = 0; k < EPT; ++k)
#pragma unroll
        for (int q = 0; q < KX; ++q) xp[k][q] = {(T)0, (T)0};
    if (has_plus && jin) {
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int i = r0 + RS * k;
            if (i < N && i != j) {
#pragma unroll
                for (int q = 0; q < KX; ++q) {
                    // Hermitian: modes of state i; general: modes of state i,
                    // then of state j; all at (i, j)
                    const int s = (q < KP) ? i : j, qq = (q < KP) ? q : q - KP;
                    const int m0 = sBegin[s];
                    if (qq < sBegin[s + 1] - m0) xp[k][q] = ld<T>(sPptr[sModes[m0 + qq]], i * N + j);
                }
            }
        }
    }


    // 4. Coupling sums Z into the sigma planes; the stage bases in flight.
    //    The first kPrefRows "-" links are wave-uniform (scalar registers);
    //    mmask marks the states with a "-" link.
    T* sZre = sSre;
    T* sZim = sSim;
    uint64_t mmask = 0;
#pragma unroll
    for (int a = 0; a < kPrefRows; ++a)
        if (lsite[a] >= 0) mmask |= 1ull << lsite[a];
    for (int a = kPrefRows; a < Dm; ++a) {
        const int s = uniform(sMsite[a]);
        if (s >= 0) mmask |= 1ull << s;
    }
    if (jin) {
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int i = r0 + RS * k;
            if (i >= N) continue;
            T zr = 0, zi = 0;
            if (has_plus && i != j) {
#pragma unroll
                for (int pass = 0; pass < (HERM ? 1 : 2); ++pass) {
                    const int s = pass == 0 ? i : j;
                    const int m0 = sBegin[s], cnt = sBegin[s + 1] - m0;
                    T pr = 0, pi = 0;
#pragma unroll
                    for (int q = 0; q < KP; ++q) {
                        if (q < cnt) {
                            const T w = sPa[sModes[m0 + q]];
                            pr += w * xp[k][pass * KP + q].re;
                            pi += w * xp[k][pass * KP + q].im;
                        }
                    }
                    for (int q = KP; q < cnt; ++q) {
                        const int l = sModes[m0 + q];
                        const C x = ld<T>(sPptr[l], i * N + j);
                        pr += sPa[l] * x.re;
                        pi += sPa[l] * x.im;
                    }
                    // i * w * (V^x x): +1 for the modes of state i, -1 for those of j
                    if (pass == 0) {
                        zr -= pi;
                        zi += pr;
                    } else {
                        zr += pi;
                        zi -= pr;
                    }
                }
            }
            const bool row_i = (mmask >> i) & 1;
            const bool row_j = !HERM && ((mmask >> j) & 1);
            if (row_i || row_j) {
                // "-" link a of state s with weights (ml, mc) on element (i, j)
                auto minus = [&](int a, int s, T ml, T mc) {
                    if (HERM) {
                        if (s != i) return;
                        const C x = a < n_rows ? C{sRow[2 * (a * N + j)], sRow[2 * (a * N + j) + 1]}
                                               : load_nb<T>(nbs, sMnb[a], i, j);
                        if (i == j) {
                            zr += 2 * ml * x.re;
                            zi += 2 * ml * x.im;
                        } else {
                            zr += ml * x.re - mc * x.im;
                            zi += ml * x.im + mc * x.re;
                        }
                    } else {
                        if (s != i && s != j) return;
                        const C x = load_nb<T>(nbs, sMnb[a], i, j);
                        const T vx = (T)((i == s) - (j == s)), vo = (T)((i == s) + (j == s));
                        const T thr = ml * vo, thi = mc * vx;
                        zr += thr * x.re - thi * x.im;
                        zi += thr * x.im + thi * x.re;
                    }
                };
#pragma unroll
                for (int a = 0; a < kPrefRows; ++a)
                    if (lsite[a] >= 0) minus(a, lsite[a], lml[a], lmc[a]);
                for (int a = kPrefRows; a < Dm; ++a)
                    if (sMsite[a] >= 0) minus(a, sMsite[a], sMml[a], sMmc[a]);
            }
            // Z is stored only where it can be non-zero (read under the same test)
            if (has_plus || row_i || row_j) {
                sZre[i * LX + j] = zr;
                sZim[i * LX + j] = zi;
            }
        }
    }
    if constexpr (NBASE > 1) {
#pragma unroll
        for (int m = 0; m < NBASE; ++m) {
            if (m < sp.nbase) {
#pragma unroll
                for (int k = 0; k < EPT; ++k) {
                    const int i = r0 + RS * k;
                    bv[m][k] = ld<T>(bptr[m], min(i, N - 1) * N + jc);  // unused outside N x N
                }
            }
        }
    }
    __syncthreads();

    // 5. Elementwise: -i[H, sigma], damping, correction, couplings, and the
    //    stage combination.
    if (!jin) return;
    const T h = (T)(sp.hmul * J.dt), w_in = (T)sp.w_in;
    char* outp = reinterpret_cast<char*>(J.rest[sp.out]) + (size_t)(u - 1) * tile_bytes;
    const T dj = sDelta[j];
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const int i = r0 + RS * k;
        if (i >= N) continue;
        const bool off = i != j;
        T cr, ci, zr, zi;
        const bool zi_row = has_plus || ((mmask >> i) & 1), zj_row = has_plus || ((mmask >> j) & 1);
        zr = zi = (T)0;
        if (HERM) {
            cr = sXre[i * LX + j] - sXre[j * LX + i];
            ci = sXim[i * LX + j] + sXim[j * LX + i];
            if (zi_row) {
                zr = sZre[i * LX + j];
                zi = sZim[i * LX + j];
            }
            if (off && zj_row) {
                zr += sZre[j * LX + i];
                zi -= sZim[j * LX + i];
            }
        } else {
            cr = sXre[i * LX + j] - sYre[i * LS + j];
            ci = sXim[i * LX + j] - sYim[i * LS + j];
            if (zi_row || zj_row) {
                zr = sZre[i * LX + j];
                zi = sZim[i * LX + j];
            }
        }
        const T sr = cur[k].re, si = cur[k].im;
        const T g = gam + (off ? sDelta[i] + dj : (T)0);
        const T fr = ci - g * sr + zr, fi = -cr - g * si + zi;
        T yr = w_in * sr + h * fr, yi = w_in * si + h * fi;
#pragma unroll
        for (int m = 0; m < NBASE; ++m) {
            if (m < sp.nbase) {
                const T w = (T)sp.wbase[m];
                yr += w * bv[m][k].re;
                yi += w * bv[m][k].im;
            }
        }
        st<T>(outp, i * N + j, C{yr, yi});
    }
}


#include "heom_stage_persist.inc"
#include "heom_stage_small.inc"

// Bulk RK4 stage on Hermitian-packed FP32 storage (P as defined at pk_nb).
// Same thread layout and matrix-core product as k_bulk_mfma on its
// Hermitian path; the sigma planes are unpacked from P in LDS.  In P-space
// the right-hand side of element (i, j) is, with X = H sigma = Xr + i Xi:
//   commutator    i <= j: Xi[i][j] + Xi[j][i];   i > j: Xr[i][j] - Xr[j][i]
//   damping       -(gamma_u + (Delta_i + Delta_j if i != j)) P[i][j]
//   "+" modes l   (sum over modes of j - sum over modes of i) w_l P_{u+e_l}[j][i]
//   "-" link a of state s in {i, j}, i != j:
//                 lambda nu_a w_a P_{u-e_a}[i][j] + (s == j ? 1 : -1) c_a w_a P_{u-e_a}[j][i]
//   "-" link a of state s = i = j: 2 lambda nu_a w_a P_{u-e_a}[i][i]
// (the real and imaginary parts of Z[i][j] + conj(Z[j][i]) in the notation
// of k_bulk_mfma).  Each thread reads the "+" neighbours at its own (i, j)
// and hands the weighted sum to element (j, i) through LDS; row s and
// column s of the first "-" neighbours are staged in LDS while the matrix
// cores run.  Every global access of an ADO's own data is coalesced.
template <int NB, int NBASE>
__global__ __launch_bounds__((128 * NB * mfma_ados_per_wg<float, NB>())) __attribute__((
    amdgpu_waves_per_eu(mfma_waves_per_eu<float, NB, true>()))) void k_bulk_mfma_pk(Job single,
                                                                                   StageSpec sp,
                                                                                   int total_tiles,
                                                                                   unsigned lds_stride,
                                                                                   int s0_blocks,
                                                                                   unsigned lds_total) {
    using T = float;
    constexpr int NT = 128 * NB;
    constexpr int AW = mfma_ados_per_wg<T, NB>();
    extern __shared__ char smem_raw[];
    if ((int)blockIdx.x < s0_blocks) {
        sigma0_stage<T, false, false, true>(single, nullptr, blockIdx.x, sp, lds_total, smem_raw);
        return;
    }
    using L = MfmaLds<T, NB, true>;
    constexpr int NP = L::NP, LS = L::LS, LX = L::LX, PLANE = L::PLANE, XPLANE = L::XPLANE;
    constexpr int KS = 4 * NB;
    constexpr int EPT = 2 * NB;
    constexpr int RS = NT / NP;
    constexpr int KP = 2;  // "+" modes per state loaded ahead (more are read late)
    using acc_t = typename mfma_acc<T>::type;

    const int sub = AW > 1 ? uniform((int)threadIdx.x / NT) : 0;
    const int tid = (int)threadIdx.x - sub * NT;
    const int lane = tid & 63, wave = tid >> 6;
    const int mt = wave >> 1, half = wave & 1;
    const int n_first = min((single.n_low + AW - 1) / AW, (int)gridDim.x - s0_blocks);
    const int tile = xcd_remap_low(blockIdx.x - s0_blocks, gridDim.x - s0_blocks, n_first) * AW + sub;
    const bool active = tile < total_tiles;
    const Job& J = single;
    const Tables& t = J.t;
    const int N = t.N, NN = N * N, W = t.W, D = t.D, Dm = D > 0 ? D : 1;
    const int u = active ? 1 + tile : 1;
    const T* rest_in = reinterpret_cast<const T*>(J.rest[sp.in]);
    const T* own = rest_in + (size_t)(u - 1) * NN;
    const NbSrc<T> nbs{J.sig0[sp.in], J.rest[sp.in], N};
    const int n_rows = L::n_rows(D);

    T* sSre = reinterpret_cast<T*>(smem_raw + (size_t)sub * lds_stride);  // sigma, then Q (stride LX)
    T* sSim = sSre + PLANE;
    T* sXre = sSim + PLANE;
    T* sXim = sXre + XPLANE;
    T* sRow = sXim + XPLANE;  // [n_rows][N] rows s, then [n_rows][N] columns s
    T* sCol = sRow + n_rows * N;
    const T** sPptr = reinterpret_cast<const T**>(sRow + 2 * n_rows * N);  // [W]
    T* sMml = reinterpret_cast<T*>(sPptr + W);
    T* sMmc = sMml + Dm;
    T* sDelta = sMmc + Dm;
    T* sPa = sDelta + N;
    int* sBegin = reinterpret_cast<int*>(sPa + W);
    int* sModes = sBegin + N + 1;
    int* sMsite = sModes + W;
    int* sMnb = sMsite + Dm;

    const int r0 = tid / NP, j = tid - (tid / NP) * NP;
    const bool jin = active && j < N;

    // 1. Own P values (clamped unpredicated loads, zeroed outside N x N), H,
    //    link tables.
    T cur[EPT];
    const int jc = min(j, N - 1);
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const int i = r0 + RS * k;
        const T m = (jin && i < N) ? (T)1 : (T)0;
        cur[k] = G(own)[min(i, N - 1) * N + jc] * m;
    }
    T hreg[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const int r = min(16 * mt + (lane & 15), N - 1), c = min(4 * ks + (lane >> 4), N - 1);
        hreg[ks] = h_entry<T>(t, r * N + c);
    }
    const int lev = G(t.level)[u];
    const T gam = (T)G(t.damping)[u];
    const bool has_plus = lev < D;
    int lsite[kPrefRows];
    T lml[kPrefRows], lmc[kPrefRows];
#pragma unroll
    for (int a = 0; a < kPrefRows; ++a) {
        const size_t at = (size_t)u * Dm + min(a, Dm - 1);
        lsite[a] = a < Dm ? G(t.mlist_site)[at] : -1;
        const pair_f w = G(reinterpret_cast<const pair_f*>(t.mlist_w32))[at];
        lml[a] = w.x;
        lmc[a] = w.y;
    }
    const T* bptr[NBASE];
#pragma unroll
    for (int m = 0; m < NBASE; ++m)
        bptr[m] = reinterpret_cast<const T*>(J.rest[sp.base[m < sp.nbase ? m : 0]]) + (size_t)(u - 1) * NN;
    for (int a = tid; a < Dm; a += NT) {
        const pair_d w = G(reinterpret_cast<const pair_d*>(t.mlist_w))[(size_t)u * Dm + a];
        sMnb[a] = G(reinterpret_cast<const pair_i*>(t.mlist))[(size_t)u * Dm + a].x;
        sMsite[a] = G(t.mlist_site)[(size_t)u * Dm + a];
        sMml[a] = (T)w.x;
        sMmc[a] = (T)w.y;
    }
    if (has_plus) {
        for (int l = tid; l < W; l += NT) {
            const int nb = G(t.plus)[(size_t)u * W + l];
            sPptr[l] = rest_in + (size_t)(nb - 1) * NN;
            sPa[l] = (T)G(t.plus_w)[(size_t)u * W + l];
            sModes[l] = G(t.state_modes)[l];
        }
        for (int x = tid; x <= N; x += NT) sBegin[x] = G(t.state_mode_begin)[x];
    }
    for (int x = tid; x < N; x += NT) sDelta[x] = (T)G(t.delta_state)[x];
    // Unpack into the sigma planes in two passes: P row-major into the X
    // plane (free until the matrix cores write it), then each thread reads
    // P[j][i] (odd stride: distinct banks) and writes Re and Im of its own
    // cells row-major.  Zero outside the N x N block.
#pragma unroll
    for (int k = 0; k < EPT; ++k) sXre[(r0 + RS * k) * LX + j] = cur[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const int i = r0 + RS * k;
        const T pt = sXre[j * LX + i];
        sSre[i * LS + j] = i <= j ? cur[k] : pt;
        sSim[i * LS + j] = i < j ? pt : (i > j ? -cur[k] : (T)0);
    }
    __syncthreads();

    // 2. Row s and column s of the first "-" neighbours in flight; X = H sigma.
    //    With a complex copy of the input's lower levels, one contiguous row
    //    s of sigma_{u-e_a} gives both (P[s][c] and P[c][s]); otherwise the
    //    column is read from the packed ADO.
    const void* mir_in = sp.mirror_in ? J.mirror[sp.mirror_in - 1] : nullptr;
    T pre = 0, pre2 = 0;
    const int nrn = n_rows * N;
    bool has_pre;
    if (mir_in) {
        has_pre = tid < nrn && sMnb[tid / N] >= 0;
        if (has_pre) {
            const int a = tid / N, c = tid - (tid / N) * N, s = sMsite[a], nb = sMnb[a];
            const cpx<T> x = nb == 0 ? load_nb<T>(nbs, 0, s, c) : ld<T>(mir_in, (size_t)(nb - 1) * NN + s * N + c);
            pre = c >= s ? x.re : -x.im;  // P[s][c]
            pre2 = c > s ? x.im : x.re;   // P[c][s]
        }
    } else {
        has_pre = tid < 2 * nrn && sMnb[(tid < nrn ? tid : tid - nrn) / N] >= 0;
        if (has_pre) {
            const int x = tid < nrn ? tid : tid - nrn;
            const int a = x / N, c = x - (x / N) * N, s = sMsite[a];
            pre = tid < nrn ? pk_nb(nbs, sMnb[a], s, c) : pk_nb(nbs, sMnb[a], c, s);
        }
    }
    // the stage bases: one base is in flight through the matrix-core phase,
    // three are read after the couplings (registers)
    T bv[NBASE][EPT];
    if constexpr (NBASE == 1) {
#pragma unroll
        for (int m = 0; m < NBASE; ++m) {
            if (m < sp.nbase) {
#pragma unroll
                for (int k = 0; k < EPT; ++k) {
                    const int i = r0 + RS * k;
                    bv[m][k] = G(bptr[m])[min(i, N - 1) * N + jc];  // unused outside N x N
                }
            }
        }
    }
    {
        const T* plane = half ? sSim : sSre;
        T* out = half ? sXim : sXre;
        acc_t acc[NB];
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) acc[cb] = acc_t{0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            T bval[NB];
#pragma unroll
            for (int cb = 0; cb < NB; ++cb)
                bval[cb] = plane[(4 * ks + (lane >> 4)) * LS + 16 * cb + (lane & 15)];
#pragma unroll
            for (int cb = 0; cb < NB; ++cb) acc[cb] = mfma16(hreg[ks], bval[cb], acc[cb]);
        }
#pragma unroll
        for (int cb = 0; cb < NB; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                out[(16 * mt + mfma_row<T>(lane, r)) * LX + 16 * cb + (lane & 15)] = acc[cb][r];
    }
    if (has_pre) {
        sRow[tid] = pre;
        if (mir_in) sCol[tid] = pre2;
    }
    __syncthreads();  // sigma planes are free from here on

    // 3. "+" neighbours at the thread's own elements: modes of state i, then of j.
    T xp[EPT][2 * KP];
#pragma unroll
    for (int k = 0; k < EPT; ++k)
#pragma unroll
        for (int q = 0; q < 2 * KP; ++q) xp[k][q] = (T)0;
    if (has_plus && jin) {
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int i = r0 + RS * k;
            if (i < N && i != j) {
#pragma unroll
                for (int q = 0; q < 2 * KP; ++q) {
                    const int s = q < KP ? i : j, qq = q < KP ? q : q - KP;
                    const int m0 = sBegin[s];
                    if (qq < sBegin[s + 1] - m0) xp[k][q] = G(sPptr[sModes[m0 + qq]])[i * N + j];
                }
            }
        }
    }
    // 4. Q[i][j] = (sum over modes of i - sum over modes of j) w_l P_{u+e_l}[i][j],
    //    read by element (j, i); the stage bases in flight.
    T* sQ = sSre;
    if (has_plus && jin) {
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int i = r0 + RS * k;
            if (i >= N || i == j) continue;
            T q = 0;
#pragma unroll
            for (int pass = 0; pass < 2; ++pass) {
                const int s = pass == 0 ? i : j;
                const int m0 = sBegin[s], cnt = sBegin[s + 1] - m0;
                T acc = 0;
#pragma unroll
                for (int qq = 0; qq < KP; ++qq)
                    if (qq < cnt) acc += sPa[sModes[m0 + qq]] * xp[k][pass * KP + qq];
                for (int qq = KP; qq < cnt; ++qq) {
                    const int l = sModes[m0 + qq];
                    acc += sPa[l] * G(sPptr[l])[i * N + j];
                }
                q += pass == 0 ? acc : -acc;
            }
            sQ[i * LX + j] = q;
        }
    }
    if constexpr (NBASE > 1) {
#pragma unroll
        for (int m = 0; m < NBASE; ++m) {
            if (m < sp.nbase) {
#pragma unroll
                for (int k = 0; k < EPT; ++k) {
                    const int i = r0 + RS * k;
                    bv[m][k] = G(bptr[m])[min(i, N - 1) * N + jc];  // unused outside N x N
                }
            }
        }
    }
    uint64_t mmask = 0;
#pragma unroll
    for (int a = 0; a < kPrefRows; ++a)
        if (lsite[a] >= 0) mmask |= 1ull << lsite[a];
    // "-" links past the staged rows (depth > kPrefRows): their terms here,
    // so that the elementwise phase issues no global loads (a wait for
    // those would also wait for its own stores).
    T fl[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) fl[k] = (T)0;
    for (int a = kPrefRows; a < Dm; ++a) {
        const int s = uniform(sMsite[a]);
        if (s < 0) continue;
        mmask |= 1ull << s;
        if (!jin) continue;
        const T ml = sMml[a], mc = sMmc[a];
        const int nb = sMnb[a];
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int i = r0 + RS * k;
            if (i >= N || (s != i && s != j)) continue;
            const T pij = pk_nb(nbs, nb, i, j);
            if (i == j) {
                fl[k] += 2 * ml * pij;
            } else {
                const T pji = pk_nb(nbs, nb, j, i);
                fl[k] += ml * pij + (s == j ? mc : -mc) * pji;
            }
        }
    }
    __syncthreads();

    // 5. Elementwise right-hand side in P-space and the stage combination.
    const T h = (T)(sp.hmul * J.dt), w_in = (T)sp.w_in;
    T* outp = reinterpret_cast<T*>(J.rest[sp.out]) + (size_t)(u - 1) * NN;
    const T dj = sDelta[j < N ? j : 0];
    const bool row_j = (mmask >> j) & 1;
    T yv[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const int i = r0 + RS * k;
        yv[k] = 0;
        if (!jin || i >= N) continue;
        const T p = cur[k];
        T f;
        if (i == j) {
            f = 2 * sXim[i * LX + i] - gam * p;
        } else {
            f = i < j ? sXim[i * LX + j] + sXim[j * LX + i] : sXre[i * LX + j] - sXre[j * LX + i];
            f -= (gam + sDelta[i] + dj) * p;
            if (has_plus) f += sQ[j * LX + i];
        }
        if (((mmask >> i) & 1) || row_j) {
            // staged "-" link a (a < n_rows) of state s, with
            // P_{u-e_a}[i][j] = pij and P_{u-e_a}[j][i] = pji
#pragma unroll
            for (int a = 0; a < kPrefRows; ++a) {
                const int s = lsite[a];
                if (s < 0 || (s != i && s != j)) continue;
                const T pij = s == i ? sRow[a * N + j] : sCol[a * N + i];
                const T pji = s == i ? sCol[a * N + j] : sRow[a * N + i];
                if (i == j)
                    f += 2 * lml[a] * pij;
                else
                    f += lml[a] * pij + (s == j ? lmc[a] : -lmc[a]) * pji;
            }
            f += fl[k];
        }
        T y = w_in * p + h * f;
#pragma unroll
        for (int m = 0; m < NBASE; ++m)
            if (m < sp.nbase) y += (T)sp.wbase[m] * bv[m][k];
        G(outp)[i * N + j] = y;
        yv[k] = y;
    }
    // 6. The complex copy of a lower-level output (the next stage's "-"
    //    rows): P_out[j][i] from a transposed LDS read.  Workgroup-uniform
    //    test (its ADOs are u0 and u0 + 1), so that every thread reaches the
    //    barrier.
    const int u0 = 1 + xcd_remap_low(blockIdx.x - s0_blocks, gridDim.x - s0_blocks, n_first) * AW;
    if (sp.mirror_out && u0 <= J.n_low) {
        T* sY = sSim;  // free since the matrix-core phase
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int i = r0 + RS * k;
            if (jin && i < N) sY[i * LX + j] = yv[k];
        }
        __syncthreads();
        if (jin && u <= J.n_low) {
            void* mir_out = J.mirror[sp.mirror_out - 1];
#pragma unroll
            for (int k = 0; k < EPT; ++k) {
                const int i = r0 + RS * k;
                if (i >= N) continue;
                const T yt = sY[j * LX + i];
                const cpx<T> v = i <= j ? cpx<T>{yv[k], i < j ? yt : (T)0} : cpx<T>{yt, -yv[k]};
                st<T>(mir_out, (size_t)(u - 1) * NN + i * N + j, v);
            }
        }
    }
}

// Complex64 copy of packed ADOs: M[u][i][j] = sigma_u(i, j), u < n.
__global__ __launch_bounds__(256) void k_pk_mirror(const float* P, void* M, int N, int64_t total) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= total) return;
    const int NN = N * N;
    const int64_t u = idx / NN;
    const int e = (int)(idx - u * NN), i = e / N, j = e - (e / N) * N;
    const float* p = P + u * NN;
    const float x = G(p)[min(i, j) * N + max(i, j)], y = G(p)[max(i, j) * N + min(i, j)];
    st<float>(M, (size_t)idx, cpx<float>{x, i < j ? y : (i > j ? -y : 0.0f)});
}

}  // namespace

int bulk_mfma_blocks(int N, bool h_complex, int precision) {
    if (N < 16 || h_complex || (precision == 0 && N > 48)) return 0;
    return (N + 15) / 16;
}

std::atomic<int> g_max_workgroups{0}, g_max_ados_per_tile{0};

int bulk_ados_per_tile(int N, int W, int D, int tsize) {
    const int NN = N * N;
    const int nt = fma_block(tsize, N);
    int g = NN >= nt ? 1 : nt / NN;
    const int cap = g_max_ados_per_tile.load();
    if (cap > 0) g = std::min(g, cap);
    // keep a tile's LDS (matrices plus staged links) within 64 KiB
    while (g > 1 && fma_lds(N, W, D, g, tsize).total > 64 * 1024) --g;
    return g;
}

hipError_t launch_pk_mirror(const void* packed_rest, void* mirror, int N, int n, hipStream_t stream) {
    const int64_t total = (int64_t)n * N * N;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pk_mirror, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream,
                       static_cast<const float*>(packed_rest), mirror, N, total);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// Coherence-block form of absorption (section "Linear absorption spectra"):
// with the ground state g uncoupled from the baths and from the excited
// states, and sigma_0(0) = mu_p^+ |g><g|, every ADO keeps only its column g
// on the excited states.  The N x 3 block Y_u[a][p] = sigma_u^{(p)}[a][g]
// holds the three directions.  Restricted to that column, eq. HEOM reads
//   f[a][p] = -i (H Y)[a][p] - (gamma_u + Delta_a) Y[a][p]
//             + sum over "+" modes l of state a of i w_l Y_{u+e_l}[a][p]
//             + sum over "-" links of state a of (lambda nu + i c) w Y_{u-e_l}[a][p]
// (V^x and V^o act as the row mask delta_{a,s}; V^x V^x as delta_{a,s};
// the ground energy is 0 in the frame of the excited block).  FP64, one
// thread per element, ADO 0 included.
// --------------------------------------------------------------------------
struct BlockBases {
    const void* p[3];
    double w[3];
};

// One element idx = (u * N + a) * 3 + p of a stage; shared by the
// single-request and the batched kernels so both round the same way.
__device__ __forceinline__ void block_stage_elem(const Tables& t, const void* in, void* out,
                                                 const BlockBases& bb, int nbase, double w_in,
                                                 double h, int64_t idx) {
    const int N = t.N, W = t.W, D = t.D, Dm = D > 0 ? D : 1, R = 3 * N;
    const int64_t u = idx / R;
    const int r = (int)(idx - u * R), a = r / 3, p = r - (r / 3) * 3;
    auto Y = [&](int64_t v, int row) { return ld<double>(in, (size_t)(v * N + row) * 3 + p); };
    // -i H Y with the diagonal shift restored (the ground energy is 0, so
    // the shift does not cancel here)
    double cr = t.h_shift * Y(u, a).re, ci = t.h_shift * Y(u, a).im;
    for (int b = 0; b < N; ++b) {
        const double hr = G(t.h_re)[a * N + b], hi = t.h_complex ? G(t.h_im)[a * N + b] : 0.0;
        const cpx<double> y = Y(u, b);
        cr = fma(hr, y.re, fma(-hi, y.im, cr));
        ci = fma(hr, y.im, fma(hi, y.re, ci));
    }
    const cpx<double> y0 = Y(u, a);
    const double g = G(t.damping)[u] + G(t.delta_state)[a];
    double fr = fma(-g, y0.re, ci), fi = fma(-g, y0.im, -cr);
    if (G(t.level)[u] < D) {
        for (int m = G(t.state_mode_begin)[a]; m < G(t.state_mode_begin)[a + 1]; ++m) {
            const int l = G(t.state_modes)[m];
            const int nb = G(t.plus)[(size_t)u * W + l];
            if (nb < 0) continue;
            const double w = G(t.plus_w)[(size_t)u * W + l];
            const cpx<double> x = Y(nb, a);
            fr = fma(-w, x.im, fr);
            fi = fma(w, x.re, fi);
        }
    }
    for (int k = 0; k < Dm; ++k) {
        const size_t at = (size_t)u * Dm + k;
        if (G(t.mlist_site)[at] != a) continue;
        const int nb = G(reinterpret_cast<const pair_i*>(t.mlist))[at].x;
        if (nb < 0) continue;
        const pair_d w = G(reinterpret_cast<const pair_d*>(t.mlist_w))[at];
        const cpx<double> x = Y(nb, a);
        fr = fma(w.x, x.re, fma(-w.y, x.im, fr));
        fi = fma(w.x, x.im, fma(w.y, x.re, fi));
    }
    double yr = fma(h, fr, w_in * y0.re), yi = fma(h, fi, w_in * y0.im);
    for (int m = 0; m < nbase; ++m) {
        const cpx<double> b = ld<double>(bb.p[m], (size_t)idx);
        yr = fma(bb.w[m], b.re, yr);
        yi = fma(bb.w[m], b.im, yi);
    }
    st<double>(out, (size_t)idx, cpx<double>{yr, yi});
}

__global__ __launch_bounds__(256) void k_block_stage(Tables t, const void* in, void* out,
                                                     BlockBases bb, int nbase, double w_in,
                                                     double h, int64_t total) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= total) return;
    block_stage_elem(t, in, out, bb, nbase, w_in, h, idx);
}

// Many coherence-block requests in one launch: job j owns the elements
// [elem_begin, elem_begin + n_ado * 3 * N) of the launch.
__global__ __launch_bounds__(256) void k_block_stage_batched(const BlockJob* jobs, int n_jobs,
                                                             StageSpec sp, int64_t total) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= total) return;
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (G(&jobs[mid].elem_begin)[0] <= idx) lo = mid;
        else hi = mid - 1;
    }
    const BlockJob& J = jobs[lo];
    BlockBases bb{};
    for (int m = 0; m < sp.nbase; ++m) {
        bb.p[m] = J.y[sp.base[m]];
        bb.w[m] = sp.wbase[m];
    }
    block_stage_elem(J.t, J.y[sp.in], J.y[sp.out], bb, sp.nbase, sp.w_in, sp.hmul * J.dt,
                     idx - J.elem_begin);
}

struct ObsArg {
    double v[3][64];
};

// P_p = sum_a obs[p][a] Y_0[a][p], written as (Re, Im) pairs at rec[2p].
template <class Obs>
__device__ __forceinline__ void block_project(const void* y, const Obs& obs, int N, int p,
                                              double* rec, int32_t* status) {
    double pr = 0.0, pi = 0.0;
    for (int a = 0; a < N; ++a) {
        const cpx<double> x = ld<double>(y, (size_t)a * 3 + p);
        const double o = obs(p, a);
        pr = fma(o, x.re, pr);
        pi = fma(o, x.im, pi);
    }
    G(rec)[2 * p] = pr;
    G(rec)[2 * p + 1] = pi;
    if (!(isfinite(pr) && isfinite(pi))) *G(status) = 1;
}

__global__ __launch_bounds__(64) void k_block_record(const void* y, ObsArg obs, int N, double* rec,
                                                     int32_t* status) {
    const int p = threadIdx.x;
    if (p >= 3) return;
    block_project(y, [&](int q, int a) { return obs.v[q][a]; }, N, p, rec, status);
}

// One workgroup per job: advance the job's step counter and, when the
// record is due, write it.
__global__ __launch_bounds__(64) void k_block_record_batched(const BlockJob* jobs) {
    const BlockJob& J = jobs[blockIdx.x];
    const int64_t s = G(J.step)[0] + 1;
    __syncthreads();
    if (threadIdx.x == 0) G(J.step)[0] = s;
    const int p = threadIdx.x;
    if (p >= 3 || s % J.record_every != 0) return;
    const double* o = J.obs;
    const int N = J.t.N;
    block_project(J.y[0], [&](int q, int a) { return G(o)[q * N + a]; }, N, p,
                  J.rec + 6 * (s / J.record_every), J.status);
}

// Fluorescence start (section "Static Fluorescence Spectra": the dipole
// operator acts on all ADOs): element (i, j) of the (N+1)-state ADO u is
// sum_b sigma_u[i-1][b] mu[b] for j = 0 < i, zero elsewhere.  One thread per
// output element; ADO 0 is complex128 on both sides.
struct MuArg {
    double mu[64];
};

template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_emission_start(const void* in_sig0, const void* in_rest,
                                                        void* out_sig0, void* out_rest, MuArg mu,
                                                        int N, int64_t total) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= total) return;
    const int M = N + 1, MM = M * M;
    const int64_t u = idx / MM;
    const int e = (int)(idx - u * MM), i = e / M, j = e - (e / M) * M;
    double yr = 0.0, yi = 0.0;
    if (j == 0 && i > 0) {
        for (int b = 0; b < N; ++b) {
            const size_t at = (size_t)(i - 1) * N + b;
            double xr, xi;
            if (u == 0) {
                const cpx<double> x = ld<double>(in_sig0, at);
                xr = x.re;
                xi = x.im;
            } else {
                const cpx<TI> x = ld<TI>(in_rest, (size_t)(u - 1) * N * N + at);
                xr = (double)x.re;
                xi = (double)x.im;
            }
            yr += xr * mu.mu[b];
            yi += xi * mu.mu[b];
        }
    }
    if (u == 0)
        st<double>(out_sig0, (size_t)e, cpx<double>{yr, yi});
    else
        st<TO>(out_rest, (size_t)(u - 1) * MM + e, cpx<TO>{(TO)yr, (TO)yi});
}

hipError_t launch_emission_start(const void* in_sig0, const void* in_rest, int in_prec,
                                 void* out_sig0, void* out_rest, int out_prec, const double* mu,
                                 int N, int64_t n_ado, hipStream_t stream) {
    if (N < 1 || N > 63 || n_ado < 1) return hipErrorInvalidValue;
    MuArg m{};
    for (int b = 0; b < N; ++b) m.mu[b] = mu[b];
    const int64_t total = n_ado * (int64_t)(N + 1) * (N + 1);
    const dim3 grid((unsigned)((total + 255) / 256)), block(256);
    if (in_prec == 0 && out_prec == 0)
        hipLaunchKernelGGL((k_emission_start<double, double>), grid, block, 0, stream, in_sig0, in_rest, out_sig0, out_rest, m, N, total);
    else if (in_prec == 0)
        hipLaunchKernelGGL((k_emission_start<double, float>), grid, block, 0, stream, in_sig0, in_rest, out_sig0, out_rest, m, N, total);
    else if (out_prec == 0)
        hipLaunchKernelGGL((k_emission_start<float, double>), grid, block, 0, stream, in_sig0, in_rest, out_sig0, out_rest, m, N, total);
    else
        hipLaunchKernelGGL((k_emission_start<float, float>), grid, block, 0, stream, in_sig0, in_rest, out_sig0, out_rest, m, N, total);
    return hipGetLastError();
}

hipError_t launch_block_stage(const Tables& t, const void* in, void* out, const void* const* base,
                              const double* wb, int nbase, double w_in, double h,
                              hipStream_t stream) {
    if (nbase < 0 || nbase > 3 || t.N < 1 || t.N > 64) return hipErrorInvalidValue;
    BlockBases bb{};
    for (int m = 0; m < nbase; ++m) {
        bb.p[m] = base[m];
        bb.w[m] = wb[m];
    }
    const int64_t total = (int64_t)t.n_ado * 3 * t.N;
    hipLaunchKernelGGL(k_block_stage, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream,
                       t, in, out, bb, nbase, w_in, h, total);
    return hipGetLastError();
}

hipError_t launch_block_record(const void* y, const double* obs, int N, double* rec,
                               int32_t* status, hipStream_t stream) {
    if (N < 1 || N > 64) return hipErrorInvalidValue;
    ObsArg o{};
    for (int p = 0; p < 3; ++p)
        for (int a = 0; a < N; ++a) o.v[p][a] = obs[p * N + a];
    hipLaunchKernelGGL(k_block_record, dim3(1), dim3(64), 0, stream, y, o, N, rec, status);
    return hipGetLastError();
}

hipError_t launch_block_stage_batched(const BlockJob* jobs_dev, int n_jobs, int64_t total,
                                      const StageSpec& sp, hipStream_t stream) {
    if (n_jobs < 1 || total <= 0) return hipSuccess;
    if (sp.nbase < 0 || sp.nbase > 3) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_block_stage_batched, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                       stream, jobs_dev, n_jobs, sp, total);
    return hipGetLastError();
}

hipError_t launch_block_record_batched(const BlockJob* jobs_dev, int n_jobs, hipStream_t stream) {
    if (n_jobs < 1) return hipSuccess;
    hipLaunchKernelGGL(k_block_record_batched, dim3((unsigned)n_jobs), dim3(64), 0, stream, jobs_dev);
    return hipGetLastError();
}

hipError_t launch_enumerate(const Tables& t, hipStream_t stream) {
    if (t.n_ado <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_enumerate, dim3((t.n_ado + 255) / 256), dim3(256), 0, stream, t);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (t.W > 0) {
        const int64_t n = (int64_t)t.n_ado * t.W;
        hipLaunchKernelGGL(k_links, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, t);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_minus_list, dim3((t.n_ado + 255) / 256), dim3(256), 0, stream, t);
    return hipGetLastError();
}

// Lets kernel `fn` take up to 160 KiB of LDS.  Called once per kernel (the
// launcher's own once_flag), so concurrent first launches do not race.
static hipError_t allow_full_lds(std::once_flag& once, hipError_t& err, const void* fn) {
    std::call_once(once, [&] {
        err = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    });
    return err;
}

template <typename T, bool BATCHED, bool PK = false>
static hipError_t launch_sigma0_t(const Job& single, const Job* jobs_dev, int n_jobs,
                                  const StageSpec& sp, size_t lds, hipStream_t stream) {
    static std::once_flag attr_once;
    static hipError_t attr_err = hipSuccess;
    if (allow_full_lds(attr_once, attr_err, reinterpret_cast<const void*>(&k_sigma0<T, BATCHED, PK>)) != hipSuccess) return attr_err;
    hipLaunchKernelGGL((k_sigma0<T, BATCHED, PK>), dim3(BATCHED ? n_jobs : 1), dim3(kBlock), lds,
                       stream, single, jobs_dev, n_jobs, sp, (unsigned)lds);
    return hipGetLastError();
}

// sigma_0 rides along with a bulk launch as n_s0 extra workgroups (placed
// first) when the kernel carries it (`allow`) and its staging fits the
// launch's LDS, which may grow up to `lds_budget` (what costs the bulk
// kernel no occupancy); otherwise it gets its own launch first.  Sets the
// number of workgroups to add and the launch's LDS.
template <typename T, bool BATCHED, bool PK = false>
static hipError_t sigma0_ride_along(const Job& single, const Job* jobs_dev, int n_jobs, int n_s0,
                                    bool allow, const StageSpec& sp, size_t lds_budget,
                                    hipStream_t stream, int* added, size_t* lds) {
    *added = 0;
    const int N = single.t.N, W = single.t.W;
    const size_t cap = std::max(*lds, lds_budget);
    // largest N and W of the batch; non-Hermitian staging needs the most LDS
    const size_t full = sigma0_lds(N, W, (int)sizeof(T), false, 160 * 1024).total;
    const size_t bare = sigma0_lds(N, W, (int)sizeof(T), false, 0).total;
    if (allow && bare <= cap) {
        *lds = std::max(*lds, full <= cap ? full : bare);
        *added = n_s0;
        return hipSuccess;
    }
    const size_t lds0 = sigma0_lds(N, W, (int)sizeof(T), false, 160 * 1024).total;
    return launch_sigma0_t<T, BATCHED, PK>(single, jobs_dev, n_jobs, sp, lds0, stream);
}

template <typename T, int NB, bool HERM, bool BATCHED, int NBASE>
static hipError_t launch_mfma_t(const Job& single, const Job* jobs_dev, int n_jobs,
                                int total_tiles, const StageSpec& sp, hipStream_t stream, int n_s0) {
    const void* fn = reinterpret_cast<const void*>(&k_bulk_mfma<T, NB, HERM, BATCHED, NBASE>);
    static std::once_flag attr_once;
    static hipError_t attr_err = hipSuccess;
    if (allow_full_lds(attr_once, attr_err, fn) != hipSuccess) return attr_err;
    constexpr int AW = mfma_ados_per_wg<T, NB>();
    const unsigned stride =
        (unsigned)((MfmaLds<T, NB, HERM>::bytes(single.t.N, single.t.W, single.t.D) + 15) & ~(size_t)15);
    // sigma_0 rides along only within the bulk workgroups' own LDS
    size_t lds = (size_t)stride * AW;
    int extra = 0;
    hipError_t e = sigma0_ride_along<T, BATCHED>(single, jobs_dev, n_jobs, n_s0, true, sp, lds, stream,
                                                 &extra, &lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_bulk_mfma<T, NB, HERM, BATCHED, NBASE>),
                       dim3(extra + (total_tiles + AW - 1) / AW), dim3(128 * NB * AW), lds, stream,
                       single, jobs_dev, n_jobs, sp, total_tiles, stride, extra, (unsigned)lds);
    return hipGetLastError();
}

template <typename T, int NB, bool HERM, bool BATCHED>
static hipError_t launch_mfma_b(const Job& single, const Job* jobs_dev, int n_jobs,
                                int total_tiles, const StageSpec& sp, hipStream_t stream, int n_s0) {
    if (sp.nbase <= 1)
        return launch_mfma_t<T, NB, HERM, BATCHED, 1>(single, jobs_dev, n_jobs, total_tiles, sp,
                                                      stream, n_s0);
    return launch_mfma_t<T, NB, HERM, BATCHED, 3>(single, jobs_dev, n_jobs, total_tiles, sp,
                                                  stream, n_s0);
}

template <typename T, int NB>
static hipError_t launch_mfma_nb(bool herm, bool batched, const Job& single, const Job* jobs_dev,
                                 int n_jobs, int total_tiles, const StageSpec& sp,
                                 hipStream_t stream, int n_s0) {
    if (herm)
        return batched ? launch_mfma_b<T, NB, true, true>(single, jobs_dev, n_jobs, total_tiles,
                                                          sp, stream, n_s0)
                       : launch_mfma_b<T, NB, true, false>(single, jobs_dev, n_jobs, total_tiles,
                                                           sp, stream, n_s0);
    return batched ? launch_mfma_b<T, NB, false, true>(single, jobs_dev, n_jobs, total_tiles, sp,
                                                       stream, n_s0)
                   : launch_mfma_b<T, NB, false, false>(single, jobs_dev, n_jobs, total_tiles, sp,
                                                        stream, n_s0);
}

template <typename T>
static hipError_t launch_mfma(int nb, bool herm, const Job& single, const Job* jobs_dev,
                              int n_jobs, int total_tiles, const StageSpec& sp,
                              hipStream_t stream, int n_s0) {
    const bool batched = jobs_dev != nullptr;
    switch (nb) {
        case 1: return launch_mfma_nb<T, 1>(herm, batched, single, jobs_dev, n_jobs, total_tiles, sp, stream, n_s0);
        case 2: return launch_mfma_nb<T, 2>(herm, batched, single, jobs_dev, n_jobs, total_tiles, sp, stream, n_s0);
        case 3: return launch_mfma_nb<T, 3>(herm, batched, single, jobs_dev, n_jobs, total_tiles, sp, stream, n_s0);
        case 4:
            // FP64 above 48 states takes the FMA kernel (LDS)
            if constexpr (sizeof(T) == 4)
                return launch_mfma_nb<T, 4>(herm, batched, single, jobs_dev, n_jobs, total_tiles, sp, stream, n_s0);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}


// Workgroups of the persistent kernel that are resident at once on the
// device (all MI355X CUs alike), cached per kernel and LDS size.
static int resident_workgroups(const void* fn, int threads, size_t lds, int max_per_cu) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    per_cu = std::min(per_cu, max_per_cu);
    static std::atomic<int> n_cu{0};
    if (n_cu.load() == 0) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus < 1)
            cus = 256;
        n_cu.store(cus);
    }
    return per_cu * n_cu.load();
}

template <int NB, int NBASE, int VEC>
static hipError_t launch_persist_t(const Job& single, int total_tiles, const StageSpec& sp,
                                   hipStream_t stream) {
    const void* fn = reinterpret_cast<const void*>(&k_stage_persist<NB, NBASE, VEC>);
    static std::once_flag attr_once;
    static hipError_t attr_err = hipSuccess;
    if (allow_full_lds(attr_once, attr_err, fn) != hipSuccess) return attr_err;
    constexpr int NT = 128 * NB;
    const size_t own = PersistLds<NB>::bytes;
    // sigma_0 rides along when its staging fits the LDS that the register
    // limit leaves to each resident workgroup
    // two workers per CU for N > 32 (measured faster than the three that the
    // registers of the stage without bases allow); up to sixteen 2-wave
    // workers for N <= 16
    const int cap = NB >= 3 ? 2 : 16;
    int by_regs = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&by_regs, fn, NT, own) != hipSuccess || by_regs < 1)
        by_regs = 1;
    by_regs = std::min(by_regs, cap);
    const size_t budget = std::max(own, (size_t)(160 * 1024 / by_regs) & ~(size_t)1023);
    size_t lds = own;
    int extra = 0;
    hipError_t e = sigma0_ride_along<float, false>(single, nullptr, 1, 1, true, sp, budget, stream,
                                                   &extra, &lds);
    if (e != hipSuccess) return e;
    int workers = std::min(total_tiles, resident_workgroups(fn, NT, lds, cap));
    if (g_max_workgroups.load() > 0) workers = std::min(workers, g_max_workgroups.load());
    hipLaunchKernelGGL((k_stage_persist<NB, NBASE, VEC>), dim3(extra + workers), dim3(NT), lds,
                       stream, single, sp, total_tiles, extra, (unsigned)lds);
    return hipGetLastError();
}

template <int NB, int VEC>
static hipError_t launch_persist_vec(const Job& single, int total_tiles, const StageSpec& sp,
                                     hipStream_t stream) {
    switch (sp.nbase) {
        case 0: return launch_persist_t<NB, 0, VEC>(single, total_tiles, sp, stream);
        case 1: return launch_persist_t<NB, 1, VEC>(single, total_tiles, sp, stream);
        case 2: return launch_persist_t<NB, 2, VEC>(single, total_tiles, sp, stream);
        case 3: return launch_persist_t<NB, 3, VEC>(single, total_tiles, sp, stream);
        default: return hipErrorInvalidValue;
    }
}

template <int NB>
static hipError_t launch_persist_nb(const Job& single, int total_tiles, const StageSpec& sp,
                                    hipStream_t stream) {
    // even N: element pairs (aligned 16-byte accesses); odd N: single elements
    return single.t.N % 2 == 0 ? launch_persist_vec<NB, 2>(single, total_tiles, sp, stream)
                               : launch_persist_vec<NB, 1>(single, total_tiles, sp, stream);
}

// The persistent matrix-core kernel takes single-job FP32 stages over
// Hermitian ADOs with a real H and 10 <= N <= 64.  Below N = 10 an ADO fills
// too little of a 16 x 16 matrix-core tile, and tiles of several ADOs on the
// FMA path are faster (the 12.3M-ADO (6, 6) FMO reference at N = 7: 17.8 ms
// per stage here, 15.9 ms on the one-launch FMA kernel, 6.6 ms on the
// persistent FMA kernel; at N = 14, 237k ADOs: 0.34 ms here against 0.49 ms
// on the persistent FMA kernel and 1.18 ms on the one-launch FMA kernel).
static int persist_blocks(const Job& single, bool batched) {
    if (batched || single.herm == 0 || single.t.h_complex != 0 || single.t.N < 10 ||
        single.t.N > 64)
        return 0;
    return (single.t.N + 15) / 16;
}

template <int NB, int NBASE>
static hipError_t launch_mfma_pk_t(const Job& single, int total_tiles, const StageSpec& sp,
                                   hipStream_t stream) {
    const void* fn = reinterpret_cast<const void*>(&k_bulk_mfma_pk<NB, NBASE>);
    static std::once_flag attr_once;
    static hipError_t attr_err = hipSuccess;
    if (allow_full_lds(attr_once, attr_err, fn) != hipSuccess) return attr_err;
    constexpr int AW = mfma_ados_per_wg<float, NB>();
    const unsigned stride =
        (unsigned)((MfmaLds<float, NB, true>::bytes(single.t.N, single.t.W, single.t.D) + 15) & ~(size_t)15);
    size_t lds = (size_t)stride * AW;
    int extra = 0;
    hipError_t e = sigma0_ride_along<float, false, true>(single, nullptr, 1, 1, true, sp, lds, stream,
                                                         &extra, &lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_bulk_mfma_pk<NB, NBASE>), dim3(extra + (total_tiles + AW - 1) / AW),
                       dim3(128 * NB * AW), lds, stream, single, sp, total_tiles, stride, extra,
                       (unsigned)lds);
    return hipGetLastError();
}

template <int NB>
static hipError_t launch_mfma_pk_nb(const Job& single, int total_tiles, const StageSpec& sp,
                                    hipStream_t stream) {
    if (sp.nbase <= 1) return launch_mfma_pk_t<NB, 1>(single, total_tiles, sp, stream);
    return launch_mfma_pk_t<NB, 3>(single, total_tiles, sp, stream);
}

template <typename T, bool BATCHED, bool HC>
static hipError_t launch_fma_t(const Job& single, const Job* jobs_dev, int n_jobs,
                               int total_tiles, const StageSpec& sp, size_t lds,
                               hipStream_t stream, int n_s0) {
    static std::once_flag attr_once;
    static hipError_t attr_err = hipSuccess;
    if (allow_full_lds(attr_once, attr_err, reinterpret_cast<const void*>(&k_bulk_fma<T, BATCHED, HC>)) != hipSuccess) return attr_err;
    // FP32 only: the FP64 sigma_0 code would cost the FP64 kernel its
    // occupancy.  Eight FP32 workgroups per CU leave 20 KiB of LDS each.
    int extra = 0;
    size_t lds_launch = lds;
    hipError_t e = sigma0_ride_along<T, BATCHED>(single, jobs_dev, n_jobs, n_s0, sizeof(T) == 4, sp,
                                                 160 * 1024 / 8, stream, &extra, &lds_launch);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_bulk_fma<T, BATCHED, HC>), dim3(total_tiles + extra), dim3(fma_block(sizeof(T), single.t.N)),
                       lds_launch, stream, single, jobs_dev, n_jobs, sp, extra, (unsigned)lds_launch);
    return hipGetLastError();
}

// Tile size of one launch of the persistent FMA kernel (and its LDS), or 0
// when it does not fit: one slot of each link table per thread, the tile's
// neighbour rows within rq per thread, and the LDS within the share of a CU
// that the kernel's occupancy leaves to each workgroup.  plus: the launch
// over the ADOs below the top level.
static int small_tile(const Job& single, int tsize, bool plus, int rq, int el, size_t budget,
                      size_t* lds) {
    const int N = single.t.N, NN = N * N, W = plus ? single.t.W : 0, D = single.t.D;
    const int Dm = std::max(D, 1);
    const bool herm = single.herm != 0;
    auto fits = [&](int GA) {
        return GA * NN <= 256 * el && GA * Dm <= 256 && GA * W <= 256 &&
               GA * (Dm + W) * N * (herm ? 1 : 2) <= 256 * rq &&
               small_lds(N, W, D, GA, tsize, herm, el).total <= budget;
    };
    int GA = std::max(1, 256 * el / NN);
    const int cap = g_max_ados_per_tile.load();
    if (cap > 0) GA = std::min(GA, cap);
    while (GA > 1 && !fits(GA)) --GA;
    if (!fits(GA)) return 0;
    *lds = small_lds(N, W, D, GA, tsize, herm, el).total;
    return GA;
}

// row slots per thread: the launch below the top level takes 8 when its
// full tile needs more than 2 (W + D rows of N per ADO), else 2, whose
// registers leave the row decode to the compiler
constexpr int kSmallRqPlusWide = 8, kSmallRqPlusNarrow = 2, kSmallRqTop = 2;
// elements per thread: the top-level launch takes two (twice the ADOs per
// tile for the same per-tile overhead)
constexpr int kSmallElPlus = 1, kSmallElTop = 2;

// LDS per workgroup when `per_cu` workgroups share a CU's 160 KiB.
static size_t small_lds_budget(int per_cu) { return (size_t)(160 * 1024 / per_cu) & ~(size_t)1023; }

// The persistent FMA kernel takes single jobs with N <= 16 and at least
// kSmallMinAdos ADOs whose tiles fit both of its launches.  Smaller
// hierarchies take the one-launch FMA kernel: with a few thousand ADOs the
// launches, not the memory traffic, set the time (FMO-like, 3060 ADOs of
// 7 x 7: 9.5 against 20 us per stage).
constexpr int kSmallMinAdos = 32768;

static bool small_plus_wide(const Job& single) {
    const int N = single.t.N, NN = N * N, Dm = std::max(single.t.D, 1);
    int GA = std::max(1, 256 / NN);
    const int cap = g_max_ados_per_tile.load();
    if (cap > 0) GA = std::min(GA, cap);
    return GA * (Dm + single.t.W) * N * (single.herm ? 1 : 2) > 256 * kSmallRqPlusNarrow;
}

static bool small_eligible(const Job& single, int tsize) {
    if (single.t.N > 16 || single.t.D < 1 || single.t.n_ado < kSmallMinAdos) return false;
    size_t l;
    const size_t bp = small_lds_budget(tsize == 4 ? small_waves<float, true>() : small_waves<double, true>());
    const size_t bt = small_lds_budget(tsize == 4 ? small_waves<float, false>() : small_waves<double, false>());
    const int rq = small_plus_wide(single) ? kSmallRqPlusWide : kSmallRqPlusNarrow;
    return small_tile(single, tsize, false, kSmallRqTop, kSmallElTop, bt, &l) > 0 &&
           (single.n_low == 0 || small_tile(single, tsize, true, rq, kSmallElPlus, bp, &l) > 0);
}

template <typename T, bool HERM, int NBASE, bool PLUS, int RQ, int EL>
static hipError_t launch_small_part(const Job& single, const StageSpec& sp, int u_begin, int u_end,
                                    bool carry_s0, hipStream_t stream) {
    const void* fn = reinterpret_cast<const void*>(&k_stage_small<T, true, HERM, NBASE, PLUS, RQ, EL>);
    static std::once_flag attr_once;
    static hipError_t attr_err = hipSuccess;
    if (allow_full_lds(attr_once, attr_err, fn) != hipSuccess) return attr_err;
    const int tsize = (int)sizeof(T);
    constexpr int per_cu = small_waves<T, PLUS>();
    size_t lds = 0;
    const int GA = small_tile(single, tsize, PLUS, RQ, EL, small_lds_budget(per_cu), &lds);
    if (GA < 1) return hipErrorInvalidValue;
    const int n_tiles = (u_end - u_begin + GA - 1) / GA;
    // sigma_0 rides along with one of the launches, in FP32 only (as in the FMA kernel)
    int extra = 0;
    size_t lds_launch = lds;
    if (carry_s0) {
        hipError_t e = sigma0_ride_along<T, false>(single, nullptr, 1, 1, sizeof(T) == 4, sp,
                                                   160 * 1024 / per_cu, stream, &extra, &lds_launch);
        if (e != hipSuccess) return e;
    }
    int workers = std::min(n_tiles, resident_workgroups(fn, 256, lds_launch, per_cu));
    if (g_max_workgroups.load() > 0) workers = std::min(workers, g_max_workgroups.load());
    hipLaunchKernelGGL((k_stage_small<T, true, HERM, NBASE, PLUS, RQ, EL>), dim3(extra + workers),
                       dim3(256), lds_launch, stream, single, sp, u_begin, u_end, GA, extra,
                       (unsigned)lds_launch);
    return hipGetLastError();
}

template <typename T, bool HERM, int NBASE>
static hipError_t launch_small_n(const Job& single, const StageSpec& sp, hipStream_t stream) {
    const int top_first = 1 + single.n_low;
    hipError_t e = hipSuccess;
    if (single.n_low > 0)
        e = small_plus_wide(single)
                ? launch_small_part<T, HERM, NBASE, true, kSmallRqPlusWide, kSmallElPlus>(
                      single, sp, 1, top_first, false, stream)
                : launch_small_part<T, HERM, NBASE, true, kSmallRqPlusNarrow, kSmallElPlus>(
                      single, sp, 1, top_first, false, stream);
    if (e == hipSuccess)
        e = launch_small_part<T, HERM, NBASE, false, kSmallRqTop, kSmallElTop>(
            single, sp, top_first, single.t.n_ado, true, stream);
    return e;
}

template <typename T, bool HERM>
static hipError_t launch_small_h(const Job& single, const StageSpec& sp, hipStream_t stream) {
    switch (sp.nbase) {
        case 0: return launch_small_n<T, HERM, 0>(single, sp, stream);
        case 1: return launch_small_n<T, HERM, 1>(single, sp, stream);
        case 2: return launch_small_n<T, HERM, 2>(single, sp, stream);
        case 3: return launch_small_n<T, HERM, 3>(single, sp, stream);
        default: return hipErrorInvalidValue;
    }
}

thread_local const char* g_launch_what = "";

template <typename T>
static hipError_t launch_stage_t(const Job& single, const Job* jobs_dev, int n_jobs,
                                 int total_tiles, const StageSpec& sp, hipStream_t stream,
                                 hipEvent_t ev_begin, hipEvent_t ev_end) {
    const int N = single.t.N;
    const bool batched = jobs_dev != nullptr;
    const int n_s0 = batched ? n_jobs : 1;  // sigma_0 workgroups, one per job
    hipError_t e;
    if (total_tiles == 0) {
        // sigma_0 only; largest N and W of the batch, non-Hermitian staging needs the most LDS
        const size_t lds0 = sigma0_lds(N, single.t.W, (int)sizeof(T), false, 160 * 1024).total;
        e = batched ? launch_sigma0_t<T, true>(single, jobs_dev, n_jobs, sp, lds0, stream)
                    : launch_sigma0_t<T, false>(single, jobs_dev, n_jobs, sp, lds0, stream);
        if (e != hipSuccess) g_launch_what = "sigma_0 stage kernel";
        return e;
    }
    // MFMA path for 16 <= N (real H); FP64 above N = 48 would need more than
    // 160 KiB of LDS and stays on the FMA path.  sigma_0 rides along with the
    // bulk launch where its LDS fits.
    const int pb = sizeof(T) == 4 ? persist_blocks(single, batched) : 0;
    if (pb > 0) {
        // one tile per ADO u >= 1 (the job's tile count may group small ADOs
        // for the FMA kernel)
        const int n_ados = single.t.n_ado - 1;
        if (ev_begin && (e = hipEventRecord(ev_begin, stream)) != hipSuccess) return e;
        switch (pb) {
            case 1: e = launch_persist_nb<1>(single, n_ados, sp, stream); break;
            case 2: e = launch_persist_nb<2>(single, n_ados, sp, stream); break;
            case 3: e = launch_persist_nb<3>(single, n_ados, sp, stream); break;
            default: e = launch_persist_nb<4>(single, n_ados, sp, stream); break;
        }
        if (e != hipSuccess) {
            g_launch_what = "persistent MFMA stage kernel";
            return e;
        }
        if (ev_end) e = hipEventRecord(ev_end, stream);
        return e;
    }
    const int nb = bulk_mfma_blocks(N, single.t.h_complex != 0, sizeof(T) == 8 ? 0 : 1);
    if (nb > 0) {
        if (ev_begin && (e = hipEventRecord(ev_begin, stream)) != hipSuccess) return e;
        e = launch_mfma<T>(nb, single.herm != 0, single, jobs_dev, n_jobs, total_tiles, sp, stream, n_s0);
        if (e != hipSuccess) g_launch_what = "MFMA bulk stage kernel";
    } else if (!batched && small_eligible(single, (int)sizeof(T))) {
        if (ev_begin && (e = hipEventRecord(ev_begin, stream)) != hipSuccess) return e;
        e = single.herm ? launch_small_h<T, true>(single, sp, stream)
                        : launch_small_h<T, false>(single, sp, stream);
        if (e != hipSuccess) g_launch_what = "persistent FMA stage kernel";
    } else {
        if (ev_begin && (e = hipEventRecord(ev_begin, stream)) != hipSuccess) return e;
        // batched launches carry the largest tile LDS of the batch
        const size_t lds = single.lds_bytes
                               ? (size_t)single.lds_bytes
                               : fma_lds(N, single.t.W, single.t.D, single.ados_per_tile,
                                         (int)sizeof(T)).total;
        if (single.any_complex_h)
            e = batched ? launch_fma_t<T, true, true>(single, jobs_dev, n_jobs, total_tiles, sp, lds, stream, n_s0)
                        : launch_fma_t<T, false, true>(single, jobs_dev, n_jobs, total_tiles, sp, lds, stream, n_s0);
        else
            e = batched ? launch_fma_t<T, true, false>(single, jobs_dev, n_jobs, total_tiles, sp, lds, stream, n_s0)
                        : launch_fma_t<T, false, false>(single, jobs_dev, n_jobs, total_tiles, sp, lds, stream, n_s0);
        if (e != hipSuccess) g_launch_what = "FMA bulk stage kernel";
    }
    if (e != hipSuccess) return e;
    if (ev_end) e = hipEventRecord(ev_end, stream);
    return e;
}

// Hermitian-packed FP32 storage: single jobs on the matrix-core path only.
static hipError_t launch_stage_pk(const Job& single, int total_tiles, const StageSpec& sp,
                                  hipStream_t stream, hipEvent_t ev_begin, hipEvent_t ev_end) {
    const int N = single.t.N;
    hipError_t e;
    if (total_tiles == 0) {
        const size_t lds0 = sigma0_lds(N, single.t.W, 4, false, 160 * 1024).total;
        e = launch_sigma0_t<float, false, true>(single, nullptr, 1, sp, lds0, stream);
        if (e != hipSuccess) g_launch_what = "sigma_0 stage kernel";
        return e;
    }
    const int nb = bulk_mfma_blocks(N, single.t.h_complex != 0, 2);
    if (nb < 1 || nb > 4) return hipErrorInvalidValue;
    if (ev_begin && (e = hipEventRecord(ev_begin, stream)) != hipSuccess) return e;
    switch (nb) {
        case 1: e = launch_mfma_pk_nb<1>(single, total_tiles, sp, stream); break;
        case 2: e = launch_mfma_pk_nb<2>(single, total_tiles, sp, stream); break;
        case 3: e = launch_mfma_pk_nb<3>(single, total_tiles, sp, stream); break;
        default: e = launch_mfma_pk_nb<4>(single, total_tiles, sp, stream); break;
    }
    if (e != hipSuccess) {
        g_launch_what = "packed MFMA bulk stage kernel";
        return e;
    }
    if (ev_end) e = hipEventRecord(ev_end, stream);
    return e;
}

const char* last_launch_failure() { return g_launch_what; }

hipError_t launch_stage(const Job& single, const Job* jobs_dev, int n_jobs, int total_tiles,
                        int precision, const StageSpec& sp, hipStream_t stream,
                        hipEvent_t ev_begin, hipEvent_t ev_end) {
    g_launch_what = "";
    if (precision == 2) {
        if (jobs_dev != nullptr) return hipErrorInvalidValue;
        return launch_stage_pk(single, total_tiles, sp, stream, ev_begin, ev_end);
    }
    if (precision == 0)
        return launch_stage_t<double>(single, jobs_dev, n_jobs, total_tiles, sp, stream,
                                      ev_begin, ev_end);
    return launch_stage_t<float>(single, jobs_dev, n_jobs, total_tiles, sp, stream, ev_begin,
                                 ev_end);
}

}  // namespace heom
