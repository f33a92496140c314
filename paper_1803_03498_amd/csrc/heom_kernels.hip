// gfx950 kernels of the HEOM library: hierarchy enumeration, +/- link tables,
// the RK4 stage kernels for sigma_0 (FP64) and for the bulk of the ADOs
// (wavefront FMA path).
//
// Equations: section "HEOM formalism" of Kramer et al., arXiv:1803.03498
// (eq. Nmatrices for the hierarchy, eq. HEOM for the right-hand side, the
// superoperator masks that follow it, and the ADO rescaling substitution).
#include <hip/hip_runtime.h>

#include <algorithm>

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
    G(t.plus)[idx] = (G(t.level)[u] < t.D) ? (int32_t)rank_with(n, W, G(t.binom), l, +1) : -1;
    G(t.minus)[idx] = (n[l] > 0) ? (int32_t)rank_with(n, W, G(t.binom), l, -1) : -1;
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

template <typename T>
__device__ __forceinline__ cpx<T> rhs_element(const Tables& t, const T* sH, const T* sS, int u,
                                              int i, int j, bool herm, const NbSrc<T>& nbs) {
    const int N = t.N, W = t.W, D = t.D;
    // -i [H, sigma]
    T cr = 0, ci = 0;
    for (int k = 0; k < N; ++k) {
        const T hr = sH[2 * (i * N + k)], hi = sH[2 * (i * N + k) + 1];
        const T sr = sS[2 * (k * N + j)], si = sS[2 * (k * N + j) + 1];
        const T tr = sS[2 * (i * N + k)], ti = sS[2 * (i * N + k) + 1];
        const T gr = sH[2 * (k * N + j)], gi = sH[2 * (k * N + j) + 1];
        cr += hr * sr - hi * si - (tr * gr - ti * gi);
        ci += hr * si + hi * sr - (tr * gi + ti * gr);
    }
    const T s_r = sS[2 * (i * N + j)], s_i = sS[2 * (i * N + j) + 1];
    T ar = ci, ai = -cr;  // -i * comm
    // second line: damping
    const T gam = (T)G(t.damping)[u];
    ar -= gam * s_r;
    ai -= gam * s_i;
    // third line: correction term, (1 - d_ij)(Delta_i + Delta_j)
    if (i != j) {
        const T dl = (T)(G(t.delta_state)[i] + G(t.delta_state)[j]);
        ar -= dl * s_r;
        ai -= dl * s_i;
    }
    const int lev = (u == 0) ? 0 : G(t.level)[u];
    gcptr<uint8_t> nu_ = G(t.tuples) + (size_t)u * W;
    const int npass = (i == j) ? 1 : 2;
    for (int pass = 0; pass < npass; ++pass) {
        const int s = pass == 0 ? i : j;
        const T vx = (T)((i == s) - (j == s));
        const T vo = (T)((i == s) + (j == s));
        const bool col = (j == s) && (i != s);
        for (int m = G(t.state_mode_begin)[s]; m < G(t.state_mode_begin)[s + 1]; ++m) {
            const int l = G(t.state_modes)[m];
            const int nl = nu_[l];
            if (lev < D && i != j) {
                const int nb = G(t.plus)[(size_t)u * W + l];
                const cpx<T> x = (herm && col) ? cconj(load_nb<T>(nbs, nb, j, i))
                                               : load_nb<T>(nbs, nb, i, j);
                const T a = (T)G(t.plus_coef)[l * (D + 1) + nl] * vx;
                ar -= a * x.im;  // i * a * x
                ai += a * x.re;
            }
            if (nl > 0) {
                const int nb = G(t.minus)[(size_t)u * W + l];
                const cpx<T> x = (herm && col) ? cconj(load_nb<T>(nbs, nb, j, i))
                                               : load_nb<T>(nbs, nb, i, j);
                const T b = (T)G(t.minus_coef)[l * (D + 1) + nl];
                const T thr = b * (T)G(t.mode_lamnu)[l] * vo;  // real part of b*theta
                const T thi = b * (T)G(t.mode_c)[l] * vx;      // imaginary part
                ar += thr * x.re - thi * x.im;
                ai += thr * x.im + thi * x.re;
            }
        }
    }
    return {ar, ai};
}

__device__ __forceinline__ int xcd_remap(int b, int nb) {
    // Workgroups are handed to the 8 XCDs round-robin; give each XCD a
    // contiguous range of tiles so neighbouring ADOs share one L2.
    const int per = nb / 8, rem = nb % 8;
    const int x = b % 8, idx = b / 8;
    return x * per + (x < rem ? x : rem) + idx;
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

template <typename T, int NB, bool BATCHED>
__global__ __launch_bounds__(256) void k_sigma0(Job single, const Job* jobs, int n_jobs,
                                                StageSpec sp, unsigned lds_cap) {
    constexpr int EPT = (16 * NB * 16 * NB + kBlock - 1) / kBlock;
    const Job& J = BATCHED ? jobs[blockIdx.x] : single;
    const Tables& t = J.t;
    const int N = t.N, NN = N * N, W = t.W, D = t.D;
    const bool herm = J.herm != 0;
    const Sigma0Lds L = sigma0_lds(N, W, (int)sizeof(T), herm, lds_cap);
    extern __shared__ char smem_s0[];
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
    const bool hc = t.h_complex != 0;
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
            const cpx<T> r = load_nb<T>(nbs, 1 + l, site, c);
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

    double nr[EPT], ni[EPT];
    const double h = sp.hmul * J.dt;
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
        const int e = tid + q * kBlock;
        nr[q] = ni[q] = 0.0;
        if (e >= NN) continue;
        const int i = e / N, j = e - (e / N) * N;
        // -i [H, sigma_0] (the damping vanishes at u = 0)
        double cr = 0, ci = 0;
        if (hc) {
            for (int k = 0; k < N; ++k) {
                const double hr = sH[2 * (i * N + k)], hi = sH[2 * (i * N + k) + 1];
                const double xr = sS[2 * (k * N + j)], xi = sS[2 * (k * N + j) + 1];
                const double yr = sS[2 * (i * N + k)], yi = sS[2 * (i * N + k) + 1];
                const double gr = sH[2 * (k * N + j)], gi = sH[2 * (k * N + j) + 1];
                cr += hr * xr - hi * xi - (yr * gr - yi * gi);
                ci += hr * xi + hi * xr - (yr * gi + yi * gr);
            }
        } else {
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
                        x = (herm && pass == 1) ? cconj(load_nb<T>(nbs, 1 + l, s, i))
                                                : load_nb<T>(nbs, 1 + l, i, j);
                    }
                    const double pa = pass == 0 ? sPa[l] : -sPa[l];
                    fr -= pa * (double)x.im;
                    fi += pa * (double)x.re;
                }
            }
        }
        // RK4 stage combination in FP64
        double yr = sp.w_in * sS[2 * e], yi = sp.w_in * sS[2 * e + 1];
        for (int m = 0; m < sp.nbase; ++m) {
            const cpx<double> bv = ld<double>(J.sig0[sp.base[m]], e);
            yr += sp.wbase[m] * bv.re;
            yi += sp.wbase[m] * bv.im;
        }
        nr[q] = yr + h * fr;
        ni[q] = yi + h * fi;
    }
    __syncthreads();  // every thread has read the old sigma_0 from LDS
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
        const int e = tid + q * kBlock;
        if (e >= NN) continue;
        st<double>(J.sig0[sp.out], e, cpx<double>{nr[q], ni[q]});
        sS[2 * e] = nr[q];
        sS[2 * e + 1] = ni[q];
    }
    if (sp.record_after) {
        __syncthreads();
        if (tid == 0) {
            const int64_t step = *G(J.step) + 1;
            *G(J.step) = step;
            if (step % J.rec_every == 0) record_sigma0(J, sS, step / J.rec_every);
        }
    }
}

// --------------------------------------------------------------------------
// Bulk stage kernel, wavefront-FMA path: a workgroup takes G consecutive ADOs
// (G = max(1, 256 / N^2)); every thread owns whole matrix elements.
// --------------------------------------------------------------------------
template <typename T, bool BATCHED>
__global__ __launch_bounds__(256) void k_bulk_fma(Job single, const Job* jobs, int n_jobs,
                                                  StageSpec sp) {
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const Job& J = JobOf<BATCHED>::get(single, jobs, n_jobs, b);
    const Tables& t = J.t;
    const int N = t.N, NN = N * N, GA = J.ados_per_tile;
    const int u0 = 1 + (b - J.tile_begin) * GA;
    const int n_here = min(GA, t.n_ado - u0);
    extern __shared__ char smem_raw[];
    T* sH = reinterpret_cast<T*>(smem_raw);  // 2*NN
    T* sS = sH + 2 * NN;                      // 2*GA*NN
    const int tid = threadIdx.x;
    for (int e = tid; e < NN; e += blockDim.x) {
        sH[2 * e] = (T)G(t.h_re)[e];
        sH[2 * e + 1] = t.h_complex ? (T)G(t.h_im)[e] : (T)0;
    }
    const size_t base = (size_t)(u0 - 1) * NN;
    const int tot = n_here * NN;
    const void* in = J.rest[sp.in];
    for (int e = tid; e < tot; e += blockDim.x) {
        const cpx<T> v = ld<T>(in, base + e);
        sS[2 * e] = v.re;
        sS[2 * e + 1] = v.im;
    }
    __syncthreads();
    const NbSrc<T> nbs{J.sig0[sp.in], J.rest[sp.in], N};
    const T h = (T)(sp.hmul * J.dt);
    const T w_in = (T)sp.w_in;
    for (int e = tid; e < tot; e += blockDim.x) {
        const int g = e / NN;
        const int ij = e - g * NN;
        const int i = ij / N, j = ij - (ij / N) * N;
        const cpx<T> f = rhs_element<T>(t, sH, sS + 2 * g * NN, u0 + g, i, j, J.herm != 0, nbs);
        T yr = w_in * sS[2 * e], yi = w_in * sS[2 * e + 1];
        for (int m = 0; m < sp.nbase; ++m) {
            const cpx<T> bv = ld<T>(J.rest[sp.base[m]], base + e);
            yr += (T)sp.wbase[m] * bv.re;
            yi += (T)sp.wbase[m] * bv.im;
        }
        yr += h * f.re;
        yi += h * f.im;
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

// Per-block LDS copies of the small per-problem tables, and the per-ADO link
// description: every mode's "+" neighbour and coefficient, and a compact list
// of the active "-" links (modes with n_l > 0, at most D of them) in mode
// order, built with a wave ballot so that the order is deterministic.
template <typename T>
struct BlockTables {
    int32_t* site;   // [W] mode -> coupled state
    T* delta;        // [N] correction coefficient per state
    int32_t* pnb;    // [W] "+" neighbour (valid when level < D)
    T* pa;           // [W] sign * sqrt((n_l+1)|c_l|)
    int32_t* msite;  // [W] active "-" links: state, neighbour, coefficients
    int32_t* mnb;
    T* mml;          // sqrt(n_l/|c_l|) * sign * lambda nu (k = 0)
    T* mmc;          // sqrt(n_l/|c_l|) * sign * c_l
    int32_t* count;  // [4] per-wave active counts, [4] = total
};

template <typename T>
__device__ __forceinline__ size_t block_tables_bytes(int N, int W) {
    return (size_t)W * (4 * sizeof(int32_t) + 3 * sizeof(T)) + (size_t)N * sizeof(T) + 8 * 4;
}

template <typename T>
__device__ __forceinline__ BlockTables<T> carve_tables(char* p, int N, int W) {
    BlockTables<T> b;
    b.pa = reinterpret_cast<T*>(p);
    b.mml = b.pa + W;
    b.mmc = b.mml + W;
    b.delta = b.mmc + W;
    b.site = reinterpret_cast<int32_t*>(b.delta + N);
    b.pnb = b.site + W;
    b.msite = b.pnb + W;
    b.mnb = b.msite + W;
    b.count = b.mnb + W;
    return b;
}

// Fill the block tables for ADO u (all threads of the block take part;
// W <= 255 so one pass of 256 threads covers every mode).  Ends with a barrier.
template <typename T>
__device__ void fill_block_tables(const Tables& t, int u, int lev, const BlockTables<T>& b) {
    const int W = t.W, D = t.D, N = t.N;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int s = tid; s < N; s += blockDim.x) b.delta[s] = (T)G(t.delta_state)[s];
    const int l = tid;
    int nl = 0;
    if (l < W) {
        nl = G(t.tuples)[(size_t)u * W + l];
        b.site[l] = G(t.mode_site)[l];
        b.pnb[l] = (lev < D) ? G(t.plus)[(size_t)u * W + l] : -1;
        b.pa[l] = (T)G(t.plus_coef)[l * (D + 1) + nl];
    }
    const bool act = (l < W) && nl > 0;
    const unsigned long long mask = __ballot(act);
    if (lane == 0) b.count[wave] = __popcll(mask);
    __syncthreads();
    if (act) {
        int slot = __popcll(mask & ((1ull << lane) - 1));
        for (int w = 0; w < wave; ++w) slot += b.count[w];
        const double coef = G(t.minus_coef)[l * (D + 1) + nl];
        b.msite[slot] = G(t.mode_site)[l];
        b.mnb[slot] = G(t.minus)[(size_t)u * W + l];
        b.mml[slot] = (T)(coef * G(t.mode_lamnu)[l]);
        b.mmc[slot] = (T)(coef * G(t.mode_c)[l]);
    }
    if (tid == 0) b.count[4] = b.count[0] + b.count[1] + b.count[2] + b.count[3];
    __syncthreads();
}

// At most this many "-" neighbour rows are prefetched into LDS per ADO
// (one element per thread for N <= 64); further links read global memory.
constexpr int kPrefRows = 4;

template <typename T, int NB, bool HERM, bool BATCHED>
__global__ __launch_bounds__(256) void k_bulk_mfma(Job single, const Job* jobs, int n_jobs,
                                                   StageSpec sp) {
    constexpr int NP = 16 * NB;                           // padded matrix dimension
    constexpr int LS = NP + 1;                            // LDS row stride (odd: no conflicts
                                                          // on the transposed reads of X)
    constexpr int KS = 4 * NB;                            // k-steps of 4 (K = NP)
    constexpr int NTC = 2 * NB;                           // column tiles of [Re | Im]
    constexpr int PLANE = NP * LS;
    constexpr int EPT = (NP * NP + kBlock - 1) / kBlock;  // elements per thread (upper bound)
    using acc_t = typename mfma_acc<T>::type;

    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const Job& J = JobOf<BATCHED>::get(single, jobs, n_jobs, b);
    const Tables& t = J.t;
    const int N = t.N, NN = N * N, W = t.W, D = t.D;
    const int u = 1 + (b - J.tile_begin);
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;

    extern __shared__ char smem_raw[];
    T* sSre = reinterpret_cast<T*>(smem_raw);
    T* sSim = sSre + PLANE;
    T* sXre = sSim + PLANE;
    T* sXim = sXre + PLANE;
    T* sYre = sXim + PLANE;  // general path only
    T* sYim = sYre + PLANE;
    T* sRow = HERM ? sYre : sYim + PLANE;  // kPrefRows x NP complex (Hermitian path)
    const BlockTables<T> bt = carve_tables<T>(
        reinterpret_cast<char*>(HERM ? sRow + 2 * kPrefRows * NP : sRow), N, W);

    // Own tile: global -> LDS planes (loads first, then the LDS writes).
    const size_t base = (size_t)(u - 1) * NN;
    {
        const void* in = J.rest[sp.in];
        cpx<T> v[EPT];
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            const int e = tid + q * kBlock;
            v[q] = (e < NN) ? ld<T>(in, base + e) : cpx<T>{(T)0, (T)0};
        }
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            const int e = tid + q * kBlock;
            if (e < NN) {
                const int i = e / N, j = e - (e / N) * N;
                sSre[i * LS + j] = v[q].re;
                sSim[i * LS + j] = v[q].im;
            }
        }
    }
    if (N < NP) {
        for (int idx = tid; idx < NP * NP; idx += kBlock) {
            const int r = idx / NP, c = idx - (idx / NP) * NP;
            if (r >= N || c >= N) {
                sSre[r * LS + c] = (T)0;
                sSim[r * LS + c] = (T)0;
            }
        }
    }
    const int lev = G(t.level)[u];
    const T gam = (T)G(t.damping)[u];
    fill_block_tables<T>(t, u, lev, bt);  // ends with a barrier (also publishes the planes)

    // Prefetch the row s of every active "-" neighbour (Hermitian path): its
    // latency hides behind the matrix-core phase.
    const NbSrc<T> nbs{J.sig0[sp.in], J.rest[sp.in], N};
    const int n_minus = bt.count[4];
    const int n_pref = HERM ? min(n_minus, kPrefRows) : 0;
    cpx<T> pre = {(T)0, (T)0};
    const bool has_pre = tid < n_pref * N;
    if (has_pre) {
        const int a = tid / N, c = tid - (tid / N) * N;
        pre = load_nb<T>(nbs, bt.mnb[a], bt.msite[a], c);
    }

    // X = H [Re S | Im S]; H is the A operand, hreg[mt][ks] = H[16 mt + lane%16][4 ks + lane/16]
    {
        T hreg[NB][KS];
#pragma unroll
        for (int mt = 0; mt < NB; ++mt)
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int r = 16 * mt + (lane & 15), c = 4 * ks + (lane >> 4);
                hreg[mt][ks] = (r < N && c < N) ? (T)G(t.h_re)[r * N + c] : (T)0;
            }
        const int ksteps = (N + 3) >> 2;
#pragma unroll
        for (int mt = 0; mt < NB; ++mt) {
            for (int nt = ((wave - mt * NTC) % 4 + 4) % 4; nt < NTC; nt += 4) {
                const T* plane = nt < NB ? sSre : sSim;
                const int c0 = 16 * (nt < NB ? nt : nt - NB);
                acc_t acc = {0, 0, 0, 0};
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) {
                    if (ks < ksteps) {
                        const T bv = plane[(4 * ks + (lane >> 4)) * LS + c0 + (lane & 15)];
                        acc = mfma16(hreg[mt][ks], bv, acc);
                    }
                }
                T* out = nt < NB ? sXre : sXim;
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    out[(16 * mt + mfma_row<T>(lane, r)) * LS + c0 + (lane & 15)] = acc[r];
            }
        }
        if (!HERM) {
            // Y = S H (H real symmetric: the B operand H[k][j] has the A layout)
#pragma unroll
            for (int mt = 0; mt < 2 * NB; ++mt) {
                const T* plane = mt < NB ? sSre : sSim;
                const int r0 = 16 * (mt < NB ? mt : mt - NB);
#pragma unroll
                for (int nt = 0; nt < NB; ++nt) {
                    if (((mt * NB + nt) & 3) != wave) continue;
                    acc_t acc = {0, 0, 0, 0};
#pragma unroll
                    for (int ks = 0; ks < KS; ++ks) {
                        if (ks < ksteps) {
                            const T av = plane[(r0 + (lane & 15)) * LS + 4 * ks + (lane >> 4)];
                            acc = mfma16(av, hreg[nt][ks], acc);
                        }
                    }
                    T* out = mt < NB ? sYre : sYim;
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        out[(r0 + mfma_row<T>(lane, r)) * LS + 16 * nt + (lane & 15)] = acc[r];
                }
            }
        }
    }
    if (has_pre) {
        sRow[2 * tid] = pre.re;
        sRow[2 * tid + 1] = pre.im;
    }
    __syncthreads();

    // Elementwise lines: -i[H, sigma], damping, correction, couplings.  Each
    // thread reads only its own elements of the sigma planes here, so the
    // stage value w_in * sigma + h * f goes back into the same slots.
    const float invN = 1.0f / (float)N;  // exact row index for e < 4096 (N <= 64)
    const T h = (T)(sp.hmul * J.dt), w_in = (T)sp.w_in;
#pragma unroll 1
    for (int e = tid; e < NN; e += kBlock) {
        const int i = (int)(((float)e + 0.5f) * invN), j = e - i * N;
        T cr, ci;
        if (HERM) {
            cr = sXre[i * LS + j] - sXre[j * LS + i];
            ci = sXim[i * LS + j] + sXim[j * LS + i];
        } else {
            cr = sXre[i * LS + j] - sYre[i * LS + j];
            ci = sXim[i * LS + j] - sYim[i * LS + j];
        }
        const T sr = sSre[i * LS + j], si = sSim[i * LS + j];
        const T g = gam + ((i != j) ? bt.delta[i] + bt.delta[j] : (T)0);
        T fr = ci - g * sr, fi = -cr - g * si;
        for (int a = 0; a < n_minus; ++a) {
            const int s = bt.msite[a];
            if (i != s && j != s) continue;
            const bool col = (j == s) && (i != s);
            cpx<T> x;
            if (a < n_pref) {
                const int c = col ? i : j;  // Hermitian: column s is conj(row s)
                x = {sRow[2 * (a * N + c)], sRow[2 * (a * N + c) + 1]};
                if (col) x = cconj(x);
            } else {
                x = (HERM && col) ? cconj(load_nb<T>(nbs, bt.mnb[a], s, i))
                                  : load_nb<T>(nbs, bt.mnb[a], i, j);
            }
            const T vx = (T)((i == s) - (j == s)), vo = (T)((i == s) + (j == s));
            const T thr = bt.mml[a] * vo, thi = bt.mmc[a] * vx;
            fr += thr * x.re - thi * x.im;
            fi += thr * x.im + thi * x.re;
        }
        if (lev < D && i != j) {
            for (int pass = 0; pass < 2; ++pass) {
                const int s = pass == 0 ? i : j;
                for (int m = G(t.state_mode_begin)[s]; m < G(t.state_mode_begin)[s + 1]; ++m) {
                    const int l = G(t.state_modes)[m];
                    const int nb = bt.pnb[l];
                    const cpx<T> x = (HERM && pass == 1) ? cconj(load_nb<T>(nbs, nb, s, i))
                                                         : load_nb<T>(nbs, nb, i, j);
                    const T pa = pass == 0 ? bt.pa[l] : -bt.pa[l];  // i * pa * vx * x
                    fr -= pa * x.im;
                    fi += pa * x.re;
                }
            }
        }
        sSre[i * LS + j] = w_in * sr + h * fr;
        sSim[i * LS + j] = w_in * si + h * fi;
    }
    // RK4 stage combination: per base array, every load first, then the sums.
    for (int m = 0; m < sp.nbase; ++m) {
        const T w = (T)sp.wbase[m];
        const void* bp = J.rest[sp.base[m]];
        cpx<T> v[EPT];
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            const int e = tid + q * kBlock;
            v[q] = (e < NN) ? ld<T>(bp, base + e) : cpx<T>{(T)0, (T)0};
        }
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            const int e = tid + q * kBlock;
            if (e < NN) {
                const int i = (int)(((float)e + 0.5f) * invN), j = e - i * N;
                sSre[i * LS + j] += w * v[q].re;
                sSim[i * LS + j] += w * v[q].im;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
        const int e = tid + q * kBlock;
        if (e < NN) {
            const int i = (int)(((float)e + 0.5f) * invN), j = e - i * N;
            st<T>(J.rest[sp.out], base + e, cpx<T>{sSre[i * LS + j], sSim[i * LS + j]});
        }
    }
}

template <typename T, int NB, bool HERM>
size_t mfma_lds_bytes(int N, int W) {
    constexpr int NP = 16 * NB;
    constexpr int LS = NP + 1;
    return sizeof(T) * ((size_t)NP * LS * (HERM ? 4 : 6) + (HERM ? 2 * kPrefRows * NP : 0)) +
           (size_t)W * (4 * 4 + 3 * sizeof(T)) + (size_t)N * sizeof(T) + 8 * 4;
}

}  // namespace

int bulk_mfma_blocks(int N, bool h_complex, int precision) {
    if (N < 16 || h_complex || (precision == 0 && N > 48)) return 0;
    return (N + 15) / 16;
}

int bulk_ados_per_tile(int N) {
    const int NN = N * N;
    return NN >= kBlock ? 1 : kBlock / NN;
}

hipError_t launch_enumerate(const Tables& t, hipStream_t stream) {
    if (t.n_ado <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_enumerate, dim3((t.n_ado + 255) / 256), dim3(256), 0, stream, t);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || t.W == 0) return e;
    const int64_t n = (int64_t)t.n_ado * t.W;
    hipLaunchKernelGGL(k_links, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, t);
    return hipGetLastError();
}

template <typename T, int NB, bool HERM, bool BATCHED>
static hipError_t launch_mfma_t(const Job& single, const Job* jobs_dev, int n_jobs,
                                int total_tiles, const StageSpec& sp, hipStream_t stream) {
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t a = hipFuncSetAttribute(
            reinterpret_cast<const void*>(&k_bulk_mfma<T, NB, HERM, BATCHED>),
            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (a != hipSuccess) return a;
        attr_set = true;
    }
    const size_t lds = mfma_lds_bytes<T, NB, HERM>(single.t.N, single.t.W);
    hipLaunchKernelGGL((k_bulk_mfma<T, NB, HERM, BATCHED>), dim3(total_tiles), dim3(kBlock), lds,
                       stream, single, jobs_dev, n_jobs, sp);
    return hipGetLastError();
}

template <typename T, int NB>
static hipError_t launch_mfma_nb(bool herm, bool batched, const Job& single, const Job* jobs_dev,
                                 int n_jobs, int total_tiles, const StageSpec& sp,
                                 hipStream_t stream) {
    if (herm)
        return batched ? launch_mfma_t<T, NB, true, true>(single, jobs_dev, n_jobs, total_tiles, sp,
                                                          stream)
                       : launch_mfma_t<T, NB, true, false>(single, jobs_dev, n_jobs, total_tiles,
                                                           sp, stream);
    return batched ? launch_mfma_t<T, NB, false, true>(single, jobs_dev, n_jobs, total_tiles, sp,
                                                       stream)
                   : launch_mfma_t<T, NB, false, false>(single, jobs_dev, n_jobs, total_tiles, sp,
                                                        stream);
}

template <typename T>
static hipError_t launch_mfma(int nb, bool herm, const Job& single, const Job* jobs_dev,
                              int n_jobs, int total_tiles, const StageSpec& sp,
                              hipStream_t stream) {
    const bool batched = jobs_dev != nullptr;
    switch (nb) {
        case 1: return launch_mfma_nb<T, 1>(herm, batched, single, jobs_dev, n_jobs, total_tiles, sp, stream);
        case 2: return launch_mfma_nb<T, 2>(herm, batched, single, jobs_dev, n_jobs, total_tiles, sp, stream);
        case 3: return launch_mfma_nb<T, 3>(herm, batched, single, jobs_dev, n_jobs, total_tiles, sp, stream);
        case 4: return launch_mfma_nb<T, 4>(herm, batched, single, jobs_dev, n_jobs, total_tiles, sp, stream);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, int NB, bool BATCHED>
static hipError_t launch_sigma0_t(const Job& single, const Job* jobs_dev, int n_jobs,
                                  const StageSpec& sp, size_t lds, hipStream_t stream) {
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t a = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sigma0<T, NB, BATCHED>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (a != hipSuccess) return a;
        attr_set = true;
    }
    hipLaunchKernelGGL((k_sigma0<T, NB, BATCHED>), dim3(BATCHED ? n_jobs : 1), dim3(kBlock), lds,
                       stream, single, jobs_dev, n_jobs, sp, (unsigned)lds);
    return hipGetLastError();
}

template <typename T, bool BATCHED>
static hipError_t launch_fma_t(const Job& single, const Job* jobs_dev, int n_jobs,
                               int total_tiles, const StageSpec& sp, size_t lds,
                               hipStream_t stream) {
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t a = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_bulk_fma<T, BATCHED>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (a != hipSuccess) return a;
        attr_set = true;
    }
    hipLaunchKernelGGL((k_bulk_fma<T, BATCHED>), dim3(total_tiles), dim3(kBlock), lds, stream,
                       single, jobs_dev, n_jobs, sp);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_stage_t(const Job& single, const Job* jobs_dev, int n_jobs,
                                 int total_tiles, const StageSpec& sp, hipStream_t stream,
                                 hipEvent_t ev_begin, hipEvent_t ev_end) {
    const int N = single.t.N;
    const bool batched = jobs_dev != nullptr;
    // sigma_0: largest N and W of the batch; non-Hermitian staging needs the most LDS
    const size_t lds0 = sigma0_lds(N, single.t.W, (int)sizeof(T), false, 160 * 1024).total;
    hipError_t e;
    switch ((N + 15) / 16) {
        case 1:
            e = batched ? launch_sigma0_t<T, 1, true>(single, jobs_dev, n_jobs, sp, lds0, stream)
                        : launch_sigma0_t<T, 1, false>(single, jobs_dev, n_jobs, sp, lds0, stream);
            break;
        case 2:
            e = batched ? launch_sigma0_t<T, 2, true>(single, jobs_dev, n_jobs, sp, lds0, stream)
                        : launch_sigma0_t<T, 2, false>(single, jobs_dev, n_jobs, sp, lds0, stream);
            break;
        case 3:
            e = batched ? launch_sigma0_t<T, 3, true>(single, jobs_dev, n_jobs, sp, lds0, stream)
                        : launch_sigma0_t<T, 3, false>(single, jobs_dev, n_jobs, sp, lds0, stream);
            break;
        default:
            e = batched ? launch_sigma0_t<T, 4, true>(single, jobs_dev, n_jobs, sp, lds0, stream)
                        : launch_sigma0_t<T, 4, false>(single, jobs_dev, n_jobs, sp, lds0, stream);
            break;
    }
    if (e != hipSuccess || total_tiles == 0) return e;
    if (ev_begin && (e = hipEventRecord(ev_begin, stream)) != hipSuccess) return e;
    // MFMA path for 16 <= N (real H); FP64 above N = 48 would need more than
    // 160 KiB of LDS and stays on the FMA path.
    const int nb = bulk_mfma_blocks(N, single.t.h_complex != 0, sizeof(T) == 8 ? 0 : 1);
    if (nb > 0) {
        e = launch_mfma<T>(nb, single.herm != 0, single, jobs_dev, n_jobs, total_tiles, sp, stream);
    } else {
        // LDS for H and the G-ADO tile: 2 n^2 (1 + G(n)) is not monotone in n, so
        // a batch whose largest matrix is N x N takes the maximum over n <= N.
        size_t lds_elems = 0;
        for (int n = 1; n <= N; ++n)
            lds_elems = std::max(lds_elems, 2 * (size_t)n * n * (1 + bulk_ados_per_tile(n)));
        const size_t lds = lds_elems * sizeof(T);
        e = batched ? launch_fma_t<T, true>(single, jobs_dev, n_jobs, total_tiles, sp, lds, stream)
                    : launch_fma_t<T, false>(single, jobs_dev, n_jobs, total_tiles, sp, lds, stream);
    }
    if (e != hipSuccess) return e;
    if (ev_end) e = hipEventRecord(ev_end, stream);
    return e;
}

hipError_t launch_stage(const Job& single, const Job* jobs_dev, int n_jobs, int total_tiles,
                        int precision, const StageSpec& sp, hipStream_t stream,
                        hipEvent_t ev_begin, hipEvent_t ev_end) {
    if (precision == 0)
        return launch_stage_t<double>(single, jobs_dev, n_jobs, total_tiles, sp, stream,
                                      ev_begin, ev_end);
    return launch_stage_t<float>(single, jobs_dev, n_jobs, total_tiles, sp, stream, ev_begin,
                                 ev_end);
}

}  // namespace heom
