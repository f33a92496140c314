// gfx950 kernels of the HEOM library: hierarchy enumeration, +/- link tables,
// the RK4 stage kernels for sigma_0 (FP64) and for the bulk of the ADOs
// (wavefront FMA path).
//
// Equations: section "HEOM formalism" of Kramer et al., arXiv:1803.03498
// (eq. Nmatrices for the hierarchy, eq. HEOM for the right-hand side, the
// superoperator masks that follow it, and the ADO rescaling substitution).
#include <hip/hip_runtime.h>

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

template <typename T>
struct vec2;
template <>
struct vec2<float> {
    using type = float2;
};
template <>
struct vec2<double> {
    using type = double2;
};

template <typename T>
__device__ __forceinline__ cpx<T> ld(const void* base, size_t idx) {
    typename vec2<T>::type v = reinterpret_cast<const typename vec2<T>::type*>(base)[idx];
    return {v.x, v.y};
}

template <typename T>
__device__ __forceinline__ void st(void* base, size_t idx, cpx<T> a) {
    typename vec2<T>::type v;
    v.x = a.re;
    v.y = a.im;
    reinterpret_cast<typename vec2<T>::type*>(base)[idx] = v;
}

// --------------------------------------------------------------------------
// Hierarchy enumeration (eq. Nmatrices): level-major, descending
// lexicographic order inside a level.  binom[m*(W+1)+k] = C(m+k, k).
//   start(L) = #tuples with sum <= L-1 = C(W+L-1, W)
//   rank(n)  = start(|n|) + sum_{i<W-1, R_i>n_i} C(R_i-n_i-1+W-1-i, W-1-i),
//              R_i = |n| - sum_{j<i} n_j  (tuples with a larger n_i come first)
// --------------------------------------------------------------------------
__device__ int64_t rank_with(const uint8_t* n, int W, const int64_t* binom, int l, int delta) {
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
    uint8_t* n = t.tuples + (size_t)u * W;
    // level: smallest L with u < C(W+L, W)
    int L = 0;
    while (L < D && (int64_t)u >= t.binom[(size_t)L * ks + W]) ++L;
    int64_t r = u - ((L == 0) ? 0 : t.binom[(size_t)(L - 1) * ks + W]);
    int R = L;
    for (int i = 0; i < W - 1; ++i) {
        int v = R;
        for (; v > 0; --v) {
            const int64_t cnt = t.binom[(size_t)(R - v) * ks + (W - 2 - i)];
            if (r < cnt) break;
            r -= cnt;
        }
        n[i] = (uint8_t)v;
        R -= v;
    }
    if (W > 0) n[W - 1] = (uint8_t)R;
    t.level[u] = (uint8_t)L;
    double damp = 0.0;
    for (int l = 0; l < W; ++l) damp += n[l] * t.mode_gamma[l];
    t.damping[u] = damp;
}

// One thread per (u, l): the "+" link (valid while |n| < D) and the "-" link
// (valid while n_l > 0) of the section "HEOM formalism".
__global__ __launch_bounds__(256) void k_links(Tables t) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int W = t.W;
    if (idx >= (int64_t)t.n_ado * W) return;
    const int u = (int)(idx / W);
    const int l = (int)(idx - (int64_t)u * W);
    const uint8_t* n = t.tuples + (size_t)u * W;
    t.plus[idx] = (t.level[u] < t.D) ? (int32_t)rank_with(n, W, t.binom, l, +1) : -1;
    t.minus[idx] = (n[l] > 0) ? (int32_t)rank_with(n, W, t.binom, l, -1) : -1;
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
    const T gam = (T)t.damping[u];
    ar -= gam * s_r;
    ai -= gam * s_i;
    // third line: correction term, (1 - d_ij)(Delta_i + Delta_j)
    if (i != j) {
        const T dl = (T)(t.delta_state[i] + t.delta_state[j]);
        ar -= dl * s_r;
        ai -= dl * s_i;
    }
    const int lev = (u == 0) ? 0 : t.level[u];
    const uint8_t* nu_ = t.tuples + (size_t)u * W;
    const int npass = (i == j) ? 1 : 2;
    for (int pass = 0; pass < npass; ++pass) {
        const int s = pass == 0 ? i : j;
        const T vx = (T)((i == s) - (j == s));
        const T vo = (T)((i == s) + (j == s));
        const bool col = (j == s) && (i != s);
        for (int m = t.state_mode_begin[s]; m < t.state_mode_begin[s + 1]; ++m) {
            const int l = t.state_modes[m];
            const int nl = nu_[l];
            if (lev < D && i != j) {
                const int nb = t.plus[(size_t)u * W + l];
                const cpx<T> x = (herm && col) ? cconj(load_nb<T>(nbs, nb, j, i))
                                               : load_nb<T>(nbs, nb, i, j);
                const T a = (T)t.plus_coef[l * (D + 1) + nl] * vx;
                ar -= a * x.im;  // i * a * x
                ai += a * x.re;
            }
            if (nl > 0) {
                const int nb = t.minus[(size_t)u * W + l];
                const cpx<T> x = (herm && col) ? cconj(load_nb<T>(nbs, nb, j, i))
                                               : load_nb<T>(nbs, nb, i, j);
                const T b = (T)t.minus_coef[l * (D + 1) + nl];
                const T thr = b * (T)t.mode_lamnu[l] * vo;  // real part of b*theta
                const T thi = b * (T)t.mode_c[l] * vx;      // imaginary part
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

__device__ __forceinline__ const Job& find_job(const Job& single, const Job* jobs, int n_jobs,
                                               int tile) {
    if (jobs == nullptr) return single;
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

// --------------------------------------------------------------------------
// sigma_0 stage kernel: one workgroup per job, FP64 throughout; reads the
// level-1 ADOs in the bulk precision T.  Also records the observables.
// --------------------------------------------------------------------------
__device__ void record_sigma0(const Job& J, const double* sS, int64_t slot) {
    // sS: interleaved complex128 [N][N] in LDS.  Caller: one thread.
    if (slot < 0 || slot >= J.n_rec_max) return;
    const int N = J.t.N;
    double* rec = J.records + slot * J.rec_doubles;
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
            pr += J.mu[a] * sS[2 * (a * N + J.ground)];
            pi += J.mu[a] * sS[2 * (a * N + J.ground) + 1];
        }
        rec[0] = pr;
        rec[1] = pi;
        rec[2] = trr;
        rec[3] = tri;
        finite = finite && isfinite(pr) && isfinite(pi);
    }
    if (!finite) *J.status = 1;
}

template <typename T>
__global__ __launch_bounds__(256) void k_sigma0(Job single, const Job* jobs, int n_jobs,
                                                StageSpec sp) {
    const Job& J = (jobs == nullptr) ? single : jobs[blockIdx.x];
    const Tables& t = J.t;
    const int N = t.N, NN = N * N;
    extern __shared__ double smem0[];
    double* sH = smem0;           // 2*NN
    double* sS = smem0 + 2 * NN;  // 2*NN
    const int tid = threadIdx.x;
    for (int e = tid; e < NN; e += blockDim.x) {
        sH[2 * e] = t.h_re[e];
        sH[2 * e + 1] = t.h_complex ? t.h_im[e] : 0.0;
        const cpx<double> v = ld<double>(J.sig0[sp.in], e);
        sS[2 * e] = v.re;
        sS[2 * e + 1] = v.im;
    }
    __syncthreads();
    if (sp.record_initial && tid == 0 && *J.step == 0) record_sigma0(J, sS, 0);
    const NbSrc<T> nbs{J.sig0[sp.in], J.rest[sp.in], N};
    const double h = sp.hmul * J.dt;
    // Values of the new sigma_0 are kept in registers until every thread has
    // read the old tile, then written back to LDS for the observables.
    double outr[kMaxStates * kMaxStates / kBlock], outi[kMaxStates * kMaxStates / kBlock];
    int q = 0;
    for (int e = tid; e < NN; e += blockDim.x, ++q) {
        const int i = e / N, j = e - (e / N) * N;
        // rhs_element<double> reads neighbours through NbSrc<double>; the
        // level-1 ADOs are stored in T, so evaluate the coupling lines here.
        cpx<double> f;
        {
            // commutator, correction term (damping is zero for u = 0)
            double cr = 0, ci = 0;
            for (int k = 0; k < N; ++k) {
                const double hr = sH[2 * (i * N + k)], hi = sH[2 * (i * N + k) + 1];
                const double sr = sS[2 * (k * N + j)], si = sS[2 * (k * N + j) + 1];
                const double tr = sS[2 * (i * N + k)], ti = sS[2 * (i * N + k) + 1];
                const double gr = sH[2 * (k * N + j)], gi = sH[2 * (k * N + j) + 1];
                cr += hr * sr - hi * si - (tr * gr - ti * gi);
                ci += hr * si + hi * sr - (tr * gi + ti * gr);
            }
            double ar = ci, ai = -cr;
            const double s_r = sS[2 * (i * N + j)], s_i = sS[2 * (i * N + j) + 1];
            if (i != j) {
                const double dl = t.delta_state[i] + t.delta_state[j];
                ar -= dl * s_r;
                ai -= dl * s_i;
            }
            if (t.D > 0 && i != j) {
                for (int pass = 0; pass < 2; ++pass) {
                    const int s = pass == 0 ? i : j;
                    const double vx = pass == 0 ? 1.0 : -1.0;
                    const bool col = pass == 1;
                    for (int m = t.state_mode_begin[s]; m < t.state_mode_begin[s + 1]; ++m) {
                        const int l = t.state_modes[m];
                        const int nb = 1 + l;  // level-1 ADO e_l
                        cpx<T> x = (J.herm && col) ? cconj(load_nb<T>(nbs, nb, j, i))
                                                   : load_nb<T>(nbs, nb, i, j);
                        const double a = t.plus_coef[l * (t.D + 1)] * vx;
                        ar -= a * (double)x.im;
                        ai += a * (double)x.re;
                    }
                }
            }
            f = {ar, ai};
        }
        double yr = sp.w_in * sS[2 * e], yi = sp.w_in * sS[2 * e + 1];
        for (int m = 0; m < sp.nbase; ++m) {
            const cpx<double> b = ld<double>(J.sig0[sp.base[m]], e);
            yr += sp.wbase[m] * b.re;
            yi += sp.wbase[m] * b.im;
        }
        yr += h * f.re;
        yi += h * f.im;
        outr[q] = yr;
        outi[q] = yi;
    }
    __syncthreads();
    q = 0;
    for (int e = tid; e < NN; e += blockDim.x, ++q) {
        st<double>(J.sig0[sp.out], e, cpx<double>{outr[q], outi[q]});
        sS[2 * e] = outr[q];
        sS[2 * e + 1] = outi[q];
    }
    if (sp.record_after) {
        __syncthreads();
        if (tid == 0) {
            const int64_t step = *J.step + 1;
            *J.step = step;
            if (step % J.rec_every == 0) record_sigma0(J, sS, step / J.rec_every);
        }
    }
}

// --------------------------------------------------------------------------
// Bulk stage kernel, wavefront-FMA path: a workgroup takes G consecutive ADOs
// (G = max(1, 256 / N^2)); every thread owns whole matrix elements.
// --------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_bulk_fma(Job single, const Job* jobs, int n_jobs,
                                                  StageSpec sp) {
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const Job& J = find_job(single, jobs, n_jobs, b);
    const Tables& t = J.t;
    const int N = t.N, NN = N * N, G = J.ados_per_tile;
    const int u0 = 1 + (b - J.tile_begin) * G;
    const int n_here = min(G, t.n_ado - u0);
    extern __shared__ char smem_raw[];
    T* sH = reinterpret_cast<T*>(smem_raw);  // 2*NN
    T* sS = sH + 2 * NN;                      // 2*G*NN
    const int tid = threadIdx.x;
    for (int e = tid; e < NN; e += blockDim.x) {
        sH[2 * e] = (T)t.h_re[e];
        sH[2 * e + 1] = t.h_complex ? (T)t.h_im[e] : (T)0;
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

}  // namespace

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

template <typename T>
static hipError_t launch_stage_t(const Job& single, const Job* jobs_dev, int n_jobs,
                                 int total_tiles, const StageSpec& sp, hipStream_t stream) {
    const int N = single.t.N;
    const int NN = N * N;
    // sigma_0: FP64 LDS for H and sigma_0
    const size_t lds0 = 4 * (size_t)NN * sizeof(double);
    // Allow dynamic LDS above 64 KiB (N up to 64 in FP64).
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t a = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sigma0<T>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (a == hipSuccess)
            a = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_bulk_fma<T>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (a != hipSuccess) return a;
        attr_set = true;
    }
    const int n0 = jobs_dev ? n_jobs : 1;
    hipLaunchKernelGGL(k_sigma0<T>, dim3(n0), dim3(kBlock), lds0, stream, single, jobs_dev, n_jobs,
                       sp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || total_tiles == 0) return e;
    // bulk: LDS for H and the G-ADO tile.  In a batched launch the largest N
    // of the batch sizes the allocation (`single` carries it).
    const int G = bulk_ados_per_tile(N);
    const size_t lds = 2 * (size_t)NN * sizeof(T) * (1 + G);
    hipLaunchKernelGGL(k_bulk_fma<T>, dim3(total_tiles), dim3(kBlock), lds, stream, single,
                       jobs_dev, n_jobs, sp);
    return hipGetLastError();
}

hipError_t launch_stage(const Job& single, const Job* jobs_dev, int n_jobs, int total_tiles,
                        int precision, const StageSpec& sp, hipStream_t stream) {
    if (precision == 0)
        return launch_stage_t<double>(single, jobs_dev, n_jobs, total_tiles, sp, stream);
    return launch_stage_t<float>(single, jobs_dev, n_jobs, total_tiles, sp, stream);
}

}  // namespace heom
