// Host runtime of the HEOM library: validation, bath coefficients, device
// table layout, and the RK4 driver behind the C ABI of include/heom.h.
//
// Coefficients follow the section "HEOM formalism" of Kramer et al.,
// arXiv:1803.03498 (gamma(b,k), c(b,k) of the Matsubara expansion, the
// correction coefficient of the third line of eq. HEOM, and the rescaled
// coupling weights of the ADO rescaling substitution), with hbar = 1.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "heom.h"
#include "heom_internal.h"

namespace {

thread_local std::string g_error;

heom_status fail(heom_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return s;
}

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(HEOM_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_));        \
    } while (0)

// 2*pi*c in rad/fs per cm^-1, and k_B/(h c) in cm^-1/K.
constexpr double kCmToRadFs = 2.0 * M_PI * 2.99792458e-5;
constexpr double kBoltzmannCm = 0.6950348004;
constexpr double kRk4RealLimit = 2.78;  // RK4 stability interval on the negative real axis
// Largest phase per step of the diagonal offset kept by the coherence-block
// form: RK4 advances e^{-i w dt} with relative error ~ (w dt)^5 / 120, 3e-4 at 0.5.
constexpr double kBlockPhaseLimit = 0.5;

constexpr size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
// one complex64 copy of n ADOs of N x N
constexpr size_t mirror_bytes(int64_t n, int N) {
    return align256(std::max<size_t>((size_t)n * N * N * 8, 1));
}

constexpr int kMaxPade = 64;

// Eigenvalues of the symmetric tridiagonal n x n matrix with zero diagonal
// and off-diagonal e[0..n-2], in descending order: bisection on the Sturm
// count (the number of negative pivots of T - x I is the number of
// eigenvalues below x).
std::vector<double> tridiag_eigenvalues_desc(const std::vector<double>& e, int n) {
    double bound = 0.0;
    for (double v : e) bound = std::max(bound, 2.0 * std::fabs(v));
    bound += 1e-300;
    auto below = [&](double x) {
        int cnt = 0;
        double q = -x;
        for (int k = 0; k < n; ++k) {
            if (k > 0) q = -x - e[k - 1] * e[k - 1] / q;
            if (std::fabs(q) < 1e-300) q = -1e-300;  // a zero pivot counts as negative
            if (q < 0.0) ++cnt;
        }
        return cnt;
    };
    std::vector<double> ev(n);
    for (int j = 1; j <= n; ++j) {  // j-th smallest
        double lo = -bound, hi = bound;
        for (int it = 0; it < 200 && hi - lo > 1e-17 * std::max(1.0, std::fabs(lo)); ++it) {
            const double mid = 0.5 * (lo + hi);
            if (below(mid) >= j)
                hi = mid;
            else
                lo = mid;
        }
        ev[n - j] = 0.5 * (lo + hi);
    }
    return ev;
}

// Pade poles xi_i and residues eta_i (i < K) of the Bose function, from the
// two tridiagonal matrices Lambda (2K x 2K, 1/sqrt((2m+1)(2m+3)) beside the
// diagonal) and Lambda' (2K-1 x 2K-1, 1/sqrt((2m+3)(2m+5))) of section "HEOM
// formalism": xi_i = 2 / (i-th largest eigenvalue of Lambda), zeta_j likewise
// from Lambda', eta_i = (K^2 + 3K/2) prod_j (zeta_j^2 - xi_i^2) / prod_{j != i}
// (xi_j^2 - xi_i^2), the factors taken in pairs to stay in range.
void pade_poles(int K, std::vector<double>& xi, std::vector<double>& eta) {
    xi.assign(K, 0.0);
    eta.assign(K, 0.0);
    if (K < 1) return;
    std::vector<double> e(2 * K - 1), ep(std::max(2 * K - 2, 0));
    for (int m = 1; m <= 2 * K - 1; ++m) e[m - 1] = 1.0 / std::sqrt((2.0 * m + 1) * (2.0 * m + 3));
    for (int m = 1; m <= 2 * K - 2; ++m) ep[m - 1] = 1.0 / std::sqrt((2.0 * m + 3) * (2.0 * m + 5));
    const std::vector<double> ev = tridiag_eigenvalues_desc(e, 2 * K);
    const std::vector<double> evp = tridiag_eigenvalues_desc(ep, 2 * K - 1);
    std::vector<double> zeta(K - 1);
    for (int i = 0; i < K; ++i) xi[i] = 2.0 / ev[i];
    for (int j = 0; j < K - 1; ++j) zeta[j] = 2.0 / evp[j];
    for (int i = 0; i < K; ++i) {
        double r = K * K + 1.5 * K;
        for (int j = 0, jd = 0; j < K - 1; ++j, ++jd) {
            if (jd == i) ++jd;
            r *= (zeta[j] * zeta[j] - xi[i] * xi[i]) / (xi[jd] * xi[jd] - xi[i] * xi[i]);
        }
        eta[i] = r;
    }
}

// Everything derived from a problem on the host.
struct Derived {
    int N = 0, W = 0, D = 0, B = 0, precision = 0;
    uint32_t flags = 0;
    int64_t n_ado = 0, n_plus = 0;
    int64_t n_low = 0;  // ADOs at levels 1..D-1
    bool h_complex = false;
    double h_shift = 0.0;            // mean of diag(H) taken off, rad/fs
    std::vector<double> h_re, h_im;  // shifted, rad/fs
    std::vector<int32_t> mode_site;
    std::vector<double> mode_gamma, mode_c_raw, mode_c, mode_lamnu;
    std::vector<double> plus_coef, minus_coef;  // [W][D+1]
    std::vector<double> delta_state;            // [N]
    std::vector<int32_t> state_mode_begin, state_modes;
    std::vector<int64_t> binom;  // [(D+2)][(W+1)]
    double rate_bound = 0.0;
};

// Table layout inside the caller's tables buffer.
struct Layout {
    size_t h_re, h_im, h_re_f32, mode_site, mode_gamma, mode_c, mode_lamnu, plus_coef, minus_coef,
        delta_state, state_mode_begin, state_modes, binom, consts_end;
    size_t tuples, level, plus, minus, mlist, mlist_site, mlist_w, mlist_w32, plus_w, damping, total;
};

Layout make_layout(int N, int W, int D, int64_t n_ado) {
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align256(o + std::max<size_t>(bytes, 1));
        return at;
    };
    const size_t NN = (size_t)N * N;
    const size_t WD = (size_t)W * (D + 1);
    L.h_re = take(NN * 8);
    L.h_im = take(NN * 8);
    L.h_re_f32 = take(NN * 4);
    L.mode_site = take(W * 4);
    L.mode_gamma = take(W * 8);
    L.mode_c = take(W * 8);
    L.mode_lamnu = take(W * 8);
    L.plus_coef = take(WD * 8);
    L.minus_coef = take(WD * 8);
    L.delta_state = take(N * 8);
    L.state_mode_begin = take((N + 1) * 4);
    L.state_modes = take(W * 4);
    L.binom = take((size_t)(D + 2) * (W + 1) * 8);
    L.consts_end = o;
    L.tuples = take((size_t)n_ado * W);
    L.level = take((size_t)n_ado);
    L.plus = take((size_t)n_ado * W * 4);
    L.minus = take((size_t)n_ado * W * 4);
    L.mlist = take((size_t)n_ado * std::max(D, 1) * 8);
    L.mlist_site = take((size_t)n_ado * std::max(D, 1) * 4);
    L.mlist_w = take((size_t)n_ado * std::max(D, 1) * 16);
    L.mlist_w32 = take((size_t)n_ado * std::max(D, 1) * 8);
    L.plus_w = take((size_t)n_ado * W * 8);
    L.damping = take((size_t)n_ado * 8);
    L.total = o;
    return L;
}

bool is_finite(double x) { return std::isfinite(x); }

// Saturating C(m+k, k) table, m in [0, D+1], k in [0, W].
std::vector<int64_t> binomial_table(int W, int D) {
    const int64_t cap = INT64_MAX / 4;
    std::vector<int64_t> b((size_t)(D + 2) * (W + 1));
    for (int m = 0; m <= D + 1; ++m)
        for (int k = 0; k <= W; ++k) {
            int64_t v;
            if (m == 0 || k == 0)
                v = 1;
            else
                v = std::min(cap, b[(size_t)m * (W + 1) + k - 1] + b[(size_t)(m - 1) * (W + 1) + k]);
            b[(size_t)m * (W + 1) + k] = v;
        }
    return b;
}

heom_status derive(const heom_problem* p, Derived& d) {
    if (!p) return fail(HEOM_E_INVAL, "problem is NULL");
    const int N = p->n_states;
    if (N < 1 || N > heom::kMaxStates)
        return fail(N < 1 ? HEOM_E_INVAL : HEOM_E_RANGE, "n_states=%d outside 1..%d", N,
                    heom::kMaxStates);
    if (p->n_baths < 0) return fail(HEOM_E_INVAL, "n_baths < 0");
    if (p->n_baths > 0 && !p->baths) return fail(HEOM_E_INVAL, "baths is NULL");
    if (!p->h_re_cm) return fail(HEOM_E_INVAL, "h_re_cm is NULL");
    if (p->depth < 0) return fail(HEOM_E_INVAL, "depth < 0");
    if (p->depth > 255) return fail(HEOM_E_RANGE, "depth > 255");
    if (p->precision != HEOM_FP64 && p->precision != HEOM_FP32_MIXED &&
        p->precision != HEOM_FP32_HERM)
        return fail(HEOM_E_INVAL, "precision %d unknown", p->precision);
    if (p->flags & ~31u) return fail(HEOM_E_INVAL, "unknown flags 0x%x", p->flags);
    if (!is_finite(p->temperature_K) || !(p->temperature_K > 0.0))
        return fail(HEOM_E_INVAL, "temperature must be finite and > 0");
    d.N = N;
    d.D = p->depth;
    d.B = p->n_baths;
    d.precision = p->precision;
    d.flags = p->flags;
    const size_t NN = (size_t)N * N;
    std::vector<double> hr(p->h_re_cm, p->h_re_cm + NN), hi(NN, 0.0);
    if (p->h_im_cm) std::copy(p->h_im_cm, p->h_im_cm + NN, hi.begin());
    double hmax = 0.0;
    for (size_t e = 0; e < NN; ++e) {
        if (!is_finite(hr[e]) || !is_finite(hi[e])) return fail(HEOM_E_INVAL, "H has a non-finite entry");
        hmax = std::max(hmax, std::hypot(hr[e], hi[e]));
    }
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            const double dr = hr[i * N + j] - hr[j * N + i];
            const double di = hi[i * N + j] + hi[j * N + i];
            if (std::hypot(dr, di) > 1e-12 * std::max(hmax, 1e-300))
                return fail(HEOM_E_INVAL, "H is not Hermitian at (%d,%d)", i, j);
        }
    // baths: validation, modes, coefficients
    const double beta = 1.0 / (kBoltzmannCm * p->temperature_K * kCmToRadFs);  // fs
    const double sign = (p->flags & HEOM_FLAG_STANDARD_GAUGE) ? -1.0 : 1.0;
    d.delta_state.assign(N, 0.0);
    int W = 0;
    for (int b = 0; b < d.B; ++b) {
        const heom_bath& bt = p->baths[b];
        if (bt.state < 0 || bt.state >= N) return fail(HEOM_E_INVAL, "bath %d state out of range", b);
        if (!is_finite(bt.lambda_cm) || bt.lambda_cm < 0.0)
            return fail(HEOM_E_INVAL, "bath %d lambda must be finite and >= 0", b);
        if (!is_finite(bt.tau_fs) || !(bt.tau_fs > 0.0))
            return fail(HEOM_E_INVAL, "bath %d tau must be finite and > 0", b);
        if (bt.n_matsubara < 0) return fail(HEOM_E_INVAL, "bath %d n_matsubara < 0", b);
        if ((p->flags & HEOM_FLAG_PADE) && bt.n_matsubara > kMaxPade)
            return fail(HEOM_E_RANGE, "bath %d: more than %d Pade poles", b, kMaxPade);
        W += 1 + bt.n_matsubara;
        if (W > 255) return fail(HEOM_E_RANGE, "more than 255 modes");
    }
    d.W = W;
    for (int b = 0; b < d.B; ++b) {
        const heom_bath& bt = p->baths[b];
        const double lam = bt.lambda_cm * kCmToRadFs;
        const double nu = 1.0 / bt.tau_fs;
        double sum_c_over_g = 0.0;
        const bool pade = (p->flags & HEOM_FLAG_PADE) != 0;
        std::vector<double> xi, eta;
        if (pade) pade_poles(bt.n_matsubara, xi, eta);
        for (int k = 0; k <= bt.n_matsubara; ++k) {
            double g, c;
            if (k == 0) {
                g = nu;
                if (pade) {
                    // Pade form of lambda nu cot(beta nu / 2), sum over the poles j
                    double s = 1.0;
                    for (size_t j = 0; j < xi.size(); ++j) {
                        const double a = xi[j] / beta;
                        s -= 2.0 * eta[j] * nu * nu / (a * a - nu * nu);
                    }
                    c = 2.0 * lam / beta * s;
                } else {
                    c = lam * nu / std::tan(0.5 * beta * nu);  // lambda nu cot(beta nu / 2)
                }
            } else {
                // Pade pole xi_k / (beta hbar), or the Matsubara frequency
                g = pade ? xi[k - 1] / beta : 2.0 * M_PI * k / beta;
                if (std::fabs(g - nu) <= 1e-12 * nu)
                    return fail(HEOM_E_INVAL, "bath %d: rate of mode %d equals nu", b, k);
                c = 4.0 * lam * nu / beta * (pade ? eta[k - 1] : 1.0) * g / (g * g - nu * nu);
            }
            sum_c_over_g += c / g;
            d.mode_site.push_back(bt.state);
            d.mode_gamma.push_back(g);
            d.mode_c_raw.push_back(c);
            d.mode_c.push_back(sign * c);
            d.mode_lamnu.push_back(k == 0 ? sign * lam * nu : 0.0);
        }
        if (!(p->flags & HEOM_FLAG_NO_TERMINATOR))
            d.delta_state[bt.state] += 2.0 * lam / (beta * nu) - sum_c_over_g;
        if (p->flags & HEOM_FLAG_ADD_REORG) hr[(size_t)bt.state * N + bt.state] += bt.lambda_cm;
    }
    // H in rad/fs, diagonal shifted by its mean (the commutator is unchanged)
    double mean = 0.0;
    for (int i = 0; i < N; ++i) mean += hr[(size_t)i * N + i];
    mean /= N;
    for (int i = 0; i < N; ++i) hr[(size_t)i * N + i] -= mean;
    d.h_shift = mean * kCmToRadFs;
    d.h_re.resize(NN);
    d.h_im.resize(NN);
    for (size_t e = 0; e < NN; ++e) {
        d.h_re[e] = hr[e] * kCmToRadFs;
        d.h_im[e] = hi[e] * kCmToRadFs;
        if (hi[e] != 0.0) d.h_complex = true;
    }
    if (d.precision == HEOM_FP32_HERM && heom::bulk_mfma_blocks(N, d.h_complex, d.precision) == 0)
        return fail(HEOM_E_INVAL,
                    "Hermitian-packed storage needs the matrix-core path (real H, 16 <= N <= 64)");
    // rescaled coupling weights (ADO rescaling substitution); |c| = 0 uses scale 1
    const int D = d.D;
    d.plus_coef.assign((size_t)W * (D + 1), 0.0);
    d.minus_coef.assign((size_t)W * (D + 1), 0.0);
    const bool rescale = !(p->flags & HEOM_FLAG_NO_RESCALE);
    for (int l = 0; l < W; ++l) {
        const double ac = std::fabs(d.mode_c_raw[l]) > 0.0 ? std::fabs(d.mode_c_raw[l]) : 1.0;
        for (int n = 0; n <= D; ++n) {
            d.plus_coef[(size_t)l * (D + 1) + n] = sign * (rescale ? std::sqrt((n + 1.0) * ac) : 1.0);
            d.minus_coef[(size_t)l * (D + 1) + n] = rescale ? std::sqrt(n / ac) : (double)n;
        }
    }
    d.state_mode_begin.assign(N + 1, 0);
    for (int l = 0; l < W; ++l) d.state_mode_begin[d.mode_site[l] + 1]++;
    for (int s = 0; s < N; ++s) d.state_mode_begin[s + 1] += d.state_mode_begin[s];
    d.state_modes.assign(W, 0);
    {
        std::vector<int32_t> fill(d.state_mode_begin.begin(), d.state_mode_begin.end() - 1);
        for (int l = 0; l < W; ++l) d.state_modes[fill[d.mode_site[l]]++] = l;
    }
    d.binom = binomial_table(W, D);
    const int64_t n_ado = d.binom[(size_t)D * (W + 1) + W];  // C(D+W, W)
    if (n_ado >= (int64_t(1) << 31)) return fail(HEOM_E_RANGE, "n_ado >= 2^31");
    d.n_ado = n_ado;
    d.n_plus = (D == 0) ? 0 : (int64_t)W * d.binom[(size_t)(D - 1) * (W + 1) + W];
    d.n_low = (D == 0) ? 0 : d.binom[(size_t)(D - 1) * (W + 1) + W] - 1;
    // Gershgorin-type bound on the generator, for the RK4 step-size check:
    // commutator 2||H||_inf, damping D max gamma, correction 2 max Delta, and
    // per element the couplings of the modes of two states.
    double hinf = 0.0;
    for (int i = 0; i < N; ++i) {
        double row = 0.0;
        for (int j = 0; j < N; ++j) row += std::hypot(d.h_re[i * N + j], d.h_im[i * N + j]);
        hinf = std::max(hinf, row);
    }
    double gmax = 0.0, dmax = 0.0, cmax = 0.0;
    for (int l = 0; l < W; ++l) gmax = std::max(gmax, d.mode_gamma[l]);
    for (int s = 0; s < N; ++s) dmax = std::max(dmax, std::fabs(d.delta_state[s]));
    for (int s = 0; s < N; ++s) {
        double acc = 0.0;
        for (int m = d.state_mode_begin[s]; m < d.state_mode_begin[s + 1]; ++m) {
            const int l = d.state_modes[m];
            double amax = 0.0, bmax = 0.0;
            for (int n = 0; n <= D; ++n) {
                if (n < D) amax = std::max(amax, std::fabs(d.plus_coef[(size_t)l * (D + 1) + n]));
                bmax = std::max(bmax, d.minus_coef[(size_t)l * (D + 1) + n]);
            }
            acc += amax + bmax * (std::fabs(d.mode_c[l]) + 2.0 * std::fabs(d.mode_lamnu[l]));
        }
        cmax = std::max(cmax, acc);
    }
    d.rate_bound = 2.0 * hinf + D * gmax + 2.0 * dmax + 2.0 * cmax;
    return HEOM_OK;
}

void fill_info(const Derived& d, heom_info* info) {
    std::memset(info, 0, sizeof *info);
    const Layout L = make_layout(d.N, d.W, d.D, d.n_ado);
    info->n_ado = d.n_ado;
    info->n_plus_edges = d.n_plus;
    info->n_states = d.N;
    info->n_modes = d.W;
    info->depth = d.D;
    info->elem_bytes = d.precision == HEOM_FP64 ? 16 : d.precision == HEOM_FP32_MIXED ? 8 : 4;
    info->tables_bytes = L.total;
    const size_t NN = (size_t)d.N * d.N;
    info->sigma0_bytes = NN * 16;
    info->rest_bytes = (size_t)(d.n_ado - 1) * NN * info->elem_bytes;
    // control block (step counter, status, mu) + three stage copies
    info->bulk_kernel = heom::bulk_mfma_blocks(d.N, d.h_complex, d.precision) > 0 ? 1 : 0;
    info->work_bytes = 1024 + align256(d.N * 8) +
                       3 * (align256(info->sigma0_bytes) + align256(std::max<size_t>(info->rest_bytes, 1)));
    // Hermitian-packed storage: two complex64 copies of the levels 1..D-1
    if (d.precision == HEOM_FP32_HERM) info->work_bytes += 2 * mirror_bytes(d.n_low, d.N);
}

int gfx950_device_check() {
    static std::mutex mu;
    static int cached = -2;  // per process: -2 unknown, 0 ok, -1 bad
    std::lock_guard<std::mutex> lk(mu);
    if (cached != -2) return cached;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        cached = -1;
    } else {
        cached = (std::strncmp(prop.gcnArchName, "gfx950", 6) == 0) ? 0 : -1;
    }
    return cached;
}

}  // namespace

struct heom_hierarchy {
    heom::Tables t;
    Derived d;
    heom_info info;
    std::vector<char> host_consts;  // source of the asynchronous constant upload
};

extern "C" {

const char* heom_last_error(void) { return g_error.c_str(); }

const char* heom_status_string(heom_status s) {
    switch (s) {
        case HEOM_OK: return "HEOM_OK";
        case HEOM_PENDING: return "HEOM_PENDING";
        case HEOM_E_INVAL: return "HEOM_E_INVAL";
        case HEOM_E_RANGE: return "HEOM_E_RANGE";
        case HEOM_E_NOMEM: return "HEOM_E_NOMEM";
        case HEOM_E_DEVICE: return "HEOM_E_DEVICE";
        case HEOM_E_NUMERIC: return "HEOM_E_NUMERIC";
        case HEOM_E_UNSTABLE: return "HEOM_E_UNSTABLE";
        case HEOM_E_NOTFOUND: return "HEOM_E_NOTFOUND";
        case HEOM_E_CANCELLED: return "HEOM_E_CANCELLED";
        default: return "HEOM_E_UNKNOWN";
    }
}

heom_status heom_plan(const heom_problem* problem, heom_info* info) {
    if (!info) return fail(HEOM_E_INVAL, "info is NULL");
    Derived d;
    heom_status s = derive(problem, d);
    if (s != HEOM_OK) return s;
    fill_info(d, info);
    g_error.clear();
    return HEOM_OK;
}

int32_t heom_record_doubles(int32_t n_states, int32_t kind) {
    return kind == HEOM_OBS_POPULATION ? n_states + 3 : 4;
}

int64_t heom_record_count(int64_t n_steps, int32_t record_every) {
    if (n_steps < 0 || record_every < 1) return 0;
    return n_steps / record_every + 1;
}

size_t heom_propagate_work_bytes(const heom_info* info, int64_t n_steps, int32_t record_every,
                                 int32_t kind) {
    if (!info) return 0;
    const size_t rec = (size_t)heom_record_count(n_steps, record_every) *
                       heom_record_doubles(info->n_states, kind) * sizeof(double);
    return info->work_bytes + align256(rec);
}

heom_status heom_build_hierarchy(const heom_problem* problem, void* tables_dev,
                                 size_t tables_bytes, void* stream, heom_hierarchy** out) {
    if (!out) return fail(HEOM_E_INVAL, "out is NULL");
    *out = nullptr;
    Derived d;
    heom_status s = derive(problem, d);
    if (s != HEOM_OK) return s;
    heom_info info;
    fill_info(d, &info);
    if (!tables_dev) return fail(HEOM_E_INVAL, "tables_dev is NULL");
    if (reinterpret_cast<uintptr_t>(tables_dev) % 256)
        return fail(HEOM_E_INVAL, "tables_dev must be 256-byte aligned");
    if (tables_bytes < info.tables_bytes)
        return fail(HEOM_E_NOMEM, "tables buffer %zu < %zu bytes", tables_bytes, info.tables_bytes);
    if (gfx950_device_check() != 0) return fail(HEOM_E_DEVICE, "no gfx950 device is current");

    auto* h = new heom_hierarchy();
    h->d = std::move(d);
    h->info = info;
    const Derived& D = h->d;
    const Layout L = make_layout(D.N, D.W, D.D, D.n_ado);
    h->host_consts.assign(L.consts_end, 0);
    char* hc = h->host_consts.data();
    auto put = [&](size_t off, const void* src, size_t bytes) {
        if (bytes) std::memcpy(hc + off, src, bytes);
    };
    const size_t NN = (size_t)D.N * D.N;
    put(L.h_re, D.h_re.data(), NN * 8);
    put(L.h_im, D.h_im.data(), NN * 8);
    std::vector<float> h32(D.h_re.begin(), D.h_re.end());
    put(L.h_re_f32, h32.data(), NN * 4);
    put(L.mode_site, D.mode_site.data(), D.W * 4);
    put(L.mode_gamma, D.mode_gamma.data(), D.W * 8);
    put(L.mode_c, D.mode_c.data(), D.W * 8);
    put(L.mode_lamnu, D.mode_lamnu.data(), D.W * 8);
    put(L.plus_coef, D.plus_coef.data(), D.plus_coef.size() * 8);
    put(L.minus_coef, D.minus_coef.data(), D.minus_coef.size() * 8);
    put(L.delta_state, D.delta_state.data(), D.N * 8);
    put(L.state_mode_begin, D.state_mode_begin.data(), (D.N + 1) * 4);
    put(L.state_modes, D.state_modes.data(), D.W * 4);
    put(L.binom, D.binom.data(), D.binom.size() * 8);

    char* base = static_cast<char*>(tables_dev);
    heom::Tables& t = h->t;
    t.N = D.N;
    t.W = D.W;
    t.D = D.D;
    t.n_ado = (int32_t)D.n_ado;
    t.h_complex = D.h_complex ? 1 : 0;
    t.h_shift = D.h_shift;
    t.h_re = reinterpret_cast<const double*>(base + L.h_re);
    t.h_im = reinterpret_cast<const double*>(base + L.h_im);
    t.h_re_f32 = reinterpret_cast<const float*>(base + L.h_re_f32);
    t.mode_site = reinterpret_cast<const int32_t*>(base + L.mode_site);
    t.mode_gamma = reinterpret_cast<const double*>(base + L.mode_gamma);
    t.mode_c = reinterpret_cast<const double*>(base + L.mode_c);
    t.mode_lamnu = reinterpret_cast<const double*>(base + L.mode_lamnu);
    t.plus_coef = reinterpret_cast<const double*>(base + L.plus_coef);
    t.minus_coef = reinterpret_cast<const double*>(base + L.minus_coef);
    t.delta_state = reinterpret_cast<const double*>(base + L.delta_state);
    t.state_mode_begin = reinterpret_cast<const int32_t*>(base + L.state_mode_begin);
    t.state_modes = reinterpret_cast<const int32_t*>(base + L.state_modes);
    t.binom = reinterpret_cast<const int64_t*>(base + L.binom);
    t.tuples = reinterpret_cast<uint8_t*>(base + L.tuples);
    t.level = reinterpret_cast<uint8_t*>(base + L.level);
    t.plus = reinterpret_cast<int32_t*>(base + L.plus);
    t.minus = reinterpret_cast<int32_t*>(base + L.minus);
    t.mlist = reinterpret_cast<int32_t*>(base + L.mlist);
    t.mlist_site = reinterpret_cast<int32_t*>(base + L.mlist_site);
    t.mlist_w = reinterpret_cast<double*>(base + L.mlist_w);
    t.mlist_w32 = reinterpret_cast<float*>(base + L.mlist_w32);
    t.plus_w = reinterpret_cast<double*>(base + L.plus_w);
    t.damping = reinterpret_cast<double*>(base + L.damping);

    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(tables_dev, hc, L.consts_end, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = heom::launch_enumerate(t, st);
    if (e != hipSuccess) {
        delete h;
        return fail(HEOM_E_DEVICE, "hierarchy build: %s", hipGetErrorString(e));
    }
    *out = h;
    g_error.clear();
    return HEOM_OK;
}

heom_status heom_copy_tables(const heom_hierarchy* h, uint8_t* tuples, int32_t* plus,
                             int32_t* minus, uint8_t* level, void* stream) {
    if (!h) return fail(HEOM_E_INVAL, "hierarchy is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t nw = (size_t)h->t.n_ado * h->t.W;
    if (tuples && nw) HIP_TRY(hipMemcpyAsync(tuples, h->t.tuples, nw, hipMemcpyDeviceToHost, st));
    if (plus && nw) HIP_TRY(hipMemcpyAsync(plus, h->t.plus, nw * 4, hipMemcpyDeviceToHost, st));
    if (minus && nw) HIP_TRY(hipMemcpyAsync(minus, h->t.minus, nw * 4, hipMemcpyDeviceToHost, st));
    if (level)
        HIP_TRY(hipMemcpyAsync(level, h->t.level, h->t.n_ado, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return HEOM_OK;
}

static void copy_coefficients(const Derived& d, double* gamma, double* c, double* lamnu,
                              double* delta_state) {
    for (int l = 0; l < d.W; ++l) {
        if (gamma) gamma[l] = d.mode_gamma[l];
        if (c) c[l] = d.mode_c_raw[l];
        if (lamnu) lamnu[l] = (d.flags & HEOM_FLAG_STANDARD_GAUGE) ? -d.mode_lamnu[l] : d.mode_lamnu[l];
    }
    if (delta_state)
        for (int s = 0; s < d.N; ++s) delta_state[s] = d.delta_state[s];
}

heom_status heom_problem_coefficients(const heom_problem* problem, double* gamma, double* c,
                                      double* lamnu, double* delta_state) {
    Derived d;
    heom_status s = derive(problem, d);
    if (s != HEOM_OK) return s;
    copy_coefficients(d, gamma, c, lamnu, delta_state);
    return HEOM_OK;
}

heom_status heom_coefficients(const heom_hierarchy* h, double* gamma, double* c, double* lamnu,
                              double* delta_state) {
    if (!h) return fail(HEOM_E_INVAL, "hierarchy is NULL");
    const Derived& d = h->d;
    for (int l = 0; l < d.W; ++l) {
        if (gamma) gamma[l] = d.mode_gamma[l];
        if (c) c[l] = d.mode_c_raw[l];
        if (lamnu) lamnu[l] = (d.flags & HEOM_FLAG_STANDARD_GAUGE) ? -d.mode_lamnu[l] : d.mode_lamnu[l];
    }
    if (delta_state)
        for (int s = 0; s < d.N; ++s) delta_state[s] = d.delta_state[s];
    return HEOM_OK;
}

}  // extern "C"

namespace {

struct TimingState {
    std::atomic<bool> enabled{false};
    std::mutex mu;
    double ms = 0.0, bytes = 0.0;
    int64_t launches = 0;
};
TimingState g_timing;

heom::Job base_job(const heom_hierarchy* h) {
    heom::Job j{};
    j.t = h->t;
    j.any_complex_h = h->t.h_complex;
    j.dt = 1.0;
    j.tile_begin = 0;
    j.n_low = (int32_t)h->d.n_low;
    j.ados_per_tile =
        heom::bulk_mfma_blocks(h->t.N, h->t.h_complex != 0, h->d.precision)
            ? 1
            : heom::bulk_ados_per_tile(h->t.N, h->t.W, h->t.D, h->d.precision == HEOM_FP64 ? 8 : 4);
    j.n_tiles = (int32_t)((h->t.n_ado - 1 + j.ados_per_tile - 1) / j.ados_per_tile);
    j.rec_every = 1;
    return j;
}

bool aligned(const void* p) { return reinterpret_cast<uintptr_t>(p) % 256 == 0; }

}  // namespace

namespace heom {

const Tables& hierarchy_tables(const heom_hierarchy* h) { return h->t; }
int hierarchy_precision(const heom_hierarchy* h) { return h->d.precision; }
double hierarchy_rate_bound(const heom_hierarchy* h) { return h->d.rate_bound; }
Job hierarchy_job(const heom_hierarchy* h) { return base_job(h); }
const heom_info& hierarchy_info(const heom_hierarchy* h) { return h->info; }

size_t control_bytes(int N) { return 1024 + align256((size_t)N * 8); }

// Workspace layout: [step @0, status @256, mu @1024][three stage copies][records].
Job bind_workspace(const heom_hierarchy* h, heom_state io, char* w, double dt, int64_t n_steps,
                   int record_every, int kind, int ground, int hermitian) {
    Job j = base_job(h);
    const int N = h->t.N;
    j.herm = hermitian ? 1 : 0;
    j.dt = dt;
    j.step = reinterpret_cast<int64_t*>(w);
    j.status = reinterpret_cast<int32_t*>(w + 256);
    j.mu = reinterpret_cast<double*>(w + 1024);
    size_t off = control_bytes(N);
    for (int k = 1; k <= 3; ++k) {
        j.sig0[k] = w + off;
        off += align256(h->info.sigma0_bytes);
        j.rest[k] = w + off;
        off += align256(std::max<size_t>(h->info.rest_bytes, 1));
    }
    j.sig0[0] = io.sigma0;
    j.rest[0] = io.rest;
    if (h->d.precision == HEOM_FP32_HERM) {
        for (int m = 0; m < 2; ++m) {
            j.mirror[m] = w + off;
            off += mirror_bytes(h->d.n_low, N);
        }
    }
    j.records = reinterpret_cast<double*>(w + off);
    j.n_rec_max = heom_record_count(n_steps, record_every);
    j.rec_every = record_every;
    j.rec_kind = kind;
    j.rec_doubles = heom_record_doubles(N, kind);
    j.ground = ground;
    return j;
}

heom_status problem_rate_bound(const heom_problem* p, double* rate) {
    Derived d;
    heom_status s = derive(p, d);
    if (s == HEOM_OK) *rate = d.rate_bound;
    return s;
}

bool block_step_ok(const heom_problem* p, double dt) {
    Derived d;
    if (derive(p, d) != HEOM_OK) return false;
    const double shift = std::fabs(d.h_shift);
    return dt * (d.rate_bound + shift) <= kRk4RealLimit && dt * shift <= kBlockPhaseLimit;
}

double rk4_real_limit() { return kRk4RealLimit; }

void set_last_error(const std::string& msg) { g_error = msg; }

double monotonic_seconds() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

void rk4_stage_specs(StageSpec sp[4]) {
    for (int k = 0; k < 4; ++k) sp[k] = StageSpec{};
    // Y2 = y + dt/2 f(y)
    sp[0].in = 0; sp[0].out = 1; sp[0].w_in = 1.0; sp[0].hmul = 0.5; sp[0].record_initial = 1;
    // Y3 = y + dt/2 f(Y2)
    sp[1].in = 1; sp[1].out = 2; sp[1].nbase = 1; sp[1].base[0] = 0; sp[1].wbase[0] = 1.0;
    sp[1].hmul = 0.5;
    // Y4 = y + dt f(Y3)
    sp[2].in = 2; sp[2].out = 3; sp[2].nbase = 1; sp[2].base[0] = 0; sp[2].wbase[0] = 1.0;
    sp[2].hmul = 1.0;
    // y' = (-y + Y2 + 2 Y3 + Y4)/3 + dt/6 f(Y4): the textbook y + dt/6 (k1 + 2k2 + 2k3 + k4)
    // with k1 = 2(Y2 - y)/dt, k2 = 2(Y3 - y)/dt, k3 = (Y4 - y)/dt
    sp[3].in = 3; sp[3].out = 0; sp[3].w_in = 1.0 / 3.0; sp[3].nbase = 3;
    sp[3].base[0] = 0; sp[3].wbase[0] = -1.0 / 3.0;
    sp[3].base[1] = 1; sp[3].wbase[1] = 1.0 / 3.0;
    sp[3].base[2] = 2; sp[3].wbase[2] = 2.0 / 3.0;
    sp[3].hmul = 1.0 / 6.0; sp[3].record_after = 1;
}

}  // namespace heom

namespace {

heom_status check_state(const heom_hierarchy* h, const heom_state& s, const char* what) {
    if (!s.sigma0) return fail(HEOM_E_INVAL, "%s.sigma0 is NULL", what);
    if (!s.rest && h->t.n_ado > 1) return fail(HEOM_E_INVAL, "%s.rest is NULL", what);
    if (!aligned(s.sigma0)) return fail(HEOM_E_INVAL, "%s.sigma0 must be 256-byte aligned", what);
    return HEOM_OK;
}

}  // namespace

extern "C" {

heom_status heom_rhs(const heom_hierarchy* h, heom_state in, heom_state out, int32_t hermitian,
                     void* stream) {
    if (!h) return fail(HEOM_E_INVAL, "hierarchy is NULL");
    heom_status s;
    if ((s = check_state(h, in, "in")) != HEOM_OK) return s;
    if ((s = check_state(h, out, "out")) != HEOM_OK) return s;
    if (h->d.precision == HEOM_FP32_HERM && !hermitian)
        return fail(HEOM_E_INVAL, "Hermitian-packed storage holds Hermitian ADOs only");
    heom::Job j = base_job(h);
    j.herm = hermitian ? 1 : 0;
    j.sig0[0] = in.sigma0;
    j.rest[0] = in.rest;
    j.sig0[1] = out.sigma0;
    j.rest[1] = out.rest;
    heom::StageSpec sp{};
    sp.in = 0;
    sp.out = 1;
    sp.w_in = 0.0;
    sp.hmul = 1.0;
    hipError_t e = heom::launch_stage(j, nullptr, 0, h->t.n_ado > 1 ? j.n_tiles : 0,
                                      h->d.precision, sp, static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return fail(HEOM_E_DEVICE, "rhs launch (%s): %s", heom::last_launch_failure(),
                    hipGetErrorString(e));
    return HEOM_OK;
}

}  // extern "C"

namespace {

// Steps from which heom_propagate replays a captured step graph.
constexpr int64_t kGraphMinSteps = 8;

// One RK4 step's launches captured on a private stream and instantiated; the
// destructor waits for the caller's stream before the graph goes away.
struct StepGraph {
    hipStream_t caller;
    hipStream_t cs = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    explicit StepGraph(hipStream_t s) : caller(s) {}
    template <class F>
    bool capture(F&& launch) {
        if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
            cs = nullptr;
            return false;
        }
        if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) return false;
        const hipError_t le = launch(cs);
        const hipError_t ee = hipStreamEndCapture(cs, &graph);
        if (le != hipSuccess || ee != hipSuccess || !graph) {
            (void)hipGetLastError();
            return false;
        }
        if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
            exec = nullptr;
            (void)hipGetLastError();
            return false;
        }
        return true;
    }
    ~StepGraph() {
        if (exec) {
            (void)hipStreamSynchronize(caller);
            (void)hipGraphExecDestroy(exec);
        }
        if (graph) (void)hipGraphDestroy(graph);
        if (cs) (void)hipStreamDestroy(cs);
    }
};

// heom_propagate on a given workspace.  `timing` allows the benchmark event
// timing (which creates HIP events) and `graphs` the step graph (which
// allocates); the no-alloc entry point passes false for both.
heom_status propagate_impl(const heom_hierarchy* h, heom_state io, void* work_dev,
                           size_t work_bytes, double dt_fs, int64_t n_steps, int32_t record_every,
                           const heom_observable* obs, int32_t hermitian, double* host_out,
                           void* stream, bool timing, bool graphs) {
    if (!h) return fail(HEOM_E_INVAL, "hierarchy is NULL");
    heom_status s;
    if ((s = check_state(h, io, "io")) != HEOM_OK) return s;
    if (!is_finite(dt_fs) || !(dt_fs > 0.0)) return fail(HEOM_E_INVAL, "dt must be finite and > 0");
    if (n_steps < 0 || record_every < 1) return fail(HEOM_E_INVAL, "n_steps < 0 or record_every < 1");
    const int kind = obs ? obs->kind : HEOM_OBS_POPULATION;
    if (kind != HEOM_OBS_POPULATION && kind != HEOM_OBS_DIPOLE)
        return fail(HEOM_E_INVAL, "observable kind %d unknown", kind);
    if (kind == HEOM_OBS_DIPOLE && (!obs->mu || obs->ground < 0 || obs->ground >= h->t.N))
        return fail(HEOM_E_INVAL, "dipole observable needs mu and a ground index in range");
    if (h->d.precision == HEOM_FP32_HERM && !hermitian)
        return fail(HEOM_E_INVAL, "Hermitian-packed storage holds Hermitian ADOs only");
    if (dt_fs * h->d.rate_bound > kRk4RealLimit)
        return fail(HEOM_E_UNSTABLE, "dt=%g fs times the rate bound %g /fs exceeds %g", dt_fs,
                    h->d.rate_bound, kRk4RealLimit);
    const size_t need = heom_propagate_work_bytes(&h->info, n_steps, record_every, kind);
    if (!work_dev || work_bytes < need)
        return fail(HEOM_E_NOMEM, "workspace %zu < %zu bytes", work_bytes, need);
    if (!aligned(work_dev)) return fail(HEOM_E_INVAL, "work_dev must be 256-byte aligned");

    const int N = h->t.N;
    const int rd = heom_record_doubles(N, kind);
    const int64_t n_rec = heom_record_count(n_steps, record_every);
    char* w = static_cast<char*>(work_dev);
    heom::Job j = heom::bind_workspace(h, io, w, dt_fs, n_steps, record_every, kind,
                                       kind == HEOM_OBS_DIPOLE ? obs->ground : 0, hermitian);

    hipStream_t st = static_cast<hipStream_t>(stream);
    // control block: step = 0, status = 0, mu (N <= 64: at most 1536 bytes)
    alignas(16) char ctl[1024 + 64 * 8] = {};
    const size_t ctl_bytes = std::min(heom::control_bytes(N), sizeof(ctl));
    if (kind == HEOM_OBS_DIPOLE) std::memcpy(ctl + 1024, obs->mu, N * 8);
    HIP_TRY(hipMemcpyAsync(w, ctl, ctl_bytes, hipMemcpyHostToDevice, st));

    heom::StageSpec sp[4];
    heom::rk4_stage_specs(sp);

    const int tiles = h->t.n_ado > 1 ? j.n_tiles : 0;
    if (h->d.precision == HEOM_FP32_HERM && j.n_low > 0 && tiles > 0) {
        // complex copies of the lower levels, alternating between the two
        // buffers: stage k reads the copy the previous stage wrote
        hipError_t e = heom::launch_pk_mirror(io.rest, j.mirror[0], N, j.n_low, st);
        if (e != hipSuccess) return fail(HEOM_E_DEVICE, "mirror launch: %s", hipGetErrorString(e));
        for (int k = 0; k < 4; ++k) {
            sp[k].mirror_in = 1 + (k & 1);
            sp[k].mirror_out = 2 - (k & 1);
        }
    }
    const bool timed = timing && g_timing.enabled.load() && tiles > 0;
    std::vector<hipEvent_t> ev;
    if (timed) {
        ev.resize(2 * (size_t)n_steps * 4);
        for (auto& x : ev) HIP_TRY(hipEventCreate(&x));
    }
    static const int kPasses[4] = {2, 3, 3, 5};
    auto launch_step = [&](int64_t step, hipStream_t s) -> hipError_t {
        for (int k = 0; k < 4; ++k) {
            hipError_t e = heom::launch_stage(j, nullptr, 0, tiles, h->d.precision, sp[k], s,
                                              timed ? ev[2 * (step * 4 + k)] : nullptr,
                                              timed ? ev[2 * (step * 4 + k) + 1] : nullptr);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    // Small hierarchies are bound by launch latency: after one step launched
    // directly (which also sets the kernels' attributes up), the four stage
    // launches of a step are captured once in a HIP graph and the graph is
    // replayed for the remaining steps.  The kernels keep the step count on
    // the device, so every replay is the same launch.  A capture that fails
    // falls back to direct launches.
    StepGraph graph(st);
    int64_t step = 0;
    if (graphs && !timed && tiles > 0 && n_steps >= kGraphMinSteps) {
        hipError_t e = launch_step(0, st);
        if (e != hipSuccess)
            return fail(HEOM_E_DEVICE, "stage launch (%s): %s", heom::last_launch_failure(),
                        hipGetErrorString(e));
        step = 1;
        if (graph.capture([&](hipStream_t cs) { return launch_step(1, cs); })) {
            for (; step < n_steps; ++step)
                if ((e = hipGraphLaunch(graph.exec, st)) != hipSuccess)
                    return fail(HEOM_E_DEVICE, "graph launch: %s", hipGetErrorString(e));
        }
    }
    for (; step < n_steps; ++step) {
        hipError_t e = launch_step(step, st);
        if (e != hipSuccess)
            return fail(HEOM_E_DEVICE, "stage launch (%s): %s", heom::last_launch_failure(),
                        hipGetErrorString(e));
    }
    if (n_steps == 0) {
        // record the initial state only: a stage-1 pass into slot 1 does it
        hipError_t e = heom::launch_stage(j, nullptr, 0, 0, h->d.precision, sp[0], st);
        if (e != hipSuccess) return fail(HEOM_E_DEVICE, "record launch: %s", hipGetErrorString(e));
    }
    int32_t status = 0;
    HIP_TRY(hipMemcpyAsync(&status, j.status, 4, hipMemcpyDeviceToHost, st));
    if (host_out)
        HIP_TRY(hipMemcpyAsync(host_out, j.records, (size_t)n_rec * rd * 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (timed) {
        double ms_total = 0.0, bytes = 0.0;
        const double pass = (double)h->info.rest_bytes;
        for (int64_t step = 0; step < n_steps; ++step)
            for (int k = 0; k < 4; ++k) {
                float ms = 0.0f;
                HIP_TRY(hipEventElapsedTime(&ms, ev[2 * (step * 4 + k)], ev[2 * (step * 4 + k) + 1]));
                ms_total += ms;
                bytes += kPasses[k] * pass;
            }
        for (auto& x : ev) (void)hipEventDestroy(x);
        std::lock_guard<std::mutex> lk(g_timing.mu);
        g_timing.ms += ms_total;
        g_timing.launches += 4 * n_steps;
        g_timing.bytes += bytes;
    }
    if (status) return fail(HEOM_E_NUMERIC, "non-finite observable");
    return HEOM_OK;
}

}  // namespace

extern "C" {

heom_status heom_propagate(const heom_hierarchy* h, heom_state io, void* work_dev,
                           size_t work_bytes, double dt_fs, int64_t n_steps, int32_t record_every,
                           const heom_observable* obs, int32_t hermitian, double* host_out,
                           void* stream) {
    return propagate_impl(h, io, work_dev, work_bytes, dt_fs, n_steps, record_every, obs,
                          hermitian, host_out, stream, true, true);
}

heom_status heom_propagate_noalloc(const heom_hierarchy* h, heom_state io, double dt_fs,
                                   int64_t n_steps, int32_t record_every,
                                   const heom_observable* obs, int32_t hermitian,
                                   double* host_out, void* stream) {
    if (!h) return fail(HEOM_E_INVAL, "hierarchy is NULL");
    if (n_steps < 0 || record_every < 1) return fail(HEOM_E_INVAL, "n_steps < 0 or record_every < 1");
    const int kind = obs ? obs->kind : HEOM_OBS_POPULATION;
    if (kind != HEOM_OBS_POPULATION && kind != HEOM_OBS_DIPOLE)
        return fail(HEOM_E_INVAL, "observable kind %d unknown", kind);
    const size_t need = heom_propagate_work_bytes(&h->info, n_steps, record_every, kind);
    if (need > heom::kScratchBytes)
        return fail(HEOM_E_NOMEM,
                    "workspace of %zu bytes exceeds the library's static scratch (%zu bytes); "
                    "use heom_propagate with a caller workspace",
                    need, heom::kScratchBytes);
    void* scratch = nullptr;
    size_t scratch_bytes = 0;
    hipError_t e = heom::scratch_buffer(&scratch, &scratch_bytes);
    if (e != hipSuccess)
        return fail(HEOM_E_DEVICE, "static scratch lookup: %s", hipGetErrorString(e));
    return propagate_impl(h, io, scratch, scratch_bytes, dt_fs, n_steps, record_every, obs,
                          hermitian, host_out, stream, false, false);
}

heom_status heom_set_launch_shape(int32_t max_workgroups, int32_t max_ados_per_tile) {
    if (max_workgroups < 0 || max_ados_per_tile < 0)
        return fail(HEOM_E_INVAL, "launch-shape caps must be >= 0");
    heom::g_max_workgroups.store(max_workgroups);
    heom::g_max_ados_per_tile.store(max_ados_per_tile);
    return HEOM_OK;
}

heom_status heom_timing_enable(int32_t enable) {
    g_timing.enabled.store(enable != 0);
    return HEOM_OK;
}

heom_status heom_timing_read(double* bulk_ms, int64_t* bulk_launches, double* bulk_bytes,
                             int32_t reset) {
    std::lock_guard<std::mutex> lk(g_timing.mu);
    if (bulk_ms) *bulk_ms = g_timing.ms;
    if (bulk_launches) *bulk_launches = g_timing.launches;
    if (bulk_bytes) *bulk_bytes = g_timing.bytes;
    if (reset) {
        g_timing.ms = 0.0;
        g_timing.launches = 0;
        g_timing.bytes = 0.0;
    }
    return HEOM_OK;
}

heom_status heom_cd_vectors(const double* R, const double* d, int32_t n_sites, double* m) {
    if (!R || !d || !m || n_sites < 1) return fail(HEOM_E_INVAL, "NULL array or n_sites < 1");
    for (int a = 0; a < n_sites; ++a) {
        const double* r = R + 3 * a;
        const double* v = d + 3 * a;
        const double c[3] = {r[1] * v[2] - r[2] * v[1], r[2] * v[0] - r[0] * v[2],
                             r[0] * v[1] - r[1] * v[0]};
        for (int p = 0; p < 3; ++p) {
            if (!is_finite(c[p])) return fail(HEOM_E_INVAL, "site %d: non-finite R or d", a);
            m[p * n_sites + a] = c[p];
        }
    }
    return HEOM_OK;
}

size_t heom_block_work_bytes(const heom_info* info, int64_t n_steps, int32_t record_every) {
    if (!info) return 0;
    const size_t copy = align256((size_t)info->n_ado * info->n_states * 3 * 16);
    const size_t rec = align256((size_t)heom_record_count(n_steps, record_every) * 6 * 8);
    return 256 + 3 * copy + rec;
}

heom_status heom_propagate_block(const heom_hierarchy* h, void* state, void* work_dev,
                                 size_t work_bytes, double dt_fs, int64_t n_steps,
                                 int32_t record_every, const double* obs, double* host_out,
                                 void* stream) {
    if (!h || !state || !obs) return fail(HEOM_E_INVAL, "NULL hierarchy, state or obs");
    if (!aligned(state)) return fail(HEOM_E_INVAL, "state must be 256-byte aligned");
    if (!is_finite(dt_fs) || !(dt_fs > 0.0)) return fail(HEOM_E_INVAL, "dt must be finite and > 0");
    if (n_steps < 0 || record_every < 1) return fail(HEOM_E_INVAL, "n_steps < 0 or record_every < 1");
    const int N = h->t.N;
    for (int e = 0; e < 3 * N; ++e)
        if (!is_finite(obs[e])) return fail(HEOM_E_INVAL, "obs[%d] is not finite", e);
    // A single column keeps the mean of diag(H) (the frame's offset from the
    // ground energy): it adds |h_shift| to the rate bound, and more than
    // kBlockPhaseLimit of phase per step means H was not given in a frame
    // rotating near the excited energies.
    const double shift = std::fabs(h->d.h_shift);
    if (dt_fs * (h->d.rate_bound + shift) > kRk4RealLimit || dt_fs * shift > kBlockPhaseLimit)
        return fail(HEOM_E_UNSTABLE,
                    "dt=%g fs: rate bound %g /fs with the diagonal offset %g rad/fs of H (limits: "
                    "%g for the bound, %g rad per step for the offset; give the excited block in a "
                    "frame rotating at the mean excited energy)",
                    dt_fs, h->d.rate_bound + shift, shift, kRk4RealLimit, kBlockPhaseLimit);
    const size_t need = heom_block_work_bytes(&h->info, n_steps, record_every);
    if (!work_dev || work_bytes < need)
        return fail(HEOM_E_NOMEM, "workspace %zu < %zu bytes", work_bytes, need);
    if (!aligned(work_dev)) return fail(HEOM_E_INVAL, "work_dev must be 256-byte aligned");
    char* w = static_cast<char*>(work_dev);
    int32_t* status = reinterpret_cast<int32_t*>(w);
    const size_t copy = align256((size_t)h->t.n_ado * N * 3 * 16);
    void* arr[4] = {state, w + 256, w + 256 + copy, w + 256 + 2 * copy};
    double* rec = reinterpret_cast<double*>(w + 256 + 3 * copy);
    const int64_t n_rec = heom_record_count(n_steps, record_every);
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIP_TRY(hipMemsetAsync(status, 0, 4, st));
    heom::StageSpec sp[4];
    heom::rk4_stage_specs(sp);
    hipError_t e = heom::launch_block_record(state, obs, N, rec, status, st);
    for (int64_t step = 0; e == hipSuccess && step < n_steps; ++step) {
        for (int k = 0; k < 4 && e == hipSuccess; ++k) {
            const void* base[3];
            for (int m = 0; m < sp[k].nbase; ++m) base[m] = arr[sp[k].base[m]];
            e = heom::launch_block_stage(h->t, arr[sp[k].in], arr[sp[k].out], base, sp[k].wbase,
                                         sp[k].nbase, sp[k].w_in, sp[k].hmul * dt_fs, st);
        }
        if (e == hipSuccess && (step + 1) % record_every == 0)
            e = heom::launch_block_record(state, obs, N, rec + 6 * ((step + 1) / record_every),
                                          status, st);
    }
    if (e != hipSuccess) return fail(HEOM_E_DEVICE, "block stage launch: %s", hipGetErrorString(e));
    int32_t bad = 0;
    HIP_TRY(hipMemcpyAsync(&bad, status, 4, hipMemcpyDeviceToHost, st));
    if (host_out)
        HIP_TRY(hipMemcpyAsync(host_out, rec, (size_t)n_rec * 6 * 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (bad) return fail(HEOM_E_NUMERIC, "a recorded correlation was not finite");
    return HEOM_OK;
}

heom_status heom_emission_start(const heom_hierarchy* exc, heom_state exc_state,
                                const heom_hierarchy* full, heom_state full_state,
                                const double* mu, void* stream) {
    if (!exc || !full || !mu) return fail(HEOM_E_INVAL, "NULL hierarchy or mu");
    heom_status rc;
    if ((rc = check_state(exc, exc_state, "exc_state")) != HEOM_OK) return rc;
    if ((rc = check_state(full, full_state, "full_state")) != HEOM_OK) return rc;
    if (full->t.N != exc->t.N + 1 || full->t.W != exc->t.W || full->t.D != exc->t.D ||
        full->t.n_ado != exc->t.n_ado)
        return fail(HEOM_E_INVAL, "full must have N + 1 states and the same modes and depth as exc");
    if (exc->d.precision == HEOM_FP32_HERM || full->d.precision == HEOM_FP32_HERM)
        return fail(HEOM_E_INVAL, "emission start takes complex storage (FP64 or FP32-mixed)");
    for (int b = 0; b < exc->t.N; ++b)
        if (!is_finite(mu[b])) return fail(HEOM_E_INVAL, "mu[%d] is not finite", b);
    hipError_t e = heom::launch_emission_start(
        exc_state.sigma0, exc_state.rest, exc->d.precision == HEOM_FP64 ? 0 : 1, full_state.sigma0,
        full_state.rest, full->d.precision == HEOM_FP64 ? 0 : 1, mu, exc->t.N, exc->t.n_ado,
        static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail(HEOM_E_DEVICE, "emission start launch: %s", hipGetErrorString(e));
    return HEOM_OK;
}

heom_status heom_get_state(const heom_hierarchy* h, heom_state s, void* host_sigma0,
                           void* host_rest, void* stream) {
    if (!h) return fail(HEOM_E_INVAL, "hierarchy is NULL");
    heom_status rc;
    if ((rc = check_state(h, s, "state")) != HEOM_OK) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (host_sigma0)
        HIP_TRY(hipMemcpyAsync(host_sigma0, s.sigma0, h->info.sigma0_bytes, hipMemcpyDeviceToHost, st));
    if (host_rest && h->info.rest_bytes)
        HIP_TRY(hipMemcpyAsync(host_rest, s.rest, h->info.rest_bytes, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return HEOM_OK;
}

heom_status heom_set_state(const heom_hierarchy* h, heom_state s, const void* host_sigma0,
                           const void* host_rest, void* stream) {
    if (!h) return fail(HEOM_E_INVAL, "hierarchy is NULL");
    heom_status rc;
    if ((rc = check_state(h, s, "state")) != HEOM_OK) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (host_sigma0)
        HIP_TRY(hipMemcpyAsync(s.sigma0, host_sigma0, h->info.sigma0_bytes, hipMemcpyHostToDevice, st));
    if (host_rest && h->info.rest_bytes)
        HIP_TRY(hipMemcpyAsync(s.rest, host_rest, h->info.rest_bytes, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    return HEOM_OK;
}

heom_status heom_spectrum(const double* P, int32_t n_dir, int64_t n_t, double dt_fs,
                          const double* omega_cm, int64_t n_omega, double* S) {
    if (!P || !omega_cm || !S || n_dir < 1 || n_t < 2 || n_omega < 0 || !(dt_fs > 0.0))
        return fail(HEOM_E_INVAL, "spectrum: bad arguments");
    // Sum the directions first (the transform is linear), then one trapezoid
    // sum per frequency with the phase advanced by a rotation per sample.
    std::vector<double> pr(n_t, 0.0), pi(n_t, 0.0);
    for (int p = 0; p < n_dir; ++p)
        for (int64_t n = 0; n < n_t; ++n) {
            pr[n] += P[2 * (p * n_t + n)];
            pi[n] += P[2 * (p * n_t + n) + 1];
        }
    for (int64_t k = 0; k < n_omega; ++k) {
        const double w = omega_cm[k] * kCmToRadFs;
        double acc = 0.0;
        for (int64_t n = 0; n < n_t; ++n) {
            const double ph = w * dt_fs * (double)n;  // exact phase per sample, no recurrence drift
            const double c = std::cos(ph), sn = std::sin(ph);
            const double wt = (n == 0 || n == n_t - 1) ? 0.5 : 1.0;
            acc += wt * (c * pr[n] - sn * pi[n]);  // Re(e^{i ph} P)
        }
        S[k] = acc * dt_fs;
    }
    return HEOM_OK;
}

heom_status heom_destroy(heom_hierarchy* h) {
    delete h;
    return HEOM_OK;
}

}  // extern "C"
