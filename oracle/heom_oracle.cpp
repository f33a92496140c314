// HEOM oracle — TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, single-threaded FP64 implementation of the hierarchical
// equations of motion (HEOM) for Drude-Lorentz baths with a Matsubara or a
// Pade expansion, integrated with textbook classic RK4.  It exists to check the GPU
// library against; nothing in the product links, loads or calls it.  Only the
// test suite, the smoke check and the CPU-baseline leg of the benchmark may
// load this library.  It shares no code, header or table with the GPU path.
//
// Every function cites the passage of Kramer, Noack, Reinefeld, Rodriguez,
// Zelinskyy, "Efficient calculation of open quantum system dynamics and
// time-resolved spectroscopy with Distributed Memory HEOM (DM-HEOM)"
// (arXiv:1803.03498) that it follows.  Section names are the paper's.
//
// Conventions (readings of the paper where it is silent or ambiguous):
//   * hbar = 1: energies are angular frequencies in rad/fs.  Inputs arrive in
//     cm^-1, fs and K and are converted here.
//   * Mode index l = (sum of K_b over earlier baths) + k, 0-based, bath-major;
//     with the same K for every bath this is the 0-based form of the mode
//     relation l = (b-1)K + k + 1 (section "HEOM formalism").
//   * ADO order: by level |n| = 0..D, and descending lexicographic order of
//     the tuple within a level (the paper only asks for a consecutive
//     numbering).
//   * If |c_l| == 0 the rescaling uses the scale 1 for that mode.
//
// Parity pins for every function live in tests/ (marker "not gpu").

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <map>
#include <vector>

namespace {

using cplx = std::complex<double>;

// 2*pi*c in rad/fs per cm^-1 (c = 2.99792458e-5 cm/fs, exact).
const double kTwoPiC = 2.0 * M_PI * 2.99792458e-5;
// Boltzmann constant in cm^-1/K (CODATA: k_B/(h c)).
const double kBoltzmannCm = 0.6950348004;

enum : uint32_t {
    kNoRescale = 1u,      // use the un-rescaled couplings of the HEOM equation
    kNoTerminator = 2u,   // drop the low-temperature correction term
    kAddReorg = 4u,       // add lambda_b to the diagonal of H (eq. h-ex)
    kStandardGauge = 8u,  // flip the sign of both coupling terms
    kPade = 16u,          // Pade poles in place of the Matsubara frequencies
};

struct Mode {
    int bath;
    int k;
    int site;
    double gamma;  // gamma(b,k), 1/fs
    double c;      // c(b,k), rad/fs^2
    double lamnu;  // lambda_b nu_b for k = 0, else 0
};

struct Model {
    int N = 0, W = 0, D = 0;
    uint32_t flags = 0;
    std::vector<cplx> H;            // [N][N], rad/fs
    std::vector<Mode> modes;        // [W]
    std::vector<int> bath_site;     // [B]
    std::vector<double> bath_delta; // [B], 1/fs
    std::vector<std::vector<uint8_t>> tuples;
    std::vector<int> level;
    std::vector<int32_t> plus, minus;  // [n_ado][W]
};

}  // namespace

extern "C" {

typedef struct {
    int32_t n_states;
    const double* h_re;  // [N*N] cm^-1, row-major
    const double* h_im;  // [N*N] cm^-1 or NULL
    int32_t n_baths;
    const int32_t* bath_state;
    const double* bath_lambda_cm;
    const double* bath_tau_fs;
    const int32_t* bath_matsubara;
    double temperature_K;
    int32_t depth;
    uint32_t flags;
} orc_problem;

}  // extern "C"

namespace {

// All tuples of W non-negative integers with sum exactly L, in descending
// lexicographic order.  Brute force: every composition is generated, then
// sorted.  (Section "HEOM formalism": tuples with sum n_i <= D.)
void compositions(int W, int L, int pos, std::vector<uint8_t>& cur,
                  std::vector<std::vector<uint8_t>>& out) {
    if (pos == W - 1) {
        cur[pos] = (uint8_t)L;
        out.push_back(cur);
        return;
    }
    for (int v = 0; v <= L; ++v) {
        cur[pos] = (uint8_t)v;
        compositions(W, L - v, pos + 1, cur, out);
    }
}

int64_t count_compositions(int W, int L, int pos) {
    if (pos == W - 1) return 1;
    int64_t n = 0;
    for (int v = 0; v <= L; ++v) n += count_compositions(W, L - v, pos + 1);
    return n;
}

// Enumerate the hierarchy and the +/- link graph (section "HEOM formalism":
// the +/- connections and the mapping u -> {u+-} computed in a first step).
void build_tables(int W, int D, Model& m) {
    m.tuples.clear();
    m.level.clear();
    if (W == 0) {
        m.tuples.push_back({});
        m.level.push_back(0);
    } else {
        for (int L = 0; L <= D; ++L) {
            std::vector<std::vector<uint8_t>> lev;
            std::vector<uint8_t> cur(W, 0);
            compositions(W, L, 0, cur, lev);
            std::sort(lev.begin(), lev.end(), std::greater<std::vector<uint8_t>>());
            for (auto& t : lev) {
                m.tuples.push_back(t);
                m.level.push_back(L);
            }
        }
    }
    std::map<std::vector<uint8_t>, int32_t> index;
    for (size_t u = 0; u < m.tuples.size(); ++u) index[m.tuples[u]] = (int32_t)u;
    const size_t n = m.tuples.size();
    m.plus.assign(n * W, -1);
    m.minus.assign(n * W, -1);
    for (size_t u = 0; u < n; ++u) {
        for (int l = 0; l < W; ++l) {
            std::vector<uint8_t> t = m.tuples[u];
            if (m.level[u] + 1 <= D) {  // "+" valid if the new sum stays <= D
                t[l] += 1;
                m.plus[u * W + l] = index.at(t);
                t[l] -= 1;
            }
            if (t[l] >= 1) {  // "-" valid if every entry stays >= 0
                t[l] -= 1;
                m.minus[u * W + l] = index.at(t);
            }
        }
    }
}

// Eigenvalues of the real symmetric n x n matrix A (row-major) by cyclic
// Jacobi rotations, in descending order.
std::vector<double> sym_eigenvalues(std::vector<double> A, int n) {
    double total = 0.0;
    for (double x : A) total += x * x;
    for (int sweep = 0; sweep < 200; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += A[p * n + q] * A[p * n + q];
        if (off <= 1e-32 * total) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = A[p * n + q];
                if (apq == 0.0) continue;
                // rotation in the (p, q) plane that zeroes A[p][q]
                const double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {  // A <- A J
                    const double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = c * akp - s * akq;
                    A[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {  // A <- J^T A
                    const double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = c * apk - s * aqk;
                    A[q * n + k] = s * apk + c * aqk;
                }
            }
    }
    std::vector<double> ev(n);
    for (int i = 0; i < n; ++i) ev[i] = A[i * n + i];
    std::sort(ev.begin(), ev.end(), [](double x, double y) { return x > y; });
    return ev;
}

// Pade poles xi_i and residues eta_i, i = 1..K, of the Bose function, in the
// form the paper takes from Hu, Xu and Yan (section "HEOM formalism", the
// replacement of the Matsubara expansion): xi_i = 2 / (i-th largest
// eigenvalue of Lambda), zeta_j = 2 / (j-th largest eigenvalue of Lambda'),
//   eta_i = (K^2 + 3K/2) prod_{j<K} (zeta_j^2 - xi_i^2) / prod_{j != i} (xi_j^2 - xi_i^2).
// Lambda (2K x 2K) and Lambda' (2K-1 x 2K-1) are zero on the diagonal with
// 1/sqrt((2m+1)(2m+3)) and 1/sqrt((2m+3)(2m+5)) beside it, m = 1, 2, ...
void pade_poles(int K, double* xi, double* eta) {
    auto tridiag = [](int n, int shift) {
        std::vector<double> A((size_t)n * n, 0.0);
        for (int m = 1; m < n; ++m) {
            const double v = 1.0 / std::sqrt((2.0 * m + shift) * (2.0 * m + shift + 2.0));
            A[(size_t)(m - 1) * n + m] = v;
            A[(size_t)m * n + m - 1] = v;
        }
        return A;
    };
    const std::vector<double> ev = sym_eigenvalues(tridiag(2 * K, 1), 2 * K);
    const std::vector<double> evp = K > 1 ? sym_eigenvalues(tridiag(2 * K - 1, 3), 2 * K - 1)
                                          : std::vector<double>();
    std::vector<double> zeta(K > 1 ? K - 1 : 0);
    for (int i = 0; i < K; ++i) xi[i] = 2.0 / ev[i];
    for (int j = 0; j + 1 < K; ++j) zeta[j] = 2.0 / evp[j];
    for (int i = 0; i < K; ++i) {
        // the K-1 factors of the numerator and of the denominator taken in
        // pairs, so that the partial products stay in range for large K
        double r = K * K + 1.5 * K;
        for (int j = 0, jd = 0; j + 1 < K; ++j, ++jd) {
            if (jd == i) ++jd;
            r *= (zeta[j] * zeta[j] - xi[i] * xi[i]) / (xi[jd] * xi[jd] - xi[i] * xi[i]);
        }
        eta[i] = r;
    }
}

// Drude-Lorentz bath exponents and weights with the Pade expansion of K
// poles (section "HEOM formalism", the Pade replacements of gamma(b,k) and
// c(b,k); the sum in c(b,0) runs over the poles j) and the same correction
// coefficient as below.  Returns -1 if a pole rate equals nu.
int bath_coefficients_pade(double lambda_cm, double tau_fs, double T, int K, double* gamma,
                           double* c, double* lamnu, double* delta) {
    const double beta = 1.0 / (kBoltzmannCm * T * kTwoPiC);
    const double lam = lambda_cm * kTwoPiC;
    const double nu = 1.0 / tau_fs;
    std::vector<double> xi(K), eta(K);
    if (K > 0) pade_poles(K, xi.data(), eta.data());
    double c0 = 1.0;
    for (int j = 0; j < K; ++j) {
        const double a = xi[j] / beta;
        if (a == nu) return -1;
        c0 -= 2.0 * eta[j] * nu * nu / (a * a - nu * nu);
    }
    gamma[0] = nu;
    c[0] = 2.0 * lam / beta * c0;
    double sum = c[0] / gamma[0];
    for (int k = 1; k <= K; ++k) {
        const double a = xi[k - 1] / beta;
        gamma[k] = a;
        c[k] = 4.0 * lam * nu / beta * eta[k - 1] * a / (a * a - nu * nu);
        sum += c[k] / gamma[k];
    }
    *lamnu = lam * nu;
    *delta = 2.0 * lam / (beta * nu) - sum;
    return 0;
}

// Drude-Lorentz bath exponents and weights with the Matsubara expansion
// (section "HEOM formalism", definitions of gamma(b,k) and c(b,k)) and the
// low-temperature correction coefficient of the third line of eq. (HEOM).
// hbar = 1, so beta*hbar = 1/(k_B T) in fs.
void bath_coefficients(double lambda_cm, double tau_fs, double T, int M,
                       double* gamma, double* c, double* lamnu, double* delta) {
    const double beta = 1.0 / (kBoltzmannCm * T * kTwoPiC);
    const double lam = lambda_cm * kTwoPiC;
    const double nu = 1.0 / tau_fs;
    double sum = 0.0;
    for (int k = 0; k <= M; ++k) {
        if (k == 0) {
            gamma[0] = nu;
            c[0] = nu * lam / std::tan(beta * nu / 2.0);
        } else {
            gamma[k] = 2.0 * M_PI * k / beta;
            c[k] = 4.0 * lam * nu / beta * gamma[k] / (gamma[k] * gamma[k] - nu * nu);
        }
        sum += c[k] / gamma[k];
    }
    *lamnu = lam * nu;
    *delta = 2.0 * lam / (beta * nu) - sum;
}

int build_model(const orc_problem* p, Model& m) {
    if (!p || p->n_states < 1 || p->depth < 0 || p->n_baths < 0) return -1;
    if (!(p->temperature_K > 0.0)) return -1;
    m.N = p->n_states;
    m.D = p->depth;
    m.flags = p->flags;
    const int N = m.N;
    m.H.assign((size_t)N * N, 0.0);
    for (int i = 0; i < N * N; ++i)
        m.H[i] = cplx(p->h_re[i], p->h_im ? p->h_im[i] : 0.0);
    m.modes.clear();
    m.bath_site.clear();
    m.bath_delta.clear();
    for (int b = 0; b < p->n_baths; ++b) {
        const int s = p->bath_state[b];
        const int M = p->bath_matsubara[b];
        if (s < 0 || s >= N || M < 0) return -1;
        if (!(p->bath_tau_fs[b] > 0.0) || !(p->bath_lambda_cm[b] >= 0.0)) return -1;
        std::vector<double> g(M + 1), c(M + 1);
        double lamnu = 0.0, delta = 0.0;
        if (m.flags & kPade) {
            if (bath_coefficients_pade(p->bath_lambda_cm[b], p->bath_tau_fs[b], p->temperature_K,
                                       M, g.data(), c.data(), &lamnu, &delta))
                return -1;
        } else {
            bath_coefficients(p->bath_lambda_cm[b], p->bath_tau_fs[b], p->temperature_K, M,
                              g.data(), c.data(), &lamnu, &delta);
        }
        for (int k = 0; k <= M; ++k)
            m.modes.push_back(Mode{b, k, s, g[k], c[k], k == 0 ? lamnu : 0.0});
        m.bath_site.push_back(s);
        m.bath_delta.push_back(delta);
        if (m.flags & kAddReorg) m.H[(size_t)s * N + s] += p->bath_lambda_cm[b];
    }
    for (auto& h : m.H) h *= kTwoPiC;
    m.W = (int)m.modes.size();
    build_tables(m.W, m.D, m);
    return 0;
}

// Right-hand side of eq. (HEOM) for one ADO u, written element by element with
// the superoperator masks of the section "HEOM formalism":
//   (V_s^x A)_ij = (d_is - d_sj) A_ij
//   (V_s^x V_s^x A)_ij = (1 - d_ij)(d_is + d_sj) A_ij
//   (V_s^o A)_ij = (d_is + d_sj) A_ij
// and the rescaled couplings sqrt((n+1)|c|) and sqrt(n/|c|) of the ADO
// rescaling substitution.
void rhs_ado(const Model& m, const cplx* in, cplx* out, size_t u) {
    const int N = m.N, W = m.W;
    const size_t NN = (size_t)N * N;
    const cplx I(0.0, 1.0);
    const cplx* s = in + u * NN;
    const std::vector<uint8_t>& n = m.tuples[u];
    const bool rescale = !(m.flags & kNoRescale);
    const double sign = (m.flags & kStandardGauge) ? -1.0 : 1.0;

    // Second line of eq. (HEOM): sum over modes of n_{u,(b,k)} gamma(b,k).
    double damp = 0.0;
    for (int l = 0; l < W; ++l) damp += n[l] * m.modes[l].gamma;

    for (int i = 0; i < N; ++i) {
        for (int j = 0; j < N; ++j) {
            // First line: -i [H, sigma_u].
            cplx comm = 0.0;
            for (int k = 0; k < N; ++k)
                comm += m.H[(size_t)i * N + k] * s[(size_t)k * N + j] -
                        s[(size_t)i * N + k] * m.H[(size_t)k * N + j];
            cplx v = -I * comm;
            v -= damp * s[(size_t)i * N + j];
            // Third line: low-temperature correction, one V^x V^x per bath.
            if (!(m.flags & kNoTerminator)) {
                for (size_t b = 0; b < m.bath_site.size(); ++b) {
                    const int sb = m.bath_site[b];
                    const double mask = (i != j) ? (double)((i == sb) + (sb == j)) : 0.0;
                    v -= m.bath_delta[b] * mask * s[(size_t)i * N + j];
                }
            }
            // Fourth and fifth lines: couplings to sigma^+ and sigma^-.
            for (int l = 0; l < W; ++l) {
                const Mode& md = m.modes[l];
                const double vx = (double)((i == md.site) - (md.site == j));
                const double vo = (double)((i == md.site) + (md.site == j));
                const double ac = std::fabs(md.c);
                const int32_t up = m.plus[u * W + l];
                if (up >= 0) {
                    double scale = 1.0;
                    if (rescale) scale = std::sqrt((n[l] + 1.0) * (ac > 0.0 ? ac : 1.0));
                    v += sign * I * scale * vx * in[(size_t)up * NN + (size_t)i * N + j];
                }
                const int32_t dn = m.minus[u * W + l];
                if (dn >= 0) {
                    double scale = (double)n[l];
                    if (rescale) scale = std::sqrt(n[l] / (ac > 0.0 ? ac : 1.0));
                    const cplx theta = I * md.c * vx + (md.k == 0 ? md.lamnu * vo : 0.0);
                    v += sign * scale * theta * in[(size_t)dn * NN + (size_t)i * N + j];
                }
            }
            out[u * NN + (size_t)i * N + j] = v;
        }
    }
}

void rhs_all(const Model& m, const cplx* in, cplx* out) {
    for (size_t u = 0; u < m.tuples.size(); ++u) rhs_ado(m, in, out, u);
}

// Observables of sigma_0 (the reduced density matrix, section "HEOM
// formalism"; polarisation P(t) = Tr[rho mu^+], eq. polarization, with the
// dipole operator of eq. mu_plusp).
//   kind 0 (populations): [Re rho_mm for m] + [Re Tr, Im Tr] + [max |rho - rho^dagger|]
//   kind 1 (dipole):      [Re P, Im P, Re Tr, Im Tr], P = sum_a mu_a rho[a][g]
void record(const Model& m, const cplx* rho, int kind, const double* mu, int ground,
            double* rec) {
    const int N = m.N;
    cplx tr = 0.0;
    for (int i = 0; i < N; ++i) tr += rho[(size_t)i * N + i];
    if (kind == 0) {
        double herm = 0.0;
        for (int i = 0; i < N; ++i) {
            rec[i] = rho[(size_t)i * N + i].real();
            for (int j = 0; j < N; ++j)
                herm = std::max(herm, std::abs(rho[(size_t)i * N + j] -
                                               std::conj(rho[(size_t)j * N + i])));
        }
        rec[N] = tr.real();
        rec[N + 1] = tr.imag();
        rec[N + 2] = herm;
    } else {
        cplx P = 0.0;
        for (int a = 0; a < N; ++a) P += mu[a] * rho[(size_t)a * N + ground];
        rec[0] = P.real();
        rec[1] = P.imag();
        rec[2] = tr.real();
        rec[3] = tr.imag();
    }
}

int record_size(int N, int kind) { return kind == 0 ? N + 3 : 4; }

}  // namespace

extern "C" {

// Number of ADOs by enumerating every tuple with sum <= D (eq. Nmatrices
// gives the closed form this must equal).  No storage.
int orc_count(int32_t W, int32_t D, int64_t* n_out) {
    if (W < 0 || D < 0 || !n_out) return -1;
    if (W == 0) {
        *n_out = 1;
        return 0;
    }
    int64_t n = 0;
    for (int L = 0; L <= D; ++L) n += count_compositions(W, L, 0);
    *n_out = n;
    return 0;
}

// Tuples [n][W] (uint8), plus/minus link tables [n][W] (int32, -1 = absent).
// Arrays must hold `capacity` ADOs; *n_out receives the count.
int orc_tables(int32_t W, int32_t D, int64_t capacity, uint8_t* tuples, int32_t* plus,
               int32_t* minus, int32_t* level, int64_t* n_out) {
    if (W < 0 || D < 0 || D > 255) return -1;
    Model m;
    build_tables(W, D, m);
    const int64_t n = (int64_t)m.tuples.size();
    *n_out = n;
    if (n > capacity) return -2;
    for (int64_t u = 0; u < n; ++u) {
        for (int l = 0; l < W; ++l) {
            if (tuples) tuples[u * W + l] = m.tuples[u][l];
            if (plus) plus[u * W + l] = m.plus[u * W + l];
            if (minus) minus[u * W + l] = m.minus[u * W + l];
        }
        if (level) level[u] = m.level[u];
    }
    return 0;
}

// Coefficients of one bath: gamma[0..M], c[0..M], lambda*nu, Delta.
int orc_bath_coefficients(double lambda_cm, double tau_fs, double T_K, int32_t M,
                          double* gamma, double* c, double* lamnu, double* delta) {
    if (M < 0 || !(T_K > 0.0) || !(tau_fs > 0.0)) return -1;
    bath_coefficients(lambda_cm, tau_fs, T_K, M, gamma, c, lamnu, delta);
    return 0;
}

// Pade poles and residues of the Bose function, K >= 1.
int orc_pade_poles(int32_t K, double* xi, double* eta) {
    if (K < 1) return -1;
    pade_poles(K, xi, eta);
    return 0;
}

// Coefficients of one bath with K Pade poles: gamma[0..K], c[0..K], lambda*nu, Delta.
int orc_bath_coefficients_pade(double lambda_cm, double tau_fs, double T_K, int32_t K,
                               double* gamma, double* c, double* lamnu, double* delta) {
    if (K < 0 || !(T_K > 0.0) || !(tau_fs > 0.0)) return -1;
    return bath_coefficients_pade(lambda_cm, tau_fs, T_K, K, gamma, c, lamnu, delta);
}

int orc_model_sizes(const orc_problem* p, int32_t* W, int64_t* n_ado) {
    Model m;
    if (build_model(p, m)) return -1;
    *W = m.W;
    *n_ado = (int64_t)m.tuples.size();
    return 0;
}

// One evaluation of eq. (HEOM) for ADOs [u_begin, u_end) (u_end < 0: all).
// `in` and `out` are interleaved complex [n_ado][N][N].
int orc_rhs(const orc_problem* p, const double* in, double* out, int64_t u_begin,
            int64_t u_end) {
    Model m;
    if (build_model(p, m)) return -1;
    const int64_t n = (int64_t)m.tuples.size();
    if (u_end < 0 || u_end > n) u_end = n;
    if (u_begin < 0) u_begin = 0;
    const cplx* ci = reinterpret_cast<const cplx*>(in);
    cplx* co = reinterpret_cast<cplx*>(out);
    for (int64_t u = u_begin; u < u_end; ++u) rhs_ado(m, ci, co, (size_t)u);
    return 0;
}

// Textbook classic RK4 (four evaluations per step, section "Distributed
// memory HEOM implementation": four copies and four evaluations per step):
//   k1 = f(y), k2 = f(y + dt/2 k1), k3 = f(y + dt/2 k2), k4 = f(y + dt k3),
//   y <- y + dt/6 (k1 + 2 k2 + 2 k3 + k4).
// `state` (interleaved complex [n_ado][N][N]) is advanced in place.  Records
// are taken at step 0 and after every `record_every` steps into
// records[n_rec][record_size].
int orc_propagate(const orc_problem* p, double* state, double dt_fs, int64_t n_steps,
                  int32_t record_every, int32_t obs_kind, const double* mu, int32_t ground,
                  double* records) {
    Model m;
    if (build_model(p, m)) return -1;
    if (record_every < 1 || n_steps < 0) return -1;
    const size_t n = m.tuples.size() * (size_t)m.N * m.N;
    cplx* y = reinterpret_cast<cplx*>(state);
    std::vector<cplx> k1(n), k2(n), k3(n), k4(n), t(n);
    const int rs = record_size(m.N, obs_kind);
    int64_t r = 0;
    if (records) record(m, y, obs_kind, mu, ground, records + (r++) * rs);
    for (int64_t step = 0; step < n_steps; ++step) {
        rhs_all(m, y, k1.data());
        for (size_t i = 0; i < n; ++i) t[i] = y[i] + 0.5 * dt_fs * k1[i];
        rhs_all(m, t.data(), k2.data());
        for (size_t i = 0; i < n; ++i) t[i] = y[i] + 0.5 * dt_fs * k2[i];
        rhs_all(m, t.data(), k3.data());
        for (size_t i = 0; i < n; ++i) t[i] = y[i] + dt_fs * k3[i];
        rhs_all(m, t.data(), k4.data());
        for (size_t i = 0; i < n; ++i)
            y[i] += dt_fs / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
        if (records && (step + 1) % record_every == 0)
            record(m, y, obs_kind, mu, ground, records + (r++) * rs);
    }
    return 0;
}

// Timing only (for the CPU baseline): the work that one orc_propagate step
// does for the ADOs u_begin, u_begin + stride, ... below u_end -- their four
// evaluations and their share of the vector updates, with the same code --
// timed on a steady clock after the model is built (table construction stays
// out of the figure); the smallest of `repeats` timings goes to *seconds.
// Neighbours that are not sampled are read as zeros (the stage arrays are
// calloc'ed and only the sampled ADOs are written); `state` is not changed.
int orc_time_step_sample(const orc_problem* p, const double* state, double dt_fs,
                         int64_t u_begin, int64_t u_end, int64_t stride, int32_t repeats,
                         double* seconds) {
    Model m;
    if (build_model(p, m) || !seconds || stride < 1 || repeats < 1) return -1;
    const int64_t n_ado = (int64_t)m.tuples.size();
    if (u_end < 0 || u_end > n_ado) u_end = n_ado;
    if (u_begin < 0) u_begin = 0;
    if (u_begin > u_end) return -1;
    const size_t NN = (size_t)m.N * m.N, n = (size_t)n_ado * NN;
    const cplx* y = reinterpret_cast<const cplx*>(state);
    cplx* buf[5];
    for (int b = 0; b < 5; ++b) {
        buf[b] = static_cast<cplx*>(std::calloc(n, sizeof(cplx)));
        if (!buf[b]) {
            for (int c = 0; c < b; ++c) std::free(buf[c]);
            return -2;
        }
    }
    cplx *k1 = buf[0], *k2 = buf[1], *k3 = buf[2], *k4 = buf[3], *t = buf[4];
    double best = 0.0;
    for (int r = 0; r < repeats; ++r) {
        const auto t0 = std::chrono::steady_clock::now();
        for (int64_t u = u_begin; u < u_end; u += stride) rhs_ado(m, y, k1, (size_t)u);
        for (int64_t u = u_begin; u < u_end; u += stride)
            for (size_t i = u * NN; i < (u + 1) * NN; ++i) t[i] = y[i] + 0.5 * dt_fs * k1[i];
        for (int64_t u = u_begin; u < u_end; u += stride) rhs_ado(m, t, k2, (size_t)u);
        for (int64_t u = u_begin; u < u_end; u += stride)
            for (size_t i = u * NN; i < (u + 1) * NN; ++i) t[i] = y[i] + 0.5 * dt_fs * k2[i];
        for (int64_t u = u_begin; u < u_end; u += stride) rhs_ado(m, t, k3, (size_t)u);
        for (int64_t u = u_begin; u < u_end; u += stride)
            for (size_t i = u * NN; i < (u + 1) * NN; ++i) t[i] = y[i] + dt_fs * k3[i];
        for (int64_t u = u_begin; u < u_end; u += stride) rhs_ado(m, t, k4, (size_t)u);
        for (int64_t u = u_begin; u < u_end; u += stride)
            for (size_t i = u * NN; i < (u + 1) * NN; ++i)
                t[i] = y[i] + dt_fs / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
        const double sec =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        best = r == 0 ? sec : std::min(best, sec);
    }
    *seconds = best;
    for (int b = 0; b < 5; ++b) std::free(buf[b]);
    return 0;
}

// Linear absorption, eq. lin_abs_mukamel, on a finite time window with the
// trapezoid rule: S(w_k) = Re sum_p sum_n w_n exp(i w_k t_n) P_p(t_n) dt,
// w_0 = w_last = 1/2.  P is interleaved complex [n_dir][n_t]; omega in cm^-1.
int orc_spectrum(const double* P, int32_t n_dir, int64_t n_t, double dt_fs,
                 const double* omega_cm, int64_t n_omega, double* S) {
    if (n_t < 2 || n_dir < 1) return -1;
    const cplx I(0.0, 1.0);
    for (int64_t k = 0; k < n_omega; ++k) {
        const double w = omega_cm[k] * kTwoPiC;
        cplx acc = 0.0;
        for (int p = 0; p < n_dir; ++p) {
            for (int64_t q = 0; q < n_t; ++q) {
                const double wt = (q == 0 || q == n_t - 1) ? 0.5 : 1.0;
                const cplx Pq(P[2 * (p * n_t + q)], P[2 * (p * n_t + q) + 1]);
                acc += wt * std::exp(I * (w * q * dt_fs)) * Pq * dt_fs;
            }
        }
        S[k] = acc.real();
    }
    return 0;
}

}  // extern "C"
