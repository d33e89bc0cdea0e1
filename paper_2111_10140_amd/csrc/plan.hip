// Plan construction and the C ABI around one matvec (host side).
//
// For each feature window the plan fixes the fast-summation parameters of
// Sec. 4.2: the period h (h >= 2 * extent, so differences of scaled nodes stay
// inside one period), the bandwidth M of the index set I_M (Sec. 4.1), the
// oversampled FFT length n and the window half-width m.  The kernel's Fourier
// coefficients b_k are the DFT of M equidistant samples of the h-periodised
// Gaussian (Sec. 4.2); they are divided by the squared window transform so
// that one multiplication performs both deconvolutions.  Points are binned
// into grid cells and sorted by grid tile for the spreading and gathering
// kernels.
#include <algorithm>
#include <map>
#include <cmath>
#include <cstring>
#include <limits>
#include <numeric>

#include "anova_internal.h"

namespace anova {

static thread_local std::string g_last_error;
void set_error(const std::string &msg) { g_last_error = msg; }
const char *get_error() { return g_last_error.c_str(); }

namespace {

constexpr double kPi = 3.14159265358979323846;

// ------------------------------------------------------------- special functions
// Modified Bessel function I0 by its power series sum ((x/2)^2k / (k!)^2):
// all terms positive, so the sum is accurate to rounding for the arguments
// used here (0 <= x <= 60).
double bessel_i0(double x) {
    const double q = 0.25 * x * x;
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 500; ++k) {
        term *= q / ((double)k * (double)k);
        sum += term;
        if (term < 1e-17 * sum) break;
    }
    return sum;
}

// Kaiser-Bessel window in grid units, phi0(t) = I0(b sqrt(1-(t/m)^2)) for
// |t| <= m, 0 outside, and its continuous Fourier transform
// 2m sinh(s)/s with s = sqrt(b^2 - (2 pi m xi)^2) (sin(s)/s past the root).
double kb_phi(double t, int m, double b) {
    if (std::fabs(t) > m) return 0.0;
    const double u = 1.0 - (t / m) * (t / m);
    return bessel_i0(b * std::sqrt(std::max(u, 0.0)));
}
double kb_phihat(double xi, int m, double b) {
    const double q = b * b - (2.0 * kPi * m * xi) * (2.0 * kPi * m * xi);
    if (q > 1e-12) {
        const double s = std::sqrt(q);
        return 2.0 * m * std::sinh(s) / s;
    }
    if (q < -1e-12) {
        const double s = std::sqrt(-q);
        return 2.0 * m * std::sin(s) / s;
    }
    return 2.0 * m;
}

// ------------------------------------------------------------- kernel coefficients
// 1-D Fourier coefficients of the h-periodised Gaussian exp(-r^2/ell^2)
// (Poisson summation); used only for the plan's error estimates.
double gauss_coeff(double k, double ell, double h) {
    const double a = kPi * ell * k / h;
    return std::sqrt(kPi) * ell / h * std::exp(-a * a);
}

// h-periodised 1-D Gaussian: sum over images r + j h.
double periodized_gauss(double r, double ell, double h) {
    double s = 0.0;
    const int J = 2 + (int)std::ceil(8.0 * ell / h);
    for (int j = -J; j <= J; ++j) {
        const double z = (r + j * h) / ell;
        s += std::exp(-z * z);
    }
    return s;
}

// b1[k + M/2], k = -M/2..M/2-1: DFT of the M equidistant samples
// samp[j + M/2] = kappa~(j h / M), j = -M/2..M/2-1, divided by M.  The
// kernel is a product over dimensions, and so is its sampled DFT:
// b_k = prod_t b1[k_t].  The samples are even in j, so the coefficients
// are real.
std::vector<double> coeffs_from_samples(const std::vector<double> &samp) {
    const int M = (int)samp.size();
    std::vector<double> b(M);
    for (int k = -M / 2; k < M / 2; ++k) {
        long double acc = 0.0L;
        for (int j = -M / 2; j < M / 2; ++j) {
            const long long kj = ((long long)k * j) % M;
            acc += (long double)samp[j + M / 2] *
                   std::cos(2.0L * (long double)kPi * (long double)kj / (long double)M);
        }
        b[k + M / 2] = (double)(acc / M);
    }
    return b;
}

// Coefficients of the h-periodised Gaussian.
std::vector<double> sampled_coeffs_1d(int M, double ell, double h) {
    std::vector<double> samp(M);
    for (int j = -M / 2; j < M / 2; ++j) samp[j + M / 2] = periodized_gauss(j * h / M, ell, h);
    return coeffs_from_samples(samp);
}

// ------------------------------------------------------------- regularised kernel
// Sec. 4.2's regularisation, applied to each 1-D factor g(r) = exp(-r^2/ell^2)
// of the Gaussian: g~ = g on [-L, L] (every coordinate difference of the
// points lies there), and on (L, h - L) the polynomial that matches g's
// derivatives of orders 0..q at r = L and those of its periodic
// continuation g(r - h) at r = h - L, so that the h-periodic g~ is q times
// continuously differentiable.  The product of the factors equals the
// kernel wherever the points can be, so only the truncation of g~'s
// Fourier series is an error there.

// j-th derivative of g at r: (-1/ell)^j H_j(r/ell) g(r), H_j the physicists'
// Hermite polynomials (H_{j+1} = 2u H_j - 2j H_{j-1}).
double gauss_deriv(int j, double r, double ell) {
    const double u = r / ell;
    double h0 = 1.0, h1 = 2.0 * u;
    double Hj = j == 0 ? h0 : h1;
    for (int k = 1; k < j; ++k) {
        const double h2 = 2.0 * u * h1 - 2.0 * k * h0;
        h0 = h1;
        h1 = h2;
        Hj = h1;
    }
    return std::pow(-1.0 / ell, j) * Hj * std::exp(-u * u);
}

// g~(r) for |r| <= h/2 (h > 2L).  On t = (|r| - L) / (h - 2L) in (0, 1) the
// two-point Taylor interpolant with A_j, B_j the t-derivatives at t = 0 and
// t = 1:  p(t) = (1-t)^(q+1) sum_j A_j t^j / j! sum_{k<=q-j} C(q+k, k) t^k
//              + t^(q+1) sum_j B_j (t-1)^j / j! sum_{k<=q-j} C(q+k, k) (1-t)^k,
// A_j = w^j g^(j)(L), B_j = (-1)^j A_j (the continuation is g mirrored).
double reg_gauss(double r, double ell, double L, double h, int q) {
    r = std::fabs(r);
    if (r <= L) return std::exp(-(r / ell) * (r / ell));
    const double w = h - 2.0 * L, t = (r - L) / w;
    double s0 = 0.0, s1 = 0.0, wj = 1.0, fact = 1.0;
    for (int j = 0; j <= q; ++j) {
        if (j > 0) {
            wj *= w;
            fact *= j;
        }
        const double Aj = wj * gauss_deriv(j, L, ell);
        const double Bj = (j % 2 ? -1.0 : 1.0) * Aj;
        double in0 = 0.0, in1 = 0.0, binom = 1.0, tk = 1.0, uk = 1.0;
        for (int k = 0; k <= q - j; ++k) {
            if (k > 0) {
                binom = binom * (q + k) / k;
                tk *= t;
                uk *= 1.0 - t;
            }
            in0 += binom * tk;
            in1 += binom * uk;
        }
        s0 += Aj * std::pow(t, j) / fact * in0;
        s1 += Bj * std::pow(t - 1.0, j) / fact * in1;
    }
    return std::pow(1.0 - t, q + 1) * s0 + std::pow(t, q + 1) * s1;
}

std::vector<double> reg_coeffs_1d(int M, double ell, double h, double L, int q) {
    std::vector<double> samp(M);
    for (int j = -M / 2; j < M / 2; ++j) samp[j + M / 2] = reg_gauss(j * h / M, ell, L, h, q);
    return coeffs_from_samples(samp);
}

// Largest error on [-L, L] of the 1-D series sum_{|k| < M/2} b1_k e^{2 pi i k r / h}
// against g, measured on 1024 points (the sampled coefficients' aliasing
// included), times 1.25 for the points between.
double reg_err1(const std::vector<double> &b1, double ell, double h, double L) {
    const int M = (int)b1.size();
    double e = 0.0;
    for (int i = 0; i <= 1024; ++i) {
        const double r = L * i / 1024.0;
        double v = b1[M / 2];
        for (int k = 1; k < M / 2; ++k) v += 2.0 * b1[k + M / 2] * std::cos(2.0 * kPi * k * r / h);
        e = std::max(e, std::fabs(v - std::exp(-(r / ell) * (r / ell))));
    }
    return 1.25 * e;
}

// Per-entry error of the d_A-fold product of factors each within e1 of
// factors of size <= 1.
double reg_trunc_dA(double e1, int dA) { return dA * e1 * std::pow(1.0 + e1, dA - 1); }

// ------------------------------------------------------------- error model
// Per-entry error estimates of one window's approximation K~_ij - K_ij for
// |x_i - x_j| <= D per coordinate, before the weight eta.
double est_images(double h, double D, double ell, int dA) {
    const double g = h - D;
    if (g <= 0) return std::numeric_limits<double>::infinity();
    return 2.0 * dA * std::exp(-(g * g) / (ell * ell));
}

// (S' + T)^d - S'^d with T the tail of the coefficient sum outside
// |k| < M/2, doubled for the aliasing of the sampled coefficients.
double est_trunc(int M, double h, double ell, int dA) {
    double inner = 0.0, tail = 0.0;
    for (int k = -(M / 2 - 1); k <= M / 2 - 1; ++k) inner += gauss_coeff(k, ell, h);
    for (int k = M / 2; k < M / 2 + 100000; ++k) {
        const double c = gauss_coeff(k, ell, h);
        tail += 2.0 * c;
        if (c < 1e-300 || c < 1e-18 * tail) break;
    }
    double d = 0.0;  // binomial expansion without cancellation
    double binom = 1.0;
    for (int j = 1; j <= dA; ++j) {
        binom = binom * (dA - j + 1) / j;
        d += binom * std::pow(inner, dA - j) * std::pow(tail, j);
    }
    return 2.0 * d;
}

// Window aliasing: for each kept frequency the relative weight of its
// aliases k + r n in the window transform, plus the jump of the truncated
// window at |t| = m; combined over dimensions and over the adjoint and the
// forward transform, weighted by the kernel coefficients.
double est_window_b(const std::vector<double> &b1, int n, int m, int dA) {
    const int M = (int)b1.size();
    const double b = kPi * m * (2.0 - (double)M / n);
    const double i0b = bessel_i0(b);
    const double jump = 1.0 / i0b;
    double B = 0.0, BA = 0.0;
    for (int k = -(M / 2 - 1); k <= M / 2 - 1; ++k) {
        const double c = std::fabs(b1[k + M / 2]);
        const double ph0 = kb_phihat((double)k / n, m, b) / i0b;
        double alias = 0.0;
        for (int r = 1; r <= 8; ++r) {
            alias += std::fabs(kb_phihat((double)(k + r * n) / n, m, b)) / i0b;
            alias += std::fabs(kb_phihat((double)(k - r * n) / n, m, b)) / i0b;
        }
        alias += 2.0 * jump;
        B += c;
        BA += c * alias / ph0;
    }
    double d = 0.0, binom = 1.0;
    for (int j = 1; j <= dA; ++j) {
        binom = binom * (dA - j + 1) / j;
        d += binom * std::pow(B, dA - j) * std::pow(BA, j);
    }
    return 2.0 * d;
}

double est_window(int M, int n, int m, double ell, double h, int dA) {
    return est_window_b(sampled_coeffs_1d(M, ell, h), n, m, dA);
}

double est_round(int precision, int n, int m, int dA) {
    const double eps = precision == ANOVA_FP64 ? 1.1e-16 : 6.0e-8;
    // plus the fixed-point spreading: each of the (2m)^dA contributions of a
    // point is rounded at 2^-51 (float64) or 2^-31 (float32) of the largest
    // |alpha| of its workgroup, at most ||alpha||_1
    const double fix = std::pow(2.0 * m, dA) * (precision == ANOVA_FP64 ? 0x1p-51 : 0x1p-31);
    return eps * 8.0 * (dA * std::log2((double)n) + 2.0 * m) + fix;
}

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// ------------------------------------------------------------- window polynomials
// Fit phi0(f + m - 1 - a) / I0(b), f in [0,1), for a = 0..2m-1, by
// interpolation at the deg+1 Chebyshev points in z = 2f-1; returns monomial
// coefficients in z ([a][deg+1]) and the largest error on a fine sample.
std::vector<double> fit_window_polys(int m, double b, int deg, double &err_out) {
    const int W = 2 * m;
    const double i0b = bessel_i0(b);
    const int npts = deg + 1;
    std::vector<double> coef((size_t)W * npts);
    double worst = 0.0;
    for (int a = 0; a < W; ++a) {
        std::vector<double> fz(npts), cheb(npts, 0.0);
        for (int i = 0; i < npts; ++i) {
            const double z = std::cos(kPi * (i + 0.5) / npts);
            fz[i] = kb_phi(0.5 * (z + 1.0) + m - 1 - a, m, b) / i0b;
        }
        for (int j = 0; j < npts; ++j) {
            double s = 0.0;
            for (int i = 0; i < npts; ++i) s += fz[i] * std::cos(kPi * j * (i + 0.5) / npts);
            cheb[j] = (j == 0 ? 1.0 : 2.0) * s / npts;
        }
        // sum_j cheb_j T_j(z) in monomials, with T_{j+1} = 2z T_j - T_{j-1}
        std::vector<double> T0(npts, 0.0), T1(npts, 0.0), mono(npts, 0.0);
        T0[0] = 1.0;
        for (int i = 0; i < npts; ++i) mono[i] += cheb[0] * T0[i];
        if (npts > 1) {
            T1[1] = 1.0;
            for (int i = 0; i < npts; ++i) mono[i] += cheb[1] * T1[i];
        }
        for (int j = 2; j < npts; ++j) {
            std::vector<double> T2(npts, 0.0);
            for (int i = 0; i < npts; ++i) {
                if (i > 0) T2[i] += 2.0 * T1[i - 1];
                T2[i] -= T0[i];
            }
            for (int i = 0; i < npts; ++i) mono[i] += cheb[j] * T2[i];
            T0 = T1;
            T1 = T2;
        }
        for (int i = 0; i < npts; ++i) coef[(size_t)a * npts + i] = mono[i];
        for (int s = 0; s <= 256; ++s) {
            const double f = s / 256.0 * (1.0 - 1e-12);
            const double z = 2.0 * f - 1.0;
            double v = 0.0;
            for (int i = deg; i >= 0; --i) v = v * z + mono[i];
            worst = std::max(worst, std::fabs(v - kb_phi(f + m - 1 - a, m, b) / i0b));
        }
    }
    err_out = worst;
    return coef;
}

// ------------------------------------------------------------- per-cell launch model
// A per-cell launch of B workgroups runs in ceil(B / R) rounds of the R
// workgroups the device holds at once; a round lasts as long as its
// workgroups' largest per-lane share of one cell's points (a chunk of K
// takes 1/K of every cell of its tile, split over S lanes) plus a fixed part
// per workgroup (set-up, flush and region sum, about four points' worth,
// as measured on the 3-D m = 3 kernels).  Returns
// the K in 1..256 with the shortest modelled time (ties: fewer chunks).
static int best_chunks(int64_t tiles, int64_t maxcnt, int S, int64_t R, double &time) {
    int bestK = 1;
    double best = std::numeric_limits<double>::infinity();
    const int kmax = (int)std::max<int64_t>(1, std::min<int64_t>(256, maxcnt / std::max(S, 1)));
    for (int K = 1; K <= kmax; ++K) {
        const int64_t rounds = (tiles * K + R - 1) / R;
        const int64_t share = ((int64_t)S * K);
        const double t = (double)rounds * (double)((maxcnt + share - 1) / share + 4);
        if (t < best) {
            best = t;
            bestK = K;
        }
    }
    time = best;
    return bestK;
}

// ------------------------------------------------------------- parameter choice
struct Choice {
    double h;
    int M, n, m;
    double e_img, e_trunc, e_win, e_round;
    double cost;     // model cost (see candidates)
    int align = 0;   // > 0: tile edge the data is aligned to (per-cell kernels)
};

// Every (n, M, m) meeting the error budget, one per FFT length n (the
// smallest M, then the smallest m), cheapest model cost first.  Fixed
// parameters give one candidate.
//
// Model cost: N (2m)^dA / eff + 4 n^dA log2(n) dA, eff the lane efficiency
// of the spreading and gathering kernels at the points' density (eff_of).
// For float32 windows that
// will run the per-cell kernels (support width supported and several points
// per cell) there is also an aligned variant: a wave of those kernels covers
// a slab of cells and runs as long as its fullest cell, so points that end
// inside a tile leave lanes idle; the variant raises h so that the points
// span a whole number of tiles (one tile fewer) with M and m chosen again
// for that h, and puts the data's lower edge on a tile boundary (centre
// chosen in make_plan).  It is placed just before its plain twin when the
// per-cell launch model (best_chunks) says it runs faster, else just after.
// Regularised kernel (prm.reg_q > 0): the period is prm.h (> 2D) or the
// cheapest of 2.5, 3 and 4 times D; at each (h, n) the smallest m, then the
// smallest M, whose measured truncation error (reg_err1) plus the window
// and rounding estimates fit the budget.  There is no image error: the
// regularised kernel equals the Gaussian wherever the points can be.
std::vector<Choice> candidates_reg(const anova_params &prm, double D, int dA, double budget,
                                   int64_t N) {
    const int prec = prm.precision;
    ANOVA_REQUIRE(prm.h <= 0 || prm.h > 2.0 * D,
                  "with reg_q, h must exceed twice the extent of the points");
    const double base = D > 0 ? D : prm.ell;
    std::vector<double> hs;
    if (prm.h > 0)
        hs.push_back(prm.h);
    else
        for (double f : {2.5, 3.0, 4.0}) hs.push_back(f * base);
    const bool fixed = prm.M > 0 && prm.m > 0 && prm.n > 0;
    // float32 (per-cell kernels): also periods for which the points span a
    // whole number k of tiles of the per-cell kernels at FFT length n, with
    // the data's lower edge on a tile boundary (centre chosen in make_plan),
    // between 2.4 and 4 times the extent; listed first, so that at equal
    // model cost they are preferred
    struct Period {
        double h;
        int n, align;  // n = 0: any FFT length
    };
    std::vector<Period> periods;
    const int T = cell_tile(dA);
    if (prm.h <= 0 && prm.center == 0 && !fixed && prec == ANOVA_FP32_NFFT && D > 0)
        for (int n = 2 * T; n <= 256; n *= 2) {
            if (prm.n > 0 && n != prm.n) continue;
            for (int k = 1; k * T <= n; ++k) {
                const double h = n * D / (k * T * (1.0 - 4e-5));
                if (h >= 2.4 * D && h <= 4.0 * D) periods.push_back(Period{h, n, T});
            }
        }
    for (double h : hs) periods.push_back(Period{h, 0, 0});
    std::vector<Choice> out;
    for (const Period &per : periods) {
        const double h = per.h;
        std::map<int, std::vector<double>> bc;
        std::map<int, double> ec;
        auto coeffs = [&](int M) -> const std::vector<double> & {
            auto it = bc.find(M);
            if (it == bc.end()) it = bc.emplace(M, reg_coeffs_1d(M, prm.ell, h, D, prm.reg_q)).first;
            return it->second;
        };
        auto etr = [&](int M) {
            auto it = ec.find(M);
            if (it == ec.end())
                it = ec.emplace(M, reg_trunc_dA(reg_err1(coeffs(M), prm.ell, h, D), dA)).first;
            return it->second;
        };
        auto fill = [&](Choice &c, int M, int n, int m) {
            c = Choice{};
            c.h = h; c.M = M; c.n = n; c.m = m;
            c.e_img = 0.0;
            c.e_trunc = etr(M);
            c.e_win = est_window_b(coeffs(M), n, m, dA);
            c.e_round = est_round(prec, n, m, dA);
            c.cost = (double)N * std::pow(2.0 * m, dA) +
                     4.0 * std::pow((double)n, dA) * std::log2((double)n) * dA;
        };
        if (fixed) {
            Choice c;
            fill(c, prm.M, prm.n, prm.m);
            out.push_back(c);
            continue;
        }
        for (int n = 8; n <= 256; n *= 2) {
            if ((prm.n > 0 && n != prm.n) || prm.M > n) continue;
            if (per.n > 0 && n != per.n) continue;
            bool found = false;
            Choice c;
            for (int m = 2; m <= 8 && !found; ++m) {
                if (prm.m > 0 && m != prm.m) continue;
                if (2 * m > n) break;
                const double avail = budget - est_round(prec, n, m, dA);
                if (avail <= 0) continue;
                const int M0 = prm.M > 0 ? prm.M : 4;
                const int M1 = prm.M > 0 ? prm.M : (4 * n) / 5;
                for (int M = M0; M <= M1; M += 2) {
                    const double et = etr(M);
                    if (et > avail) continue;
                    const double ew = est_window_b(coeffs(M), n, m, dA);
                    if (et + ew > avail) {
                        if (et < 1e-3 * avail) break;  // only the window error grows from here
                        continue;
                    }
                    fill(c, M, n, m);
                    found = true;
                    break;
                }
            }
            if (!found) continue;
            // the wide 3-D kernels walk every point of a cell per lane and
            // gain nothing from alignment
            if (per.align > 0 && !(dA == 3 && 2 * c.m > 6)) c.align = per.align;
            if (per.align > 0 && c.align == 0) continue;
            out.push_back(c);
        }
    }
    if (out.empty())
        throw Error{ANOVA_E_ACCURACY,
                    "no (M, n, m) with n <= 256 and m <= 8 meets target_err for this window"};
    // fixed parameters: the period with the smallest estimate
    std::stable_sort(out.begin(), out.end(), [&](const Choice &x, const Choice &y) {
        return fixed ? x.e_trunc + x.e_win < y.e_trunc + y.e_win : x.cost < y.cost;
    });
    if (fixed) out.resize(1);
    return out;
}

std::vector<Choice> candidates(const anova_params &prm, double D, int dA, double budget,
                               int64_t N, int share) {
    if (prm.reg_q > 0) return candidates_reg(prm, D, dA, budget, N);
    const int prec = prm.precision;
    double h0;
    if (prm.h > 0) {
        h0 = prm.h;
    } else {
        const double r = std::max(budget * 0.1, 1e-300);
        h0 = std::max(2.0 * D, D + prm.ell * std::sqrt(std::log(std::max(2.0 * dA / r, 1.0001))));
        if (h0 <= 0) h0 = 1.0;
    }
    // the smallest (M, m) at FFT length n and period h, if any
    auto search = [&](double h, int n, Choice &c) -> bool {
        c = Choice{};
        c.h = h;
        c.n = n;
        c.e_img = est_images(h, D, prm.ell, dA);
        const double rest = std::max(budget - c.e_img, budget * 0.5);
        if (prm.M > n) return false;
        // the smallest m, then the smallest M (sigma = n/M >= 1.25 unless M
        // is given), whose truncation, window and rounding estimates
        // together fit what the images leave: truncation falls and the
        // window error grows with M, so the M that fit form one run
        for (int m = 2; m <= 8; ++m) {
            if (prm.m > 0 && m != prm.m) continue;
            if (2 * m > n) break;
            const double avail = rest - est_round(prec, n, m, dA);
            if (avail <= 0) continue;
            const int M0 = prm.M > 0 ? prm.M : 4;
            const int M1 = prm.M > 0 ? prm.M : (4 * n) / 5;
            for (int M = M0; M <= M1; M += 2) {
                const double et = est_trunc(M, h, prm.ell, dA);
                if (et > avail) continue;
                if (et + est_window(M, n, m, prm.ell, h, dA) > avail) {
                    if (et < 1e-3 * avail) break;  // only the window error grows from here
                    continue;
                }
                c.M = M;
                c.m = m;
                return true;
            }
        }
        return false;
    };
    const int T = cell_tile(dA);
    auto per_cell_likely = [&](const Choice &c, double span) {
        return c.n >= 2 * T && cell_width_supported(dA, 2 * c.m, prec) &&
               (double)N >= 3.0 * std::pow(std::max(span, 1.0), dA);
    };
    auto cost = [&](const Choice &c, double eff) {
        return (double)N * std::pow(2.0 * c.m, dA) / eff +
               4.0 * std::pow((double)c.n, dA) * std::log2((double)c.n) * dA;
    };
    // lane efficiency of the spreading and gathering kernels: per cell, a
    // lane's points of one cell against the fixed work of a workgroup (about
    // four points' worth, as in best_chunks); per point, bound by int64 LDS
    // atomics, a quarter in float32 and 0.4 in float64 (as measured against
    // the per-cell kernels of each precision)
    auto eff_of = [&](const Choice &c, double span) {
        if (!per_cell_likely(c, span)) return prec == ANOVA_FP32_NFFT ? 0.25 : 0.4;
        const double steps = (double)N / std::pow(std::max(span, 1.0), dA) /
                             cell_point_splits(dA, 2 * c.m, prec);
        return steps / (steps + 4.0);
    };
    std::vector<Choice> out;
    const bool fixed = prm.M > 0 && prm.m > 0 && prm.n > 0;
    if (fixed) {
        Choice c{};
        c.h = h0; c.M = prm.M; c.n = prm.n; c.m = prm.m;
        c.e_img = est_images(h0, D, prm.ell, dA);
        c.cost = cost(c, 1.0);
        out.push_back(c);
    } else {
        for (int n = 8; n <= 256; n *= 2) {
            if (prm.n > 0 && n != prm.n) continue;
            Choice c;
            if (!search(h0, n, c)) continue;
            const double span = n * D / h0;  // cells the points cover per dimension
            c.cost = cost(c, eff_of(c, span));
            out.push_back(c);
            // the aligned variant serves the kernels with one support per
            // thread (the wide 3-D kernels' lanes walk every point of a cell,
            // which the launch model below does not describe)
            if (!per_cell_likely(c, span) || D <= 0 || (dA == 3 && 2 * c.m > 6)) continue;
            const int k1 = std::max(1, (int)std::ceil(span / T - 1e-9));
            if (k1 >= 2 && prm.h <= 0 && prm.center == 0) {
                Choice a;
                const double h1 = n * D / ((k1 - 1) * T * (1.0 - 4e-5));
                if (search(h1, n, a) && per_cell_likely(a, n * D / h1)) {
                    a.align = T;
                    // the launch model on uniformly spread points: the
                    // centred points end inside edge tiles, whose idle lanes
                    // still take a workgroup's time; the aligned ones fill
                    // k1 - 1 tiles per dimension
                    const double lo = 0.5 * n - 0.5 * span;
                    const int64_t tp = (int64_t)std::floor((lo + span) / T - 1e-9) -
                                       (int64_t)std::floor(lo / T) + 1;
                    auto launch_time = [&](const Choice &x, int64_t tiles_dim, double sp) {
                        const double avg = (double)N / std::pow(std::max(sp, 1.0), dA);
                        const int64_t maxcnt = (int64_t)std::ceil(avg + 3.0 * std::sqrt(avg));
                        const int64_t tiles = (int64_t)std::pow((double)tiles_dim, dA) * share;
                        double t = 0.0;
                        best_chunks(tiles, maxcnt, cell_point_splits(dA, 2 * x.m, prec),
                                    cell_resident_blocks(dA, 2 * x.m, prec), t);
                        return t * std::pow(2.0 * x.m, dA);
                    };
                    const bool better = launch_time(a, k1 - 1, n * D / h1) < launch_time(c, tp, span);
                    // placed just before or after the plain variant
                    a.cost = c.cost * (better ? 1.0 - 1e-9 : 1.0 + 1e-9);
                    out.push_back(a);
                }
            }
        }
        if (out.empty())
            throw Error{ANOVA_E_ACCURACY,
                        "no (M, n, m) with n <= 256 and m <= 8 meets target_err for this window"};
        std::stable_sort(out.begin(), out.end(),
                         [](const Choice &x, const Choice &y) { return x.cost < y.cost; });
    }
    for (Choice &k : out) {
        k.e_trunc = est_trunc(k.M, k.h, prm.ell, dA);
        k.e_win = est_window(k.M, k.n, k.m, prm.ell, k.h, dA);
        k.e_round = est_round(prec, k.n, k.m, dA);
    }
    return out;
}


// For every tile of the n^dA grid (tile edge `tile`, tpd = n/tile per
// dimension), the source regions (one per non-empty tile, src_tiles[k] its
// tile id) that overlap it, in increasing k.  A region starts at its tile's
// origin - m + 1
// and spans L = tile + 2m - 1 points per dimension, periodically.  Each pair
// stores the destination tile origin's offset b in the region (mod n) per
// dimension, packed as 10-bit fields.
void build_fold_lists(const std::vector<int32_t> &src_tiles, int dA, int n, int tile, int m,
                      std::vector<int32_t> &fstart, std::vector<int2> &pairs) {
    const int L = tile + 2 * m - 1;
    const int tpd = n / tile;
    int64_t ntiles = 1;
    for (int t = 0; t < dA; ++t) ntiles *= tpd;
    std::vector<std::vector<int2>> per_tile(ntiles);
    for (size_t si = 0; si < src_tiles.size(); ++si) {
        const int tl = src_tiles[si];
        const int tc[3] = {tl % tpd, (tl / tpd) % tpd, tl / (tpd * tpd)};
        std::vector<int> dest[3];
        int r0[3] = {0, 0, 0};
        for (int t = 0; t < 3; ++t) {
            if (t >= dA) {
                dest[t].push_back(0);
                continue;
            }
            r0[t] = tc[t] * tile - m + 1;
            std::vector<char> hit(tpd, 0);
            for (int e = 0; e < L; ++e) hit[(((r0[t] + e) % n + n) % n) / tile] = 1;
            for (int q = 0; q < tpd; ++q)
                if (hit[q]) dest[t].push_back(q);
        }
        for (int dz : dest[2])
            for (int dy : dest[1])
                for (int dx : dest[0]) {
                    const int dc[3] = {dx, dy, dz};
                    int packed = 0;
                    for (int t = 0; t < dA; ++t) packed |= (((dc[t] * tile - r0[t]) % n + n) % n) << (10 * t);
                    per_tile[(size_t)dx + (size_t)tpd * (dy + (size_t)tpd * dz)].push_back(
                        int2{(int)si, packed});
                }
    }
    fstart.assign(ntiles + 1, 0);
    pairs.clear();
    for (int64_t t = 0; t < ntiles; ++t) {
        fstart[t] = (int32_t)pairs.size();
        pairs.insert(pairs.end(), per_tile[t].begin(), per_tile[t].end());
    }
    fstart[ntiles] = (int32_t)pairs.size();
}

template <typename T, typename Node>
void build_window(WindowPlan &w, const Points &X, int prec) {
    const int dA = w.dA, n = w.n, m = w.m;
    const int64_t N = X.N, ldx = X.ld;
    const double *Xh = X.host;
    // binning: cell index and fractional offset per point and dimension, from
    // t = n (x - c) / h + n/2 in float64 (periodic on [0, n)); hist counts
    // the points of each grid cell (cell index x fastest).  Device points
    // are binned by the device, which keeps the per-point results.
    size_t ncells = 1;
    for (int t = 0; t < dA; ++t) ncells *= (size_t)n;
    std::vector<int32_t> hist;
    std::vector<int32_t> cellc;
    std::vector<T> frac;
    DeviceBins db;
    if (X.dev) {
        device_bin<T>(X.dev, N, ldx, w, db, hist, X.s);
    } else {
        cellc.assign((size_t)N * 3, 0);
        frac.assign((size_t)N * 3, T(0));
        hist.assign(ncells, 0);
        const double scale = (double)n / w.h;
        for (int64_t i = 0; i < N; ++i) {
            size_t lin = 0, mul = 1;
            for (int t = 0; t < dA; ++t) {
                double tt = (Xh[(size_t)i * ldx + w.feat[t]] - w.center[t]) * scale + 0.5 * n;
                tt -= n * std::floor(tt / n);
                const double cf = std::floor(tt);
                int cell = (int)cf;
                const double f = tt - cf;
                if (cell >= n) cell -= n;
                if (cell < 0) cell += n;
                frac[(size_t)i * 3 + t] = static_cast<T>(f);
                cellc[(size_t)i * 3 + t] = cell;
                lin += (size_t)cell * mul;
                mul *= (size_t)n;
            }
            ++hist[lin];
        }
    }
    size_t nocc = 0;
    for (int32_t c : hist) nocc += c > 0 ? 1 : 0;
    // dense regime: small support (float32; float64 in 3-D up to W = 6) and
    // several points per occupied cell -> per-cell register accumulation
    // with a fixed small tile
    const int W = 2 * m;
    const int dense_tile = dA == 3 ? 4 : (dA == 2 ? 16 : 64);
    const bool dense_ok = n >= dense_tile && cell_width_supported(dA, W, prec);
    w.dense = dense_ok && (double)N >= 3.0 * (double)std::max<size_t>(nocc, 1);
    // tile edge: power of two dividing n whose region (tile + 2m - 1)^dA of
    // 64-bit spreading accumulators fits in 64 KB of LDS
    int tile = dA == 3 ? 8 : (dA == 2 ? 32 : 256);
    tile = std::min(tile, n);
    auto region = [&](int t) {
        double L = t + 2.0 * m - 1.0;
        return std::pow(L, dA) * 8.0;
    };
    while (tile > 2 && region(tile) > 65536.0) tile /= 2;
    while (w.tile_cap > 0 && tile > 2 && tile > w.tile_cap) tile /= 2;
    if (w.dense) tile = dense_tile;
    w.tile = tile;
    w.tiles_per_dim = n / tile;
    int64_t ntiles = 1;
    for (int t = 0; t < dA; ++t) ntiles *= w.tiles_per_dim;
    w.n_tiles = ntiles;
    int64_t cells_per_tile = 1;
    for (int t = 0; t < dA; ++t) cells_per_tile *= tile;
    // sort key: tile, then cell inside the tile (x fastest); per-point
    // kernels keep the caller's order inside a tile (points of one cell in
    // one wave collide on the same LDS addresses)
    auto key_of = [&](const int *cell) {
        int64_t tk = 0, lk = 0, mul = 1, lmul = 1;
        for (int t = 0; t < dA; ++t) {
            tk += (int64_t)(cell[t] / tile) * mul;
            lk += (int64_t)(cell[t] % tile) * lmul;
            mul *= w.tiles_per_dim;
            lmul *= tile;
        }
        return w.dense ? tk * cells_per_tile + lk : tk * cells_per_tile;
    };
    // first sorted position of each key, from the points per cell
    const int64_t nkeys = ntiles * cells_per_tile;
    std::vector<int64_t> kstart(nkeys + 1, 0);
    for (size_t lin = 0; lin < ncells; ++lin) {
        if (hist[lin] == 0) continue;
        int cell[3] = {0, 0, 0};
        size_t r = lin;
        for (int t = 0; t < dA; ++t) {
            cell[t] = (int)(r % (size_t)n);
            r /= (size_t)n;
        }
        kstart[key_of(cell) + 1] += hist[lin];
    }
    for (int64_t k = 0; k < nkeys; ++k) kstart[k + 1] += kstart[k];
    // stable sort by key (ties by the caller's index)
    if (X.dev) {
        device_sort_nodes<T, Node>(w, N, cells_per_tile, w.dense, db, X.s);
        w.nodes = std::move(db.nodes);
        w.perm = std::move(db.perm);
    } else {
        std::vector<int64_t> fill(kstart.begin(), kstart.end() - 1);
        std::vector<int32_t> perm(N);
        for (int64_t i = 0; i < N; ++i) perm[fill[key_of(&cellc[(size_t)i * 3])]++] = (int32_t)i;
        std::vector<Node> nodes(N);
        for (int64_t j = 0; j < N; ++j) {
            const int32_t i = perm[j];
            Node nd{};
            uint32_t packed = 0;
            for (int t = 0; t < 3; ++t) {
                nd.f[t] = frac[(size_t)i * 3 + t];
                if (t < dA) packed |= (uint32_t)cellc[(size_t)i * 3 + t] << (10 * t);
            }
            nd.cell = packed;
            nodes[j] = nd;
        }
        upload(w.nodes, nodes);
        upload(w.perm, perm);
    }
    std::vector<int64_t> start(ntiles + 1);
    for (int64_t t = 0; t <= ntiles; ++t) start[t] = kstart[t * cells_per_tile];
    w.n_points = N;
    if (w.dense) {
        std::vector<int32_t> cs(nkeys + 1);
        for (int64_t k = 0; k <= nkeys; ++k) cs[k] = (int32_t)kstart[k];
        upload(w.cell_start, cs);
        std::vector<int32_t> ne;
        for (int64_t t = 0; t < ntiles; ++t)
            if (start[t + 1] > start[t]) ne.push_back((int32_t)t);
        // heaviest tiles first (by their fullest cell, which sets a
        // workgroup's duration), so that the last workgroups to start are
        // short ones and the launch's tail stays small; ties by tile id
        {
            std::vector<int64_t> heavy(ntiles, 0);
            for (int32_t t : ne)
                for (int64_t c = 0; c < cells_per_tile; ++c) {
                    const int64_t k = (int64_t)t * cells_per_tile + c;
                    heavy[t] = std::max(heavy[t], kstart[k + 1] - kstart[k]);
                }
            std::stable_sort(ne.begin(), ne.end(),
                             [&](int32_t a, int32_t b) { return heavy[a] > heavy[b]; });
        }
        w.tile_order = ne;
        upload(w.tiles_ne, ne);
        // workgroups (chunks) per tile: a thread handles its cell's share of
        // one chunk, so a workgroup takes as long as its fullest cell; tiles
        // at the edge of the data still hold full cells, so every tile gets
        // the same count, the one the launch model (best_chunks) finds
        // fastest for this window's tiles and fullest cell, with the plan's
        // windows sharing the device
        int64_t maxcnt = 0;
        for (int64_t k = 0; k < nkeys; ++k) maxcnt = std::max(maxcnt, kstart[k + 1] - kstart[k]);
        double model_time = 0.0;
        const int K = best_chunks((int64_t)ne.size() * std::max(1, w.launch_windows), maxcnt,
                                  cell_point_splits(dA, 2 * m, prec),
                                  cell_resident_blocks(dA, 2 * m, prec),
                                  model_time);
        std::vector<int32_t> cstart(ne.size() + 1);
        for (size_t k = 0; k <= ne.size(); ++k) cstart[k] = (int32_t)(k * K);
        w.chunk_start = cstart;
        w.chunks = K;
    }
    // sub-problems
    const int64_t maxsub = 1024;
    std::vector<SubProblem> subs;
    int64_t nonempty = 0;
    for (int64_t t = 0; t < ntiles; ++t) {
        const int64_t s0 = start[t], s1 = start[t + 1];
        if (s1 == s0) continue;
        ++nonempty;
        for (int64_t s = s0; s < s1; s += maxsub)
            subs.push_back(SubProblem{(int32_t)t, (int32_t)s, (int32_t)std::min(maxsub, s1 - s), 0});
    }
    w.n_nonempty = nonempty;
    w.n_sub = (int64_t)subs.size();
    w.n_regions = w.dense ? (int64_t)w.chunk_start.back() : w.n_sub;
    upload(w.subs, subs);
    // per non-empty tile: its sub-problems, and the fold lists over tiles
    {
        std::vector<int32_t> src_tiles, src_sub;
        for (size_t q = 0; q < subs.size(); ++q)
            if (q == 0 || subs[q].tile != subs[q - 1].tile) {
                src_tiles.push_back(subs[q].tile);
                src_sub.push_back((int32_t)q);
            }
        src_sub.push_back((int32_t)subs.size());
        if (w.dense) {  // chunk regions of tile k: chunk_start[k] .. chunk_start[k+1] - 1
            src_sub = w.chunk_start;
            src_tiles = w.tile_order;  // k-th non-empty tile in launch order
        }
        upload(w.src_sub, src_sub);
        std::vector<int32_t> fstart;
        std::vector<int2> pairs;
        build_fold_lists(src_tiles, dA, n, tile, m, fstart, pairs);
        w.n_pairs = (int64_t)pairs.size();
        upload(w.fold_pairs, pairs);
        upload(w.fold_start, fstart);
        // fold workgroup order: workgroups go to the chip's 8 dies in turn,
        // so the tiles that receive regions are split into 8 runs by tile
        // id, workgroup b taking entry b / 8 of run b % 8: each die folds
        // one slab of neighbouring tiles, which read the same regions
        // through its L2; the tiles that receive none follow, to be zeroed
        std::vector<int32_t> act, idle;
        for (int64_t t = 0; t < w.n_tiles; ++t)
            (fstart[t + 1] > fstart[t] ? act : idle).push_back((int32_t)t);
        const int64_t run = ((int64_t)act.size() + 7) / 8;
        std::vector<int32_t> order(8 * run, -1);
        for (int64_t b = 0; b < 8 * run; ++b) {
            const int64_t pos = (b % 8) * run + b / 8;
            if (pos < (int64_t)act.size()) order[b] = act[pos];
        }
        w.fold_act = (int32_t)order.size();
        order.insert(order.end(), idle.begin(), idle.end());
        w.fold_len = (int32_t)order.size();
        upload(w.fold_tiles, order);
    }
    // window polynomial table at the precision's fixed degree; its error
    // perturbs every weight, counted (per dimension, spread and gather) in
    // the window error relative to the window's integral
    const int deg = prec == ANOVA_FP64 ? (w.dense ? kPolyDegCell64 : PolyDeg<double>::of(2 * m))
                                       : PolyDeg<float>::of(2 * m);
    double fit_err = 0.0;
    std::vector<double> coef = fit_window_polys(m, w.kb_b, deg, fit_err);
    w.poly_deg = deg;
    w.fit_err = fit_err;
    {
        const double phi0_int = kb_phihat(0.0, m, w.kb_b) / bessel_i0(w.kb_b);
        const double e_fit = std::fabs(w.eta) * 2.0 * dA * (2.0 * m) * fit_err / phi0_int;
        w.err_window += e_fit;
        w.err_total += e_fit;
    }
    std::vector<T> coefT(coef.begin(), coef.end());
    upload(w.poly, coefT);
    // per-axis multiplier: b1_k / phihat(k/n)^2 for |k| < M/2, else 0
    std::vector<double> bd(n, 0.0);
    const double i0b = bessel_i0(w.kb_b);
    const std::vector<double> bk = w.reg_q > 0 ? reg_coeffs_1d(w.M, w.ell, w.h, w.extent, w.reg_q)
                                               : sampled_coeffs_1d(w.M, w.ell, w.h);
    for (int k = 0; k < n; ++k) {
        const int ks = k < n / 2 ? k : k - n;
        if (std::abs(ks) >= w.M / 2) continue;
        const double ph = kb_phihat((double)ks / n, m, w.kb_b) / i0b;
        bd[k] = bk[ks + w.M / 2] / (ph * ph);
    }
    upload(w.bconv, std::vector<T>(bd.begin(), bd.end()));
    // the same filter as circular-convolution taps (small grids): the
    // multiplier is real and even, so its inverse transform is the real,
    // even c_d = sum_k b_k cos(2 pi k d / n)
    {
        std::vector<T> taps(n);
        for (int d = 0; d < n; ++d) {
            double c = 0.0;
            for (int k = 0; k < n; ++k) c += bd[k] * std::cos(2.0 * kPi * (double)((int64_t)k * d % n) / n);
            taps[d] = static_cast<T>(c);
        }
        upload(w.ctaps, taps);
    }
    // twiddles exp(-2 pi i j / n), j < n/2
    std::vector<T> tw(n);
    for (int j = 0; j < n / 2; ++j) {
        const long double ang = -2.0L * (long double)kPi * j / n;
        tw[2 * j] = static_cast<T>(std::cos(ang));
        tw[2 * j + 1] = static_cast<T>(std::sin(ang));
    }
    upload(w.twiddle, tw);
}

void validate(const double *X, int64_t N, int32_t d, int64_t ldx, const anova_window *win,
              int32_t P, const anova_params *prm) {
    ANOVA_REQUIRE(X != nullptr, "X is NULL");
    ANOVA_REQUIRE(win != nullptr, "win is NULL");
    ANOVA_REQUIRE(prm != nullptr, "prm is NULL");
    ANOVA_REQUIRE(N >= 1 && N <= 2147483647LL, "N must be in [1, 2^31-1]");
    ANOVA_REQUIRE(d >= 1, "d must be >= 1");
    ANOVA_REQUIRE(ldx >= d, "ldx must be >= d");
    ANOVA_REQUIRE(P >= 1 && P <= 64, "P must be in [1, 64]");
    ANOVA_REQUIRE(std::isfinite(prm->ell) && prm->ell > 0, "ell must be finite and > 0");
    ANOVA_REQUIRE(prm->precision == ANOVA_FP64 || prm->precision == ANOVA_FP32_NFFT,
                  "precision must be ANOVA_FP64 or ANOVA_FP32_NFFT");
    ANOVA_REQUIRE(prm->M >= 0 && prm->M % 2 == 0 && prm->M <= 256, "M must be even, 0 or 4..256");
    ANOVA_REQUIRE(prm->M == 0 || prm->M >= 4, "M must be >= 4");
    ANOVA_REQUIRE(prm->n == 0 || (is_pow2(prm->n) && prm->n >= 8 && prm->n <= 256),
                  "n must be 0 or a power of two in [8, 256]");
    ANOVA_REQUIRE(prm->n == 0 || prm->M == 0 || prm->n >= prm->M, "n must be >= M");
    ANOVA_REQUIRE(prm->m == 0 || (prm->m >= 2 && prm->m <= 8), "m must be 0 or in [2, 8]");
    ANOVA_REQUIRE(prm->n == 0 || prm->m == 0 || 2 * prm->m <= prm->n, "2m must be <= n");
    ANOVA_REQUIRE(std::isfinite(prm->h) && prm->h >= 0, "h must be finite and >= 0");
    ANOVA_REQUIRE(std::isfinite(prm->target_err) && prm->target_err >= 0, "target_err must be >= 0");
    ANOVA_REQUIRE(prm->center == 0 || prm->center == 1, "center must be 0 or 1");
    ANOVA_REQUIRE(prm->residual == ANOVA_RESIDUAL_FP64 || prm->residual == ANOVA_RESIDUAL_SAME,
                  "residual must be ANOVA_RESIDUAL_FP64 or ANOVA_RESIDUAL_SAME");
    ANOVA_REQUIRE(prm->tune == 0 || prm->tune == 1, "tune must be 0 or 1");
    ANOVA_REQUIRE(prm->reg_q >= 0 && prm->reg_q <= 12, "reg_q must be in [0, 12]");
    for (int l = 0; l < P; ++l) {
        const anova_window &w = win[l];
        ANOVA_REQUIRE(w.d_A >= 1 && w.d_A <= 3, "window d_A must be 1, 2 or 3");
        ANOVA_REQUIRE(std::isfinite(w.eta), "window weight eta must be finite");
        for (int t = 0; t < w.d_A; ++t) {
            ANOVA_REQUIRE(w.feat[t] >= 0 && w.feat[t] < d, "feature index out of range");
            for (int u = 0; u < t; ++u)
                ANOVA_REQUIRE(w.feat[u] != w.feat[t], "repeated feature inside a window");
        }
    }
}

}  // namespace

std::recursive_mutex &device_mutex() {
    // never destroyed: buffers held by other static objects are released
    // during exit, after function-local statics constructed later are gone
    static std::recursive_mutex *mu = new std::recursive_mutex();
    return *mu;
}

namespace {
// A released block may still be read by work queued before its release (on
// any stream), so it waits in `pending` until a device synchronisation
// after its release, one for every kPendingFlush releases, and only then
// becomes reusable.
constexpr size_t kPendingFlush = 512;
struct SmallCache {
    std::map<size_t, std::vector<void *>> free;  // size class -> reusable blocks
    std::vector<std::pair<void *, size_t>> pending;
    size_t bytes = 0;  // free and pending
};
std::map<int, SmallCache> &small_caches() {
    // per device; guarded by device_mutex(); never destroyed (as the mutex)
    static std::map<int, SmallCache> *c = new std::map<int, SmallCache>();
    return *c;
}
// (runs inside buffer releases, destructors included: a failed
// synchronisation leaves the blocks pending instead of throwing)
void flush_pending(int dev, SmallCache &c) {
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return;
    if (cur != dev && hipSetDevice(dev) != hipSuccess) return;
    const hipError_t e = hipDeviceSynchronize();
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess) return;
    for (auto &b : c.pending) c.free[b.second].push_back(b.first);
    c.pending.clear();
}
}  // namespace

void *small_block_take(int dev, size_t cls) {
    SmallCache &c = small_caches()[dev];
    auto it = c.free.find(cls);
    if (it == c.free.end() || it->second.empty()) return nullptr;
    void *p = it->second.back();
    it->second.pop_back();
    c.bytes -= cls;
    return p;
}

bool small_block_give(int dev, void *p, size_t cls) {
    SmallCache &c = small_caches()[dev];
    if (c.bytes + cls > kSmallCacheBytes) return false;
    c.pending.emplace_back(p, cls);
    c.bytes += cls;
    if (c.pending.size() >= kPendingFlush) flush_pending(dev, c);
    return true;
}

hipEvent_t pool_event(anova_plan_s *p) {
    if (!p->event_pool.empty()) {
        hipEvent_t e = p->event_pool.back();
        p->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    ANOVA_HIP_CHECK(hipEventCreate(&e));
    return e;
}

// out = (K~ + beta I) alpha for nrhs columns: one batched launch per stage
// over all windows and columns; the launch tables are rebuilt only when the
// vectors, their layout or the shift change (after the previous product on
// the caller's stream has finished reading them).
void plan_matvec(anova_plan_s *p, const double *alpha, double *out, int nrhs, int64_t ld,
                 double beta, hipStream_t s) {
    BatchProblem bp;
    bp.plan = p;
    bp.alpha = alpha;
    bp.out = out;
    bp.nrhs = nrhs;
    bp.ld = ld;
    bp.beta = beta;
    run_cached(p->mv_cache, {bp}, s, p);
}

// out = K~(Z, X) alpha for nrhs columns (rows: the plan's targets), batched
// like plan_matvec.
void plan_predict(anova_plan_s *p, const double *alpha, double *out, int nrhs, int64_t lda,
                  int64_t ldo, hipStream_t s) {
    BatchProblem bp;
    bp.plan = p;
    bp.alpha = alpha;
    bp.out = out;
    bp.nrhs = nrhs;
    bp.ld = lda;
    bp.ld_out = ldo;
    bp.predict = true;
    run_cached(p->pred_cache, {bp}, s, p);
}

}  // namespace anova

using namespace anova;

size_t anova::plan_device_bytes(const anova_plan_s *p) {
    size_t b = 0;
    for (const std::vector<WindowPlan> *ws : {&p->win, &p->win64, &p->tgt})
      for (const WindowPlan &w : *ws)
        for (const DevBuf *d : {&w.nodes, &w.perm, &w.subs, &w.poly, &w.bconv, &w.ctaps, &w.twiddle,
                                &w.src_sub, &w.cell_start, &w.tiles_ne, &w.fold_pairs,
                                &w.fold_start, &w.fold_tiles})
            b += d->bytes;
    for (const auto &c : {&p->mv_cache, &p->pred_cache})
        for (const auto &bt : *c) b += bt->device_bytes();
    return b;
}

// Centre of each dimension: the bounding-box centre, or (aligned choices)
// the point that puts the lowest coordinate just above a tile boundary, so
// that the points fill whole tiles of the per-cell kernels; with
// center = 1 the plain scaling x/h.
static void set_centers(WindowPlan &w, const Choice &c, const double *lo, const double *hi,
                        const anova_params &prm) {
    for (int t = 0; t < w.dA; ++t) {
        if (prm.center == 1) {
            w.center[t] = 0.0;
        } else if (c.align > 0) {
            const double T = c.align, n = c.n;
            const double span = n * (hi[t] - lo[t]) / c.h;
            const double k0 = std::floor((0.5 * n - 0.5 * span) / T);
            // t(lo) = n (lo - centre) / h + n/2 = T k0 + 1e-5 T
            w.center[t] = lo[t] - (T * k0 + 1e-5 * T - 0.5 * n) * c.h / n;
        } else {
            w.center[t] = 0.5 * (lo[t] + hi[t]);
        }
    }
}

// Parameters and error estimates of one choice into a window.
static void apply_choice(WindowPlan &w, const Choice &c, const anova_params &prm) {
    w.h = c.h; w.M = c.M; w.n = c.n; w.m = c.m;
    w.kb_b = kPi * w.m * (2.0 - (double)w.M / w.n);
    const double ae = std::fabs(w.eta);
    w.err_images = ae * c.e_img;
    w.err_trunc = ae * c.e_trunc;
    w.err_window = ae * c.e_win;
    w.err_round = ae * c.e_round;
    w.err_total = w.err_images + w.err_trunc + w.err_window + w.err_round;
    w.ell = prm.ell;
    w.reg_q = prm.reg_q;
}

static void build_for(WindowPlan &w, const Points &X, int prec) {
    if (prec == ANOVA_FP64)
        build_window<double, NodeF64>(w, X, prec);
    else
        build_window<float, NodeF32>(w, X, prec);
}

// Device time of one product of a one-window plan (the best of 3 after a
// warm-up), on a stream of its own.
// Product time of a one-window plan launched `copies` times together, as the
// plan's windows share their launches (out: copies columns of one.N).
static double time_window(anova_plan_s &one, const double *alpha, double *out, int copies) {
    hipStream_t s = nullptr;
    ANOVA_HIP_CHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float best = std::numeric_limits<float>::infinity();
    try {
        Batch b;
        std::vector<BatchProblem> bps((size_t)std::max(copies, 1));
        for (size_t k = 0; k < bps.size(); ++k) {
            BatchProblem &bp = bps[k];
            bp.plan = &one;
            bp.alpha = alpha;
            bp.out = out + (size_t)k * (size_t)one.N;
            bp.nrhs = 1;
            bp.ld = one.N;
            bp.beta = 1.0;
        }
        b.build(bps);
        ANOVA_HIP_CHECK(hipEventCreate(&e0));
        ANOVA_HIP_CHECK(hipEventCreate(&e1));
        b.run(s);
        for (int r = 0; r < 3; ++r) {
            ANOVA_HIP_CHECK(hipEventRecord(e0, s));
            b.run(s);
            ANOVA_HIP_CHECK(hipEventRecord(e1, s));
            ANOVA_HIP_CHECK(hipEventSynchronize(e1));
            float ms = 0.0f;
            ANOVA_HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
            best = std::min(best, ms);
        }
        ANOVA_HIP_CHECK(hipStreamSynchronize(s));
    } catch (...) {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(s);
    return best;
}

// Minimum and maximum of each of the d features of the points, which must
// all be finite (`what` names them in the error).
static void feature_bounds(const Points &X, int d, std::vector<double> &lo,
                           std::vector<double> &hi, const char *what) {
    lo.assign(d, 0.0);
    hi.assign(d, 0.0);
    if (X.dev) {
        bool finite = true;
        device_bounds(X.dev, X.N, X.ld, d, lo.data(), hi.data(), finite, X.s);
        ANOVA_REQUIRE(finite, std::string(what) + " holds a non-finite value");
        return;
    }
    for (int t = 0; t < d; ++t) lo[t] = hi[t] = X.host[t];
    for (size_t i = 0; i < (size_t)X.N; ++i)
        for (int t = 0; t < d; ++t) {
            const double v = X.host[i * X.ld + t];
            ANOVA_REQUIRE(std::isfinite(v), std::string(what) + " holds a non-finite value");
            lo[t] = std::min(lo[t], v);
            hi[t] = std::max(hi[t], v);
        }
}

// Plan from validated arguments and the points X (host or device); with
// targets Z (Z.N > 0) also a prediction plan, whose periods and centres are
// chosen for both point sets together.
static anova_status make_plan(anova_plan_t *out, const Points &X, int32_t d,
                              const anova_window *win, int32_t P, const anova_params *prm,
                              const Points &Z = Points{}) {
    anova_plan_s *p = nullptr;
    const int64_t N = X.N;
    const bool targets = Z.N > 0;
    anova_status st = guarded([&] {
        std::vector<double> xlo, xhi, zlo, zhi;
        feature_bounds(X, d, xlo, xhi, "X");
        if (targets) feature_bounds(Z, d, zlo, zhi, "Z");
        p = new anova_plan_s();
        ANOVA_HIP_CHECK(hipGetDevice(&p->device));
        p->N = N; p->d = d; p->P = P; p->precision = prm->precision; p->ell = prm->ell;
        p->Nz = targets ? Z.N : 0;
        p->win.resize(P);
        double eta_abs = 0.0;
        for (int l = 0; l < P; ++l) eta_abs += std::fabs(win[l].eta);
        if (eta_abs == 0.0) eta_abs = 1.0;
        const double target = prm->target_err > 0 ? prm->target_err
                              : (prm->precision == ANOVA_FP64 ? 1e-9 : 1e-4);
        const double budget = target / eta_abs;
        DevBuf tune_alpha, tune_out;  // measured choice: a vector of ones and its product
        for (int l = 0; l < P; ++l) {
            WindowPlan &w = p->win[l];
            w.dA = win[l].d_A;
            w.eta = win[l].eta;
            double D = 0.0, lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
            for (int t = 0; t < w.dA; ++t) {
                w.feat[t] = win[l].feat[t];
                lo[t] = xlo[w.feat[t]];
                hi[t] = xhi[w.feat[t]];
                // targets: every difference z - x enters the periodised
                // kernel, so the box holds both sets (Sec. 4.2 scales both
                // into the same torus)
                if (targets) {
                    lo[t] = std::min(lo[t], zlo[w.feat[t]]);
                    hi[t] = std::max(hi[t], zhi[w.feat[t]]);
                }
                D = std::max(D, hi[t] - lo[t]);
            }
            w.extent = D;
            w.launch_windows = P;
            const std::vector<Choice> cands = candidates(*prm, D, w.dA, budget, N, P);
            for (const Choice &c : cands) {
                ANOVA_REQUIRE(c.h > D || (D == 0 && c.h > 0),
                              "h must exceed the extent of the points");
                ANOVA_REQUIRE(prm->reg_q == 0 || c.h > 2.0 * D,
                              "with reg_q, h must exceed twice the extent of the points");
            }
            // the candidates fit the budget before the window polynomials'
            // fit error, which building adds: a candidate whose total then
            // exceeds the window's share of the target is passed over
            const double share = std::fabs(w.eta) * budget;
            auto build_choice = [&](WindowPlan &v, const Choice &c, int cap) {
                v.dA = w.dA; v.eta = w.eta; v.extent = w.extent;
                v.launch_windows = w.launch_windows;  // chunks as in the full plan
                v.tile_cap = cap;
                for (int t = 0; t < 3; ++t) v.feat[t] = w.feat[t];
                set_centers(v, c, lo, hi, *prm);
                apply_choice(v, c, *prm);
                build_for(v, X, prm->precision);
                return v.err_total <= share;
            };
            // first candidate that fits once built (the last one otherwise,
            // for the plan's final check to report)
            auto build_first_fit = [&]() {
                for (size_t k = 0; k < cands.size(); ++k) {
                    WindowPlan v;
                    if (build_choice(v, cands[k], 0) || k + 1 == cands.size()) {
                        w = std::move(v);
                        return;
                    }
                }
            };
            if (prm->tune == 0 || cands.size() == 1) {
                build_first_fit();
                continue;
            }
            // measured choice: build the cheapest candidates (model cost
            // within 8x of the cheapest, at most 4) on these points and keep
            // the one whose product runs fastest, timed with P copies of the
            // window in each launch as the plan's P windows will be
            if (!tune_alpha.ptr) {
                upload(tune_alpha, std::vector<double>((size_t)N, 1.0));
                tune_out.alloc((size_t)N * (size_t)P * sizeof(double));
            }
            // (per-point windows: also with tiles of half the edge, whose
            // regions hold fewer halo points per point but add fold work)
            double best_t = std::numeric_limits<double>::infinity();
            for (size_t k = 0; k < cands.size() && k < 4; ++k) {
                if (cands[k].cost > 8.0 * cands.front().cost) break;
                int cap = 0;
                for (int variant = 0; variant < 2; ++variant) {
                    anova_plan_s one;
                    one.N = N; one.d = d; one.P = 1; one.precision = prm->precision;
                    one.ell = prm->ell; one.device = p->device;
                    one.win.resize(1);
                    WindowPlan &v = one.win[0];
                    if (!build_choice(v, cands[k], cap)) break;  // both variants share the estimate
                    const double t =
                        time_window(one, tune_alpha.as<double>(), tune_out.as<double>(), P);
                    const bool halve = !v.dense && v.tile > 2;
                    const int tile = v.tile;
                    if (t < best_t) {
                        best_t = t;
                        w = std::move(v);
                    }
                    if (!halve) break;
                    cap = tile / 2;
                }
            }
            if (best_t == std::numeric_limits<double>::infinity()) build_first_fit();
        }
        if (prm->precision == ANOVA_FP32_NFFT && prm->residual == ANOVA_RESIDUAL_FP64) {
            // the same windows and parameters in float64, for CG's residuals
            p->win64.resize(P);
            for (int l = 0; l < P; ++l) {
                const WindowPlan &w = p->win[l];
                WindowPlan &v = p->win64[l];
                v.dA = w.dA; v.eta = w.eta; v.ell = w.ell; v.h = w.h; v.extent = w.extent;
                v.M = w.M; v.n = w.n; v.m = w.m; v.kb_b = w.kb_b; v.reg_q = w.reg_q;
                for (int t = 0; t < 3; ++t) { v.feat[t] = w.feat[t]; v.center[t] = w.center[t]; }
                build_window<double, NodeF64>(v, X, ANOVA_FP64);
            }
        }
        if (targets) {
            // the targets binned on the same grids, in the plan's precision
            p->tgt.resize(P);
            for (int l = 0; l < P; ++l) {
                const WindowPlan &w = p->win[l];
                WindowPlan &v = p->tgt[l];
                v.dA = w.dA; v.eta = w.eta; v.ell = w.ell; v.h = w.h; v.extent = w.extent;
                v.M = w.M; v.n = w.n; v.m = w.m; v.kb_b = w.kb_b; v.reg_q = w.reg_q;
                v.launch_windows = w.launch_windows;
                v.err_images = w.err_images; v.err_trunc = w.err_trunc;
                v.err_window = w.err_window; v.err_round = w.err_round;
                v.err_total = w.err_total;
                for (int t = 0; t < 3; ++t) { v.feat[t] = w.feat[t]; v.center[t] = w.center[t]; }
                build_for(v, Z, prm->precision);
            }
        }
        if (prm->target_err > 0) {
            double tot = 0.0;
            for (auto &w : p->win) tot += w.err_total;
            if (tot > prm->target_err)
                throw Error{ANOVA_E_ACCURACY, "estimated per-entry error " + std::to_string(tot) +
                                                  " exceeds target_err"};
        }
        // every upload above was a synchronous copy: the plan is complete and
        // other streams' work is not waited for
    });
    if (st != ANOVA_OK) {
        delete p;
        return st;
    }
    *out = p;
    return ANOVA_OK;
}

extern "C" anova_status anova_fastsum_plan(anova_plan_t *out, const double *X, int64_t N,
                                           int32_t d, int64_t ldx, const anova_window *win,
                                           int32_t P, const anova_params *prm, void *stream) {
    if (!out) {
        set_error("out is NULL");
        return ANOVA_E_INVALID;
    }
    *out = nullptr;
    const anova_status st = guarded([&] { validate(X, N, d, ldx, win, P, prm); });
    if (st != ANOVA_OK) return st;
    // the points stay on the device: bounds, binning and sorting run there
    Points pts;
    pts.dev = X;
    pts.N = N;
    pts.ld = ldx;
    pts.s = (hipStream_t)stream;
    return make_plan(out, pts, d, win, P, prm);
}

extern "C" anova_status anova_fastsum_plan_host(anova_plan_t *out, const double *X, int64_t N,
                                                int32_t d, int64_t ldx, const anova_window *win,
                                                int32_t P, const anova_params *prm) {
    if (!out) {
        set_error("out is NULL");
        return ANOVA_E_INVALID;
    }
    *out = nullptr;
    const anova_status st = guarded([&] { validate(X, N, d, ldx, win, P, prm); });
    if (st != ANOVA_OK) return st;
    Points pts;
    pts.host = X;
    pts.N = N;
    pts.ld = ldx;
    return make_plan(out, pts, d, win, P, prm);
}

static void validate_targets(const double *Z, int64_t Nz, int32_t d, int64_t ldz) {
    ANOVA_REQUIRE(Z != nullptr, "Z is NULL");
    ANOVA_REQUIRE(Nz >= 1 && Nz <= 2147483647LL, "Nz must be in [1, 2^31-1]");
    ANOVA_REQUIRE(ldz >= d, "ldz must be >= d");
}

extern "C" anova_status anova_predict_plan(anova_plan_t *out, const double *X, int64_t N,
                                           const double *Z, int64_t Nz, int32_t d, int64_t ldx,
                                           int64_t ldz, const anova_window *win, int32_t P,
                                           const anova_params *prm, void *stream) {
    if (!out) {
        set_error("out is NULL");
        return ANOVA_E_INVALID;
    }
    *out = nullptr;
    const anova_status st = guarded([&] {
        validate(X, N, d, ldx, win, P, prm);
        validate_targets(Z, Nz, d, ldz);
    });
    if (st != ANOVA_OK) return st;
    Points px, pz;
    px.dev = X; px.N = N; px.ld = ldx; px.s = (hipStream_t)stream;
    pz.dev = Z; pz.N = Nz; pz.ld = ldz; pz.s = (hipStream_t)stream;
    return make_plan(out, px, d, win, P, prm, pz);
}

extern "C" anova_status anova_predict_plan_host(anova_plan_t *out, const double *X, int64_t N,
                                                const double *Z, int64_t Nz, int32_t d,
                                                int64_t ldx, int64_t ldz, const anova_window *win,
                                                int32_t P, const anova_params *prm) {
    if (!out) {
        set_error("out is NULL");
        return ANOVA_E_INVALID;
    }
    *out = nullptr;
    const anova_status st = guarded([&] {
        validate(X, N, d, ldx, win, P, prm);
        validate_targets(Z, Nz, d, ldz);
    });
    if (st != ANOVA_OK) return st;
    Points px, pz;
    px.host = X; px.N = N; px.ld = ldx;
    pz.host = Z; pz.N = Nz; pz.ld = ldz;
    return make_plan(out, px, d, win, P, prm, pz);
}

extern "C" anova_status anova_predict(anova_plan_t p, const double *alpha, double *out,
                                      int32_t nrhs, int64_t lda, int64_t ldo, void *stream) {
    return guarded([&] {
        ANOVA_REQUIRE(p != nullptr, "NULL plan");
        ANOVA_REQUIRE(p->Nz > 0 && (int)p->tgt.size() == p->P, "the plan has no targets");
        ANOVA_REQUIRE(alpha != nullptr && out != nullptr, "NULL vector");
        ANOVA_REQUIRE(nrhs >= 1, "nrhs must be >= 1");
        ANOVA_REQUIRE(lda >= p->N, "lda must be >= N");
        ANOVA_REQUIRE(ldo >= p->Nz, "ldo must be >= Nz");
        plan_predict(p, alpha, out, nrhs, lda, ldo, (hipStream_t)stream);
    });
}

extern "C" anova_status anova_plan_destroy(anova_plan_t p) {
    if (!p) return ANOVA_OK;
    return guarded([&] {
        (void)hipDeviceSynchronize();
        for (auto &t : p->timed) {
            (void)hipEventDestroy(t.start);
            (void)hipEventDestroy(t.stop);
        }
        for (auto e : p->event_pool) (void)hipEventDestroy(e);
        delete p;
    });
}

extern "C" anova_status anova_plan_set_timing(anova_plan_t p, int32_t enable) {
    return guarded([&] {
        ANOVA_REQUIRE(p != nullptr, "NULL plan");
        p->timing = enable != 0;
    });
}

extern "C" anova_status anova_plan_stage_times(anova_plan_t p, double *ms, int64_t *launches) {
    return guarded([&] {
        ANOVA_REQUIRE(p != nullptr && ms != nullptr && launches != nullptr, "NULL argument");
        for (int k = 0; k < kStageKinds; ++k) { ms[k] = 0.0; launches[k] = 0; }
        ANOVA_HIP_CHECK(hipDeviceSynchronize());
        for (auto &t : p->timed) {
            float e = 0.0f;
            ANOVA_HIP_CHECK(hipEventElapsedTime(&e, t.start, t.stop));
            ms[t.kind] += e;
            launches[t.kind] += 1;
            p->event_pool.push_back(t.start);
            p->event_pool.push_back(t.stop);
        }
        p->timed.clear();
    });
}

extern "C" const char *anova_last_error(void) { return get_error(); }

extern "C" anova_status anova_plan_query(anova_plan_t p, int32_t l, anova_window_info *info) {
    return guarded([&] {
        ANOVA_REQUIRE(p != nullptr && info != nullptr, "NULL argument");
        ANOVA_REQUIRE(l >= 0 && l < p->P, "window index out of range");
        const WindowPlan &w = p->win[l];
        anova_window_info r{};
        r.d_A = w.dA; r.M = w.M; r.n = w.n; r.m = w.m; r.h = w.h;
        for (int t = 0; t < 3; ++t) r.center[t] = w.center[t];
        r.extent = w.extent;
        r.err_images = w.err_images; r.err_trunc = w.err_trunc; r.err_window = w.err_window;
        r.err_round = w.err_round; r.err_total = w.err_total;
        r.n_tiles = w.n_nonempty;
        r.n_subproblems = w.n_regions;
        r.per_cell = w.dense ? 1 : 0;
        r.tile = w.tile;
        *info = r;
    });
}

extern "C" anova_status anova_plan_shape(anova_plan_t p, int64_t *N, int32_t *P, int32_t *precision) {
    return guarded([&] {
        ANOVA_REQUIRE(p != nullptr, "NULL plan");
        if (N) *N = p->N;
        if (P) *P = p->P;
        if (precision) *precision = p->precision;
    });
}

extern "C" anova_status anova_matvec(anova_plan_t p, const double *alpha, double *out,
                                     int32_t nrhs, int64_t ld, double beta, void *stream) {
    return guarded([&] {
        ANOVA_REQUIRE(p != nullptr, "NULL plan");
        ANOVA_REQUIRE(alpha != nullptr && out != nullptr, "NULL vector");
        ANOVA_REQUIRE(nrhs >= 1, "nrhs must be >= 1");
        ANOVA_REQUIRE(ld >= p->N, "ld must be >= N");
        ANOVA_REQUIRE(std::isfinite(beta), "beta must be finite");
        plan_matvec(p, alpha, out, nrhs, ld, beta, (hipStream_t)stream);
    });
}

// one-window batches over the caller's grid (stage entry points)
static void stage_run(anova_plan_s *p, int32_t l, const double *alpha, double *out, void *grid,
                      unsigned mask, hipStream_t s) {
    BatchProblem bp;
    bp.plan = p;
    bp.alpha = alpha;
    bp.out = out;
    bp.nrhs = 1;
    bp.ld = p->N;
    bp.only_window = l;
    bp.grid_override = grid;
    Batch b;
    b.build({bp});
    b.run(s, nullptr, mask);
    ANOVA_HIP_CHECK(hipStreamSynchronize(s));  // the batch's work space dies here
}

extern "C" anova_status anova_stage_spread(anova_plan_t p, int32_t l, const double *alpha,
                                           void *grid, void *stream) {
    return guarded([&] {
        ANOVA_REQUIRE(p != nullptr && alpha != nullptr && grid != nullptr, "NULL argument");
        ANOVA_REQUIRE(l >= 0 && l < p->P, "window index out of range");
        stage_run(p, l, alpha, nullptr, grid, (1u << kStagePermute) | (1u << kStageSpread) |
                      (1u << kStageTileSum) | (1u << kStageFold),
                  (hipStream_t)stream);
    });
}

extern "C" anova_status anova_stage_convolve(anova_plan_t p, int32_t l, void *grid, void *stream) {
    return guarded([&] {
        ANOVA_REQUIRE(p != nullptr && grid != nullptr, "NULL argument");
        ANOVA_REQUIRE(l >= 0 && l < p->P, "window index out of range");
        // the coefficient column is not read by the convolution
        stage_run(p, l, static_cast<const double *>(grid), nullptr, grid, 1u << kStageConvolve,
                  (hipStream_t)stream);
    });
}

extern "C" anova_status anova_stage_gather(anova_plan_t p, int32_t l, const void *grid,
                                           double *out, void *stream) {
    return guarded([&] {
        ANOVA_REQUIRE(p != nullptr && grid != nullptr && out != nullptr, "NULL argument");
        ANOVA_REQUIRE(l >= 0 && l < p->P, "window index out of range");
        stage_run(p, l, out, out, const_cast<void *>(grid),
                  (1u << kStageGather) | (1u << kStageCombine), (hipStream_t)stream);
    });
}
