// Host FP64 construction of the per-axis grid-convolution coefficients.
//
// The fast summation of Section 3 replaces the Gaussian by the trigonometric
// polynomial k~(t) = sum_{k in I_N} b_k e^{2 pi i k t} and evaluates
// sum_k b_k (sum_i v_i e^{-2 pi i k x_i}) e^{2 pi i k x_j} with an adjoint and a
// forward NFFT. Here:
//  * every feature of a window is mapped affinely onto the box
//    |u| <= (1/2 - eps_b)/2, so all pairwise differences satisfy
//    |u_i - u_j| <= 1/2 - eps_b and the Gaussian width becomes sigma * scale;
//  * the Gaussian of one axis is made 1-periodic and smooth by a two-point
//    Taylor (Hermite) polynomial of degree 2p-1 on [1/2 - eps_b, 1/2 + eps_b]
//    that matches p-1 derivatives at both ends; its N samples give the b_k
//    (trigonometric interpolation), real and even; the unpaired frequency -N/2
//    is split evenly between +-N/2 so the interpolant is real;
//  * the NFFT deconvolution by the Kaiser-Bessel transform on both sides folds
//    into B_k = b_k / (n phi_hat(k))^2, and the composition FFT -> multiply by
//    B -> inverse FFT along one axis is the real symmetric circulant with first
//    column circ[d] = sum_k B_k cos(2 pi k d / n). Because the window kernel is
//    a product of one-dimensional Gaussians, the d-dimensional grid step is the
//    product of these one-axis circulants.
#include <cmath>
#include <limits>

#include "common.hpp"

namespace anv {

static double bessel_i0(double x) {
    // power series sum ((x/2)^{2j} / (j!)^2): positive terms, no cancellation
    double q = 0.25 * x * x, term = 1.0, sum = 1.0;
    for (int j = 1; j < 500; ++j) {
        term *= q / (double(j) * double(j));
        sum += term;
        if (term < 1e-18 * sum) break;
    }
    return sum;
}

double kb_window(double u, int m, double b) {
    double s2 = double(m) * m - u * u;
    double s = s2 > 0 ? std::sqrt(s2) : 0.0;
    double v = s > 0 ? std::sinh(b * s) / (M_PI * s) : b / M_PI;
    double v0 = std::sinh(b * m) / (M_PI * m);
    return v / v0;
}

double kb_hat(int k, int n, int m, double b) {
    double w = 2.0 * M_PI * k / n;
    double arg = b * b - w * w;
    double v0 = std::sinh(b * m) / (M_PI * m);
    double h;
    if (arg >= 0) {
        h = bessel_i0(m * std::sqrt(arg));
    } else {  // I0(i x) = J0(x), power series sum (-1)^j (x/2)^{2j} / (j!)^2
        double q = -0.25 * double(m) * m * arg, term = 1.0;
        h = 1.0;
        for (int j = 1; j < 200; ++j) {
            term *= -q / (double(j) * double(j));
            h += term;
            if (std::fabs(term) < 1e-18) break;
        }
    }
    return h / (double(n) * v0);
}

// j-th derivative of exp(-t^2/s^2): (-1/s)^j H_j(t/s) exp(-(t/s)^2), with the
// physicists' Hermite polynomials H_0 = 1, H_1 = 2u, H_{j+1} = 2u H_j - 2j H_{j-1}.
static double gauss_deriv(double t, double s, int j) {
    double u = t / s;
    double h0 = 1.0, h1 = 2.0 * u;
    double hj = (j == 0) ? h0 : h1;
    for (int i = 1; i < j; ++i) {
        double h2 = 2.0 * u * h1 - 2.0 * i * h0;
        h0 = h1;
        h1 = h2;
        hj = h2;
    }
    return std::pow(-1.0 / s, j) * hj * std::exp(-u * u);
}

// Periodic regularised Gaussian g_R(t), t in [-1/2, 1/2].
static double g_reg(double t, double s, double eps, int p) {
    double a = std::fabs(t);
    double t0 = 0.5 - eps;
    if (a <= t0) return std::exp(-(a / s) * (a / s));
    double h = 2.0 * eps;
    double x = (a - t0) / h;  // in [0, 1]
    double res = 0.0;
    double fact = 1.0;
    for (int j = 0; j < p; ++j) {
        if (j > 0) fact *= j;
        double hj = std::pow(h, j);
        double f0 = gauss_deriv(t0, s, j) * hj;
        double f1 = gauss_deriv(-t0, s, j) * hj;  // derivative of g(t - 1) at t = 1/2 + eps
        double A = 0.0, B = 0.0, c = 1.0;
        for (int k = 0; k < p - j; ++k) {
            if (k > 0) c = c * (p - 1 + k) / k;  // binomial(p-1+k, k)
            A += c * std::pow(x, k + j);
            B += c * std::pow(1.0 - x, k + j);
        }
        double sgn = (j % 2) ? -1.0 : 1.0;
        res += (std::pow(1.0 - x, p) * A * f0 + std::pow(x, p) * B * sgn * f1) / fact;
    }
    return res;
}

static void fourier_coeffs(double s, double eps, int p, int nbw, std::vector<double>& bk) {
    // b_k for k = -nbw/2 .. nbw/2-1 (index k + nbw/2)
    std::vector<double> g(nbw);
    for (int j = 0; j < nbw; ++j) g[j] = g_reg(double(j - nbw / 2) / nbw, s, eps, p);
    bk.assign(nbw, 0.0);
    for (int k = -nbw / 2; k < nbw / 2; ++k) {
        double acc = 0.0;
        for (int j = 0; j < nbw; ++j) acc += g[j] * std::cos(2.0 * M_PI * double(j - nbw / 2) * k / nbw);
        bk[k + nbw / 2] = acc / nbw;
    }
}

static double interp_error(const std::vector<double>& bk, double s, double eps, int nbw) {
    double half = 0.5 - eps, err = 0.0;
    const int npts = 400;
    for (int i = 0; i <= npts; ++i) {
        double t = half * double(i) / npts;  // the Gaussian is even
        double val = bk[0] * std::cos(M_PI * nbw * t);  // split Nyquist term
        for (int k = -nbw / 2 + 1; k < nbw / 2; ++k) val += bk[k + nbw / 2] * std::cos(2.0 * M_PI * k * t);
        err = std::max(err, std::fabs(val - std::exp(-(t / s) * (t / s))));
    }
    return err;
}

AxisCoef build_axis(double lo, double hi, double sigma, const NfftParams& prm) {
    AxisCoef ax;
    ax.lo = lo;
    ax.hi = hi;
    ax.center = 0.5 * (lo + hi);
    double half = 0.5 * (0.5 - prm.eps_b);  // box is [-half, half]
    ax.scale = (hi > lo) ? 2.0 * half / (hi - lo) : 1.0;
    ax.sigma_a = sigma * ax.scale;
    const int nbw = prm.n_bw, n = prm.n_os, m = prm.m;
    std::vector<double> bk;
    if (prm.reg_p > 0) {
        ax.reg_p = prm.reg_p;
        fourier_coeffs(ax.sigma_a, prm.eps_b, prm.reg_p, nbw, bk);
        ax.kerr = interp_error(bk, ax.sigma_a, prm.eps_b, nbw);
    } else {
        double best = std::numeric_limits<double>::infinity();
        std::vector<double> tmp;
        for (int p = 2; p <= 14; ++p) {
            fourier_coeffs(ax.sigma_a, prm.eps_b, p, nbw, tmp);
            double e = interp_error(tmp, ax.sigma_a, prm.eps_b, nbw);
            if (e < best) {
                best = e;
                bk = tmp;
                ax.reg_p = p;
            }
        }
        ax.kerr = best;
    }
    const double b = M_PI * (2.0 - double(nbw) / n);
    // B_k for k = 0..nbw/2 (even in k); the Nyquist entry carries half of b_{-nbw/2}
    std::vector<double> Bk(nbw / 2 + 1);
    for (int k = 0; k <= nbw / 2; ++k) {
        double bkv = (k == nbw / 2) ? 0.5 * bk[0] : bk[k + nbw / 2];
        double ph = double(n) * kb_hat(k, n, m, b);
        Bk[k] = bkv / (ph * ph);
    }
    ax.bk = bk;
    ax.circ.assign(n, 0.0);
    for (int dlt = 0; dlt < n; ++dlt) {
        double acc = Bk[0];
        for (int k = 1; k <= nbw / 2; ++k) acc += 2.0 * Bk[k] * std::cos(2.0 * M_PI * k * dlt / n);
        ax.circ[dlt] = acc;
    }
    return ax;
}

}  // namespace anv
