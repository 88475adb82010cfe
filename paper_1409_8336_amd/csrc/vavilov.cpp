// Vavilov energy-loss straggling tables (Sec. II.A.2 of arXiv:1409.8336: a
// Vavilov-Gaussian model of the loss fluctuations).
//
// The loss of a step is <Delta> + sigma W with sigma^2 the Bohr variance and
// W standardised.  For kappa = xi / T_max in [0.01, 10) the transport draws W
// from Vavilov's distribution of (kappa, beta^2) by mapping the step's normal
// score z through the quantile function G(z) = F_W^-1(Phi(z)); outside that
// range W = z (Gaussian).  G is tabulated here for the device:
//   [beta^2 = k/10, k < 5][log10 kappa = -2 + j/10, j < 31][z = -6 + i/8, i < 97]
// and interpolated trilinearly by the kernel.
//
// Vavilov's model: energy transfers v T_max, v in (0, 1], to free electrons
// with density kappa (1 - beta^2 v) / v^2.  X = (Delta - <Delta>) / T_max then
// has ln E[exp(itX)] = kappa (A(t) + i B(t)) with, in closed form through the
// sine and cosine integrals,
//   A(t) = 1 - cos t - t Si(t) - beta^2 (Ci(t) - Euler - ln t),
//   B(t) = t - sin t + t (Ci(t) - Euler - ln t) - beta^2 (Si(t) - t),
// and W = X / sqrt(kappa (1 - beta^2 / 2)).  The density of X is the inverse
// Fourier integral f(x) = (1/pi) Int_0^inf exp(kappa A) cos(kappa B - t x) dt
// (trapezoidal rule), its distribution function the running integral of f
// over a grid dense in the Landau-like core, and G follows by inverse
// interpolation.
#include <algorithm>
#include <cmath>
#include <complex>
#include <mutex>
#include <thread>
#include <vector>

#include "tables.hpp"

namespace pmc {

namespace {

constexpr double kEuler = 0.57721566490153286;

// Si(t) and Cin(t) = Euler + ln t - Ci(t) for t > 0: power series up to t = 2,
// beyond that E1(i t) = -Ci(t) + i (Si(t) - pi/2) from its continued fraction
// (modified Lentz).
void sine_cosine_integrals(double t, double* si, double* cin)
{
    if (t <= 2.0) {
        double term_s = t, sum_s = t;          // Si = sum (-1)^n t^(2n+1) / ((2n+1)(2n+1)!)
        double term_c = 1.0, sum_c = 0.0;      // Cin = sum (-1)^(n+1) t^(2n) / (2n (2n)!)
        for (int n = 1; n < 30; ++n) {
            term_s *= -t * t / ((2.0 * n) * (2.0 * n + 1.0));
            sum_s += term_s / (2.0 * n + 1.0);
            term_c *= -t * t / ((2.0 * n - 1.0) * (2.0 * n));
            sum_c -= term_c / (2.0 * n);
        }
        *si = sum_s;
        *cin = sum_c;
        return;
    }
    const std::complex<double> z(0.0, t);
    const double tiny = 1e-300;
    std::complex<double> b = z + 1.0, c = 1.0 / tiny, d = 1.0 / b, h = d;
    for (int i = 1; i < 100000; ++i) {
        const double a = -(double)i * i;
        b += 2.0;
        d = 1.0 / (a * d + b);
        c = b + a / c;
        const std::complex<double> del = c * d;
        h *= del;
        if (std::abs(del - 1.0) < 1e-16) break;
    }
    const std::complex<double> e1 = h * std::exp(-z);
    *si = e1.imag() + 0.5 * M_PI;
    *cin = kEuler + std::log(t) + e1.real();     // Ci = -Re E1
}

// support of X used for the inversion: negligible mass (far below 1e-9) outside
void window(double kappa, double* lo, double* hi)
{
    *lo = -8.0 * std::sqrt(kappa) - 0.1;
    *hi = 4.0 + 8.0 * std::sqrt(kappa);
}

// quantile nodes G[i], z_i = -6 + i/8, of W for one (kappa, beta^2)
void quantile_nodes(double kappa, double beta2, float* g)
{
    double lo, hi;
    window(kappa, &lo, &hi);
    // trapezoidal frequency step: the periodic images of the density lie two
    // window widths apart; nodes until exp(kappa A) < e^-45
    const double dt = M_PI / (hi - lo);
    std::vector<double> amp, ph, tt;
    for (int j = 0;; ++j) {
        const double t = j * dt;
        double a, b;
        if (j == 0) {
            a = 0.0;
            b = 0.0;
        } else {
            double si, cin;
            sine_cosine_integrals(t, &si, &cin);
            a = 1.0 - std::cos(t) - t * si + beta2 * cin;
            b = t - std::sin(t) - t * cin - beta2 * (si - t);
        }
        if (kappa * a < -45.0) break;
        amp.push_back((j == 0 ? 0.5 : 1.0) * std::exp(kappa * a));
        ph.push_back(kappa * b);
        tt.push_back(t);
    }
    // points: uniform in lambda = X/kappa - (1 - Euler) - ln kappa (step
    // 1/40) through the core, then uniform in X to the window's end
    const double shift = (1.0 - kEuler) + std::log(kappa);
    const double l0 = std::max(-8.0, lo / kappa - shift);
    const double l_end = hi / kappa - shift;
    const double l1 = std::min(25.0, l_end);
    const int n1 = (int)std::ceil((l1 - l0) * 40.0) + 1, n2 = l_end > l1 ? 400 : 0;
    std::vector<double> x(n1 + n2), f(n1 + n2), cdf(n1 + n2);
    for (int i = 0; i < n1; ++i) x[i] = kappa * (l0 + (l1 - l0) * i / (n1 - 1) + shift);
    for (int i = 0; i < n2; ++i) x[n1 + i] = x[n1 - 1] + (hi - x[n1 - 1]) * (i + 1) / n2;
    for (size_t i = 0; i < x.size(); ++i) {
        double s = 0.0;
        for (size_t j = 0; j < amp.size(); ++j) s += amp[j] * std::cos(ph[j] - tt[j] * x[i]);
        f[i] = std::max(0.0, s * dt / M_PI);
    }
    // running trapezoidal integral, normalised to its end value
    cdf[0] = 0.0;
    for (size_t i = 1; i < x.size(); ++i) cdf[i] = cdf[i - 1] + 0.5 * (f[i] + f[i - 1]) * (x[i] - x[i - 1]);
    const double total = cdf.back();
    for (double& v : cdf) v /= total;
    const double c = std::sqrt(kappa * (1.0 - 0.5 * beta2));
    size_t at = 1;
    for (int q = 0; q < kVavNZ; ++q) {
        const double u = 0.5 * std::erfc(-(-6.0 + q / 8.0) / std::sqrt(2.0));
        while (at < x.size() - 1 && cdf[at] < u) ++at;
        const double fa = cdf[at - 1], fb = cdf[at];
        double xq = x[at];
        if (fb > fa) xq = x[at - 1] + (x[at] - x[at - 1]) * std::min(1.0, std::max(0.0, (u - fa) / (fb - fa)));
        g[q] = (float)(xq / c);
    }
}

}  // namespace

const std::vector<float>& vavilov_table()
{
    static std::vector<float> table;
    static std::once_flag once;
    std::call_once(once, [] {
        table.assign((size_t)kVavNB * kVavNK * kVavNZ, 0.f);
        const int rows = kVavNB * kVavNK;
        const int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        std::vector<std::thread> pool;
        for (int w = 0; w < nth; ++w)
            pool.emplace_back([w, nth, rows] {
                for (int r = w; r < rows; r += nth) {
                    const int b = r / kVavNK, j = r % kVavNK;
                    quantile_nodes(std::pow(10.0, -2.0 + j / 10.0), 0.1 * b, table.data() + (size_t)r * kVavNZ);
                }
            });
        for (auto& th : pool) th.join();
    });
    return table;
}

}  // namespace pmc
