// Molière multiple-scattering tables (Sec. II.A.2 of arXiv:1409.8336 names a
// full Molière option beside the scaled Highland formula), in Bethe's form:
//   f(theta) theta dtheta = v dv [f0(v) + f1(v)/B + f2(v)/B^2],
//   v = theta / (chi_c sqrt B), f0 = 2 exp(-v^2),
//   fn(v) = (1/n!) Int_0^inf u J0(v u) exp(-u^2/4) [(u^2/4) ln(u^2/4)]^n du.
// The transport draws v from its distribution with q = -ln u through
// v^2 = q R(q, 1/B); ln R is tabulated here at
//   [1/B = 1/20 + j (2/9 - 1/20)/12, j < 13][q = k/8, k < 161]
// and interpolated bilinearly by the kernel.
//
// Route: the densities fn on a v grid (Gauss-Legendre panels over u, the C
// library's Bessel J0), their
// running integrals Fn(v) = Int_0^v fn v' dv' (Simpson), continued beyond
// v = 20 by the single-scattering asymptotics F1 = -(v^-2 + 2 v^-4) and
// F2 proportional to ln v / v^4; then P(V > v) = exp(-v^2) - F1/B - F2/B^2
// inverted by bisection.
#include <algorithm>
#include <cmath>
#include <math.h>
#include <mutex>
#include <thread>
#include <vector>

#include "tables.hpp"

namespace pmc {

namespace {

constexpr double kEuler = 0.57721566490153286;
constexpr double kVMax = 20.0;
constexpr int kNV = 2001;                 // v grid 0 .. 20, step 0.01
constexpr double kDV = kVMax / (kNV - 1);

// 16-point Gauss-Legendre nodes and weights on [-1, 1] by Newton's method on
// the Legendre polynomial
struct GaussLegendre {
    double x[16], w[16];
    GaussLegendre()
    {
        const int n = 16;
        for (int i = 0; i < n; ++i) {
            double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
            for (int it = 0; it < 100; ++it) {
                double p0 = 1.0, p1 = z;
                for (int k = 2; k <= n; ++k) {
                    const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                    p0 = p1;
                    p1 = p2;
                }
                dp = n * (z * p1 - p0) / (z * z - 1.0);
                const double dz = p1 / dp;
                z -= dz;
                if (std::fabs(dz) < 1e-16) break;
            }
            x[i] = z;
            w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
        }
    }
};

// fn(v), n = 1, 2: u in [0, 14] (exp(-u^2/4) < 1e-21 beyond) in 224 panels
double density(int n, double v, const GaussLegendre& gl)
{
    const int panels = 224;
    const double h = 14.0 / panels;
    double s = 0.0;
    for (int p = 0; p < panels; ++p) {
        const double c = (p + 0.5) * h;
        for (int i = 0; i < 16; ++i) {
            const double u = c + 0.5 * h * gl.x[i];
            const double y = 0.25 * u * u;
            const double t = y * std::log(y);
            const double g = std::exp(-y) * (n == 1 ? t : 0.5 * t * t);
            s += 0.5 * h * gl.w[i] * u * ::j0(v * u) * g;
        }
    }
    return s;
}

struct Running {
    std::vector<double> f1, f2;   // F1, F2 at v = i kDV
};

const Running& running()
{
    static Running r;
    static std::once_flag once;
    std::call_once(once, [] {
        const GaussLegendre gl;
        // densities on the grid and at the half steps
        std::vector<double> d1(2 * kNV - 1), d2(2 * kNV - 1);
        const int m = 2 * kNV - 1;
        const int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        std::vector<std::thread> pool;
        for (int w = 0; w < nth; ++w)
            pool.emplace_back([&, w] {
                for (int i = w; i < m; i += nth) {
                    const double v = 0.5 * i * kDV;
                    d1[i] = density(1, v, gl) * v;
                    d2[i] = density(2, v, gl) * v;
                }
            });
        for (auto& th : pool) th.join();
        r.f1.assign(kNV, 0.0);
        r.f2.assign(kNV, 0.0);
        for (int i = 1; i < kNV; ++i) {
            const int a = 2 * (i - 1), b = 2 * i - 1, c = 2 * i;
            r.f1[i] = r.f1[i - 1] + kDV / 6.0 * (d1[a] + 4.0 * d1[b] + d1[c]);
            r.f2[i] = r.f2[i - 1] + kDV / 6.0 * (d2[a] + 4.0 * d2[b] + d2[c]);
        }
    });
    return r;
}

// P(V > v) for 1/B = x
double survival(const Running& r, double x, double v)
{
    double f1, f2;
    if (v >= kVMax) {
        const double s = kVMax / v;
        f1 = -(1.0 / (v * v) + 2.0 / (v * v * v * v));
        f2 = r.f2[kNV - 1] * s * s * s * s * std::log(v) / std::log(kVMax);
    } else {
        const double t = v / kDV;
        const int i = std::min((int)t, kNV - 2);
        const double fr = t - i;
        f1 = r.f1[i] + fr * (r.f1[i + 1] - r.f1[i]);
        f2 = r.f2[i] + fr * (r.f2[i + 1] - r.f2[i]);
    }
    return std::exp(-v * v) - x * f1 - x * x * f2;
}

}  // namespace

const std::vector<float>& moliere_table()
{
    static std::vector<float> table;
    static std::once_flag once;
    std::call_once(once, [] {
        const Running& r = running();
        table.assign((size_t)kMolNX * kMolNQ, 0.f);
        const double f1_0 = 2.0 * (1.0 - kEuler);
        const double f2_0 = 2.0 * ((1.5 - kEuler) * (1.5 - kEuler) + M_PI * M_PI / 6.0 - 1.25);
        for (int j = 0; j < kMolNX; ++j) {
            const double x = 0.05 + j * (2.0 / 9.0 - 0.05) / (kMolNX - 1);
            // q = 0: v^2 / q -> 2 / f(0) as v -> 0
            table[(size_t)j * kMolNQ] = (float)std::log(2.0 / (2.0 + x * f1_0 + x * x * f2_0));
            for (int k = 1; k < kMolNQ; ++k) {
                const double q = k / 8.0, target = std::exp(-q);
                double lo = 0.0, hi = 1.0e5;
                for (int it = 0; it < 200; ++it) {
                    const double mid = 0.5 * (lo + hi);
                    if (survival(r, x, mid) > target) lo = mid;
                    else hi = mid;
                }
                const double v = 0.5 * (lo + hi);
                table[(size_t)j * kMolNQ + k] = (float)std::log(v * v / q);
            }
        }
    });
    return table;
}

void moliere_material(const double w[kNEl], float out[kMolMatFloats])
{
    // per element: weight w Z (Z + 1) / A, screening log ln chi_0^2 p^2 c^2 =
    // ln (0.0042134917^2 Z^(2/3)), Born parameter term 3.76 (Z alpha)^2
    constexpr double kChi0 = 0.0042134917;     // hbar c / (0.885 a_0), MeV
    constexpr double kAlpha = 0.0072973525693;
    double s1 = 0.0;
    for (int e = 0; e < kNEl; ++e) s1 += w[e] * kElemZ[e] * (kElemZ[e] + 1.0) / kElemA[e];
    double c = 0.0;
    for (int e = 0; e < kNEl; ++e) {
        const double z = kElemZ[e];
        const double om = s1 > 0.0 ? w[e] * z * (z + 1.0) / kElemA[e] / s1 : 0.0;
        c += om * std::log(kChi0 * kChi0 * std::cbrt(z * z));
        out[2 + e] = (float)om;
        out[2 + kNEl + e] = (float)(3.76 * (z * kAlpha) * (z * kAlpha));
    }
    out[0] = (float)s1;
    out[1] = (float)c;
}

}  // namespace pmc
