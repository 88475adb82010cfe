// Host-side physics tables (see tables.hpp).
#include "tables.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>

namespace pmc {

const double kElemZ[kNEl] = {1, 6, 7, 8, 15, 20, 22};
const double kElemA[kNEl] = {1.00794, 12.0107, 14.0067, 15.9994, 30.973762, 40.078, 47.867};
const int kElemMassNumber[kNEl] = {1, 12, 14, 16, 31, 40, 48};

double grid_log_step() { return std::log(kEMax / kEMin) / (kNE - 1); }

double grid_energy(int i) { return kEMin * std::pow(kEMax / kEMin, double(i) / (kNE - 1)); }

// Bethe-Bloch mass stopping power without shell, density-effect or Barkas
// terms (the paper's tabulated water/titanium stopping powers are replaced by
// this closed form).
double bethe_bloch(double t, double za, double i_ev)
{
    const double m = kProtonMeV, me = kElectronMeV;
    const double e_tot = t + m;
    const double bg2 = t * (t + 2.0 * m) / (m * m);
    const double b2 = t * (t + 2.0 * m) / (e_tot * e_tot);
    const double gam = e_tot / m;
    const double ratio = me / m;
    const double tmax = 2.0 * me * bg2 / (1.0 + 2.0 * gam * ratio + ratio * ratio);
    const double i = i_ev * 1.0e-6;
    const double log_term = 0.5 * std::log(2.0 * me * bg2 * tmax / (i * i));
    return kBetheK * za / b2 * (log_term - b2);
}

// Below its maximum the formula drops towards zero; the tables hold S flat
// there (only titanium-like media reach it above 0.1 MeV).
double bethe_bloch_peak(double za, double i_ev)
{
    double lo = std::log(1.0e-3), hi = std::log(10.0);
    // ternary search on the unimodal curve
    for (int it = 0; it < 400 && hi - lo > 1e-14; ++it) {
        const double a = lo + (hi - lo) / 3.0, b = hi - (hi - lo) / 3.0;
        if (bethe_bloch(std::exp(a), za, i_ev) < bethe_bloch(std::exp(b), za, i_ev)) lo = a;
        else hi = b;
    }
    return std::exp(0.5 * (lo + hi));
}

double water_z_over_a()
{
    const double mass = 2.0 * kElemA[0] + kElemA[3];
    return (2.0 * kElemZ[0] + kElemZ[3]) / mass;
}

// Tsai's radiation length (as tabulated by the PDG), Bragg additivity in 1/X0.
static double element_radiation_length(int e)
{
    const double z = kElemZ[e], a = kElemA[e];
    const double alpha = 1.0 / 137.035999084;
    const double y = (alpha * z) * (alpha * z);
    const double fc = y * (1.0 / (1.0 + y) + 0.20206 - 0.0369 * y + 0.0083 * y * y - 0.002 * y * y * y);
    double l_rad, l_rad_p;
    if (e == 0) {
        l_rad = 5.31;
        l_rad_p = 6.144;
    } else {
        l_rad = std::log(184.15 / std::cbrt(z));
        l_rad_p = std::log(1194.0 / std::cbrt(z * z));
    }
    return 716.408 * a / (z * z * (l_rad - fc) + z * l_rad_p);
}

double radiation_length(const double w[kNEl])
{
    double inv = 0.0;
    for (int e = 0; e < kNEl; ++e)
        if (w[e] > 0) inv += w[e] / element_radiation_length(e);
    return 1.0 / inv;
}

// Range on the grid: integrate 1/S cell by cell (8-point Gauss-Legendre on
// four sub-cells in ln E, with the stopping-power kink of a flat-held region
// split out), R(0.1 MeV) = 0.
RangeTable build_range_table(double za, double i_ev)
{
    static const double gx[8] = {-0.9602898564975363, -0.7966664774136267, -0.5255324099163290,
                                 -0.1834346424956498, 0.1834346424956498, 0.5255324099163290,
                                 0.7966664774136267, 0.9602898564975363};
    static const double gw[8] = {0.1012285362903763, 0.2223810344533745, 0.3137066458778873,
                                 0.3626837833783620, 0.3626837833783620, 0.3137066458778873,
                                 0.2223810344533745, 0.1012285362903763};
    const double e_star = bethe_bloch_peak(za, i_ev);
    auto stop = [&](double e) { return bethe_bloch(std::max(e, e_star), za, i_ev); };
    auto integrate = [&](double la, double lb) {   // int E/S dlnE over [la, lb]
        const double half = 0.5 * (lb - la), mid = 0.5 * (la + lb);
        double acc = 0.0;
        for (int q = 0; q < 8; ++q) {
            const double e = std::exp(mid + half * gx[q]);
            acc += gw[q] * e / stop(e);
        }
        return acc * half;
    };
    std::vector<double> r(kNE, 0.0);
    const double ls = std::log(e_star);
    for (int i = 1; i < kNE; ++i) {
        const double la = std::log(grid_energy(i - 1)), lb = std::log(grid_energy(i));
        std::vector<double> cuts = {la};
        if (ls > la && ls < lb) cuts.push_back(ls);
        cuts.push_back(lb);
        double acc = 0.0;
        for (size_t k = 0; k + 1 < cuts.size(); ++k) {
            const double step = (cuts[k + 1] - cuts[k]) / 4.0;
            for (int s = 0; s < 4; ++s) acc += integrate(cuts[k] + s * step, cuts[k] + (s + 1) * step);
        }
        r[i] = r[i - 1] + acc;
    }
    RangeTable t;
    t.lnr.resize(kNE);
    for (int i = 1; i < kNE; ++i) t.lnr[i] = float(std::log(r[i]));
    t.lnr[0] = t.lnr[1];
    t.r_first = std::exp(double(t.lnr[1]));
    t.ln_r1 = t.lnr[1];
    const double span = double(t.lnr[kNE - 1]) - double(t.lnr[1]);
    t.inv_step = (kInvN - 1) / span;
    t.inv.resize(kInvN);
    int j = 1;
    for (int c = 0; c < kInvN; ++c) {
        const double target = double(t.lnr[1]) + c * span / (kInvN - 1);
        while (j < kNE - 2 && double(t.lnr[j + 1]) <= target) ++j;
        t.inv[c] = uint16_t(j);
    }
    return t;
}

std::string build_materials(int n_bins, const int16_t* hu_lo, const float* rho_lo,
                            const float* rho_hi, const float* mass_frac, const float* i_ev,
                            const int32_t* own, std::vector<Material>& out)
{
    if (n_bins < 1 || n_bins > kMaxMat) return "material table: n_bins must be in [1, 16]";
    if (!hu_lo || !rho_lo || !rho_hi || !mass_frac || !i_ev || !own)
        return "material table: NULL array";
    if (hu_lo[0] > -1000) return "material table: hu_lo[0] must be <= -1000";
    int n_own = 0;
    out.assign(n_bins, Material{});
    const double s_water = bethe_bloch(kFRefMeV, water_z_over_a(), kWaterIeV);
    for (int b = 0; b < n_bins; ++b) {
        Material& m = out[b];
        if (b > 0 && hu_lo[b] <= hu_lo[b - 1]) return "material table: hu_lo must ascend";
        if (hu_lo[b] > 3000) return "material table: hu_lo above 3000";
        if (!(rho_lo[b] > 0.f) || !(rho_hi[b] > 0.f)) return "material table: density must be > 0";
        if (!(i_ev[b] > 0.f)) return "material table: mean excitation energy must be > 0";
        m.hu_lo = hu_lo[b];
        m.hu_hi = b + 1 < n_bins ? hu_lo[b + 1] : 3000;
        m.rho_lo = rho_lo[b];
        m.rho_hi = rho_hi[b];
        m.i_ev = i_ev[b];
        m.own = own[b] != 0;
        n_own += m.own;
        double sum = 0.0;
        for (int e = 0; e < kNEl; ++e) {
            const double w = mass_frac[b * kNEl + e];
            if (!(w >= 0.0)) return "material table: negative mass fraction";
            m.w[e] = w;
            sum += w;
            m.za += w * kElemZ[e] / kElemA[e];
            m.nuclei_per_g_barn[e] = w * kAvogadro / kElemA[e] * 1.0e-24;
        }
        if (std::fabs(sum - 1.0) > 1e-4) return "material table: mass fractions must sum to 1";
        m.x0 = radiation_length(m.w);
        m.f = m.own ? 1.0 : bethe_bloch(kFRefMeV, m.za, m.i_ev) / s_water;   // Eq. 1
    }
    if (n_own > 1) return "material table: at most one own-table bin is supported";
    return "";
}

}  // namespace pmc
