// Host-side physics tables of the engine (Sec. II.A.1-2 of arXiv:1409.8336):
// Bethe-Bloch stopping power, CSDA range on the shared 1000-point log grid,
// the water-equivalence factor of Eq. 1, radiation lengths and nuclear
// cross sections per gram.  Built once per load in double precision and
// stored as float32 tables for the device.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace pmc {

constexpr int kNE = 1000;           // energy grid points
constexpr double kEMin = 0.1;       // MeV; also the termination energy
constexpr double kEMax = 250.0;     // MeV
constexpr int kNEl = 7;             // H C N O P Ca Ti
constexpr int kInvN = 1024;         // coarse ln(range) index cells
constexpr int kMaxMat = 16;
constexpr int kSecNuc = 6, kSecBins = 25, kSecMult = 5, kSecCdf = 33;

constexpr double kProtonMeV = 938.272088;
constexpr double kElectronMeV = 0.51099895;
constexpr double kAmuMeV = 931.49410242;
constexpr double kBetheK = 0.307075;          // MeV cm^2 / mol
constexpr double kAvogadro = 6.02214076e23;
constexpr double kWaterIeV = 75.0;
constexpr double kFRefMeV = 100.0;            // f_m is evaluated here

extern const double kElemZ[kNEl];
extern const double kElemA[kNEl];
extern const int kElemMassNumber[kNEl];

double grid_energy(int i);                    // E_i = 0.1 * 2500^(i/999)
double grid_log_step();                       // ln(2500)/999
double bethe_bloch(double t_mev, double za, double i_ev);      // MeV cm^2/g, raw formula
double bethe_bloch_peak(double za, double i_ev);               // energy of its maximum
double water_z_over_a();
double radiation_length(const double w[kNEl]);                 // g/cm^2

// ln(range) table of one stopping medium on the grid, plus the coarse inverse
// index: lnr[i] = ln R(E_i) for i >= 1 (lnr[0] = lnr[1]; bin 0 is linear in
// range from 0 at 0.1 MeV), inv[c] = largest j in [1, 998] with
// lnr[j] <= lnr[1] + c * (lnr[999]-lnr[1])/(kInvN-1).
struct RangeTable {
    std::vector<float> lnr;
    std::vector<uint16_t> inv;
    double r_first = 0;          // R(E_1), cm * g/cm^3
    double inv_step = 0;         // kInvN-1 over the ln range span
    double ln_r1 = 0;
};
RangeTable build_range_table(double za, double i_ev);

struct Material {
    double za = 0, i_ev = 0, f = 1, x0 = 0;   // Z/A, I, Eq. 1 factor, X0 g/cm^2
    double nuclei_per_g_barn[kNEl] = {};     // n_i/rho * 1e-24 (cm^2 per barn per g)
    double w[kNEl] = {};
    double rho_lo = 0, rho_hi = 0;
    int hu_lo = 0, hu_hi = 0;
    bool own = false;
};

// Vavilov straggling quantile table (built once per process):
// [beta^2 = k/10][log10 kappa = -2 + j/10][z = -6 + i/8], standardised loss W.
constexpr int kVavNB = 5, kVavNK = 31, kVavNZ = 97;
const std::vector<float>& vavilov_table();

// Molière sampling table (built once per process): ln(v^2 / q) at
// [1/B = 1/20 + j (2/9 - 1/20)/12][q = k/8]; and the per-material constants
// the kernel's step needs: {sum w Z(Z+1)/A, sum_i omega_i ln chi_0,i^2 (pc)^2,
// omega_i (i < 7), 3.76 (Z_i alpha)^2 (i < 7)}, omega_i the Z(Z+1)/A weights.
constexpr int kMolNX = 13, kMolNQ = 161, kMolMatFloats = 16;
const std::vector<float>& moliere_table();
void moliere_material(const double w[kNEl], float out[kMolMatFloats]);

// Validates and derives the per-bin materials; returns "" or an error text.
std::string build_materials(int n_bins, const int16_t* hu_lo, const float* rho_lo,
                            const float* rho_hi, const float* mass_frac, const float* i_ev,
                            const int32_t* own, std::vector<Material>& out);

}  // namespace pmc
