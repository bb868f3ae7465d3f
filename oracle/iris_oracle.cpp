// FP64 reference ray-marcher for 13CO(2-1) position-position-velocity cubes.
//
// TEST INFRASTRUCTURE ONLY. This file is the oracle that the HIP library is
// checked against. Only the test suite, the smoke check and the CPU-baseline
// leg of the benchmark load it; the product path never does. It shares no
// source, header, table or constant generator with the HIP library.
//
// What it computes (paper sections named by title):
//  * RT equation, total and continuum split        -- "The Radiative Transfer Equation"
//  * dust: alpha = kappa*rho, blackbody source     -- "Dust Emission and Absorption"
//  * line j and alpha from level populations        -- "Line Emission and Absorption"
//  * Gaussian Doppler profile (+ microturbulence)   -- "Line Emission and Absorption"
//  * Einstein B from A                              -- "Einstein Coefficients, Collisions, and the Detailed Balance"
//  * LTE (Boltzmann) level populations              -- "Synthetic Observation Versus Density-Tracing"
//  * Doppler-shifted profile, T_inf cut             -- "Observability Determination"
//  * background intensity as initial condition      -- "Transfer Solution: Overview"
//  * formal (exponential) step, far -> near         -- "Transfer Solution: Formal and Smooth Integration ..."
//  * smooth integration: trapezoidal first step,    -- same section, BDF2 and TR step solutions
//    BDF2 after it, each step clamped at zero
//  * optically thin transfer: no absorption, the    -- "Transfer Solution: Optically Thin Transfer"
//    path integral of the emission with the channel-
//    averaged (erf) profile; midpoint sum (formal) or
//    Simpson panels over the nodes (smooth)
//  * selectively thin transfer: the line absorbs    -- "Transfer Solution: Selectively Thin Transfer"
//    the continuum but not itself; formal steps or
//    the smooth (TR, BDF2) steps with the mode's
//    substitution
//  * output units: Rayleigh-Jeans kelvin, specific   -- "Intensity Versus Temperature"
//    intensity, or the Planck brightness temperature
//    (inverse of the Planck function) of [T], [C], [B]
//  * continuum subtraction in intensity space       -- "Continuum Subtraction"
//  * velocity subsampling: march a fine grid of      -- "Transfer Solution: Optically Thick Transfer"
//    2 f n_chan + 1 velocities (channel edges and
//    2f - 1 points inside each channel), then each
//    channel's intensity is the composite Simpson
//    average over its 2f fine steps (f = 0: profile
//    at channel centres only)
//
// Everything runs in cgs units and double precision, densely over every
// (cell, channel) pair, in the order the paper states the method. The scalar
// type is a template parameter so that the same forward code runs on
// std::complex<double> for complex-step derivatives, which pin the
// hand-written reverse mode below.
//
// Readings where the paper is silent or garbled (also listed in the design
// notes of the repository):
//  * level energies: rigid rotor scaled so E_u - E_l = h nu0 / k exactly
//    (energy_mode 0), or the literal E_u with E_J proportional to J(J+1)
//    (energy_mode 1); partition sum over J = 0..j_max inclusive;
//  * profile in velocity space: phi_nu = (c/nu0) exp(-((v_k - v)/b)^2)/(b sqrt(pi)),
//    b^2 = 2kT/m + 2 sigma_turb^2, v > 0 receding, channel centres
//    v_k = v_lo + (k + 1/2) dv;
//  * continuum evaluated at the rest frequency (REST), so [C], [D], [B] are
//    channel independent;
//  * sightline index 0 is the far side; the background enters there;
//  * [B] = background attenuated by the dust column, [D] = dust emission
//    marched from zero intensity, [L] = [T] - [C];
//  * smooth integration: the nodes of the integrator are the cells, each
//    carrying its own coefficients; the background is the intensity at node
//    0 (the far cell), so N cells take N - 1 steps; [C], [D] and [B] are
//    integrated the same way as [T], each from its own start (background,
//    zero, background with no emission);
//  * optically thin transfer: the channel-averaged profile is the mean of
//    the Gaussian over the channel, (1/dv) (1/2) [erf(x_hi) - erf(x_lo)] in
//    velocity with x = (v_edge - v)/b; the formal integrator sums h f over
//    every cell, the smooth one takes Simpson panels of two cells over the
//    nodes 0 .. 2P, P = floor((N - 1)/2), leaving out the last cell when N
//    is even; the background is not attenuated;
//  * selectively thin transfer: within a cell's formal step the continuum
//    intensity absorbed by the line is the continuum after that cell (the
//    continuum step is solved first, then used in the total's step); under
//    the smooth integrator the node's continuum is solved first in the same
//    way and enters the emission of the total's TR or BDF2 step; every step
//    of the total, formal or smooth, is clamped at zero (the paper applies
//    its ReLU to each step of the selective mode).

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <type_traits>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// CODATA 2018 (cgs).
constexpr double kH = 6.62607015e-27;      // erg s
constexpr double kK = 1.380649e-16;        // erg / K
constexpr double kC = 2.99792458e10;       // cm / s
constexpr double kAMU = 1.66053906660e-24; // g
constexpr double kPi = 3.14159265358979323846;

using cplx = std::complex<double>;

inline double re(double x) { return x; }
inline double re(const cplx& z) { return z.real(); }
inline double ex(double x) { return std::exp(x); }
inline cplx ex(const cplx& z) { return std::exp(z); }
inline double sq(double x) { return std::sqrt(x); }
inline cplx sq(const cplx& z) { return std::sqrt(z); }
inline double em1(double x) { return std::expm1(x); }
// exp(z) - 1 for complex z = x + iy without cancellation in the real part:
// e^x cos y - 1 = expm1(x) cos y - 2 sin^2(y/2).
inline cplx em1(const cplx& z) {
  const double s = std::sin(0.5 * z.imag());
  return cplx(std::expm1(z.real()) * std::cos(z.imag()) - 2.0 * s * s,
              std::exp(z.real()) * std::sin(z.imag()));
}

}  // namespace

extern "C" {

// Line, dust and background constants. Mirrors the physical inputs of the
// library's own line struct but is declared here independently.
typedef struct {
  double nu0_hz;          // rest frequency of the transition
  double a_ul;            // Einstein A, s^-1
  double e_u_k;           // upper-level energy / k (used by energy_mode 1)
  int32_t j_u;            // upper rotational level (lower = j_u - 1)
  int32_t j_max;          // partition sum runs over J = 0..j_max
  double m_tracer_amu;    // tracer molecular mass
  double sigma_turb_kms;  // 1-D microturbulent velocity dispersion
  double kappa_dust;      // dust opacity per gram of dust, cm^2/g
  double dust_to_gas;     // dust-to-gas mass ratio
  double mu_amu;          // gas mass per H2 molecule, amu
  double t_bg_k;          // background (CMB) temperature
  double t_inf_k;         // no line emission/absorption above this temperature
  int32_t energy_mode;    // 0: E_u - E_l = h nu0/k exactly; 1: literal E_u
  int32_t units;          // outputs: 0 Rayleigh-Jeans K, 1 intensity (cgs), 2 Planck T_B
  int32_t integrator;     // 0 formal (exponential) steps, 1 smooth (TR, then BDF2)
  int32_t transfer;       // 0 optically thick, 1 optically thin, 2 selectively thin
} oracle_line;

}  // extern "C"

namespace {

struct Geometry {
  int64_t nx, ny, nz;
  int axis;
  int64_t n_los() const { return axis == 0 ? nx : axis == 1 ? ny : nz; }
  int64_t n_pix() const { return nx * ny * nz / n_los(); }
  // Flat C-order index of sightline position s (0 = far side) of pixel p.
  // Pixels enumerate the two remaining axes in C order.
  int64_t cell(int64_t p, int64_t s) const {
    if (axis == 0) { const int64_t y = p / nz, z = p % nz; return (s * ny + y) * nz + z; }
    if (axis == 1) { const int64_t x = p / nz, z = p % nz; return (x * ny + s) * nz + z; }
    const int64_t x = p / ny, y = p % ny;
    return (x * ny + y) * nz + s;
  }
};

struct Inputs {
  const double* lnn;    // ln n_H2 [cm^-3]
  const double* tkin;   // K
  const double* vlos;   // km/s, > 0 receding
  const double* xab;    // n(tracer)/n(H2)
  const double* tdust;  // K, or null for T_dust = T_kin
  Geometry g;
  double cell_cm;
  int n_chan;
  double v_lo_kms, dv_kms;
  int simpson_f;  // Simpson panels per channel; 0 = channel centres
  oracle_line line;
  // Non-LTE (optically thin level balance) populations of the observed
  // transition per cell, native layout, when given: FU = (g_l/g_u) f_u and
  // FL = f_l - FU, f the fractional populations (null: LTE).
  const double* ot_fu = nullptr;
  const double* ot_fl = nullptr;
};

// Level energy E_J / k in kelvin.
double level_energy(const oracle_line& L, int J) {
  if (L.energy_mode == 0) {
    // E_u - E_l = theta * 2 J_u = h nu0 / k.
    const double theta = kH * L.nu0_hz / kK / (2.0 * L.j_u);
    return theta * J * (J + 1.0);
  }
  const double theta = L.e_u_k / (L.j_u * (L.j_u + 1.0));
  return theta * J * (J + 1.0);
}

// Planck intensity B_nu(T), erg s^-1 cm^-2 Hz^-1 sr^-1 (dust source function
// and background, "Dust Emission and Absorption").
template <class S>
S planck(double nu, const S& T) {
  if (!(re(T) > 0.0)) return S(0.0);  // zero-temperature limit
  return (2.0 * kH * nu * nu * nu / (kC * kC)) / em1((kH * nu / kK) / T);
}

// Per-cell coefficients, all cgs.
template <class S>
struct CellCoef {
  S jL0, aL0;   // frequency-integrated line emission / absorption ("Line Emission and Absorption")
  S aD, jD;     // dust absorption and emission
  S b_cms;      // Doppler parameter
  S v_cms;      // line-of-sight velocity
  S Z, n_u, n_l, N;
};

template <class S>
CellCoef<S> cell_coefficients(const oracle_line& L, const S& lnn, const S& T, const S& v_kms,
                              const S& X, const S& Td) {
  CellCoef<S> c;
  const S nH2 = ex(lnn);
  c.N = X * nH2;
  // Boltzmann populations n_i = N g_i exp(-E_i/kT) / Z.
  S Z = S(0.0);
  for (int J = 0; J <= L.j_max; ++J) Z += (2.0 * J + 1.0) * ex(-level_energy(L, J) / T);
  c.Z = Z;
  const int Ju = L.j_u, Jl = L.j_u - 1;
  const double gu = 2.0 * Ju + 1.0, gl = 2.0 * Jl + 1.0;
  c.n_u = c.N * gu * ex(-level_energy(L, Ju) / T) / Z;
  c.n_l = c.N * gl * ex(-level_energy(L, Jl) / T) / Z;
  // Einstein relations.
  const double nu = L.nu0_hz;
  const double Bul = kC * kC * L.a_ul / (2.0 * kH * nu * nu * nu);
  const double Blu = gu / gl * Bul;
  const double e0 = kH * nu / (4.0 * kPi);
  if (re(T) > L.t_inf_k) {
    c.jL0 = S(0.0);
    c.aL0 = S(0.0);
  } else {
    c.jL0 = e0 * c.n_u * L.a_ul;
    c.aL0 = e0 * (c.n_l * Blu - c.n_u * Bul);
  }
  // Thermal plus microturbulent Doppler parameter.
  const double m = L.m_tracer_amu * kAMU;
  const double st = L.sigma_turb_kms * 1e5;
  c.b_cms = sq(2.0 * kK * T / m + 2.0 * st * st);
  c.v_cms = v_kms * 1e5;
  // Dust: alpha = kappa_dust * (dust/gas) * rho_gas; Kirchhoff source.
  const S rho = L.mu_amu * kAMU * nH2;
  c.aD = L.kappa_dust * L.dust_to_gas * rho;
  c.jD = c.aD * planck(nu, Td);
  return c;
}

// Line profile phi_nu (per Hz) at channel velocity vk_cms: the Gaussian of
// "Line Emission and Absorption" written in velocity, with the Jacobian c/nu0.
template <class S>
S profile(const CellCoef<S>& c, double vk_cms, double nu0) {
  const S x = (vk_cms - c.v_cms) / c.b_cms;
  return (kC / nu0) * ex(-x * x) / (c.b_cms * std::sqrt(kPi));
}

// One formal step through a cell of length h with constant j, alpha:
// I' = I e^{-tau} + (j/alpha)(1 - e^{-tau}), tau = h alpha; the tau = 0 limit
// is I + h j.
template <class S>
S formal_step(const S& I, const S& j, const S& a, double h) {
  const S tau = h * a;
  if (re(tau) == 0.0) return I + h * j;
  return I * ex(-tau) - (j / a) * em1(-tau);
}

// Smooth integration of dI/ds = j - alpha I between nodes one cell apart.
// Step n >= 1 gives I_n from I_{n-1} (I1) and I_{n-2} (I2): the trapezoidal
// rule for the first step, which also needs the coefficients j1, a1 of node
// n - 1, and the two-step backward differentiation formula (BDF2) after it.
// The equation is linear in I, so both implicit relations solve in closed
// form. Every step is clamped at zero intensity.
template <class S>
S smooth_step(int64_t n, const S& I1, const S& I2, const S& j1, const S& a1, const S& j,
              const S& a, double h) {
  S I = n == 1 ? (h * (j1 + j) + (2.0 - h * a1) * I1) / (2.0 + h * a)
               : (2.0 * h * j + 4.0 * I1 - I2) / (3.0 + 2.0 * h * a);
  if (re(I) < 0.0) I = S(0.0);
  return I;
}

// State of one smoothly integrated intensity: the two latest nodes and the
// coefficients of the latest.
template <class S>
struct SmoothRun {
  S I1, I2, j1, a1;
  int64_t n = 0;  // nodes taken
  explicit SmoothRun(const S& start) : I1(start), I2(start), j1(S(0.0)), a1(S(0.0)) {}
  void node(const S& j, const S& a, double h) {
    if (n > 0) {
      const S I = smooth_step(n, I1, I2, j1, a1, j, a, h);
      I2 = I1;
      I1 = I;
    }
    j1 = j;
    a1 = a;
    ++n;
  }
};

// Optically thin transfer ("Transfer Solution: Optically Thin Transfer"):
// no absorption, so every intensity is the background plus the path
// integral of its emission, sum over cells of weight * h * f. The formal
// integrator weighs every cell by 1 (each cell is the midpoint of its own
// step); the smooth one takes Simpson panels of two cells, weights
// 1 4 2 4 ... 4 1 / 3 over the nodes 0 .. 2P, P = floor((N - 1)/2).
double thin_weight(int integrator, int64_t n, int64_t N) {
  if (integrator == 0) return 1.0;
  const int64_t last = 2 * ((N - 1) / 2);
  if (last == 0 || n > last) return 0.0;
  if (n == 0 || n == last) return 1.0 / 3.0;
  return n % 2 ? 4.0 / 3.0 : 2.0 / 3.0;
}

double channel_velocity_cms(const Inputs& in, int k) {
  return (in.v_lo_kms + (k + 0.5) * in.dv_kms) * 1e5;
}

// Velocities the march samples: channel centres (f = 0), or the fine grid
// v_lo + j dv / (2f), j = 0 .. 2 f n_chan, whose points 2fk and 2f(k+1) are
// the edges of channel k.
int march_samples(const Inputs& in) {
  return in.simpson_f > 0 ? 2 * in.simpson_f * in.n_chan + 1 : in.n_chan;
}
double sample_velocity_cms(const Inputs& in, int j) {
  if (in.simpson_f == 0) return channel_velocity_cms(in, j);
  return (in.v_lo_kms + j * in.dv_kms / (2.0 * in.simpson_f)) * 1e5;
}

// Channel average of the line profile ("Transfer Solution: Selectively Thin
// Transfer", the integrated profile; the optically thin mode uses the same):
// phibar_k = (c/nu0) (1/dv) (1/2) [erf(x_hi) - erf(x_lo)], x = (v_edge - v)/b
// at the edges v_lo + k dv and v_lo + (k + 1) dv of channel k.
double channel_profile(const Inputs& in, const CellCoef<double>& c, int k) {
  const double dv = in.dv_kms * 1e5;
  const double lo = (in.v_lo_kms * 1e5 + k * dv - c.v_cms) / c.b_cms;
  const double hi = (in.v_lo_kms * 1e5 + (k + 1) * dv - c.v_cms) / c.b_cms;
  return (kC / in.line.nu0_hz) / dv * 0.5 * (std::erf(hi) - std::erf(lo));
}
// Weight of fine sample 2fk + i (i = 0 .. 2f) in the average of channel k:
// composite Simpson over 2f steps, 1 4 2 4 ... 2 4 1, divided by 6f.
double simpson_weight(int f, int i) {
  const double w = (i == 0 || i == 2 * f) ? 1.0 : (i % 2 ? 4.0 : 2.0);
  return w / (6.0 * f);
}

// Optional complex perturbation of one field value of one cell.
struct Perturb {
  int field = -1;       // 0 lnn, 1 T, 2 v, 3 X, 4 Tdust
  int64_t cell = -1;
  double h = 0.0;
};

template <class S>
S field_value(const double* a, int64_t idx, int field, const Perturb* pt) {
  S v = S(a[idx]);
  if (pt && pt->field == field && pt->cell == idx) v += S(cplx(0.0, pt->h));
  return v;
}
template <>
double field_value<double>(const double* a, int64_t idx, int, const Perturb*) { return a[idx]; }

// Line coefficients from non-LTE populations of the observed transition
// ("Level Populations: Mathematical Solution" for f; "Line Emission and
// Absorption" for j and alpha): n_u = N f_u, n_l = N f_l with
// f_u = (g_u/g_l) FU, f_l = FL + FU; where FL is not positive the cell
// carries no line.
template <class S>
void ot_line_coefficients(const oracle_line& L, double FU, double FL, const S& T,
                          CellCoef<S>& c) {
  const double gu = 2.0 * L.j_u + 1.0, gl = 2.0 * L.j_u - 1.0;
  if (!(FL > 0.0) || re(T) > L.t_inf_k) {
    c.n_u = c.n_l = c.jL0 = c.aL0 = S(0.0);
    return;
  }
  const double nu = L.nu0_hz;
  const double Bul = kC * kC * L.a_ul / (2.0 * kH * nu * nu * nu);
  const double Blu = gu / gl * Bul;
  const double e0 = kH * nu / (4.0 * kPi);
  c.n_u = c.N * (gu / gl * FU);
  c.n_l = c.N * (FL + FU);
  c.jL0 = e0 * c.n_u * L.a_ul;
  c.aL0 = e0 * (c.n_l * Blu - c.n_u * Bul);
}

template <class S>
CellCoef<S> coefficients_at(const Inputs& in, int64_t idx, const Perturb* pt) {
  const S lnn = field_value<S>(in.lnn, idx, 0, pt);
  const S T = field_value<S>(in.tkin, idx, 1, pt);
  const S v = field_value<S>(in.vlos, idx, 2, pt);
  const S X = field_value<S>(in.xab, idx, 3, pt);
  const S Td = in.tdust ? field_value<S>(in.tdust, idx, 4, pt) : T;
  CellCoef<S> c = cell_coefficients<S>(in.line, lnn, T, v, X, Td);
  if (in.ot_fu) ot_line_coefficients<S>(in.line, in.ot_fu[idx], in.ot_fl[idx], T, c);
  return c;
}

// Forward march of one sightline; outputs in the line's units. outT/outL
// have n_chan entries; C, D, B are channel independent (REST). [L] and [D]
// are intensity-space quantities (a difference, and an emission marched
// from zero): under Planck brightness temperature units they stay in
// Rayleigh-Jeans kelvin.
template <class S>
void march(const Inputs& in, int64_t p, const Perturb* pt, S* outT, S* outC, S* outD, S* outB,
           S* outL) {
  const int C = in.n_chan;
  const double nu = in.line.nu0_hz;
  const double h = in.cell_cm;
  const S Ibg = planck(nu, S(in.line.t_bg_k));
  const int M = march_samples(in);
  std::vector<S> IT(M, Ibg);
  S IC = Ibg, ID = S(0.0), tauD = S(0.0);
  const int64_t N = in.g.n_los();
  S IB = Ibg;
  if (in.line.transfer == 1) {
    // Optically thin: the emission of each cell with the channel average
    // of its profile, phibar_k = (c/nu0) (1/dv) (1/2) [erf(x_hi) - erf(x_lo)],
    // x = (v_edge - v)/b at the channel's edges v_lo + k dv, v_lo + (k+1) dv.
    if constexpr (std::is_same<S, double>::value) {
      for (int64_t s = 0; s < N; ++s) {
        const double w = thin_weight(in.line.integrator, s, N) * h;
        if (w == 0.0) continue;
        const CellCoef<S> c = coefficients_at<S>(in, in.g.cell(p, s), pt);
        for (int k = 0; k < M; ++k) IT[k] += w * (c.jL0 * channel_profile(in, c, k) + c.jD);
        IC += w * c.jD;
        ID += w * c.jD;
      }
    } else {
      for (int k = 0; k < M; ++k) IT[k] = S(NAN);  // no complex erf: not differentiated
      IC = ID = IB = S(NAN);
    }
  } else if (in.line.transfer == 2 && in.line.integrator == 0) {
    // Selectively thin ("Transfer Solution: Selectively Thin Transfer"): the
    // line does not absorb itself. Each cell's continuum step is solved
    // first; the total then takes the formal step with the dust absorption
    // only and the emission jbar_L + j_D - alphabar_L I_C, I_C the continuum
    // just solved for this cell, with the channel-averaged profile. As every
    // step of the selective mode ("Transfer Solution: Formal and Smooth
    // Integration ...", the ReLU of the selective substitution), each formal
    // step of the total is clamped at zero intensity: a line colder than the
    // continuum it absorbs can otherwise drive the total negative.
    if constexpr (std::is_same<S, double>::value) {
      for (int64_t s = 0; s < N; ++s) {
        const CellCoef<S> c = coefficients_at<S>(in, in.g.cell(p, s), pt);
        IC = formal_step(IC, c.jD, c.aD, h);
        ID = formal_step(ID, c.jD, c.aD, h);
        tauD += h * c.aD;
        for (int k = 0; k < M; ++k)
          IT[k] = std::max(0.0, formal_step(IT[k], (c.jL0 - c.aL0 * IC) * channel_profile(in, c, k)
                                                       + c.jD, c.aD, h));
      }
      IB = Ibg * ex(-tauD);
    } else {
      for (int k = 0; k < M; ++k) IT[k] = S(NAN);  // no complex erf: not differentiated
      IC = ID = IB = S(NAN);
    }
  } else if (in.line.integrator == 1) {
    // Smooth integration: every intensity is integrated over the nodes.
    // Selectively thin: the substitution of the selective mode, the
    // channel-averaged profile with the emission jbar_L + j_D - alphabar_L I_C
    // (I_C the continuum at the same node, solved first) and the dust
    // absorption only.
    std::vector<SmoothRun<S>> RT(M, SmoothRun<S>(Ibg));
    SmoothRun<S> RC(Ibg), RD(S(0.0)), RB(Ibg);
    for (int64_t s = 0; s < N; ++s) {
      const CellCoef<S> c = coefficients_at<S>(in, in.g.cell(p, s), pt);
      RC.node(c.jD, c.aD, h);
      RD.node(c.jD, c.aD, h);
      RB.node(S(0.0), c.aD, h);
      if (in.line.transfer == 2) {
        if constexpr (std::is_same<S, double>::value) {
          for (int k = 0; k < M; ++k)
            RT[k].node((c.jL0 - c.aL0 * RC.I1) * channel_profile(in, c, k) + c.jD, c.aD, h);
        } else {
          for (int k = 0; k < M; ++k) RT[k].node(S(NAN), S(NAN), h);  // no complex erf
        }
        continue;
      }
      for (int k = 0; k < M; ++k) {
        const S phi = profile(c, sample_velocity_cms(in, k), nu);
        RT[k].node(c.jL0 * phi + c.jD, c.aL0 * phi + c.aD, h);
      }
    }
    for (int k = 0; k < M; ++k) IT[k] = RT[k].I1;
    IC = RC.I1;
    ID = RD.I1;
    IB = RB.I1;
  } else {
    for (int64_t s = 0; s < N; ++s) {
      const CellCoef<S> c = coefficients_at<S>(in, in.g.cell(p, s), pt);
      for (int k = 0; k < M; ++k) {
        const S phi = profile(c, sample_velocity_cms(in, k), nu);
        const S a = c.aL0 * phi + c.aD;
        const S j = c.jL0 * phi + c.jD;
        IT[k] = formal_step(IT[k], j, a, h);
      }
      IC = formal_step(IC, c.jD, c.aD, h);
      ID = formal_step(ID, c.jD, c.aD, h);
      tauD += h * c.aD;
    }
    IB = Ibg * ex(-tauD);
  }
  if (in.simpson_f > 0) {
    // Channel averages of the emergent intensity (post-transfer integration).
    const int f = in.simpson_f;
    std::vector<S> avg(C, S(0.0));
    for (int k = 0; k < C; ++k)
      for (int i = 0; i <= 2 * f; ++i) avg[k] += simpson_weight(f, i) * IT[2 * f * k + i];
    IT.swap(avg);
  }
  const double rj = kC * kC / (2.0 * kK * nu * nu);  // T_RJ per unit intensity
  if (in.line.units == 2) {
    // Planck brightness temperature: the T with B_nu(T) = I, inverting
    // B = (2 h nu^3 / c^2) / (e^{h nu / k T} - 1).
    const double a = 2.0 * kH * nu * nu * nu / (kC * kC), t0 = kH * nu / kK;
    auto tb = [&](const S& I) { return I == S(0.0) ? S(0.0) : t0 / std::log(1.0 + a / I); };
    for (int k = 0; k < C; ++k) outT[k] = tb(IT[k]);
    *outC = tb(IC);
    *outB = tb(IB);
    *outD = rj * ID;
    for (int k = 0; k < C; ++k) outL[k] = rj * (IT[k] - IC);
    return;
  }
  const double u = in.line.units == 1 ? 1.0 : rj;  // output units per unit intensity
  for (int k = 0; k < C; ++k) outT[k] = u * IT[k];
  *outC = u * IC;
  *outD = u * ID;
  *outB = u * IB;
  for (int k = 0; k < C; ++k) outL[k] = outT[k] - *outC;
}

// ---------------------------------------------------------------------------
// Hand-written reverse mode of march<double>, for the loss
//   L = sum_k gT_k [T]_k + gC_k [C] + gD_k [D] + gL_k [L]_k + gB_k [B].
// Gradients are with respect to the stored field values (ln n_H2, T_kin,
// v_los in km/s, X, and T_dust when given).

struct StepAdj { double dI, dj, da; };

// Adjoint of formal_step for output cotangent g.
StepAdj formal_step_adj(double I, double j, double a, double h, double g) {
  const double tau = h * a;
  if (tau == 0.0) return {g, g * h, g * (-h * I - 0.5 * h * h * j)};
  const double e = std::exp(-tau);
  const double f = -std::expm1(-tau);
  StepAdj r;
  r.dI = g * e;
  r.dj = g * f / a;
  // d/da of (j/a) f(h a) and of I e^{-h a}.
  r.da = g * (-j * f / (a * a) + (j / a - I) * h * e);
  return r;
}

// With non-LTE populations given per cell (in.ot_fu, in.ot_fl), the line
// coefficients' share of the chain rule stops at those two inputs: their
// gradients go to gfu, gfl (the populations' own dependence on the fields is
// the caller's).
void march_adjoint(const Inputs& in, int64_t p, const double* gT, const double* gC,
                   const double* gD, const double* gL, const double* gB, double* glnn,
                   double* gt, double* gv, double* gx, double* gtd, double* gfu = nullptr,
                   double* gfl = nullptr) {
  const int C = in.n_chan;
  const double nu = in.line.nu0_hz;
  const double h = in.cell_cm;
  const int64_t N = in.g.n_los();
  const double Ibg = planck(nu, in.line.t_bg_k);
  // Output units per unit intensity (Rayleigh-Jeans kelvin or intensity).
  const double rj = in.line.units == 1 ? 1.0 : kC * kC / (2.0 * kK * nu * nu);

  // Forward sweep over the marched samples, keeping the state entering
  // each cell.
  const int M = march_samples(in);
  std::vector<CellCoef<double>> cc(N);
  std::vector<double> IT_in((size_t)N * M), IC_in(N), ID_in(N);
  std::vector<double> IT(M, Ibg);
  double IC = Ibg, ID = 0.0, tauD = 0.0;
  std::vector<double> phi((size_t)N * M);
  for (int64_t s = 0; s < N; ++s) {
    cc[s] = coefficients_at<double>(in, in.g.cell(p, s), nullptr);
    const CellCoef<double>& c = cc[s];
    std::memcpy(&IT_in[(size_t)s * M], IT.data(), sizeof(double) * M);
    IC_in[s] = IC;
    ID_in[s] = ID;
    for (int k = 0; k < M; ++k) {
      const double ph = profile(c, sample_velocity_cms(in, k), nu);
      phi[(size_t)s * M + k] = ph;
      IT[k] = formal_step(IT[k], c.jL0 * ph + c.jD, c.aL0 * ph + c.aD, h);
    }
    IC = formal_step(IC, c.jD, c.aD, h);
    ID = formal_step(ID, c.jD, c.aD, h);
    tauD += h * c.aD;
  }

  // Output cotangents -> intensity cotangents (through the channel average
  // onto the fine samples when subsampled).
  std::vector<double> bIT(M, 0.0);
  double bIC = 0.0, bID = 0.0, btauD = 0.0;
  for (int k = 0; k < C; ++k) {
    const double gt_k = (gT ? gT[k] : 0.0) + (gL ? gL[k] : 0.0);
    if (in.simpson_f > 0) {
      const int f = in.simpson_f;
      for (int i = 0; i <= 2 * f; ++i) bIT[2 * f * k + i] += rj * gt_k * simpson_weight(f, i);
    } else {
      bIT[k] = rj * gt_k;
    }
    bIC += rj * ((gC ? gC[k] : 0.0) - (gL ? gL[k] : 0.0));
    bID += rj * (gD ? gD[k] : 0.0);
    // [B] = rj Ibg exp(-tauD)
    btauD += -(gB ? gB[k] : 0.0) * rj * Ibg * std::exp(-tauD);
  }

  const oracle_line& L = in.line;
  const int Ju = L.j_u, Jl = L.j_u - 1;
  const double gu = 2.0 * Ju + 1.0, gl = 2.0 * Jl + 1.0;
  const double Bul = kC * kC * L.a_ul / (2.0 * kH * nu * nu * nu);
  const double Blu = gu / gl * Bul;
  const double e0 = kH * nu / (4.0 * kPi);
  const double m = L.m_tracer_amu * kAMU;
  const double Eu = level_energy(L, Ju), El = level_energy(L, Jl);

  for (int64_t s = N - 1; s >= 0; --s) {
    const CellCoef<double>& c = cc[s];
    double bjL0 = 0.0, baL0 = 0.0, baD = 0.0, bjD = 0.0, bv = 0.0, bb = 0.0;
    if (in.line.transfer == 1) {
      // Optically thin: I_k gains w h (jL0 phibar_k + jD), [C] and [D] gain
      // w h jD; nothing attenuates, so the cotangents pass unchanged. With
      // A = (c/nu0)/(2 dv) and the channel edges' x = (v_edge - v)/b,
      // d phibar/d v = A (2/sqrt(pi)) (e^{-lo^2} - e^{-hi^2}) / b and
      // d phibar/d b = A (2/sqrt(pi)) (lo e^{-lo^2} - hi e^{-hi^2}) / b.
      const double w = thin_weight(in.line.integrator, s, N) * h;
      if (w != 0.0) {
        const double dvc = in.dv_kms * 1e5;
        const double A2 = (kC / nu) / dvc * 0.5 * 2.0 / std::sqrt(kPi);
        for (int k = 0; k < M; ++k) {
          const double g = w * bIT[k];
          bjL0 += g * channel_profile(in, c, k);
          bjD += g;
          const double lo = (in.v_lo_kms * 1e5 + k * dvc - c.v_cms) / c.b_cms;
          const double hi = (in.v_lo_kms * 1e5 + (k + 1) * dvc - c.v_cms) / c.b_cms;
          const double el = std::exp(-lo * lo), eh = std::exp(-hi * hi);
          bv += g * c.jL0 * A2 * (el - eh) / c.b_cms;
          bb += g * c.jL0 * A2 * (lo * el - hi * eh) / c.b_cms;
        }
        bjD += w * (bIC + bID);
      }
    } else {
    for (int k = 0; k < M; ++k) {
      const double ph = phi[(size_t)s * M + k];
      const double a = c.aL0 * ph + c.aD, j = c.jL0 * ph + c.jD;
      const StepAdj r = formal_step_adj(IT_in[(size_t)s * M + k], j, a, h, bIT[k]);
      bIT[k] = r.dI;
      baL0 += r.da * ph;
      bjL0 += r.dj * ph;
      baD += r.da;
      bjD += r.dj;
      const double bphi = r.da * c.aL0 + r.dj * c.jL0;
      // phi = (c/nu)/(b sqrt(pi)) exp(-x^2), x = (v_k - v)/b
      const double x = (sample_velocity_cms(in, k) - c.v_cms) / c.b_cms;
      bv += bphi * ph * 2.0 * x / c.b_cms;
      bb += bphi * ph * (2.0 * x * x - 1.0) / c.b_cms;
    }
    {
      const StepAdj rc = formal_step_adj(IC_in[s], c.jD, c.aD, h, bIC);
      bIC = rc.dI;
      baD += rc.da;
      bjD += rc.dj;
      const StepAdj rd = formal_step_adj(ID_in[s], c.jD, c.aD, h, bID);
      bID = rd.dI;
      baD += rd.da;
      bjD += rd.dj;
      baD += btauD * h;
    }
    }
    // Chain rule to the stored fields of this cell.
    const int64_t idx = in.g.cell(p, s);
    const double lnn = in.lnn[idx], T = in.tkin[idx], X = in.xab[idx];
    const double Td = in.tdust ? in.tdust[idx] : T;
    const double nH2 = std::exp(lnn);
    double blnn = 0.0, bT = 0.0, bX = 0.0, bTd = 0.0;
    // jD = aD B(Td); B'(T) = B x e^x / (T expm1(x)), x = h nu / k T.
    const double B = planck(nu, Td);
    const double xd = kH * nu / (kK * Td);
    const double dB = B * xd * std::exp(xd) / (Td * std::expm1(xd));
    baD += bjD * B;
    bTd += bjD * c.aD * dB;
    // aD proportional to n_H2 = e^lnn.
    blnn += baD * c.aD;
    // Line coefficients (zero with no gradient above T_inf).
    if (in.ot_fu) {
      // n_u = N (g_u/g_l) FU, n_l = N (FL + FU), N = X n_H2; no line where
      // FL is not positive.
      const double FU = in.ot_fu[idx], FL = in.ot_fl[idx];
      double bFU = 0.0, bFL = 0.0;
      if (FL > 0.0 && T <= L.t_inf_k) {
        const double bnu = bjL0 * e0 * L.a_ul - baL0 * e0 * Bul;
        const double bnl = baL0 * e0 * Blu;
        const double Ntr = X * nH2;
        const double bN = bnu * (gu / gl * FU) + bnl * (FL + FU);
        bX += bN * nH2;
        blnn += bN * Ntr;
        bFU = Ntr * (bnu * gu / gl + bnl);
        bFL = Ntr * bnl;
      }
      gfu[idx] = bFU;
      gfl[idx] = bFL;
    } else if (T <= L.t_inf_k) {
      const double bnu = bjL0 * e0 * L.a_ul - baL0 * e0 * Bul;
      const double bnl = baL0 * e0 * Blu;
      double Z = 0.0, ZT = 0.0;
      for (int J = 0; J <= L.j_max; ++J) {
        const double E = level_energy(L, J);
        const double w = (2.0 * J + 1.0) * std::exp(-E / T);
        Z += w;
        ZT += w * E / (T * T);
      }
      const double fu = gu * std::exp(-Eu / T) / Z, fl = gl * std::exp(-El / T) / Z;
      const double dfu = fu * (Eu / (T * T) - ZT / Z), dfl = fl * (El / (T * T) - ZT / Z);
      const double Ntr = X * nH2;
      const double bN = bnu * fu + bnl * fl;
      bT += Ntr * (bnu * dfu + bnl * dfl);
      bX += bN * nH2;
      blnn += bN * Ntr;
    }
    // b = sqrt(2kT/m + 2 sigma^2)
    bT += bb * (kK / m) / c.b_cms;
    gv[idx] = bv * 1e5;  // v_cms = 1e5 v_kms
    if (in.tdust) {
      gtd[idx] = bTd;
    } else {
      bT += bTd;
    }
    glnn[idx] = blnn;
    gt[idx] = bT;
    gx[idx] = bX;
  }
}

Inputs make_inputs(const double* lnn, const double* tkin, const double* vlos, const double* x,
                   const double* tdust, int nx, int ny, int nz, int axis, double cell_cm,
                   int n_chan, double v_lo, double dv, int simpson_f,
                   const oracle_line* line) {
  Inputs in;
  in.lnn = lnn;
  in.tkin = tkin;
  in.vlos = vlos;
  in.xab = x;
  in.tdust = tdust;
  in.g = Geometry{nx, ny, nz, axis};
  in.cell_cm = cell_cm;
  in.n_chan = n_chan;
  in.v_lo_kms = v_lo;
  in.dv_kms = dv;
  in.simpson_f = simpson_f;
  in.line = *line;
  return in;
}

int check_args(int nx, int ny, int nz, int axis, int n_chan, double cell_cm, double dv,
               int simpson_f, const oracle_line* line) {
  if (!line || line->integrator < 0 || line->integrator > 1) return 1;
  if (line->transfer < 0 || line->transfer > 2) return 1;
  if (line->transfer != 0 && simpson_f != 0) return 1;  // the erf profile is the channel average
  if (nx <= 0 || ny <= 0 || nz <= 0 || axis < 0 || axis > 2 || n_chan <= 0) return 1;
  if (simpson_f < 0 || simpson_f > 64) return 1;
  if (!(cell_cm > 0.0) || !(dv > 0.0)) return 1;
  return 0;
}

}  // namespace

extern "C" {

// Forward cube for pixels [pix_begin, pix_end). Outputs are [n][n_chan] with
// n = pix_end - pix_begin; C, D, B are written for every channel. Any output
// pointer may be null. Returns 0 on success, 1 on bad arguments.
int oracle_forward(const double* lnn, const double* tkin, const double* vlos, const double* x,
                   const double* tdust, int nx, int ny, int nz, int axis, double cell_cm,
                   int n_chan, double v_lo, double dv, int simpson_f, const oracle_line* line,
                   int64_t pix_begin,
                   int64_t pix_end, double* outT, double* outC, double* outD, double* outL,
                   double* outB, int n_threads) {
  if (check_args(nx, ny, nz, axis, n_chan, cell_cm, dv, simpson_f, line)) return 1;
  const Inputs in = make_inputs(lnn, tkin, vlos, x, tdust, nx, ny, nz, axis, cell_cm, n_chan,
                                v_lo, dv, simpson_f, line);
  if (pix_begin < 0 || pix_end > in.g.n_pix() || pix_begin > pix_end) return 1;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int64_t p = pix_begin; p < pix_end; ++p) {
    std::vector<double> T(n_chan), Lc(n_chan);
    double Cv, Dv, Bv;
    march<double>(in, p, nullptr, T.data(), &Cv, &Dv, &Bv, Lc.data());
    const size_t o = (size_t)(p - pix_begin) * n_chan;
    for (int k = 0; k < n_chan; ++k) {
      if (outT) outT[o + k] = T[k];
      if (outC) outC[o + k] = Cv;
      if (outD) outD[o + k] = Dv;
      if (outL) outL[o + k] = Lc[k];
      if (outB) outB[o + k] = Bv;
    }
  }
  return 0;
}

// The forward cube with non-LTE populations of the observed transition given
// per cell (FU, FL in the native layout), otherwise as oracle_forward.
int oracle_forward_ot(const double* lnn, const double* tkin, const double* vlos, const double* x,
                      const double* tdust, int nx, int ny, int nz, int axis, double cell_cm,
                      int n_chan, double v_lo, double dv, int simpson_f, const oracle_line* line,
                      const double* ot_fu, const double* ot_fl, double* outT, double* outC,
                      double* outD, double* outL, double* outB, int n_threads) {
  if (check_args(nx, ny, nz, axis, n_chan, cell_cm, dv, simpson_f, line)) return 1;
  if (!ot_fu || !ot_fl) return 1;
  Inputs in = make_inputs(lnn, tkin, vlos, x, tdust, nx, ny, nz, axis, cell_cm, n_chan, v_lo, dv,
                          simpson_f, line);
  in.ot_fu = ot_fu;
  in.ot_fl = ot_fl;
  const int64_t n_pix = in.g.n_pix();
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int64_t p = 0; p < n_pix; ++p) {
    std::vector<double> T(n_chan), Lc(n_chan);
    double Cv, Dv, Bv;
    march<double>(in, p, nullptr, T.data(), &Cv, &Dv, &Bv, Lc.data());
    const size_t o = (size_t)p * n_chan;
    for (int k = 0; k < n_chan; ++k) {
      if (outT) outT[o + k] = T[k];
      if (outC) outC[o + k] = Cv;
      if (outD) outD[o + k] = Dv;
      if (outL) outL[o + k] = Lc[k];
      if (outB) outB[o + k] = Bv;
    }
  }
  return 0;
}

// Reverse-mode gradient of L = sum(g_X * [X]) over pixels [pix_begin,
// pix_end). Cotangents are [pix_end - pix_begin][n_chan] (null = zero);
// gradients are written in the native field layout for the cells of those
// pixels only (g_td only when tdust is given). Returns 0 on success.
int oracle_adjoint(const double* lnn, const double* tkin, const double* vlos, const double* x,
                   const double* tdust, int nx, int ny, int nz, int axis, double cell_cm,
                   int n_chan, double v_lo, double dv, int simpson_f, const oracle_line* line,
                   int64_t pix_begin,
                   int64_t pix_end, const double* gT, const double* gC, const double* gD,
                   const double* gL, const double* gB, double* g_lnn, double* g_t, double* g_v,
                   double* g_x, double* g_td, int n_threads) {
  if (check_args(nx, ny, nz, axis, n_chan, cell_cm, dv, simpson_f, line)) return 1;
  if (line->units == 2) return 2;  // reverse mode written for linear output units only
  if (line->transfer == 2) return 2;  // not for selectively thin transfer
  if (line->transfer == 0 && line->integrator != 0) return 2;  // thick: formal step only
  const Inputs in = make_inputs(lnn, tkin, vlos, x, tdust, nx, ny, nz, axis, cell_cm, n_chan,
                                v_lo, dv, simpson_f, line);
  if (pix_begin < 0 || pix_end > in.g.n_pix() || pix_begin > pix_end) return 1;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int64_t p = pix_begin; p < pix_end; ++p) {
    const size_t o = (size_t)(p - pix_begin) * n_chan;
    march_adjoint(in, p, gT ? gT + o : nullptr, gC ? gC + o : nullptr, gD ? gD + o : nullptr,
                  gL ? gL + o : nullptr, gB ? gB + o : nullptr, g_lnn, g_t, g_v, g_x, g_td);
  }
  return 0;
}

// The same with non-LTE populations of the observed transition given per cell
// (as oracle_forward_ot): the field gradients hold every path but the one
// through the populations, whose gradients are written to g_fu, g_fl.
int oracle_adjoint_ot(const double* lnn, const double* tkin, const double* vlos, const double* x,
                      const double* tdust, int nx, int ny, int nz, int axis, double cell_cm,
                      int n_chan, double v_lo, double dv, int simpson_f, const oracle_line* line,
                      const double* ot_fu, const double* ot_fl, const double* gT,
                      const double* gC, const double* gD, const double* gL, const double* gB,
                      double* g_lnn, double* g_t, double* g_v, double* g_x, double* g_td,
                      double* g_fu, double* g_fl, int n_threads) {
  if (check_args(nx, ny, nz, axis, n_chan, cell_cm, dv, simpson_f, line)) return 1;
  if (!ot_fu || !ot_fl || !g_fu || !g_fl) return 1;
  if (line->units == 2 || line->integrator != 0 || line->transfer != 0) return 2;
  Inputs in = make_inputs(lnn, tkin, vlos, x, tdust, nx, ny, nz, axis, cell_cm, n_chan, v_lo, dv,
                          simpson_f, line);
  in.ot_fu = ot_fu;
  in.ot_fl = ot_fl;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int64_t p = 0; p < in.g.n_pix(); ++p) {
    const size_t o = (size_t)p * n_chan;
    march_adjoint(in, p, gT ? gT + o : nullptr, gC ? gC + o : nullptr, gD ? gD + o : nullptr,
                  gL ? gL + o : nullptr, gB ? gB + o : nullptr, g_lnn, g_t, g_v, g_x, g_td, g_fu,
                  g_fl);
  }
  return 0;
}

// Complex-step derivative d L / d field[cell] of the same loss, with L built
// from the sightline through that cell only (the others do not depend on it).
// field: 0 ln n_H2, 1 T_kin, 2 v_los, 3 X, 4 T_dust. Returns NaN on bad input.
double oracle_complex_step(const double* lnn, const double* tkin, const double* vlos,
                           const double* x, const double* tdust, int nx, int ny, int nz, int axis,
                           double cell_cm, int n_chan, double v_lo, double dv,
                           int simpson_f, const oracle_line* line, const double* gT, const double* gC,
                           const double* gD, const double* gL, const double* gB, int field,
                           int64_t cell, double h) {
  if (check_args(nx, ny, nz, axis, n_chan, cell_cm, dv, simpson_f, line)) return NAN;
  if (field == 4 && !tdust) return NAN;
  if (line->transfer != 0) return NAN;  // the thin profile's erf has no complex form here
  const Inputs in = make_inputs(lnn, tkin, vlos, x, tdust, nx, ny, nz, axis, cell_cm, n_chan,
                                v_lo, dv, simpson_f, line);
  // Locate the pixel owning this cell.
  const int64_t nz_ = in.g.nz, ny_ = in.g.ny;
  const int64_t xi = cell / (ny_ * nz_), yi = (cell / nz_) % ny_, zi = cell % nz_;
  int64_t p;
  if (axis == 0) p = yi * nz_ + zi;
  else if (axis == 1) p = xi * nz_ + zi;
  else p = xi * ny_ + yi;
  Perturb pt;
  pt.field = field;
  pt.cell = cell;
  pt.h = h;
  std::vector<cplx> T(n_chan), Lc(n_chan);
  cplx Cv = 0.0, Dv = 0.0, Bv = 0.0;
  march<cplx>(in, p, &pt, T.data(), &Cv, &Dv, &Bv, Lc.data());
  const size_t o = (size_t)p * n_chan;
  cplx acc = 0.0;
  for (int k = 0; k < n_chan; ++k) {
    if (gT) acc += gT[o + k] * T[k];
    if (gC) acc += gC[o + k] * Cv;
    if (gD) acc += gD[o + k] * Dv;
    if (gL) acc += gL[o + k] * Lc[k];
    if (gB) acc += gB[o + k] * Bv;
  }
  return acc.imag() / h;
}

// Per-cell coefficients (cgs) for tests of the level populations and source
// functions: out = {jL0, aL0, aD, jD, b_cms, Z, n_u, n_l, N}.
int oracle_cell(const oracle_line* line, double lnn, double T, double v, double X, double Td,
                double* out9) {
  const CellCoef<double> c = cell_coefficients<double>(*line, lnn, T, v, X, Td);
  const double v9[9] = {c.jL0, c.aL0, c.aD, c.jD, c.b_cms, c.Z, c.n_u, c.n_l, c.N};
  std::memcpy(out9, v9, sizeof v9);
  return 0;
}

// Planck intensity and its Rayleigh-Jeans temperature at frequency nu.
double oracle_planck(double nu, double T) { return planck(nu, T); }
double oracle_rj_per_intensity(double nu) { return kC * kC / (2.0 * kK * nu * nu); }

}  // extern "C"
