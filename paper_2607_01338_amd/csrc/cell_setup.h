// Per-cell setup shared by the forward and adjoint march kernels: LTE level
// populations, line and dust optical depths of one cell, source functions
// and the channel window of the line. One lane computes one cell.
#pragma once

#include "device_util.h"

namespace iris {

struct CellIn {
  float lnn, T, X, Td;
  double v;
};

struct CellOut {
  // physics
  double n;      // n_H2, cm^-3
  double Z;      // partition function
  double fl;     // lower-level fraction n_l / N
  float stim;    // 1 - exp(-dE/T): stimulated-emission correction
  float b;       // Doppler parameter, km/s
  float kL;      // line-centre optical depth of the cell
  float kD;      // dust optical depth of the cell (clamped at kRebaseTau)
  float JL;      // line source function, RJ K
  float JD;      // dust source function, RJ K
  // profile evaluation: t_k = (m_k * A - R), m_k = k - kc (exact integer),
  // tau_k * log2(e) = 2^(lk - t_k^2)
  float A, R, lk;
  float df;      // (float)(kstart - kc)
  int packed;    // kstart | npass << 24; 0 = no line pass for this cell
};

template <typename FT>
__device__ __forceinline__ CellIn load_cell(const FT* const* f, int64_t off, bool valid,
                                            bool has_td) {
  CellIn in;
  if (valid) {
    in.lnn = to_f32(f[0][off]);
    in.T = to_f32(f[1][off]);
    in.v = to_f64(f[2][off]);
    in.X = to_f32(f[3][off]);
    in.Td = has_td ? to_f32(f[4][off]) : in.T;
  } else {
    in.lnn = 0.f;
    in.T = 100.f;
    in.v = 0.0;
    in.X = 0.f;
    in.Td = 100.f;
  }
  return in;
}

// `line_min`: apply the forward-only cut kappa_L >= kL_min to the window.
__device__ __forceinline__ CellOut cell_setup(const Folded& c, const CellIn& in, bool valid,
                                              bool line_min) {
  CellOut o;
  const float T = in.T;
  o.n = exp((double)in.lnn);
  const float n = (float)o.n;
  // Partition sum over J = 0..j_max, term (2J+1) q^{J(J+1)}, q = e^{-theta/T},
  // by the exact recurrence q^{(J+1)(J+2)} = q^{J(J+1)} q^{2(J+1)} in FP64.
  const double q = exp2(-c.th2 / (double)T);
  const double q2 = q * q;
  double Z = 0.0, r = 1.0, m = q2, rl = 0.0;
  for (int J = 0; J <= c.j_max; ++J) {
    if (J == c.j_l) rl = r;
    Z = fma((double)(2 * J + 1), r, Z);
    r *= m;
    m *= q2;
  }
  o.Z = Z;
  o.fl = c.g_l * rl / Z;
  o.stim = -expm1f(-c.dE / T);
  o.b = sqrtf(fmaf(c.bT, T, c.bt2));
  float kL = c.kL * in.X * n * (float)o.fl * o.stim / o.b;
  if (!(T <= c.t_inf)) kL = 0.f;
  o.kL = kL;
  o.JD = c.T0 / expm1f(c.T0 / in.Td);
  o.JL = c.general ? c.T0 / expm1f(c.dE / T) : o.JD;
  o.kD = fminf(c.kD * n, kRebaseTau);

  // Channel window: |v_k - v| <= x_w b with x_w^2 = ln(max(kappa_L,1)/eps).
  const double u = (in.v - c.v_lo) * c.inv_dv - 0.5;  // line centre in channel units
  const float xw2 = c.xw2min + __logf(fmaxf(kL, 1.f));
  const float hw = sqrtf(xw2) * o.b * (float)c.inv_dv;
  double klo = ceil(u - (double)hw), khi = floor(u + (double)hw);
  klo = fmax(klo, 0.0);
  khi = fmin(khi, (double)(c.n_chan - 1));
  const bool line = valid && (T > 0.f) && (T <= c.t_inf) && (klo <= khi) &&
                    (!line_min || kL >= c.kL_min);
  double kc = rint(u);
  kc = fmin(fmax(kc, klo - 64.0), khi + 64.0);
  const double rr = in.v - (c.v_lo + (kc + 0.5) * c.dv);
  const float a = kSqrtLog2e / o.b;
  o.A = (float)(c.dv * (double)a);
  o.R = (float)rr * a;
  o.lk = log2f(fmaxf(kL * kLog2e, 1e-20f));
  if (line) {
    const int kstart = (int)klo;
    const int npass = (int)(khi - klo) / 64 + 1;
    o.df = (float)(klo - kc);
    o.packed = kstart | (npass << 24);
  } else {
    o.df = 0.f;
    o.packed = 0;
  }
  return o;
}

}  // namespace iris
