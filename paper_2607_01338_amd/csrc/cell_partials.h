// Derivatives of the per-cell quantities of cell_setup.h with respect to the
// stored fields, for the adjoint's chain rule. One lane per cell. Inside the
// temperature tables the T-dependence comes from their cubics, in FP32 (about
// 1e-7 relative, far below the gradient tolerance); outside, from the
// partition sum in FP64.
#pragma once

#include "cell_setup.h"

namespace iris {

struct CellPartials {
  double kL;       // line-centre optical depth
  double dkL_dT;   // total d kappa_L / d T (populations, stimulated emission, 1/b)
  double dkL_dX;   // d kappa_L / d X
  double b;        // Doppler parameter, km/s
  double db_dT;
  double dJ_dT;    // d J(T) / d T of the source function J = T0 / expm1(T0/T)
  double dJL_dT;   // d JL(T) / d T of the LTE line source function T0 / expm1(dE/T)
  // Non-LTE populations from the level grid only (zero otherwise):
  double dkL_dlnn; // d kappa_L / d ln n_H2 beyond kappa_L's proportionality to n_H2
  double dJL_dlnn; // d JL / d ln n_H2
  bool line_src;   // false: the cell carries no line and JL is the dust's J_D
  double kD;       // dust optical depth used by the march (clamped)
  double kD_free;  // unclamped dust optical depth (for the background)
  bool kD_clamped;
};

// Fast path: FL(T) and J(T) with their derivatives from the temperature
// tables (cubic Hermite in u = log2 T; d/dT = (d/du) / (T ln 2)), in FP32 like
// the march itself (n, b and the clamp decision are the forward's own
// expressions): partials to about 1e-7 relative, far below the gradient
// tolerance. Returns false outside the tabulated range.
template <bool GEN>
__device__ __forceinline__ bool cell_partials_tab(const Folded& c, double lnn, double T,
                                                  double X, CellPartials& p) {
  int idx;
  float t;
  const float Tf = (float)T;
  if (!tab_coord(Tf, idx, t)) return false;
  const float4 qf = gload((const float4*)c.tab + idx);
  const float4 qj = gload((const float4*)c.tab + kTabN + idx);
  const float FL = fmaf(t, fmaf(t, fmaf(t, qf.w, qf.z), qf.y), qf.x);
  const float dFL_du = fmaf(t, fmaf(t, 3.f * qf.w, 2.f * qf.z), qf.y) * (float)kTabPerOctave;
  const float dJ_du = fmaf(t, fmaf(t, 3.f * qj.w, 2.f * qj.z), qj.y) * (float)kTabPerOctave;
  const float du_dT = __builtin_amdgcn_rcpf(Tf) * kLog2e;  // 1 / (T ln 2)
  const float n = ex2((float)lnn * kLog2e);
  const float b2 = fmaf(c.bT, Tf, c.bt2);
  const float b = __builtin_amdgcn_sqrtf(b2), rb = __builtin_amdgcn_rcpf(b);
  p.b = b;
  p.db_dT = 0.5f * c.bT * rb;
  const float dlnb = 0.5f * c.bT * rb * rb;
  const float base = c.kL * n * FL * rb;  // kappa_L per unit X
  if (Tf <= c.t_inf && FL > 0.f) {
    const float kL = base * (float)X;
    p.kL = kL;
    p.dkL_dX = base;
    p.dkL_dT = kL * fmaf(dFL_du * du_dT, __builtin_amdgcn_rcpf(FL), -dlnb);
  } else {
    p.kL = p.dkL_dX = p.dkL_dT = 0.0;
  }
  p.dJ_dT = dJ_du * du_dT;
  p.dkL_dlnn = p.dJL_dlnn = 0.0;
  p.line_src = true;
  if (GEN) {
    const float4 ql = gload((const float4*)c.tab + 2 * kTabN + idx);
    p.dJL_dT = fmaf(t, fmaf(t, 3.f * ql.w, 2.f * ql.z), ql.y) * (float)kTabPerOctave * du_dT;
  } else {
    p.dJL_dT = p.dJ_dT;
  }
  const float kDf = c.kD * n;
  p.kD_free = kDf;
  p.kD_clamped = kDf > kRebaseTau;
  p.kD = p.kD_clamped ? (double)kRebaseTau : (double)kDf;
  return true;
}

template <bool GEN>
__device__ __forceinline__ CellPartials cell_partials(const Folded& c, double lnn, double T,
                                                      double X) {
  CellPartials p;
  if (cell_partials_tab<GEN>(c, lnn, T, X, p)) return p;
  const double n = exp(lnn);
  // Z = sum (2J+1) q^{J(J+1)} and E-weighted sum for dZ/dT, with
  // q^{J(J+1)} = e^{-E_J/T}, E_J = theta J(J+1), theta = th2 / log2(e).
  const double q = exp2(-c.th2 / T);
  const double q2 = q * q;
  const double theta = c.th2 * 0.69314718055994530942;
  double Z = 0.0, ZE = 0.0, r = 1.0, m = q2, rl = 0.0;
  for (int J = 0; J <= c.j_max; ++J) {
    if (J == c.j_l) rl = r;
    const double w = (2.0 * J + 1.0) * r;
    Z += w;
    ZE += w * (double)J * (J + 1.0);
    r *= m;
    m *= q2;
  }
  const double fl = c.g_l * rl / Z;
  const double El = theta * c.j_l * (c.j_l + 1.0);
  // d ln f_l / dT = E_l/T^2 - <E>/T^2, <E> = theta ZE / Z.
  const double dlnfl = (El - theta * ZE / Z) / (T * T);
  const double dE = (double)c.dE;
  const double em = exp(-dE / T);
  const double stim = -expm1(-dE / T);
  const double dlnstim = -em * dE / (T * T) / stim;
  const double b2 = (double)c.bT * T + (double)c.bt2;
  p.b = sqrt(b2);
  p.db_dT = 0.5 * (double)c.bT / p.b;
  const double dlnb = 0.5 * (double)c.bT / b2;
  const double base = (double)c.kL * n * fl * stim / p.b;  // kappa_L per unit X
  if (T <= (double)c.t_inf) {
    p.kL = base * X;
    p.dkL_dX = base;
    p.dkL_dT = p.kL * (dlnfl + dlnstim - dlnb);
  } else {
    p.kL = p.dkL_dX = p.dkL_dT = 0.0;
  }
  const double T0 = (double)c.T0;
  const double x = T0 / T;
  const double J = T0 / expm1(x);
  p.dJ_dT = J * J * exp(x) / (T * T);
  // JL = T0 / (e^y - 1), y = dE/T: dJL/dT = JL^2 e^y dE / (T0 T^2).
  const double y = dE / T;
  const double JL = T0 / expm1(y);
  p.dJL_dT = JL * JL * exp(y) * dE / (T0 * T * T);
  p.dkL_dlnn = p.dJL_dlnn = 0.0;
  p.line_src = true;
  p.kD_free = (double)c.kD * n;
  p.kD_clamped = (float)p.kD_free > kRebaseTau;
  p.kD = p.kD_clamped ? (double)kRebaseTau : p.kD_free;
  return p;
}

// d J / d T of the Planck source function J(T) = T0 / expm1(T0/T) at any
// temperature (a dust temperature, or T_kin with non-LTE populations): from
// the table's cubic inside its range, else directly.
__device__ __forceinline__ double planck_rj_dT(const Folded& c, double T) {
  int idx;
  float t;
  const float Tf = (float)T;
  if (tab_coord(Tf, idx, t)) {
    const float4 qj = gload((const float4*)c.tab + kTabN + idx);
    const float du_dT = __builtin_amdgcn_rcpf(Tf) * kLog2e;
    return fmaf(t, fmaf(t, 3.f * qj.w, 2.f * qj.z), qj.y) * (float)kTabPerOctave * du_dT;
  }
  if (!(T > 0.0)) return 0.0;
  const double x = (double)c.T0 / T;
  const double J = (double)c.T0 / expm1(x);
  return J * J * exp(x) / (T * T);
}


// Partials with non-LTE populations interpolated from the level grid (the
// cell setup's ot_functions): FL (the line opacity factor) and
// JL = T0 FU / FL are multilinear in (ln n_H2, ln T) on the grid interval
// the cell falls in, so their derivatives are that interval's slopes (the
// edge interval's beyond the grid, as the interpolation itself); kappa_L
// = kL X n FL / b. Where FL is not positive the cell carries no line and JL
// is the dust's source function. `dJ_dT` is the Planck derivative at T_kin.
__device__ __forceinline__ CellPartials cell_partials_ot(const Folded& c, double lnn_d, double T_d,
                                                         double X) {
  CellPartials p;
  const float lnn = (float)lnn_d, T = (float)T_d;
  const float2* Gd = (const float2*)c.ot;
  const float un = (lnn - c.ot_n0) * c.ot_dn_inv;
  const float in_ = fminf(fmaxf(floorf(un), 0.f), (float)max(c.ot_nn - 2, 0));
  const float tn = un - in_;
  const float lt = __builtin_amdgcn_logf(fmaxf(T, 1e-30f)) * kLn2;
  const float ut = (lt - c.ot_t0) * c.ot_dt_inv;
  const float it = fminf(fmaxf(floorf(ut), 0.f), (float)max(c.ot_nt - 2, 0));
  const float tt = ut - it;
  const int sn = c.ot_nn > 1 ? 1 : 0;
  const int st = c.ot_nt > 1 ? c.ot_nn : 0;
  const int sc = c.ot_nc > 1 ? c.ot_nt * c.ot_nn : 0;
  const int b0 = (c.ot_ic * c.ot_nt + (int)it) * c.ot_nn + (int)in_;
  // Per molecular-fraction plane: value and slopes in the local coordinates.
  float fu[2], fl[2], fu_n[2], fl_n[2], fu_t[2], fl_t[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int b = b0 + q * sc;
    const float2 g00 = gload(Gd + b), g01 = gload(Gd + b + sn);
    const float2 g10 = gload(Gd + b + st), g11 = gload(Gd + b + st + sn);
    const float du0 = g01.x - g00.x, du1 = g11.x - g10.x;
    const float dl0 = g01.y - g00.y, dl1 = g11.y - g10.y;
    const float u0 = fmaf(tn, du0, g00.x), u1 = fmaf(tn, du1, g10.x);
    const float l0 = fmaf(tn, dl0, g00.y), l1 = fmaf(tn, dl1, g10.y);
    fu[q] = fmaf(tt, u1 - u0, u0);
    fl[q] = fmaf(tt, l1 - l0, l0);
    fu_n[q] = fmaf(tt, du1 - du0, du0);
    fl_n[q] = fmaf(tt, dl1 - dl0, dl0);
    fu_t[q] = u1 - u0;
    fl_t[q] = l1 - l0;
  }
  const float tc = c.ot_tc;
  const double FU = fmaf(tc, fu[1] - fu[0], fu[0]);
  const double FL = fmaf(tc, fl[1] - fl[0], fl[0]);
  const double dtn = (double)c.ot_dn_inv;         // d tn / d ln n_H2
  const double dtt = (double)c.ot_dt_inv / T_d;   // d tt / d T
  const double FU_n = fmaf(tc, fu_n[1] - fu_n[0], fu_n[0]) * dtn;
  const double FL_n = fmaf(tc, fl_n[1] - fl_n[0], fl_n[0]) * dtn;
  const double FU_t = fmaf(tc, fu_t[1] - fu_t[0], fu_t[0]) * dtt;
  const double FL_t = fmaf(tc, fl_t[1] - fl_t[0], fl_t[0]) * dtt;
  const double n = exp(lnn_d);
  const double b2 = (double)c.bT * T_d + (double)c.bt2;
  p.b = sqrt(b2);
  p.db_dT = 0.5 * (double)c.bT / p.b;
  const double dlnb = 0.5 * (double)c.bT / b2;
  p.line_src = FL > 0.0;
  if (p.line_src && T_d <= (double)c.t_inf) {
    const double base = (double)c.kL * n * FL / p.b;  // kappa_L per unit X
    p.kL = base * X;
    p.dkL_dX = base;
    p.dkL_dT = p.kL * (FL_t / FL - dlnb);
    p.dkL_dlnn = p.kL * FL_n / FL;
  } else {
    p.kL = p.dkL_dX = p.dkL_dT = p.dkL_dlnn = 0.0;
  }
  if (p.line_src) {
    const double T0 = (double)c.T0;
    p.dJL_dT = T0 * (FU_t * FL - FU * FL_t) / (FL * FL);
    p.dJL_dlnn = T0 * (FU_n * FL - FU * FL_n) / (FL * FL);
  } else {
    p.dJL_dT = p.dJL_dlnn = 0.0;
  }
  p.dJ_dT = planck_rj_dT(c, T_d);
  p.kD_free = (double)c.kD * n;
  p.kD_clamped = (float)p.kD_free > kRebaseTau;
  p.kD = p.kD_clamped ? (double)kRebaseTau : p.kD_free;
  return p;
}

}  // namespace iris
