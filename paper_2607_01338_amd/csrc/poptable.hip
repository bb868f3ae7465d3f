// Temperature tables of the LTE line and of the source functions.
//
// The paper precomputes its level populations on a grid and interpolates
// them at run time ("Grid Precomputation"). Here, with LTE populations, the
// per-cell quantities that depend on temperature alone are
//   FL(T) = f_l(T) (1 - e^{-dE/T}),  f_l = g_l e^{-E_l/T} / Z(T)
//   J(T)  = T0 / expm1(T0 / T)       (Planck source in RJ kelvin)
//   JL(T) = T0 / expm1(dE / T)       (LTE line source; = J when dE = T0)
// so kappa_L = kL X n_H2 FL(T) / b(T). Each is evaluated exactly in FP64
// (partition sum over J = 0..j_max) at the nodes of a grid in u = log2(T)
// with kTabPerOctave intervals per octave over T in [2^kTabOct0, 2^kTabOct1),
// and stored per interval as the cubic Hermite polynomial
//   y(t) = y0 + t (m0 + t (c2 + t c3)),  t in [0, 1),
// built from the values and exact u-derivatives at both ends. Its
// interpolation error is below 1e-9 relative over the grid, far under FP32
// rounding. Temperatures outside the grid use the direct formulas.

#include "device_util.h"

namespace iris {

// Value and derivative d/du (u = log2 T) of FL, J and JL at T, in FP64.
struct TabNode {
  double fl, dfl, j, dj, jl, djl;
};

__device__ inline TabNode tab_node(const TabParams& tp, double u) {
  const double T = exp2(u);
  const double ln2 = 0.69314718055994530942;
  TabNode r;
  // Partition sum and its E-weighted sum, E_J = theta J(J+1).
  double Z = 0.0, ZE = 0.0;
  for (int J = 0; J <= tp.j_max; ++J) {
    const double E = tp.theta * J * (J + 1.0);
    const double w = (2.0 * J + 1.0) * exp(-E / T);
    Z += w;
    ZE += w * E;
  }
  const double El = tp.theta * tp.j_l * (tp.j_l + 1.0);
  const double em = exp(-tp.dE / T);
  const double stim = -expm1(-tp.dE / T);
  r.fl = tp.g_l * exp(-El / T) * stim / Z;
  // d ln FL / dT = E_l/T^2 - <E>/T^2 - (dE/T^2) e^{-dE/T} / (1 - e^{-dE/T})
  const double dln = (El - ZE / Z) / (T * T) - tp.dE / (T * T) * em / stim;
  r.dfl = r.fl * dln * T * ln2;
  const double x = tp.T0 / T;
  r.j = tp.T0 / expm1(x);
  r.dj = r.j * r.j * exp(x) * ln2 / T;
  const double y = tp.dE / T;
  const double ey = expm1(y);
  r.jl = tp.T0 / ey;
  r.djl = tp.T0 * (ey + 1.0) * y * ln2 / (ey * ey);
  return r;
}

__device__ inline float4 hermite(double y0, double d0, double y1, double d1, double h) {
  const double m0 = d0 * h, m1 = d1 * h;
  const double c2 = 3.0 * (y1 - y0) - 2.0 * m0 - m1;
  const double c3 = 2.0 * (y0 - y1) + m0 + m1;
  return make_float4((float)y0, (float)m0, (float)c2, (float)c3);
}

__global__ void pop_table_kernel(const TabParams tp, float4* tab) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kTabN) return;
  const double h = 1.0 / kTabPerOctave;
  const double u0 = kTabOct0 + i * h;
  const TabNode a = tab_node(tp, u0), b = tab_node(tp, u0 + h);
  tab[i] = hermite(a.fl, a.dfl, b.fl, b.dfl, h);
  tab[kTabN + i] = hermite(a.j, a.dj, b.j, b.dj, h);
  tab[2 * kTabN + i] = hermite(a.jl, a.djl, b.jl, b.djl, h);
}

int launch_pop_table(const TabParams& tp, void* tab, void* stream) {
  hipLaunchKernelGGL(pop_table_kernel, dim3((kTabN + 255) / 256), dim3(256), 0,
                     (hipStream_t)stream, tp, (float4*)tab);
  return (int)hipGetLastError();
}

}  // namespace iris
