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
  float b;       // Doppler parameter, km/s
  float kL;      // line-centre optical depth of the cell
  float kD;      // dust optical depth of the cell (clamped at kRebaseTau)
  float JL;      // line source function, RJ K
  float JD;      // dust source function, RJ K
  // profile evaluation: t_k = (m_k * A - R), m_k = k - kc (exact integer),
  // tau_k * log2(e) = 2^(lk - t_k^2); c0 = t at the window's first channel
  float A, R, lk;
  float df;      // (float)(kstart - kc)
  float c0;
  int kstart;    // first channel of the line window
  int nwin;      // channels in the window; 0 = the cell carries no line
};

// Passes of `w` lanes needed to cover a window of `nwin` channels.
__device__ __forceinline__ int window_passes(int nwin, int w) {
  return (int)(((unsigned)nwin + (unsigned)w - 1u) / (unsigned)w);
}

// The stored values of one cell, not yet converted, so that a load issued
// ahead of its use is not waited for by the conversion.
template <typename FT>
struct RawCell {
  FT lnn, T, v, X, Td;
};

template <typename FT>
__device__ __forceinline__ RawCell<FT> fetch_cell(const FT* const* f, int64_t off, bool valid,
                                                  bool has_td) {
  RawCell<FT> r{};
  if (valid) {
    r.lnn = gload(f[0] + off);
    r.T = gload(f[1] + off);
    r.v = gload(f[2] + off);
    r.X = gload(f[3] + off);
    r.Td = has_td ? gload(f[4] + off) : r.T;
  }
  return r;
}

// Invalid cells (beyond the sightline or of a dead group) get harmless values.
template <typename FT>
__device__ __forceinline__ CellIn decode_cell(const RawCell<FT>& r, bool valid) {
  CellIn in;
  if (valid) {
    in.lnn = to_f32(r.lnn);
    in.T = to_f32(r.T);
    in.v = to_f64(r.v);
    in.X = to_f32(r.X);
    in.Td = to_f32(r.Td);
  } else {
    in.lnn = 0.f;
    in.T = 100.f;
    in.v = 0.0;
    in.X = 0.f;
    in.Td = 100.f;
  }
  return in;
}

// Field access of one sightline: compile-time storage type. fetch() issues
// the loads; decode() converts.
template <typename FT>
struct Loader {
  using Raw = RawCell<FT>;
  const FT* f[5];
  bool has_td;
  __device__ __forceinline__ Loader(const void* const* base, int64_t first) {
#pragma unroll
    for (int i = 0; i < 5; ++i) f[i] = base[i] ? (const FT*)base[i] + first : nullptr;
    has_td = base[4] != nullptr;
  }
  __device__ __forceinline__ Raw fetch(int64_t off, bool valid) const {
    return fetch_cell<FT>(f, off, valid, has_td);
  }
  __device__ __forceinline__ CellIn decode(const Raw& r, bool valid) const {
    return decode_cell<FT>(r, valid);
  }
  __device__ __forceinline__ CellIn operator()(int64_t off, bool valid) const {
    return decode(fetch(off, valid), valid);
  }
};

// Field access with the storage type chosen at run time (batched plans mix
// storage types in one launch); the switch is uniform across the wavefront.
// Raw holds the stored bits: 16- and 32-bit elements as loaded, v of FP64
// storage as its 64-bit pattern; the other FP64 fields are narrowed to FP32
// at the load (FP64 storage is the exactness reference, not a fast path).
struct DynRaw {
  uint32_t lnn, T, X, Td;
  uint64_t v;
};

struct DynLoader {
  using Raw = DynRaw;
  const void* const* base;
  int64_t first;
  int32_t dt;
  __device__ __forceinline__ DynLoader(const void* const* b, int64_t fst, int32_t dtype)
      : base(b), first(fst), dt(dtype) {}

  template <typename FT>
  __device__ __forceinline__ Raw fetch_bits(int64_t off, bool valid) const {
    const RawCell<FT> r = Loader<FT>(base, first).fetch(off, valid);
    Raw w;
    if constexpr (sizeof(FT) == 8) {
      w.lnn = __float_as_uint((float)r.lnn);
      w.T = __float_as_uint((float)r.T);
      w.X = __float_as_uint((float)r.X);
      w.Td = __float_as_uint((float)r.Td);
      w.v = (uint64_t)__double_as_longlong(r.v);
    } else if constexpr (sizeof(FT) == 4) {
      w.lnn = __float_as_uint(r.lnn);
      w.T = __float_as_uint(r.T);
      w.X = __float_as_uint(r.X);
      w.Td = __float_as_uint(r.Td);
      w.v = __float_as_uint(r.v);
    } else {
      w.lnn = bits16(r.lnn);
      w.T = bits16(r.T);
      w.X = bits16(r.X);
      w.Td = bits16(r.Td);
      w.v = bits16(r.v);
    }
    return w;
  }
  static __device__ __forceinline__ uint32_t bits16(bf16_t x) { return x.bits; }
  static __device__ __forceinline__ uint32_t bits16(_Float16 x) {
    return (uint32_t)__builtin_bit_cast(uint16_t, x);
  }

  __device__ __forceinline__ Raw fetch(int64_t off, bool valid) const {
    switch (dt) {
      case IRIS_F64: return fetch_bits<double>(off, valid);
      case IRIS_BF16: return fetch_bits<bf16_t>(off, valid);
      case IRIS_F16: return fetch_bits<_Float16>(off, valid);
      default: return fetch_bits<float>(off, valid);
    }
  }

  __device__ __forceinline__ float narrow(uint32_t w) const {
    switch (dt) {
      case IRIS_BF16: return __uint_as_float(w << 16);
      case IRIS_F16: return (float)__builtin_bit_cast(_Float16, (uint16_t)w);
      default: return __uint_as_float(w);  // FP32, or FP64 narrowed at the load
    }
  }

  __device__ __forceinline__ CellIn decode(const Raw& w, bool valid) const {
    CellIn in;
    if (valid) {
      in.lnn = narrow(w.lnn);
      in.T = narrow(w.T);
      in.X = narrow(w.X);
      in.Td = narrow(w.Td);
      in.v = dt == IRIS_F64 ? __longlong_as_double((long long)w.v) : (double)narrow((uint32_t)w.v);
    } else {
      in.lnn = 0.f;
      in.T = 100.f;
      in.v = 0.0;
      in.X = 0.f;
      in.Td = 100.f;
    }
    return in;
  }

  __device__ __forceinline__ CellIn operator()(int64_t off, bool valid) const {
    return decode(fetch(off, valid), valid);
  }
};

// Coordinates of T in the temperature tables: interval index and local t.
// Branch-free; false (with idx = 0, t = 0) outside the tabulated range.
__device__ __forceinline__ bool tab_coord(float T, int& idx, float& t) {
  int e;
  const float m = frexpf(T, &e);  // T = m 2^e, m in [0.5, 1)
  const int oct = e - 1 - kTabOct0;
  const bool in = (T > 0.f) && oct >= 0 && oct < kTabOct1 - kTabOct0;
  const float f = __builtin_amdgcn_logf(2.f * m) * (float)kTabPerOctave;  // [0, 128)
  const float fi = fminf(fmaxf(floorf(f), 0.f), (float)(kTabPerOctave - 1));
  idx = in ? oct * kTabPerOctave + (int)fi : 0;
  t = in ? f - fi : 0.f;
  return in;
}

__device__ __forceinline__ float tab_eval(const Folded& c, int which, int idx, float t) {
  const float4 q = gload((const float4*)c.tab + which * kTabN + idx);
  return fmaf(t, fmaf(t, fmaf(t, q.w, q.z), q.y), q.x);
}

// Direct evaluation (FP64) for temperatures outside the tables.
__device__ __forceinline__ void temp_direct(const Folded& c, float Tf, float& FL, float& J,
                                         float& JL) {
  const double T = (double)Tf;
  const double theta = c.th2 * 0.69314718055994530942;
  double Z = 0.0;
  for (int j = 0; j <= c.j_max; ++j) Z += (2.0 * j + 1.0) * exp(-theta * j * (j + 1.0) / T);
  const double El = theta * c.j_l * (c.j_l + 1.0);
  FL = (float)(c.g_l * exp(-El / T) * -expm1(-(double)c.dE / T) / Z);
  J = (float)((double)c.T0 / expm1((double)c.T0 / T));
  JL = (float)((double)c.T0 / expm1((double)c.dE / T));
  if (!(Tf > 0.f)) FL = J = JL = 0.f;
}

// FL(T) = f_l (1 - e^{-dE/T}), the Planck source J(T) and (GEN) the LTE line
// source JL(T) from the tables (poptable.hip); without GEN, JL = J. The rare
// temperatures outside the tables are evaluated first, in a divergent branch,
// so that the table loads and their uses sit in one block with the rest of
// the cell setup, which hides their latency.
template <bool GEN>
__device__ __forceinline__ void temp_functions(const Folded& c, float T, float& FL, float& J,
                                               float& JL) {
  int idx;
  float t;
  const bool in = tab_coord(T, idx, t);
  float FLd = 0.f, Jd = 0.f, JLd = 0.f;
  if (!in) temp_direct(c, T, FLd, Jd, JLd);
  const float FLt = tab_eval(c, 0, idx, t);  // idx is valid for every lane
  const float Jt = tab_eval(c, 1, idx, t);
  FL = in ? FLt : FLd;
  J = in ? Jt : Jd;
  if (GEN) {
    const float JLt = tab_eval(c, 2, idx, t);
    JL = in ? JLt : JLd;
  } else {
    JL = J;
  }
}

__device__ __forceinline__ float planck_rj(const Folded& c, float T) {
  int idx;
  float t;
  const bool in = tab_coord(T, idx, t);
  float FLd = 0.f, Jd = 0.f, JLd = 0.f;
  if (!in) temp_direct(c, T, FLd, Jd, JLd);
  const float Jt = tab_eval(c, 1, idx, t);
  return in ? Jt : Jd;
}

// Non-LTE populations of the observed transition from the (FU, FL) grid:
// multilinear in (ln n_H2, ln T) on the two molecular-fraction planes that
// bracket the launch's fraction, then linear between those planes; interval
// indices are clamped to the grid and the local coordinates are not, so the
// interpolation extends linearly beyond it. FL is the factor of the line
// opacity (f_l - (g_l/g_u) f_u) and the line source function is T0 FU / FL;
// where FL is not positive the cell carries no line (FL = 0, JL = JD).
__device__ __forceinline__ void ot_functions(const Folded& c, float lnn, float T, float JD,
                                             float& FL, float& JL) {
  const float2* G = (const float2*)c.ot;
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
  float fu[2], fl[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int b = b0 + q * sc;
    const float2 g00 = gload(G + b), g01 = gload(G + b + sn);
    const float2 g10 = gload(G + b + st), g11 = gload(G + b + st + sn);
    const float u0 = fmaf(tn, g01.x - g00.x, g00.x), u1 = fmaf(tn, g11.x - g10.x, g10.x);
    const float l0 = fmaf(tn, g01.y - g00.y, g00.y), l1 = fmaf(tn, g11.y - g10.y, g10.y);
    fu[q] = fmaf(tt, u1 - u0, u0);
    fl[q] = fmaf(tt, l1 - l0, l0);
  }
  const float FU = fmaf(c.ot_tc, fu[1] - fu[0], fu[0]);
  const float FLi = fmaf(c.ot_tc, fl[1] - fl[0], fl[0]);
  const bool pos = FLi > 0.f;
  FL = pos ? FLi : 0.f;
  JL = pos ? c.T0 * FU / FLi : JD;
}

// `line_min`: apply the forward-only cut kappa_L >= kL_min to the window.
// GEN: separate line and dust source functions (energy mode 1 or a dust
// temperature field); must equal c.general.
template <bool GEN>
__device__ __forceinline__ CellOut cell_setup(const Folded& c, const CellIn& in, bool valid,
                                              bool line_min) {
  CellOut o;
  const float T = in.T;
  const float n = ex2(in.lnn * kLog2e);  // ~4e-7 relative: far inside the FP32 budget
  o.n = (double)n;
  float FL, JT, JLT;
  temp_functions<GEN>(c, T, FL, JT, JLT);
  // Non-LTE populations (a line whose source function is its own, GEN).
  const float JDc = GEN ? planck_rj(c, in.Td) : JT;
  if (GEN && c.ot) ot_functions(c, in.lnn, T, JDc, FL, JLT);
  // Hardware square root and logarithm (about 1 ulp): the arguments are
  // positive normal numbers, and the profile needs b and lk to ~1e-7 only.
  o.b = __builtin_amdgcn_sqrtf(fmaf(c.bT, T, c.bt2));
  const float rb = __builtin_amdgcn_rcpf(o.b);
  float kL = c.kL * in.X * n * FL * rb;
  if (!(T <= c.t_inf)) kL = 0.f;
  o.kL = kL;
  o.JD = JDc;
  o.JL = GEN ? JLT : o.JD;
  o.kD = fminf(c.kD * n, kRebaseTau);
  o.lk = __builtin_amdgcn_logf(fmaxf(kL * kLog2e, 1e-20f));

  // Channel window: |v_k - v| <= x_w b with x_w^2 = ln(max(kappa_L,1)/eps);
  // ln kappa_L = (lk - log2(log2 e)) ln 2.
  // Line centre in channel units, FP32: its rounding (~1e-4 channel) can move
  // a window edge by one channel where the profile is ~eps, and the centre
  // channel kc by one, which only changes the reference of rr (kept in FP64).
  const float inv_dv = (float)c.inv_dv;
  const float u = fmaf((float)(in.v - c.v_lo), inv_dv, -0.5f);
  const float xw2 = c.xw2min + fmaxf(0.f, (o.lk - 0.52876637f) * kLn2);
  const float hw = __builtin_amdgcn_sqrtf(xw2) * o.b * inv_dv;
  const float klo = fmaxf(ceilf(u - hw), 0.f);
  const float khi = fminf(floorf(u + hw), (float)(c.n_chan - 1));
  const bool line = valid && (T > 0.f) && (T <= c.t_inf) && (klo <= khi) &&
                    (!line_min || kL >= c.kL_min);
  const float kc = fminf(fmaxf(rintf(u), klo - 64.f), khi + 64.f);
  const double rr = in.v - (c.v_lo + ((double)kc + 0.5) * c.dv);
  const float a = kSqrtLog2e * rb;
  o.A = (float)c.dv * a;
  o.R = (float)rr * a;
  if (line) {
    o.kstart = (int)klo;
    o.nwin = (int)(khi - klo) + 1;
    o.df = klo - kc;
  } else {
    o.kstart = 0;
    o.nwin = 0;
    o.df = 0.f;
  }
  o.c0 = fmaf(o.df, o.A, -o.R);
  return o;
}

// Formal step ("Transfer Solution: Formal and Smooth Integration ...") of the
// scaled line excess over a line depth tau = x ln 2 (x = tau log2 e, the
// exponent the profile gives): Psi' = (Psi + g) e^{-tau} - g. Written so, the
// rounding of e^{-tau} near 1 (half an ulp of 1) costs |Psi + g| 6e-8 per step
// whatever tau is, which for a faint line (g, the continuum's distance from
// the line source function, far above the line's own change g tau) is a large
// relative error of the line. The step is taken as
// Psi - (Psi + g)(1 - 2^{-x}) instead, with 1 - 2^{-x} from three terms of its
// series below x = 0.044 (the first omitted term is under 1.2e-6 of the sum)
// and as 1 - 2^{-x} above (there 1 - e^{-tau} > 0.03, so the rounding of the
// exponential is under 2e-6 of the step; the subtraction is exact while
// 2^{-x} >= 1/2).
constexpr float kSeriesX = 0.044f;
__device__ __forceinline__ float formal_line_step(float ps, float g, float x) {
  float q = fmaf(x, 0.0555041087f, -0.2402265070f);  // (ln 2)^3/6, -(ln 2)^2/2
  q = fmaf(x, q, 0.6931471806f);                      // ln 2
  const float om = x < kSeriesX ? x * q : 1.f - ex2(-x);  // 1 - e^{-tau}
  return fmaf(-(ps + g), om, ps);
}

}  // namespace iris
