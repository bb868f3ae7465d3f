// Smooth integration of the transfer equation, far side to observer, one
// sightline per wavefront.
//
// Method (paper, "Transfer Solution: Formal and Smooth Integration of
// Optically Thick and Selectively Thin Transfer", the TR and BDF2 step
// solutions): dI/ds = j - alpha I is integrated over nodes one cell apart,
// each node carrying its cell's coefficients, from the background at node 0.
// The first step is the implicit trapezoidal rule,
//   I_1 = (h (j_0 + j_1) + (2 - h alpha_0) I_0) / (2 + h alpha_1),
// every later one the two-step backward differentiation formula,
//   I_n = (2 h j_n + 4 I_{n-1} - I_{n-2}) / (3 + 2 h alpha_n),
// and each result is clamped at zero. [C], [D] and [B] are integrated the
// same way with the dust terms only (from the background, from zero, and
// with no emission from the background).
//
// How it is organised on gfx950:
//  * Unlike the formal step, a BDF2 step changes the intensity of every
//    channel in every cell, line or not (it carries two intensities, and the
//    difference of two channels decays by a factor of about 1/3 per cell), so
//    the work is dense in (cell, channel). Channel k of the marched grid is
//    slot k / 64 of lane k % 64; each lane keeps two nodes of its slots in
//    registers (S slots: up to 64 S channels).
//  * The per-channel state is the line excess Delta = I - C over the
//    continuum C of the same node (C integrated by the same steps), so that
//    it carries no rounding of the continuum's size and [L] keeps its
//    accuracy under a bright continuum. Every step is taken in increment
//    form, X_n = X_{n-1} + (...) / (3 + 2 tau), whose rounding is unbiased:
//    the product form (4 X_{n-1} - X_{n-2}) r, r = 1 / (3 + 2 tau), turns
//    the rounding of r into a relative drift of order 1e-5 over 500 cells.
//    With C_n the (clamped) continuum step and E its clamp correction (zero
//    unless the continuum's own clamp acted), the step of the total
//    intensity, clamped at zero, becomes
//      Delta_n = max(Delta_{n-1} + (2 tau_L (J_L - C_n) + E (3 + 2 tau_D)
//                    + Delta_{n-1} - Delta_{n-2} - 2 (tau_L + tau_D) Delta_{n-1})
//                    / (3 + 2 tau_L + 2 tau_D), -C_n).
//    Outside a cell's line window (tau_L = 0) that is three FMA-class
//    operations and a maximum with per-cell constants.
//  * Per-cell coefficients are computed lane-parallel for 64 cells at a time
//    (cell_setup.h) into an LDS table; the march reads a cell's row as
//    uniform 128-bit loads.
//  * The two nodes trade roles every step, so the cell loop takes two cells
//    per iteration and never moves a register.
//
// Selectively thin transfer (paper, "Transfer Solution: Selectively Thin
// Transfer", with the same section's substitution for the smooth steps):
// the profile is the channel average, the emission of the total is
// jbar_L + j_D - alphabar_L C_n (C_n the continuum of the same node) and its
// absorption the dust alone. The line then changes only the numerator:
//   Delta_n = max(Delta_{n-1} + (2 taubar (J_L - C_n) + E (3 + 2 tau_D)
//                 + Delta_{n-1} - Delta_{n-2} - 2 tau_D Delta_{n-1})
//                 / (3 + 2 tau_D), -C_n),
// i.e. the line-free step plus 2 taubar (J_L - C_n) r in the window's slots.
// taubar_k is the centre depth times (sqrt(pi)/2)(b/dv)[erf(x_hi) - erf(x_lo)],
// x = (v_edge - v)/b at the edges of channel k, the erf difference formed
// from erfc(|x|) at both edges (erfc_table.h) so that it keeps its relative
// accuracy in the tails; the window is the channels whose extent meets the
// line's (edges, not centres, as a line narrower than a channel still lands
// in one).

#include <array>
#include <utility>

#include "cell_setup.h"
#include "epilogue.h"
#include "erfc_table.h"
#include "host_common.h"

namespace iris {

// Per-cell table row (16 floats, 128-bit loads):
//   0: A, c0, lk, 2 J_L  profile argument t_k = (k - lo) A + c0, line optical
//                        depth tau_L = 2^(lk - t_k^2), line source term
//                        (selectively thin: x0, xs, amp, 2 J_L, the lower edge
//                        argument x_k = (k - lo) xs + x0 and taubar_k =
//                        amp [erf(x_k + xs) - erf(x_k)])
//   1: 3 + 2 tau_D, 2 h j_D, r, -2 tau_D   (r = 1 / (3 + 2 tau_D))
//   2: -, lo, hi, -                        line window [lo, hi] (int bits; hi < lo: none)
//   3: tau_D, h j_D, -, -                  (trapezoidal first step)
// Optical depths are per cell (h alpha); h j is in Rayleigh-Jeans kelvin.
enum : int { kSmRow = 16 };

constexpr int kSmoothMaxChannels = 2048;

// LDS floats per wavefront: the cell table and the line excess of every
// marched velocity for the epilogue.
__host__ __device__ inline int smooth_wave_floats(int n_chan) {
  return 64 * kSmRow + ((n_chan + 3) & ~3);
}

// One cell's table row in registers; lo and hi are uniform.
struct SmRow {
  float4 q0, q1, q2;
  int lo, hi;
};

__device__ __forceinline__ SmRow load_row(const float* row) {
  SmRow r;
  r.q0 = *(const float4*)row;
  r.q1 = *(const float4*)(row + 4);
  r.q2 = *(const float4*)(row + 8);
  r.lo = __builtin_amdgcn_readfirstlane(__float_as_int(r.q2.y));
  r.hi = __builtin_amdgcn_readfirstlane(__float_as_int(r.q2.z));
  return r;
}

// Channel-averaged line depth of slot m of this lane for the cell of row q0
// (selectively thin): amp [erf(x_hi) - erf(x_lo)] from erfc(|x|) at both
// edges, the difference of the two erfc values within one tail.
__device__ __forceinline__ float tau_bar(const float4& q0, int lo, int m, float lanef,
                                         const float4* etab) {
  const float x = fmaf((float)(64 * m - lo) + lanef, q0.y, q0.x);
  const float xh = x + q0.y;
  const float H = erfc_tab(etab, fabsf(x)), Hh = erfc_tab(etab, fabsf(xh));
  const float d = x >= 0.f ? H - Hh : (xh < 0.f ? Hh - H : 2.f - H - Hh);
  return q0.z * d;
}

// BDF2 step of the channel-independent intensities of one node: continuum,
// dust emission and background (no emission), from `newer` (node n-1) and
// `older` (node n-2) into `older`. Returns the new continuum C_n and its
// clamp correction E (the unclamped step minus C_n) for the channel step.
__device__ __forceinline__ void bdf2_continuum(float (&older)[3], const float (&newer)[3],
                                               const SmRow& r, float& Cn, float& E) {
  const float rr = r.q1.z, m2t = r.q1.w, e2 = r.q1.y;
  const float Cu = fmaf(rr, fmaf(m2t, newer[0], (newer[0] - older[0]) + e2), newer[0]);
  Cn = fmaxf(Cu, 0.f);
  E = Cu - Cn;
  older[0] = Cn;
  older[1] = fmaxf(fmaf(rr, fmaf(m2t, newer[1], (newer[1] - older[1]) + e2), newer[1]), 0.f);
  older[2] = fmaxf(fmaf(rr, fmaf(m2t, newer[2], newer[2] - older[2]), newer[2]), 0.f);
}

// One BDF2 step of the line excess in the S channel slots of this lane, from
// `newer` (node n-1) and `older` (node n-2) into `older`. Cn and E come from
// the continuum step of the same node. HAS_E: the continuum's clamp acted at
// this node (E != 0). Each slot tests one bit of a uniform mask of the slots
// the line window touches. SEL: selectively thin transfer.
template <int S, bool HAS_E, bool SEL>
__device__ __forceinline__ void bdf2_slots(float (&older)[S], const float (&newer)[S],
                                           float lanef, const SmRow& r, float Cn, float E,
                                           const float4* etab) {
  const int mlo = r.lo >> 6, mhi = min(r.hi >> 6, S - 1);
  const int nw = r.hi < r.lo ? 0 : mhi - mlo + 1;
  const uint32_t wm = nw >= 32 ? ~0u : ((1u << nw) - 1u) << mlo;
  const float rr = r.q1.z, m2t = r.q1.w, nC = -Cn;
#pragma unroll
  for (int m = 0; m < S; ++m) {
    const float D1 = newer[m];
    const float d = D1 - older[m];
    // The step without the line, taken in every slot (no branch around it);
    // the few slots the window touches take the full step instead.
    float x = fmaf(rr, fmaf(m2t, D1, d), D1);
    if (HAS_E) x += E;
    if (SEL && (wm & (1u << m))) {
      // Line-free step plus 2 taubar (J_L - C_n) r.
      const float src = fmaf(-2.f, Cn, r.q0.w);  // 2 (J_L - C_n)
      x = fmaf(tau_bar(r.q0, r.lo, m, lanef, etab) * src, rr, x);
    } else if (wm & (1u << m)) {
      const float t = fmaf((float)(64 * m - r.lo) + lanef, r.q0.x, r.q0.y);
      const float tl = ex2(fmaf(-t, t, r.q0.z));  // line optical depth
      const float den = fmaf(2.f, tl, r.q1.x);    // 3 + 2 (tau_L + tau_D)
      const float src = fmaf(-2.f, Cn, r.q0.w);   // 2 (J_L - C_n)
      const float w = fmaf(-2.f, tl, m2t);        // -2 (tau_L + tau_D)
      const float dE = HAS_E ? fmaf(E, r.q1.x, d) : d;
      const float num = fmaf(src, tl, fmaf(w, D1, dE));
      x = fmaf(num, __builtin_amdgcn_rcpf(den), D1);
    }
    // max(x, -C_n) as a median with +FLT_MAX: one instruction, no NaN quieting.
    older[m] = __builtin_amdgcn_fmed3f(x, nC, 3.402823466e38f);
  }
}

// A cell's step: continuum first, then the channels.
template <int S, bool SEL>
__device__ __forceinline__ void bdf2_cell(float (&older)[S], const float (&newer)[S],
                                          float (&cold)[3], const float (&cnew)[3], float lanef,
                                          const SmRow& r, const float4* etab) {
  float Cn, E;
  bdf2_continuum(cold, cnew, r, Cn, E);
  if (__builtin_amdgcn_readfirstlane(__float_as_uint(E)) == 0u)
    bdf2_slots<S, false, SEL>(older, newer, lanef, r, Cn, E, etab);
  else
    bdf2_slots<S, true, SEL>(older, newer, lanef, r, Cn, E, etab);
}

// Two values per slot stay live through the per-cell setup of each
// chunk, so wider variants take more registers per wavefront (fewer
// wavefronts per SIMD); their slots keep the SIMD busy on their own.
template <int S>
constexpr int smooth_waves_per_eu() { return S <= 4 ? 4 : S <= 16 ? 3 : 2; }

// S = ceil(C / 64) exactly, one kernel per slot count, so that no slot test
// or padding costs anything in the march; the storage type is taken at run
// time in the per-cell setup. GEN: separate line and dust source functions.
// SEL: selectively thin transfer (erfc_pieces: the erfc table, staged in LDS).
template <bool GEN, int S, bool SEL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(smooth_waves_per_eu<S>())))
void smooth_kernel(const FwdParams P, const float4* erfc_pieces) {
  extern __shared__ float lds[];
  __shared__ float4 etab[SEL ? kErfcN : 1];
  if (SEL) {
    // Staged before any wavefront leaves.
    for (int i = threadIdx.x; i < kErfcN; i += blockDim.x) etab[i] = gload(erfc_pieces + i);
    __syncthreads();
  }
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int tile = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  const int64_t pix = (int64_t)tile * kWavesPerBlock + wave;
  if (pix >= P.n_pix) return;  // whole wavefront
  const Folded& c = P.c;
  const int C = c.n_chan;
  float* tbl = lds + (size_t)wave * smooth_wave_floats(C);
  float* psi = tbl + 64 * kSmRow;
  const float lanef = (float)lane;
  const float Ibg = (float)c.J_bg;
  const DynLoader load(P.f, P.at.base(pix), P.dtype);

  // X and Y hold the line excess of nodes n-2 and n-1 at the start of each
  // pair of steps; the step of the first cell of a pair writes X, the second
  // Y. cX, cY: the same for continuum, dust emission and background.
  float X[S], Y[S], cX[3], cY[3];
  bool odd = false;  // after an unpaired last step, X holds the newest

  DynLoader::Raw pre = load.fetch((int64_t)lane * P.at.los, lane < P.n_los);
  for (int s0 = 0; s0 < P.n_los; s0 += 64) {
    const int s = s0 + lane;
    const bool valid = s < P.n_los;
    const CellIn in = load.decode(pre, valid);
    const CellOut o = cell_setup<GEN>(c, in, valid, true);
    {
      // The unclamped dust depth: no rescaling here, and the step needs it.
      const float tD = valid ? c.kD * (float)o.n : 0.f;
      const float hjD = tD * o.JD;
      const float r = 1.f / fmaf(2.f, tD, 3.f);
      float* row = tbl + lane * kSmRow;
      if constexpr (SEL) {
        // Channels whose extent meets |v' - v| <= x_w b (the window test of
        // the thick march at channel edges), clipped to the grid. The edge
        // argument is taken from the nearest channel centre kc and the FP64
        // offset of v from it: x at the lower edge of channel e is
        // ((e - kc) dv - (v - v_kc) - dv/2) / b, with b / dv = sqrt(log2 e) / A.
        const float u = fmaf((float)(in.v - c.v_lo), (float)c.inv_dv, -0.5f);
        const float kc = fminf(fmaxf(rintf(u), -1.f), (float)C);
        const double rv = in.v - (c.v_lo + ((double)kc + 0.5) * c.dv);
        const float Rt = (float)rv * (o.A / (float)c.dv);
        const float xw =
            __builtin_amdgcn_sqrtf(c.xw2min + fmaxf(0.f, (o.lk - 0.52876637f) * kLn2));
        const float hw = xw * kSqrtLog2e / o.A;
        const float e0f = fmaxf(ceilf(u - hw - 0.5f), 0.f);
        const float e1f = fminf(floorf(u + hw + 0.5f), (float)(C - 1));
        const bool line = valid && o.kL > 0.f && o.kL >= c.kL_min && e0f <= e1f;
        const int e0 = line ? (int)e0f : 0;
        const float isl = 1.f / kSqrtLog2e;
        // amp: the centre depth times (sqrt(pi)/2)(b/dv), half of the channel
        // mean's factor sqrt(pi) (b/dv) over the erf difference.
        *(float4*)row = line ? make_float4((fmaf((float)e0 - kc, o.A, -Rt) - 0.5f * o.A) * isl,
                                           o.A * isl,
                                           o.kL * (0.88622692545275801f * kSqrtLog2e) / o.A,
                                           2.f * o.JL)
                             : make_float4(0.f, 0.f, 0.f, 2.f * o.JL);
        *(float4*)(row + 8) = make_float4(0.f, __int_as_float(e0),
                                          __int_as_float(line ? (int)e1f : -1), 0.f);
      } else {
        const bool line = o.nwin > 0;
        *(float4*)row = make_float4(o.A, o.c0, line ? o.lk - 0.52876637f : -256.f, 2.f * o.JL);
        *(float4*)(row + 8) = make_float4(0.f, __int_as_float(o.kstart),
                                          __int_as_float(line ? o.kstart + o.nwin - 1 : -1), 0.f);
      }
      *(float4*)(row + 4) = make_float4(fmaf(2.f, tD, 3.f), 2.f * hjD, r, -2.f * tD);
      *(float4*)(row + 12) = make_float4(tD, hjD, 0.f, 0.f);
    }
    wave_order();
    pre = load.fetch((int64_t)(s0 + 64 + lane) * P.at.los, s0 + 64 + lane < P.n_los);
    const int nv = min(64, P.n_los - s0);

    int i = 0;
    if (s0 == 0) {
      // Node 0 is the background. The trapezoidal first step needs the
      // coefficients of nodes 0 and 1 in every channel:
      // I_1 = (hj_0 + (2 - tau_0) I_0 + hj_1) / (2 + tau_1), taken in
      // intensity once; the excess at node 0 is zero.
      const float* r0 = tbl;
      const float4 p0 = *(const float4*)r0;
      const float4 d0 = *(const float4*)(r0 + 12);
#pragma unroll
      for (int m = 0; m < S; ++m) {
        if constexpr (SEL) {
          // hj_0 = taubar (J_L - C_0) + h j_D with C_0 the background; the
          // absorption is the dust's.
          const float tb = tau_bar(p0, __float_as_int(r0[9]), m, lanef, etab);
          X[m] = fmaf(2.f - d0.x, Ibg, fmaf(0.5f * p0.w - Ibg, tb, d0.y));
        } else {
          const float t =
              fmaf((float)(64 * m) + lanef - (float)__float_as_int(r0[9]), p0.x, p0.y);
          const float tl = ex2(fmaf(-t, t, p0.z));
          const float hj = fmaf(0.5f * p0.w, tl, d0.y);
          X[m] = fmaf(2.f - tl - d0.x, Ibg, hj);  // carried into step 1
        }
        Y[m] = 0.f;
      }
      cX[0] = fmaf(2.f - d0.x, Ibg, d0.y);
      cX[1] = d0.y;
      cX[2] = (2.f - d0.x) * Ibg;
      cY[0] = Ibg;
      cY[1] = 0.f;
      cY[2] = Ibg;
      if (nv > 1) {
        const float* r1 = tbl + kSmRow;
        const float4 p1 = *(const float4*)r1;
        const float4 d1 = *(const float4*)(r1 + 12);
        const float rc = __builtin_amdgcn_rcpf(2.f + d1.x);
        const float c1 = fmaxf((cX[0] + d1.y) * rc, 0.f);
        const float e1 = fmaxf((cX[1] + d1.y) * rc, 0.f);
        const float b1 = fmaxf(cX[2] * rc, 0.f);
#pragma unroll
        for (int m = 0; m < S; ++m) {
          float I1;
          if constexpr (SEL) {
            const float tb = tau_bar(p1, __float_as_int(r1[9]), m, lanef, etab);
            I1 = fmaxf((X[m] + fmaf(0.5f * p1.w - c1, tb, d1.y)) * rc, 0.f);
          } else {
            const float t =
                fmaf((float)(64 * m) + lanef - (float)__float_as_int(r1[9]), p1.x, p1.y);
            const float tl = ex2(fmaf(-t, t, p1.z));
            const float hj = fmaf(0.5f * p1.w, tl, d1.y);
            I1 = fmaxf((X[m] + hj) * __builtin_amdgcn_rcpf(2.f + tl + d1.x), 0.f);
          }
          X[m] = 0.f;  // node 0: the background is the continuum
          Y[m] = I1 - c1;
        }
        cX[0] = cY[0];
        cX[1] = cY[1];
        cX[2] = cY[2];
        cY[0] = c1;
        cY[1] = e1;
        cY[2] = b1;
      }
      i = min(2, nv);
    }
    for (; i + 2 <= nv; i += 2) {
      // Both rows first: the second one's loads wait behind the first step.
      const SmRow ra = load_row(tbl + i * kSmRow);
      const SmRow rb = load_row(tbl + (i + 1) * kSmRow);
      bdf2_cell<S, SEL>(X, Y, cX, cY, lanef, ra, etab);
      bdf2_cell<S, SEL>(Y, X, cY, cX, lanef, rb, etab);
    }
    if (i < nv) {
      // Unpaired last cell (only in the last chunk: the others hold 64
      // cells, and the first one's two trapezoidal nodes keep it even).
      bdf2_cell<S, SEL>(X, Y, cX, cY, lanef, load_row(tbl + i * kSmRow), etab);
      odd = true;
    }
    wave_order();
  }

  // Line excess over the continuum per marched velocity, then the outputs.
  const float Cn = odd ? cX[0] : cY[0];
  const float Dn = odd ? cX[1] : cY[1];
  const float Bn = odd ? cX[2] : cY[2];
#pragma unroll
  for (int m = 0; m < S; ++m) {
    const int k = 64 * m + lane;
    if (k < C) psi[k] = odd ? X[m] : Y[m];
  }
  wave_order();
  write_outputs<64>(c, P.out, pix, psi, lane, c.out_scale, Cn, (double)Dn, (double)Bn);
}

size_t smooth_lds_bytes(int n_chan) {
  return (size_t)kWavesPerBlock * smooth_wave_floats(n_chan) * sizeof(float);
}

int smooth_max_channels() { return kSmoothMaxChannels; }

template <bool GEN, bool SEL, int... I>
constexpr auto smooth_kernels(std::integer_sequence<int, I...>) {
  return std::array<void (*)(FwdParams, const float4*), sizeof...(I)>{
      &smooth_kernel<GEN, I + 1, SEL>...};
}

template <bool SEL>
static int launch_smooth_t(iris_dtype dt, const FwdParams& p, const void* table, void* stream) {
  using Slots = std::make_integer_sequence<int, kSmoothMaxChannels / 64>;
  static constexpr auto shared = smooth_kernels<false, SEL>(Slots{});
  static constexpr auto general = smooth_kernels<true, SEL>(Slots{});
  if (p.c.n_chan < 1 || p.c.n_chan > kSmoothMaxChannels || p.n_los < 1 ||
      p.dtype != (int32_t)dt || (SEL && !table))
    return (int)hipErrorInvalidValue;
  const int ns = (p.c.n_chan + 63) / 64;
  const int blocks = (int)((p.n_pix + kWavesPerBlock - 1) / kWavesPerBlock);
  FwdParams arg = p;
  const float4* tab = (const float4*)table;
  void* args[] = {&arg, &tab};
  const auto& kernels = p.c.general ? general : shared;
  return (int)hipLaunchKernel((const void*)kernels[ns - 1], dim3(blocks), dim3(64 * kWavesPerBlock),
                              args, smooth_lds_bytes(p.c.n_chan), (hipStream_t)stream);
}

int launch_smooth(iris_dtype dt, const FwdParams& p, void* stream) {
  return launch_smooth_t<false>(dt, p, nullptr, stream);
}

int launch_smooth_selective(iris_dtype dt, const FwdParams& p, const void* table, void* stream) {
  return launch_smooth_t<true>(dt, p, table, stream);
}

}  // namespace iris
