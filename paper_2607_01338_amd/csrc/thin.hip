// Optically thin and selectively thin transfer.
//
// Method (paper, "Transfer Solution: Optically Thin Transfer"): absorption
// and stimulation are ignored, so each intensity is the background plus the
// path integral of its emission. The line profile is replaced by its mean
// over each channel, (1/dv) (1/2) [erf(x_hi) - erf(x_lo)] with
// x = (v_edge - v)/b at the channel's edges, so no velocity subsampling is
// needed. The formal integrator sums every cell (each cell the midpoint of
// its own step); the smooth one takes Simpson panels of two cells over the
// nodes 0 .. 2P, P = floor((N - 1)/2), weights 1 4 2 4 ... 4 1 / 3.
// Selectively thin transfer (paper, "Transfer Solution: Selectively Thin
// Transfer", formal steps): the line absorbs the continuum but not itself;
// each cell's continuum step is solved first, and the line excess takes the
// formal step with the dust depth and the source taubar (J_L - C_n), the
// total clamped at zero after every step.
//
// How it is organised on gfx950:
//  * G = 1, 2 or 4 sightlines per wavefront, W = 64/G lanes each. Per-cell
//    coefficients are computed lane-parallel for W cells of each sightline at
//    a time (cell_setup.h) into an LDS table.
//  * The line sum of every channel is kept in LDS. A cell adds to the
//    channels whose extent meets its line window (the thick march's window
//    test taken at channel edges, so that a line narrower than a channel
//    still lands in it): W - 1 channels per pass of W lanes, lane l of a
//    group evaluating the channel edge e0 + l, the upper edge coming from
//    lane l + 1 by a DPP wave shift. The edge function is erfc(|x|), so that
//    the difference of two edges in the same tail keeps its relative
//    accuracy.
//  * erfc on [0, 6) comes from a table of cubic Hermite pieces (values and
//    derivatives, -2/sqrt(pi) e^{-x^2}, built in FP64 by a small kernel per
//    call and staged in LDS per workgroup): 512 pieces of width 6/512 leave
//    an interpolation error below 1e-9, under the FP32 rounding of the
//    result; beyond 6, erfc < 3e-17 is taken as zero. An edge then costs a
//    table read and three FMAs instead of a rational approximation.
//  * Optically thin: the dust emission is a group sum per chunk, carried in
//    FP64; the background is not attenuated. Selectively thin: the
//    continuum and the dust depth come from DPP scans per chunk, and the
//    line sums are kept scaled to the depth at the chunk's end.

#include "cell_partials.h"
#include "cell_setup.h"
#include "epilogue.h"
#include "erfc_table.h"

namespace iris {

// Row of a cell in the chunk table: x0, xs, amp, e0 | ne << 16 (int bits);
// selectively thin adds the floor of the scaled sums (padded to 6 floats for
// 8-byte accesses). Short rows leave LDS for four wavefronts per SIMD at 800
// channels (three with 8-float rows).
__host__ __device__ constexpr int thin_row(bool sel) { return sel ? 6 : 4; }
constexpr int kDppWaveShl1 = 0x130;  // lane i receives lane i + 1 (lane 63: 0)
// Piece i of erfc on [x_i, x_i + h], h = kErfcMax / kErfcN, as the cubic
// c0 + c1 s + c2 s^2 + c3 s^3 in s = (x - x_i)/h through the values and
// derivatives at both ends (FP64, rounded once).
__global__ void erfc_table_kernel(float4* tab) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kErfcN) return;
  const double h = (double)kErfcMax / kErfcN;
  const double x0 = i * h, x1 = (i + 1) * h;
  const double k = -1.1283791670955126;  // -2/sqrt(pi)
  const double f0 = erfc(x0), f1 = erfc(x1);
  const double d0 = k * exp(-x0 * x0) * h, d1 = k * exp(-x1 * x1) * h;
  tab[i] = make_float4((float)f0, (float)d0, (float)(3.0 * (f1 - f0) - 2.0 * d0 - d1),
                       (float)(2.0 * (f0 - f1) + d0 + d1));
}

// Weight of node n of N in the path integral (times the cell length, which
// the per-cell optical depths already carry).
__device__ __forceinline__ float thin_weight(bool smooth, int n, int N) {
  if (!smooth) return 1.f;
  const int last = 2 * ((N - 1) / 2);
  if (last == 0 || n > last) return 0.f;
  if (n == 0 || n == last) return 1.f / 3.f;
  return (n & 1) ? 4.f / 3.f : 2.f / 3.f;
}

// Inclusive scan of affine maps x -> A x + B within aligned groups of W lanes
// (lane i ends with the composition of lanes 0..i, the lowest applied first),
// on DPP moves: row shifts inside each row of 16, then row broadcasts, as the
// prefix sums of the march (lanes without a source take the identity).
template <int Ctrl, int RowMask>
__device__ __forceinline__ void affine_step(float& A, float& B) {
  const float Ap = __int_as_float(__builtin_amdgcn_update_dpp(
      __float_as_int(1.f), __float_as_int(A), Ctrl, RowMask, 0xF, false));
  const float Bp = __int_as_float(
      __builtin_amdgcn_update_dpp(0, __float_as_int(B), Ctrl, RowMask, 0xF, false));
  B = fmaf(A, Bp, B);
  A *= Ap;
}
template <int W>
__device__ __forceinline__ void group_scan_affine(float& A, float& B) {
  affine_step<kDppRowShr + 1, 0xF>(A, B);
  affine_step<kDppRowShr + 2, 0xF>(A, B);
  affine_step<kDppRowShr + 4, 0xF>(A, B);
  affine_step<kDppRowShr + 8, 0xF>(A, B);
  if (W >= 32) affine_step<kDppRowBcast15, 0xA>(A, B);
  if (W == 64) affine_step<kDppRowBcast31, 0xC>(A, B);
}

// Floats of LDS per wavefront: the cell table of 64 rows and, per sightline
// group, the line sum of every channel (multiple of 4, with W spare).
__host__ __device__ inline int thin_state_stride(int n_chan, int groups) {
  return (n_chan + 64 / groups + 3) & ~3;
}
__host__ __device__ inline int thin_wave_floats(int n_chan, int groups, bool sel) {
  return 64 * thin_row(sel) + groups * thin_state_stride(n_chan, groups);
}

// G sightlines per wavefront, W = 64/G lanes each: a pass covers W - 1
// channels of every group's cell at once. SEL: selectively thin transfer
// (formal steps) instead of optically thin.
template <bool GEN, int G, bool SEL>
__global__ __launch_bounds__(256) void thin_kernel(const FwdParams P, int smooth,
                                                   const float4* erfc_pieces) {
  constexpr int W = 64 / G;
  __shared__ float4 etab[kErfcN];
  extern __shared__ float lds[];
  // Stage the erfc table before any wavefront leaves.
  for (int i = threadIdx.x; i < kErfcN; i += blockDim.x) etab[i] = gload(erfc_pieces + i);
  __syncthreads();
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int sub = lane / W, sl = lane % W;
  const int tile = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  const int64_t pix0 = ((int64_t)tile * kWavesPerBlock + wave) * G;
  if (pix0 >= P.n_pix) return;  // whole wavefront
  const int64_t pix = pix0 + sub;
  const bool live = pix < P.n_pix;
  const Folded& c = P.c;
  const int C = c.n_chan;
  const int stride = thin_state_stride(C, G);
  constexpr int kRow = thin_row(SEL);
  float* lw = lds + (size_t)wave * thin_wave_floats(C, G, SEL);
  float* tbl = lw + sub * W * kRow;
  float* psi = lw + 64 * kRow + sub * stride;
  for (int k = sl; k < stride; k += W) psi[k] = 0.f;
  const DynLoader load(P.f, P.at.base(live ? pix : P.n_pix - 1), P.dtype);
  const float isl = 1.f / kSqrtLog2e;  // profile argument t = x sqrt(log2 e)
  double Dsum = 0.0;
  // Selectively thin: the continuum map of the sightline so far,
  // I -> Atot I + Btot (FP64), applied to the background.
  double Atot = 1.0, Btot = 0.0;

  for (int s0 = 0; s0 < P.n_los; s0 += W) {
    const int s = s0 + sl;
    const bool valid = live && s < P.n_los;
    const CellIn in = load(s * P.at.los, valid);
    const CellOut o = cell_setup<GEN>(c, in, valid, true);
    const float w = valid ? thin_weight(smooth != 0, s, P.n_los) : 0.f;
    const int nv = min(W, P.n_los - s0);
    // Optically thin: the dust emission h j_D = tau_D J_D is summed (the
    // unclamped depth: nothing is attenuated). Selectively thin: the line
    // excess takes the formal step Delta_n = a Delta_{n-1} + taubar (J_L - C_n)
    // (1 - a)/tau_D, a = e^{-tau_D}, C_n the continuum after cell n. It is kept
    // scaled by e^{P_n - base}, base = the dust depth at the end of the chunk
    // (so every factor is at most 1): the cell's weight below carries
    // (J_L - C_n)(1 - a)/tau_D e^{P_n - P_end}, and the sums are rescaled by
    // e^{-(chunk depth)} before the chunk's cells are added.
    float lw_line = 1.f;
    float flo = 0.f;  // selectively thin: lowest scaled line sum, -C_n e^{P_n - base}
    if (SEL) {
      const float tD = valid ? c.kD * (float)o.n : 0.f;
      const float om = tD >= 0.25f ? one_minus_exp_neg(tD) : one_minus_exp_neg_small(tD);
      float A = valid ? 1.f - om : 1.f, B = valid ? o.JD * om : 0.f;
      group_scan_affine<W>(A, B);
      const float Pin = group_scan_dpp<W>(tD);
      const int last = sub * W + nv - 1;
      const float Pend = __shfl(Pin, last, 64);
      const float Alast = __shfl(A, last, 64), Blast = __shfl(B, last, 64);
      const float Cn = fmaf(A, (float)(Atot * c.J_bg + Btot), B);
      const float fD = tD > 1e-4f ? om / tD : 1.f - 0.5f * tD;
      const float esc = ex2((Pin - Pend) * kLog2e);
      lw_line = (o.JL - Cn) * fD * esc;
      flo = -Cn * esc;
      const float resc = ex2(-Pend * kLog2e);
      for (int k = sl; k < C; k += W) psi[k] *= resc;
      Btot = (double)Alast * Btot + (double)Blast;
      Atot *= (double)Alast;
    } else {
      Dsum += (double)group_allsum<W>(w * (c.kD * (float)o.n) * o.JD);
    }
    {
      // Channels whose extent meets |v' - v| <= x_w b (the thick march's
      // window test, at channel edges instead of centres), clipped to the
      // grid. The line centre sits at u channels (centre units); the profile
      // argument is taken from the nearest channel centre kc and the FP64
      // offset of v from it, as in the cell setup, but for every cell (the
      // setup's own reference exists only where its centre window is not
      // empty): x at the lower edge of channel e is
      // ((e - kc) dv - (v - v_kc) - dv/2) / b, with b / dv = sqrt(log2 e) / A.
      const float u = fmaf((float)(in.v - c.v_lo), (float)c.inv_dv, -0.5f);
      const float kc = fminf(fmaxf(rintf(u), -1.f), (float)C);
      const double rr = in.v - (c.v_lo + ((double)kc + 0.5) * c.dv);
      const float Rt = (float)rr * (o.A / (float)c.dv);  // (v - v_kc) sqrt(log2 e) / b
      const float xw = __builtin_amdgcn_sqrtf(c.xw2min + fmaxf(0.f, (o.lk - 0.52876637f) * kLn2));
      const float hw = xw * kSqrtLog2e / o.A;
      const float e0f = fmaxf(ceilf(u - hw - 0.5f), 0.f);
      const float e1f = fminf(floorf(u + hw + 0.5f), (float)(C - 1));
      const bool line = w > 0.f && o.kL > 0.f && o.kL >= c.kL_min && e0f <= e1f;
      const int e0 = line ? (int)e0f : 0;
      float* row = tbl + sl * kRow;
      // Channel mean of the line depth over the centre depth: (sqrt(pi)/2) (b/dv) d.
      const float4 rv = make_float4(
          (fmaf((float)e0 - kc, o.A, -Rt) - 0.5f * o.A) * isl, o.A * isl /* dv / b */,
          w * o.kL * (SEL ? lw_line : o.JL) * (0.88622692545275801f * kSqrtLog2e) / o.A,
          __int_as_float(e0 | ((line ? (int)e1f - e0 + 1 : 0) << 16)));
      if (SEL) {
        ((float2*)row)[0] = make_float2(rv.x, rv.y);
        ((float2*)row)[1] = make_float2(rv.z, rv.w);
        ((float2*)row)[2] = make_float2(flo, 0.f);
      } else {
        *(float4*)row = rv;
      }
    }
    wave_order();
    // A cell's row: x0, dv/b, amplitude and the packed window (one 16-byte
    // read, or two 8-byte reads for the 6-float selective rows), plus the
    // selective floor.
    struct Row {
      float4 q;
      float floor;
    };
    auto read_row = [&](int i) {
      const float* r = tbl + i * kRow;
      Row o;
      if (SEL) {
        const float2 a = *(const float2*)r, b = *(const float2*)(r + 2);
        o.q = make_float4(a.x, a.y, b.x, b.y);
        o.floor = r[4];
      } else {
        o.q = *(const float4*)r;
        o.floor = 0.f;
      }
      return o;
    };
    // Channel mean of a cell's line in the channel of this lane in pass q
    // (0 outside the window): erf(x_hi) - erf(x_lo) from erfc(|x|) at both
    // edges, the upper one from the next lane (the last lane of a group
    // evaluates only that edge). Branch-free, so that the scheduler can
    // interleave the table reads of two cells.
    auto contribution = [&](const Row& r, int ne, int q) {
      const int j = (W - 1) * q + sl;
      const float x = fmaf((float)j, r.q.y, r.q.x);
      const float H = erfc_tab(etab, fabsf(x));
      const float Hn = __int_as_float(
          __builtin_amdgcn_update_dpp(0, __float_as_int(H), kDppWaveShl1, 0xF, 0xF, false));
      const float xh = x + r.q.y;
      const float dpos = H - Hn;           // both edges above the centre
      const float dmid = 2.f - H - Hn;     // the centre inside the channel
      const float d = x >= 0.f ? dpos : (xh < 0.f ? -dpos : dmid);
      return (sl < W - 1 && j < ne) ? r.q.z * d : 0.f;
    };
    // Passes of cell i: the widest window over the groups.
    auto max_ne = [&](int ne) { return groups_max<G>(ne); };
    // A cell's update of one channel. Selectively thin: every step of the
    // total is clamped at zero intensity, I_T = C_n + Delta_n >= 0, i.e. the
    // scaled line sum at -C_n e^{P_n - base} (the row's floor); outside a
    // cell's window the total takes a dust-only step from a non-negative value
    // and needs no clamp.
    auto add = [&](float* pp, float v, const Row& r) {
      *pp = SEL ? fmaxf(*pp + v, r.floor) : *pp + v;
    };
    int i = 0;
    // Two cells at a time where every window fits one pass: their profiles do
    // not depend on the sums, so they are evaluated before the two
    // read-modify-writes, in order.
    for (; i + 2 <= nv; i += 2) {
      const Row ra = read_row(i), rb = read_row(i + 1);
      const int pa = __float_as_int(ra.q.w), pb = __float_as_int(rb.q.w);
      const int na = pa >> 16, nb = pb >> 16, ea = pa & 0xFFFF, eb = pb & 0xFFFF;
      const int ma = max_ne(na), mb = max_ne(nb);
      if (ma <= W - 1 && mb <= W - 1) {
        const float ca = contribution(ra, na, 0);
        const float cb = contribution(rb, nb, 0);
        if (sl < na) add(psi + ea + sl, ca, ra);
        wave_order();
        if (sl < nb) add(psi + eb + sl, cb, rb);
        wave_order();
        continue;
      }
      for (int q = 0; (W - 1) * q < ma; ++q) {
        const float ca = contribution(ra, na, q);
        if (sl < W - 1 && (W - 1) * q + sl < na) add(psi + ea + (W - 1) * q + sl, ca, ra);
      }
      wave_order();
      for (int q = 0; (W - 1) * q < mb; ++q) {
        const float cb = contribution(rb, nb, q);
        if (sl < W - 1 && (W - 1) * q + sl < nb) add(psi + eb + (W - 1) * q + sl, cb, rb);
      }
      wave_order();
    }
    if (i < nv) {
      const Row ra = read_row(i);
      const int pa = __float_as_int(ra.q.w);
      const int na = pa >> 16, ea = pa & 0xFFFF;
      const int ma = max_ne(na);
      for (int q = 0; (W - 1) * q < ma; ++q) {
        const float ca = contribution(ra, na, q);
        if (sl < W - 1 && (W - 1) * q + sl < na) add(psi + ea + (W - 1) * q + sl, ca, ra);
      }
    }
    wave_order();
  }
  if (!live) return;
  if (SEL)
    write_outputs<W>(c, P.out, pix, psi, sl, c.out_scale, (float)(Atot * c.J_bg + Btot), Btot,
                     Atot * c.J_bg);
  else
    write_outputs<W>(c, P.out, pix, psi, sl, c.out_scale, (float)(c.J_bg + Dsum), Dsum, c.J_bg);
}

// Reverse mode of optically thin transfer ("differentiability modes" in
// "Synthetic Observation Implementation and Algorithms"). Nothing attenuates,
// so the loss is linear in each cell's emission and the cells are
// independent: per cell, three sums over its window of the line cotangent g_k
// (times the output units) against the channel mean d_k = erf(x_hi) - erf(x_lo)
// and the parts of its derivatives in v and b,
//   S1 = sum g d,  Sv = sum g (e^{-x_lo^2} - e^{-x_hi^2}),
//   Sb = sum g (x_lo e^{-x_lo^2} - x_hi e^{-x_hi^2}),
// (d d / d v = (2/sqrt(pi)) (e^{-x_lo^2} - e^{-x_hi^2}) / b, d d / d b the same
// with Sb's weights), then the chain rule of the cell's line amplitude
// w (sqrt(pi)/2) Q J_L / dv, Q = kappa_L b (which does not depend on b), and
// of its dust emission w tau_D J_D, whose cotangent is the sum over the
// channels of [T], [C] and [D]'s. Windows, weights and packing are the
// forward's; each lane walks its own cell's window, so no sum crosses lanes.
// LDS per wavefront: per group the line cotangent row.
__host__ __device__ inline int thin_adj_wave_floats(int n_chan, int groups) {
  return groups * thin_state_stride(n_chan, groups);
}

template <bool GEN, int G>
__global__ __launch_bounds__(256) void thin_adj_kernel(const AdjParams P, int smooth,
                                                       const float4* erfc_pieces) {
  constexpr int W = 64 / G;
  __shared__ float4 etab[kErfcN];
  extern __shared__ float lds[];
  for (int i = threadIdx.x; i < kErfcN; i += blockDim.x) etab[i] = gload(erfc_pieces + i);
  __syncthreads();
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int sub = lane / W, sl = lane % W;
  const int tile = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  const int64_t pix0 = ((int64_t)tile * kWavesPerBlock + wave) * G;
  if (pix0 >= P.n_pix) return;  // whole wavefront
  const int64_t pix = pix0 + sub;
  const bool live = pix < P.n_pix;
  const Folded& c = P.c;
  const int C = c.n_chan;
  const int stride = thin_state_stride(C, G);
  float* gl = lds + (size_t)wave * thin_adj_wave_floats(C, G) + sub * stride;
  const float* gT = live && P.cot[0] ? P.cot[0] + pix * C : nullptr;
  const float* gC = live && P.cot[1] ? P.cot[1] + pix * C : nullptr;
  const float* gD = live && P.cot[2] ? P.cot[2] + pix * C : nullptr;
  const float* gL = live && P.cot[3] ? P.cot[3] + pix * C : nullptr;
  // Line cotangent per channel ([L] = [T] - [C]) and the continuum's, the sum
  // over the channels of the [T], [C] and [D] cotangents (the dust emission
  // enters all three).
  double sc = 0.0;
  for (int k = sl; k < stride; k += W) {
    float v = 0.f;
    if (k < C) {
      const float t = gT ? gload(gT + k) : 0.f, l = gL ? gload(gL + k) : 0.f;
      v = (t + l) * c.out_scale;
      sc += (double)t + (gC ? (double)gload(gC + k) : 0.0) + (gD ? (double)gload(gD + k) : 0.0);
    }
    gl[k] = v;
  }
  const double SC = group_sum<W>(sc) * (double)c.out_scale;
  wave_order();
  const DynLoader load(P.f, P.at.base(live ? pix : P.n_pix - 1), P.dtype);
  const bool has_td = GEN && P.f[4] != nullptr;
  const float isl = 1.f / kSqrtLog2e;

  for (int s0 = 0; s0 < P.n_los; s0 += W) {
    const int s = s0 + sl;
    const bool valid = live && s < P.n_los;
    const CellIn in = load(s * P.at.los, valid);
    const CellOut o = cell_setup<GEN>(c, in, valid, true);
    const float w = valid ? thin_weight(smooth != 0, s, P.n_los) : 0.f;
    // The forward's window and profile argument (thin_kernel). Lane sl walks
    // its own cell's window channel by channel (no sums across lanes), each
    // channel's upper edge the next one's lower.
    const float u = fmaf((float)(in.v - c.v_lo), (float)c.inv_dv, -0.5f);
    const float kc = fminf(fmaxf(rintf(u), -1.f), (float)C);
    const double rr = in.v - (c.v_lo + ((double)kc + 0.5) * c.dv);
    const float Rt = (float)rr * (o.A / (float)c.dv);
    const float xw = __builtin_amdgcn_sqrtf(c.xw2min + fmaxf(0.f, (o.lk - 0.52876637f) * kLn2));
    const float hw = xw * kSqrtLog2e / o.A;
    const float e0f = fmaxf(ceilf(u - hw - 0.5f), 0.f);
    const float e1f = fminf(floorf(u + hw + 0.5f), (float)(C - 1));
    const bool line = w > 0.f && o.kL > 0.f && o.kL >= c.kL_min && e0f <= e1f;
    const int e0 = line ? (int)e0f : 0;
    const int ne = line ? (int)e1f - e0 + 1 : 0;
    const float x0 = (fmaf((float)e0 - kc, o.A, -Rt) - 0.5f * o.A) * isl;
    const float dvb = o.A * isl;  // dv / b
    float x = x0;
    float H = erfc_tab(etab, fabsf(x)), ex = ex2(-x * x * kLog2e);
    float s1 = 0.f, sv = 0.f, sb = 0.f;
#pragma unroll 4
    for (int j = 0; j < ne; ++j) {
      const float xn = fmaf((float)(j + 1), dvb, x0);
      const float Hn = erfc_tab(etab, fabsf(xn));
      const float exn = ex2(-xn * xn * kLog2e);
      const float xh = x + dvb;
      const float dpos = H - Hn;
      const float d = x >= 0.f ? dpos : (xh < 0.f ? -dpos : 2.f - H - Hn);
      const float g = gl[e0 + j];
      s1 = fmaf(g, d, s1);
      sv = fmaf(g, ex - exn, sv);
      sb = fmaf(g, fmaf(x, ex, -xn * exn), sb);
      x = xn;
      H = Hn;
      ex = exn;
    }
    if (valid) {
      const float4 rs = make_float4(s1, sv, sb, 0.f);
      const CellPartials cp =
          GEN && c.ot ? cell_partials_ot(c, (double)in.lnn, (double)in.T, (double)in.X)
                      : cell_partials<GEN>(c, (double)in.lnn, (double)in.T, (double)in.X);
      const double JL = (double)o.JL;
      const double Q = cp.kL * cp.b;                       // kappa_L b
      const double a = (double)w * 0.88622692545275801 / c.dv;  // w (sqrt(pi)/2) / dv
      const double bQ = (double)rs.x * a * JL, bJL = (double)rs.x * a * Q;
      const double vb = (double)w * Q * JL / (c.dv * cp.b);  // amplitude (2/sqrt(pi)) / b
      const double gv = vb * (double)rs.y;
      double gT = vb * (double)rs.z * cp.db_dT + bQ * (cp.dkL_dT * cp.b + cp.kL * cp.db_dT) +
                  bJL * (GEN ? cp.dJL_dT : cp.dJ_dT);
      double glnn = bQ * cp.b * (cp.kL + cp.dkL_dlnn) + bJL * cp.dJL_dlnn;
      const double gX = bQ * cp.b * cp.dkL_dX;
      // Dust emission w kappa_D n J_D (unclamped: nothing is attenuated).
      const double bDe = SC * (double)w;
      const double kDn = (double)(c.kD * (float)o.n);
      glnn += bDe * kDn * (double)o.JD;
      double gTd = 0.0;
      if (has_td) gTd = bDe * kDn * planck_rj_dT(c, (double)in.Td);
      else gT += bDe * kDn * cp.dJ_dT;
      const int64_t off = P.gat.base(pix) + (int64_t)s * P.gat.los;
      gstore(P.grad[0] + off, glnn);
      gstore(P.grad[1] + off, gT);
      gstore(P.grad[2] + off, gv);
      gstore(P.grad[3] + off, gX);
      if (has_td) gstore(P.grad[4] + off, gTd);
    }
    wave_order();
  }
}

template <bool GEN, int G>
static void launch_thin_adj_g(const AdjParams& p, int sm, const float4* tab, hipStream_t st) {
  const int64_t waves = (p.n_pix + G - 1) / G;
  const int blocks = (int)((waves + kWavesPerBlock - 1) / kWavesPerBlock);
  const size_t lds = (size_t)kWavesPerBlock * thin_adj_wave_floats(p.c.n_chan, G) * sizeof(float);
  hipLaunchKernelGGL((thin_adj_kernel<GEN, G>), dim3(blocks), dim3(64 * kWavesPerBlock), lds, st,
                     p, sm, tab);
}

size_t thin_adj_lds_bytes(int n_chan, int groups) {
  return (size_t)kWavesPerBlock * thin_adj_wave_floats(n_chan, groups) * sizeof(float) +
         (size_t)kErfcN * sizeof(float4);
}

// Dynamic LDS of a workgroup (the erfc table is static LDS on top).
size_t thin_lds_bytes(int n_chan, int groups, bool selective) {
  return (size_t)kWavesPerBlock * thin_wave_floats(n_chan, groups, selective) * sizeof(float);
}
size_t thin_static_lds_bytes() { return (size_t)kErfcN * sizeof(float4); }
size_t thin_table_bytes() { return (size_t)kErfcN * sizeof(float4); }

template <bool GEN, int G, bool SEL>
static void launch_thin_g(const FwdParams& p, int sm, const float4* tab, hipStream_t st) {
  const int64_t waves = (p.n_pix + G - 1) / G;
  const int blocks = (int)((waves + kWavesPerBlock - 1) / kWavesPerBlock);
  hipLaunchKernelGGL((thin_kernel<GEN, G, SEL>), dim3(blocks), dim3(64 * kWavesPerBlock),
                     thin_lds_bytes(p.c.n_chan, G, SEL), st, p, sm, tab);
}

template <bool SEL>
static void launch_thin_s(const FwdParams& p, int sm, int groups, const float4* tab,
                          hipStream_t st) {
  if (p.c.general) {
    if (groups == 4) launch_thin_g<true, 4, SEL>(p, sm, tab, st);
    else if (groups == 2) launch_thin_g<true, 2, SEL>(p, sm, tab, st);
    else launch_thin_g<true, 1, SEL>(p, sm, tab, st);
  } else {
    if (groups == 4) launch_thin_g<false, 4, SEL>(p, sm, tab, st);
    else if (groups == 2) launch_thin_g<false, 2, SEL>(p, sm, tab, st);
    else launch_thin_g<false, 1, SEL>(p, sm, tab, st);
  }
}

void launch_erfc_table(void* table, void* stream) {
  hipLaunchKernelGGL(erfc_table_kernel, dim3((kErfcN + 255) / 256), dim3(256), 0,
                     (hipStream_t)stream, (float4*)table);
}

int launch_thin_adjoint(const AdjParams& p, bool smooth, int groups, void* table, void* stream) {
  if (p.c.n_chan < 1 || p.n_los < 1 || !table || (groups != 1 && groups != 2 && groups != 4))
    return (int)hipErrorInvalidValue;
  const hipStream_t st = (hipStream_t)stream;
  const float4* tab = (const float4*)table;
  launch_erfc_table(table, stream);
  const int sm = smooth ? 1 : 0;
  if (p.c.general) {
    if (groups == 4) launch_thin_adj_g<true, 4>(p, sm, tab, st);
    else if (groups == 2) launch_thin_adj_g<true, 2>(p, sm, tab, st);
    else launch_thin_adj_g<true, 1>(p, sm, tab, st);
  } else {
    if (groups == 4) launch_thin_adj_g<false, 4>(p, sm, tab, st);
    else if (groups == 2) launch_thin_adj_g<false, 2>(p, sm, tab, st);
    else launch_thin_adj_g<false, 1>(p, sm, tab, st);
  }
  return (int)hipGetLastError();
}

int launch_thin(const FwdParams& p, bool smooth, bool selective, int groups, void* table,
                void* stream) {
  if (p.c.n_chan < 1 || p.n_los < 1 || !table || (groups != 1 && groups != 2 && groups != 4) ||
      (selective && smooth))
    return (int)hipErrorInvalidValue;
  const hipStream_t st = (hipStream_t)stream;
  float4* tab = (float4*)table;
  launch_erfc_table(table, stream);
  const int sm = smooth ? 1 : 0;
  if (selective) launch_thin_s<true>(p, sm, groups, tab, st);
  else launch_thin_s<false>(p, sm, groups, tab, st);
  return (int)hipGetLastError();
}

}  // namespace iris
