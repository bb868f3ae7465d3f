// Forward march, far side to observer, G sightlines per wavefront.
//
// Method (paper, "Transfer Solution: Formal and Smooth Integration of
// Optically Thick and Selectively Thin Transfer", formal step):
//   I_n = S_n + (I_{n-1} - S_n) e^{-tau_n}, tau = h (alpha_L phi + alpha_D),
// for the total intensity per channel and, with the dust terms only, for the
// continuum; both start from the background at the far side ("Transfer
// Solution: Overview").
//
// How it is organised on gfx950:
//  * A wavefront holds G sightlines in groups of W = 64/G lanes. G is chosen
//    so that a cell's line window (about 2 x 4.6 Doppler widths of channels)
//    fits one W-lane pass, which keeps most lanes of a pass useful.
//  * Per-cell physics (LTE populations, optical depths, source functions,
//    channel window of the line) is computed lane-parallel for W cells of
//    each sightline at a time from coalesced loads (cell_setup.h). The
//    results go to a small LDS table that the march reads back as uniform
//    128-bit loads, one row per cell.
//  * The continuum march and the dust optical-depth prefix P_n are
//    channel-independent prefix sums over those lanes: FP32 inside a chunk
//    (at most W terms, relative to the chunk's base), FP64 across chunks. A
//    cell's entry prefix is read from its predecessor's lane, so entry and
//    exit scales agree bit for bit.
//  * Per channel the kernel keeps the line excess over the continuum,
//    Delta_k = I_k - C, scaled by the dust transmission:
//        Psi_k = Delta_k e^{P - base}.
//    Where the line profile of a cell is negligible in channel k, Psi_k does
//    not change, so a cell only touches the channels of its line window.
//    Inside the window the formal step becomes
//        Psi <- (Psi + G) e^{-tau_L} - G,  G = (C_{n-1} - J) e^{P_{n-1} - base}
//    (plus a term when the line and dust source functions differ). G is
//    accumulated as G_n = G_{n-1} + (J_{n-1} - J_n) e^{P_{n-1} - base}, the
//    scaled continuum deficit, which stays accurate when the dust is thick
//    and C and J agree to many digits.
//    Psi lives in LDS.
//  * `base` moves up to the running P only when the dust depth above it
//    passes kRebaseAt at a chunk end (a chunk is cut early where it would
//    pass kCutTau), so the scale factors stay in FP32 range and thin-dust
//    sightlines never rescale their state.
//  * Optional checkpoints of Delta and of (C, D, P) every K cells feed the
//    adjoint.

#include "cell_setup.h"
#include "epilogue.h"

namespace iris {

// Fields of the per-cell LDS table. The table of a sightline is field-major
// (field f of cell i at f * W + i): each lane writes its cell's fields to
// consecutive words, and the march reads one field of four cells at once.
// The profile argument of lane sl in pass q is t = (sl + W q) A + c0.
enum : int { kRowG = 0, kRowA, kRowC0, kRowLk, kRowKstart, kRowPacked, kRowEmPex,
             kRowH, kRowKd, kRowEk };
// Fields per cell: the source-function split (GEN) adds three.
__host__ __device__ constexpr int fwd_row_fields(bool general) { return general ? 10 : 7; }

// Scaled-state range of the march: a chunk is cut before the first cell
// whose dust depth above the current base exceeds kCutTau, and the base is
// moved up to the running depth at a chunk end once that exceeds
// kRebaseAt. With per-cell depths clamped at kRebaseTau,
// kRebaseAt + kRebaseTau <= kCutTau guarantees progress, and e^{kCutTau}
// (6e27) times a W-lane sum of source functions up to 1e8 K stays in FP32.
constexpr float kCutTau = 64.f;
constexpr float kRebaseAt = 4.f;
static_assert(kRebaseAt + kRebaseTau <= kCutTau, "a chunk must take its first cell");

// Floats of LDS per sightline for the channel state (multiple of 4, >= C + W).
__host__ __device__ inline int fwd_state_stride(int n_chan, int groups) {
  return (n_chan + 64 / groups + 3) & ~3;
}
// The cell tables of the G sightlines of a wavefront start kTblSkew floats
// apart beyond their length, so that the G rows read together (one per
// sightline, each broadcast to its lanes) sit in different LDS banks.
constexpr int kTblSkew = 4;
// Floats of LDS per wavefront: G channel states plus the 64-row cell table.
__host__ __device__ inline int fwd_wave_floats(int n_chan, int groups, bool general) {
  return groups * fwd_state_stride(n_chan, groups) + 64 * fwd_row_fields(general) +
         groups * kTblSkew;
}

// Field loader of sightline `pix` for a compile-time or run-time storage type.
template <typename L>
struct LoaderMaker;
template <typename FT>
struct LoaderMaker<Loader<FT>> {
  static __device__ __forceinline__ Loader<FT> make(const FwdParams& P, int64_t pix) {
    return Loader<FT>(P.f, P.at.base(pix));
  }
};
template <>
struct LoaderMaker<DynLoader> {
  static __device__ __forceinline__ DynLoader make(const FwdParams& P, int64_t pix) {
    return DynLoader(P.f, P.at.base(pix), P.dtype);
  }
};

// March of the G sightlines pix0 .. pix0+G-1 by one wavefront. `lw` is the
// wavefront's LDS (fwd_wave_floats floats, 16-byte aligned). CKPT: write the
// adjoint's checkpoints every P.ckpt_K cells.
template <typename LoaderT, bool GEN, int G, bool CKPT>
__device__ __forceinline__ void fwd_wave(const FwdParams& P, int64_t pix0, float* lw) {
  constexpr int W = 64 / G;
  constexpr int TF = fwd_row_fields(GEN);
  const int lane = threadIdx.x & 63;
  const int sub = lane / W, sl = lane % W;
  const int64_t pix = pix0 + sub;
  const bool live = pix < P.n_pix;
  const Folded& c = P.c;
  const int C = c.n_chan;
  const int stride = fwd_state_stride(C, G);
  float* psi = lw + sub * stride;
  float* tbl = lw + G * stride + sub * (W * TF + kTblSkew);
  for (int k = sl; k < C + W; k += W) psi[k] = 0.f;

  const int64_t pixc = live ? pix : P.n_pix - 1;  // address of a dead group is never loaded
  const LoaderT load = LoaderMaker<LoaderT>::make(P, pixc);
  const float slf = (float)sl;
  const int K = CKPT ? P.ckpt_K : 0;

  // State relative to `base`, the dust depth the scaled quantities refer to
  // (Psi = Delta e^{P - base}): Pabs = base (FP64), Pb = depth at the chunk
  // start above base; scaled carries at the chunk start (FP64): dust
  // emission D, background attenuated by the clamped column (constant
  // between rebasings), and the continuum deficit G = (C - J_prev); J of the
  // cell before the chunk; the unclamped column for [B]. Before the first
  // cell, C = J_bg and J_{-1} := J_bg.
  double Pabs = 0.0, Dcar = 0.0, Bsc = c.J_bg, Ptrue = 0.0;
  float Pb = 0.f;
  float Jcar = (float)c.J_bg;
  double Gcar = c.J_bg - (double)Jcar;

  // The fields of the next chunk are loaded while this chunk marches, for a
  // chunk that starts where this one would end uncut (s0 + W); a chunk cut
  // short by the dust depth reloads its successor.
  int s0 = 0;
  int s_pre = 0;
  typename LoaderT::Raw pre = load.fetch((int64_t)sl * P.at.los, live && sl < P.n_los);
  while (s0 < P.n_los) {
    const int s = s0 + sl;
    const bool valid = live && s < P.n_los;
    const CellIn in =
        load.decode(s0 == s_pre ? pre : load.fetch((int64_t)s * P.at.los, valid), valid);
    const CellOut o = cell_setup<GEN>(c, in, valid, true);

    // Dust prefix: FP32 scan inside the chunk (at most W terms) on top of Pb.
    const float kD = valid ? o.kD : 0.f;
    const float Prel = group_scan_dpp<W>(kD);
    const float Pin = Pb + Prel;
    // The entry scale of a cell is its predecessor's exit scale, bit for bit.
    const float Pup = lane_up1(Pin);
    const float Pex = sl == 0 ? Pb : Pup;
    const uint64_t over = __ballot(valid && Pin > kCutTau);
    int nv = min(W, P.n_los - s0);
    if (over) {
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const uint64_t m = W == 64 ? over : (over >> (g * W)) & ((1ull << (W & 63)) - 1);
        if (m) nv = min(nv, __ffsll((unsigned long long)m) - 1);
      }
    }
    nv = __builtin_amdgcn_readfirstlane(nv);  // uniform: lets the march loops unroll
    const bool act = sl < nv;

    const float eex = ex2(Pex * kLog2e);  // e^{P_{n-1} - base}
    const float ein = ex2(Pin * kLog2e);  // e^{P_n - base}
    // Dust emission entering the continuum, scaled: J_D (1 - e^{-kD}) e^{P_n - base}.
    const float om = __any(act && o.kD >= 0.25f) ? one_minus_exp_neg(o.kD)
                                                 : one_minus_exp_neg_small(o.kD);
    const float w = act ? o.JD * om * ein : 0.f;
    const float Sin = group_scan_dpp<W>(w);
    const float Sex = Sin - w;
    // Line source term G_n = (C_{n-1} - J_n) e^{P_{n-1} - base} by its own
    // recursion G_n = G_{n-1} + (J_{n-1} - J_n) e^{P_{n-1} - base} (the
    // deficit after cell n-1 equals G_{n-1}), so that G is never the small
    // difference of two terms of size J e^{P}.
    const float Jup = __int_as_float(__builtin_amdgcn_update_dpp(
        0, __float_as_int(o.JD), kDppWaveShr1, 0xF, 0xF, false));
    const float tJ = act ? ((sl == 0 ? Jcar : Jup) - o.JD) * eex : 0.f;
    const float Gsc = group_scan_dpp<W>(tJ);
    const float Gn = (float)(Gcar + (double)Gsc);

    if (CKPT && act && valid && ((s & (K - 1)) == 0)) {
      const double emx = exp(-(double)Pex);
      const double Cprev = Dcar + Bsc + (double)Sex;  // C_{n-1} e^{P_{n-1} - base}
      double* cs = P.ck_scal + ((int64_t)(s / K) * P.n_pix + pix) * kCkScal;
      gstore(cs + kCkC, Cprev * emx);
      gstore(cs + kCkD, (Dcar + (double)Sex) * emx);
      gstore(cs + kCkP, Pabs + (double)Pex);
      gstore(cs + kCkA, (Gcar + (double)Gsc) * emx);
      gstore(cs + kCkB, Bsc * emx);
    }

    // Table row of this lane's cell. A cell without a line gets g = 0 and
    // an optical-depth exponent that flushes to zero, so that a pass over it
    // leaves the state bit-identical.
    const int np = act ? window_passes(o.nwin, W) : 0;
    // The lean march needs one pass per cell (the general loop's pass bounds
    // across groups are not needed then).
    const bool lean = !__any(np > 1);

    {
      int packed = o.kstart | (np << 13);
      if (!lean) {
        const int npmax = cross_group_max<W>(np);
        const int npmin = cross_group_min<W>(np);
        packed |= (npmax << 21) | ((npmin == npmax) << 29);
      }
      float* r = tbl + sl;
      r[kRowG * W] = np ? Gn : 0.f;
      r[kRowA * W] = o.A;
      r[kRowC0 * W] = o.c0;
      r[kRowLk * W] = np ? o.lk : -256.f;
      r[kRowKstart * W] = __int_as_float(np ? o.kstart : 0);
      r[kRowPacked * W] = __int_as_float(packed);
      if (CKPT) r[kRowEmPex * W] = ex2(-Pex * kLog2e);
      if (GEN) {
        r[kRowH * W] = (float)((double)(o.JL - o.JD) * (double)eex);
        r[kRowKd * W] = o.kD;
        r[kRowEk * W] = ex2(o.kD * kLog2e);
      }
    }
    wave_order();

    s_pre = s0 + W;
    pre = load.fetch((int64_t)(s_pre + sl) * P.at.los, live && s_pre + sl < P.n_los);

    // One channel's step: the formal step of the shared source function, and
    // with separate line and dust source functions (GEN) the term of the
    // line source's own part, beta h (e^{-kD} - e^{-tau_L}) scaled, beta the
    // line's share of the total depth.
    auto gen_step = [&](float ps, float g, float x, float h, float kd, float ek) {
      float nw = formal_line_step(ps, g, x);
      if (GEN) {
        const float E = ex2(-x);  // e^{-tau_L}
        const float tL = x * kLn2;
        const float beta = tL * __builtin_amdgcn_rcpf(fmaxf(tL + kd, 1e-30f));
        nw = fmaf(beta * h, ek - E, nw);
      }
      return nw;
    };
    if (lean) {
      // Lean march: every window fits one W-lane pass. Per cell and lane:
      // profile argument, two exponentials (the line depth and the step,
      // whose series form serves below x = kSeriesX), one LDS
      // read-modify-write. Four cells at a time: their table rows and
      // exponentials do not depend on the state, so they are computed ahead of
      // the four updates.
      // Checkpoints (line excess entering cell s0 + i, for the adjoint) are
      // written before the cell that starts a checkpoint interval; a group of
      // four with such a cell after its first goes one cell at a time.
      auto checkpoint = [&](int i) {
        if (CKPT && (((s0 + i) & (K - 1)) == 0) && live) {
          float* dst = P.ck_state + ((int64_t)((s0 + i) / K) * P.n_pix + pix) * C;
          const float emp = tbl[kRowEmPex * W + i];
          for (int k = sl; k < C; k += W) gstore(dst + k, psi[k] * emp);
          wave_order();
        }
      };
      int i = 0;
      for (; i + 4 <= nv; i += 4) {
        if (CKPT) {
          if (((s0 + i) & (K - 1)) > K - 4) break;
          checkpoint(i);
        }
        const float4 g = *(const float4*)(tbl + kRowG * W + i);
        const float4 A = *(const float4*)(tbl + kRowA * W + i);
        const float4 c0 = *(const float4*)(tbl + kRowC0 * W + i);
        const float4 lk = *(const float4*)(tbl + kRowLk * W + i);
        const int4 off = *(const int4*)(tbl + kRowKstart * W + i);
        const float x0 = ex2(fmaf(-fmaf(slf, A.x, c0.x), fmaf(slf, A.x, c0.x), lk.x));
        const float x1 = ex2(fmaf(-fmaf(slf, A.y, c0.y), fmaf(slf, A.y, c0.y), lk.y));
        const float x2 = ex2(fmaf(-fmaf(slf, A.z, c0.z), fmaf(slf, A.z, c0.z), lk.z));
        const float x3 = ex2(fmaf(-fmaf(slf, A.w, c0.w), fmaf(slf, A.w, c0.w), lk.w));
        float4 h = make_float4(0.f, 0.f, 0.f, 0.f), kd = h, ek = h;
        if (GEN) {
          h = *(const float4*)(tbl + kRowH * W + i);
          kd = *(const float4*)(tbl + kRowKd * W + i);
          ek = *(const float4*)(tbl + kRowEk * W + i);
        }
        float* p0 = psi + off.x + sl;
        *p0 = gen_step(*p0, g.x, x0, h.x, kd.x, ek.x);
        wave_order();
        float* p1 = psi + off.y + sl;
        *p1 = gen_step(*p1, g.y, x1, h.y, kd.y, ek.y);
        wave_order();
        float* p2 = psi + off.z + sl;
        *p2 = gen_step(*p2, g.z, x2, h.z, kd.z, ek.z);
        wave_order();
        float* p3 = psi + off.w + sl;
        *p3 = gen_step(*p3, g.w, x3, h.w, kd.w, ek.w);
        wave_order();
      }
      for (; i < nv; ++i) {
        checkpoint(i);
        const float g = tbl[kRowG * W + i], A = tbl[kRowA * W + i];
        const float c0 = tbl[kRowC0 * W + i], lk = tbl[kRowLk * W + i];
        const float t = fmaf(slf, A, c0);
        float* pp = psi + __float_as_int(tbl[kRowKstart * W + i]) + sl;
        *pp = GEN ? gen_step(*pp, g, ex2(fmaf(-t, t, lk)), tbl[kRowH * W + i],
                             tbl[kRowKd * W + i], tbl[kRowEk * W + i])
                  : gen_step(*pp, g, ex2(fmaf(-t, t, lk)), 0.f, 0.f, 0.f);
        wave_order();
      }
    } else {
      for (int i = 0; i < nv; ++i) {
        const float* r = tbl + i;
        if (CKPT && (((s0 + i) & (K - 1)) == 0) && live) {
          // Line excess entering cell s0+i: Delta = Psi e^{-(P_{n-1} - base)}.
          float* dst = P.ck_state + ((int64_t)((s0 + i) / K) * P.n_pix + pix) * C;
          const float emp = r[kRowEmPex * W];
          for (int k = sl; k < C; k += W) gstore(dst + k, psi[k] * emp);
        }
        const int pk = __float_as_int(r[kRowPacked * W]);
        const int pku = __builtin_amdgcn_readfirstlane(pk);
        const int npm = (pku >> 21) & 0xFF;
        if (npm == 0) continue;
        const int npo = (pk >> 13) & 0xFF;
        const float g = r[kRowG * W], A = r[kRowA * W], c0 = r[kRowC0 * W], lk = r[kRowLk * W];
        float h = 0.f, kd = 0.f, ek = 0.f;
        if (GEN) {
          h = r[kRowH * W];
          kd = r[kRowKd * W];
          ek = r[kRowEk * W];
        }
        float* pp = psi + (pk & 0x1FFF) + sl;
        for (int q = 0; q < npm; ++q) {
          if (q < npo) {
            const float t = fmaf(slf + (float)(W * q), A, c0);
            const float tl = ex2(fmaf(-t, t, lk));  // tau_L * log2(e)
            pp[W * q] = gen_step(pp[W * q], g, tl, h, kd, ek);
          }
        }
        wave_order();
      }
    }

    // Chunk end. The unclamped dust column (only [B], a pure transmission,
    // resolves depths beyond the clamp) grows by the chunk's depth, plus
    // the clamped-off excess where a cell was clamped.
    const int last = sub * W + nv - 1;
    const float Pend = __shfl(Pin, last, 64);
    Ptrue += (double)__shfl(Prel, last, 64);
    const bool clamped = act && c.kD * (float)o.n > kRebaseTau;
    if (__any(clamped)) Ptrue += (double)group_sum<W>(clamped ? c.kD * (float)o.n - o.kD : 0.f);
    Dcar += (double)__shfl(Sin, last, 64);
    Gcar += (double)__shfl(Gsc, last, 64);
    Jcar = __shfl(o.JD, last, 64);
    Pb = Pend;
    if (Pb > kRebaseAt) {
      // Move the base up to the running depth (per group).
      const double f = exp(-(double)Pb);
      Dcar *= f;
      Bsc *= f;
      Gcar *= f;
      Pabs += (double)Pb;
      Pb = 0.f;
      const float fs = (float)f;
      for (int k = sl; k < C; k += W) psi[k] *= fs;
    }
    wave_order();
    s0 += nv;
  }

  if (!live) return;
  // The adjoint needs the unclamped dust column of [B]: slot 3 of checkpoint 0.
  if (CKPT && sl == 0) gstore(P.ck_scal + pix * kCkScal + kCkPtrue, Ptrue);

  // Outputs, unscaled by e^{-(P_N - base)}: [L] = Delta, [C] = D + B,
  // [T] = [C] + [L].
  const double fend = exp(-(double)Pb);
  const double Bout = c.J_bg * exp(-Ptrue);
  const double Dout = Dcar * fend;
  write_outputs<W>(c, P.out, pix, psi, sl, (float)fend * c.out_scale, (float)(Dout + Bout), Dout,
                   Bout);
}

template <typename FT, bool GEN, int G, bool CKPT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void fwd_kernel(
    const FwdParams P) {
  extern __shared__ float lds[];
  const int wave = threadIdx.x >> 6;
  const int tile = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  const int64_t pix0 = ((int64_t)tile * kWavesPerBlock + wave) * G;
  if (pix0 >= P.n_pix) return;  // whole wavefront
  fwd_wave<Loader<FT>, GEN, G, CKPT>(P, pix0,
                                      lds + (size_t)wave * fwd_wave_floats(P.c.n_chan, G, GEN));
}

int fwd_state_floats(int n_chan, int groups) { return fwd_state_stride(n_chan, groups); }

size_t fwd_lds_bytes(int n_chan, int groups, bool general) {
  return (size_t)kWavesPerBlock * fwd_wave_floats(n_chan, groups, general) * sizeof(float);
}

template <typename FT, int G>
static int launch_g(const FwdParams& p, void* stream) {
  const int64_t waves = (p.n_pix + G - 1) / G;
  const int blocks = (int)((waves + kWavesPerBlock - 1) / kWavesPerBlock);
  const size_t lds = fwd_lds_bytes(p.c.n_chan, G, p.c.general != 0);
  const dim3 grid(blocks), block(64 * kWavesPerBlock);
  const hipStream_t st = (hipStream_t)stream;
  const bool ck = p.ckpt_K > 0;
  if (p.c.general) {
    if (ck) hipLaunchKernelGGL((fwd_kernel<FT, true, G, true>), grid, block, lds, st, p);
    else hipLaunchKernelGGL((fwd_kernel<FT, true, G, false>), grid, block, lds, st, p);
  } else {
    if (ck) hipLaunchKernelGGL((fwd_kernel<FT, false, G, true>), grid, block, lds, st, p);
    else hipLaunchKernelGGL((fwd_kernel<FT, false, G, false>), grid, block, lds, st, p);
  }
  return (int)hipGetLastError();
}

template <typename FT>
static int launch_t(const FwdParams& p, void* stream) {
  switch (p.groups) {
    case 1: return launch_g<FT, 1>(p, stream);
    case 2: return launch_g<FT, 2>(p, stream);
    case 4: return launch_g<FT, 4>(p, stream);
  }
  return (int)hipErrorInvalidValue;
}

int launch_forward(iris_dtype dt, const FwdParams& p, void* stream) {
  switch (dt) {
    case IRIS_F64: return launch_t<double>(p, stream);
    case IRIS_F32: return launch_t<float>(p, stream);
    case IRIS_BF16: return launch_t<bf16_t>(p, stream);
    case IRIS_F16: return launch_t<_Float16>(p, stream);
  }
  return (int)hipErrorInvalidValue;
}

// --- batched persistent launch -------------------------------------------------

// One wavefront per work item (a cube and its G sightlines), taken from the
// sliced queue (ItemClaim) until it is empty. Storage type, G and the
// source-function variant are taken per cube at run time.
template <int G, bool CKPT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void plan_fwd_kernel(
    const PlanFwdParams Q) {
  extern __shared__ float lds[];
  const int wave = threadIdx.x >> 6;
  float* lw = lds + (size_t)wave * Q.wave_floats;
  ItemClaim claim(kWavesPerBlock, wave, Q.static_rounds != 0);
  while (true) {
    const int idx = claim.next(Q.slice_begin, Q.counter);
    if (idx < 0) break;
    // The previous item's last LDS reads used another lane mapping.
    wave_order();
    // Item and cube parameters are uniform: scalar loads into registers.
    const WorkItem wi = Q.items[idx];
    const int cube = __builtin_amdgcn_readfirstlane(wi.cube);
    const int64_t pix0 = __builtin_amdgcn_readfirstlane(wi.pix0);
    // Read-only for the whole launch: through the constant address space the
    // parameters load with scalar loads and may be reloaded instead of kept.
    const FwdParams& P =
        *(const FwdParams*)((const __attribute__((address_space(4))) FwdParams*)Q.cubes + cube);
    if (P.c.general)
      fwd_wave<DynLoader, true, G, CKPT>(P, pix0, lw);
    else
      fwd_wave<DynLoader, false, G, CKPT>(P, pix0, lw);
  }
}

template <int G, bool CKPT>
static int launch_plan_t(const PlanFwdParams& q, int blocks, void* stream) {
  const size_t lds = (size_t)kWavesPerBlock * q.wave_floats * sizeof(float);
  hipLaunchKernelGGL((plan_fwd_kernel<G, CKPT>), dim3(blocks), dim3(64 * kWavesPerBlock), lds,
                     (hipStream_t)stream, q);
  return (int)hipGetLastError();
}

int launch_plan_forward(const PlanFwdParams& q, int groups, bool ckpt, int blocks, void* stream) {
  switch (groups * 2 + (ckpt ? 1 : 0)) {
    case 2: return launch_plan_t<1, false>(q, blocks, stream);
    case 3: return launch_plan_t<1, true>(q, blocks, stream);
    case 4: return launch_plan_t<2, false>(q, blocks, stream);
    case 5: return launch_plan_t<2, true>(q, blocks, stream);
    case 8: return launch_plan_t<4, false>(q, blocks, stream);
    case 9: return launch_plan_t<4, true>(q, blocks, stream);
  }
  return (int)hipErrorInvalidValue;
}

template <int G, bool CKPT>
static int occupancy_t(int wave_floats) {
  int nb = 0;
  const size_t lds = (size_t)kWavesPerBlock * wave_floats * sizeof(float);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, plan_fwd_kernel<G, CKPT>,
                                                   64 * kWavesPerBlock, lds) != hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

int plan_forward_occupancy(int wave_floats, int groups, bool ckpt) {
  switch (groups * 2 + (ckpt ? 1 : 0)) {
    case 2: return occupancy_t<1, false>(wave_floats);
    case 3: return occupancy_t<1, true>(wave_floats);
    case 4: return occupancy_t<2, false>(wave_floats);
    case 5: return occupancy_t<2, true>(wave_floats);
    case 8: return occupancy_t<4, false>(wave_floats);
    case 9: return occupancy_t<4, true>(wave_floats);
  }
  return 1;
}

}  // namespace iris
