// Forward march: one wavefront per sightline, far side to observer.
//
// Method (paper, "Transfer Solution: Formal and Smooth Integration of
// Optically Thick and Selectively Thin Transfer", formal step):
//   I_n = S_n + (I_{n-1} - S_n) e^{-tau_n}, tau = h (alpha_L phi + alpha_D),
// for the total intensity per channel and, with the dust terms only, for the
// continuum; both start from the background at the far side ("Transfer
// Solution: Overview").
//
// How it is organised on gfx950:
//  * Per-cell physics (LTE populations, optical depths, source functions,
//    channel window of the line) is computed lane-parallel for 64 cells at a
//    time from coalesced loads along the sightline (cell_setup.h).
//  * The continuum march and the dust optical-depth prefix P_n are
//    channel-independent: they are prefix sums over those 64 lanes in FP64.
//  * Per channel the kernel keeps the line excess over the continuum,
//    Delta_k = I_k - C, scaled by the dust transmission:
//        Psi_k = Delta_k e^{P - base}.
//    Where the line profile of a cell is negligible in channel k, Psi_k does
//    not change at all, so a cell only touches the channels inside its line
//    window (|v_k - v| <= x_w b). Inside the window the formal step becomes
//        Psi <- (Psi + G) e^{-tau_L} - G,  G = (C_{n-1} - J) e^{P_{n-1} - base}
//    (plus a term when the line and dust source functions differ).
//    Psi lives in LDS; a cell's window is covered by 64-lane passes starting
//    at its first in-window channel.
//  * `base` is rebased to the running P at the end of every 64-cell chunk
//    (and earlier if the dust depth inside a chunk would exceed kRebaseTau),
//    so the scale factors stay in FP32 range.
//  * Optional checkpoints of Delta and of (C, D, P) every K cells feed the
//    adjoint.

#include "cell_setup.h"

namespace iris {

template <typename FT, bool GEN>
__global__ __launch_bounds__(256) void fwd_kernel(const FwdParams P) {
  extern __shared__ float lds[];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t pix = (int64_t)blockIdx.x * kWavesPerBlock + wave;
  if (pix >= P.n_pix) return;  // whole wavefront
  const Folded& c = P.c;
  const int C = c.n_chan;
  float* psi = lds + (size_t)wave * P.lds_per_wave;
  for (int k = lane; k < C + 64; k += 64) psi[k] = 0.f;

  const FT* f[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) f[i] = P.f[i] ? (const FT*)P.f[i] + pix * P.pix_stride : nullptr;
  const bool has_td = P.f[4] != nullptr;
  const float lanef = (float)lane;
  const int K = P.ckpt_K;

  double Pabs = 0.0;     // dust optical depth up to the chunk start
  double Dcar = 0.0;     // dust-emission march at the chunk start
  double Bcar = c.J_bg;  // attenuated background at the chunk start
  double Ptrue = 0.0;    // dust column without the per-cell clamp (for [B])

  int s0 = 0;
  while (s0 < P.n_los) {
    const int s = s0 + lane;
    const bool valid = s < P.n_los;
    const CellIn in = load_cell<FT>(f, (int64_t)s * P.los_stride, valid, has_td);
    const CellOut o = cell_setup(c, in, valid, true);

    // Dust prefix inside the chunk, relative to base = P at the chunk start.
    const double kD = valid ? (double)o.kD : 0.0;
    const double Pin = wave_scan_incl(kD, lane);
    const double Pex = Pin - kD;
    // Cut the chunk before the first cell whose scaled state could overflow.
    const uint64_t over = __ballot(valid && Pin > (double)kRebaseTau);
    int nv = min(64, P.n_los - s0);
    if (over) nv = min(nv, __ffsll((unsigned long long)over) - 1);
    const bool act = lane < nv;

    const float eex = ex2((float)Pex * kLog2e);  // e^{P_{n-1} - base}
    const float ein = ex2((float)Pin * kLog2e);  // e^{P_n - base}
    // Dust emission entering the continuum, scaled: J_D (1 - e^{-kD}) e^{P_n - base}.
    const double w = act ? (double)(o.JD * -expm1f(-o.kD) * ein) : 0.0;
    const double Sin = wave_scan_incl(w, lane);
    const double Sex = Sin - w;
    const double Cprev = Dcar + Bcar + Sex;  // C_{n-1} e^{P_{n-1} - base}
    const float G = (float)(Cprev - (double)o.JD * (double)eex);
    const float Hs = GEN ? (float)((double)(o.JL - o.JD) * (double)eex) : 0.f;
    const float eK = GEN ? ex2(o.kD * kLog2e) : 0.f;

    // Checkpoint scalars, written by the lane that owns the cell.
    if (K && act && ((s & (K - 1)) == 0)) {
      const double emx = exp(-Pex);
      double* cs = P.ck_scal + ((int64_t)(s / K) * P.n_pix + pix) * 4;
      cs[0] = Cprev * emx;
      cs[1] = (Dcar + Sex) * emx;
      cs[2] = Pabs + Pex;
      if (s > 0) cs[3] = 0.0;
    }
    const float emPex = ex2(-(float)Pex * kLog2e);

    for (int i = 0; i < nv; ++i) {
      if (K && (((s0 + i) & (K - 1)) == 0)) {
        // Line excess entering cell s0+i: Delta = Psi e^{-(P_{n-1} - base)}.
        const float sc = bcast(emPex, i);
        float* dst = P.ck_state + ((int64_t)((s0 + i) / K) * P.n_pix + pix) * C;
        wave_order();
        for (int k = lane; k < C; k += 64) dst[k] = psi[k] * sc;
      }
      const int pk = bcast(o.packed, i);
      if (pk == 0) continue;
      const float g = bcast(G, i);
      const float A = bcast(o.A, i);
      const float R = bcast(o.R, i);
      const float lk = bcast(o.lk, i);
      const float df = bcast(o.df, i);
      float h = 0.f, kd = 0.f, ek = 0.f;
      if (GEN) {
        h = bcast(Hs, i);
        kd = bcast(o.kD, i);
        ek = bcast(eK, i);
      }
      const int kstart = pk & 0xFFFFFF;
      const int npass = pk >> 24;
      wave_order();
      for (int q = 0; q < npass; ++q) {
        const int k = kstart + 64 * q + lane;
        const float mf = lanef + (df + 64.f * q);
        const float t = fmaf(mf, A, -R);
        const float tl = ex2(fmaf(-t, t, lk));  // tau_L * log2(e)
        const float E = ex2(-tl);               // e^{-tau_L}
        const float ps = psi[k];
        float nw = fmaf(ps + g, E, -g);
        if (GEN) {
          const float tL = tl * kLn2;
          const float beta = tL * __builtin_amdgcn_rcpf(fmaxf(tL + kd, 1e-30f));
          nw = fmaf(beta * h, ek - E, nw);
        }
        psi[k] = nw;
      }
      wave_order();
    }

    // Unclamped dust column: only [B] (a pure transmission) resolves the
    // difference once a cell's dust depth exceeds kRebaseTau.
    Ptrue += wave_sum(act ? (double)c.kD * o.n : 0.0);

    // Chunk end: carry the continuum and rebase Psi to the new P.
    const double Pend = bcast(Pin, nv - 1);
    const double Send = bcast(Sin, nv - 1);
    const double fD = exp(-Pend);
    Dcar = (Dcar + Send) * fD;
    Bcar = Bcar * fD;
    Pabs += Pend;
    if (Pend > 0.0) {
      const float fs = (float)fD;
      wave_order();
      for (int k = lane; k < C; k += 64) psi[k] *= fs;
      wave_order();
    }
    s0 += nv;
  }

  // The adjoint needs the unclamped dust column of [B]: slot 3 of checkpoint 0.
  if (K && lane == 0) P.ck_scal[(int64_t)pix * 4 + 3] = Ptrue;

  // Outputs: [L] = Delta, [C] = D + B, [T] = [C] + [L].
  const double Bout = c.J_bg * exp(-Ptrue);
  const float Cf = (float)(Dcar + Bout), Df = (float)Dcar, Bf = (float)Bout;
  float* oT = P.out[0] ? P.out[0] + pix * C : nullptr;
  float* oC = P.out[1] ? P.out[1] + pix * C : nullptr;
  float* oD = P.out[2] ? P.out[2] + pix * C : nullptr;
  float* oL = P.out[3] ? P.out[3] + pix * C : nullptr;
  float* oB = P.out[4] ? P.out[4] + pix * C : nullptr;
  wave_order();
  for (int k = lane; k < C; k += 64) {
    const float d = psi[k];
    if (oT) oT[k] = Cf + d;
    if (oC) oC[k] = Cf;
    if (oD) oD[k] = Df;
    if (oL) oL[k] = d;
    if (oB) oB[k] = Bf;
  }
}

template <typename FT>
static int launch_t(const FwdParams& p, void* stream) {
  const int blocks = (p.n_pix + kWavesPerBlock - 1) / kWavesPerBlock;
  const size_t lds = (size_t)kWavesPerBlock * p.lds_per_wave * sizeof(float);
  if (p.c.general)
    hipLaunchKernelGGL((fwd_kernel<FT, true>), dim3(blocks), dim3(64 * kWavesPerBlock), lds,
                       (hipStream_t)stream, p);
  else
    hipLaunchKernelGGL((fwd_kernel<FT, false>), dim3(blocks), dim3(64 * kWavesPerBlock), lds,
                       (hipStream_t)stream, p);
  return (int)hipGetLastError();
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

}  // namespace iris
