// Adjoint (reverse mode) of the forward march: gradient of
//   Loss = sum_k gT_k [T]_k + gC_k [C] + gD_k [D] + gL_k [L]_k + gB_k [B]
// with respect to the stored per-cell fields (ln n_H2, T_kin, v_los, X, and
// T_dust where it is given).
// The paper makes its pipeline differentiable through autograd ("Synthetic
// Observation Implementation and Algorithms", differentiability modes); here
// the reverse pass is written by hand.
//
// Base-free recurrences, per sightline, reversing cell n = N-1 .. 0
// (Delta = line excess I - C, a_n = C_{n-1} - J_n, e_n = e^{-kD_n},
// E_nk = e^{-tau_L,nk}; forward in-window step
// Delta_n = e_n [(Delta_{n-1} + a_n) E - a_n], out of window Delta_n = e_n Delta_{n-1}):
//   lambda_{n-1,k} = lambda_{n,k} e_n E_nk
//   abar_n        = sum_k lambda_{n,k} e_n (E_nk - 1)           (window only)
//   taubar_{n,k}  = -E_nk lambda_{n,k} e_n (Delta_{n-1,k} + a_n)  (window only)
//   Q_n           = sum_k lambda_{n,k} Delta_{n,k} (all channels); out of the
//                   window lambda*Delta is invariant, so Q_{n-1} = Q_n - a_n abar_n
//   kDbar_n       = -Q_n - e_n [gamma_n (C_{n-1} - J_n) + delta_n (D_{n-1} - J_n)]
//   Jbar_n        = (gamma_n + delta_n)(1 - e_n) - abar_n
//   gamma_{n-1}   = gamma_n e_n + abar_n,   delta_{n-1} = delta_n e_n
// with gamma = dLoss/dC, delta = dLoss/dD. In the kernel lambda is scaled like
// Psi: lambda~ = lambda e^{-(P - base)}, which is invariant outside a cell's
// window; then lambda~_{n-1} = lambda~_n E, abar_n = e^{P_{n-1}-base} sum lambda~ (E-1),
// and taubar = -E lambda~ (Psi_{n-1} + G_n) with the forward's G_n. The base
// of a cell is the segment start's depth plus a multiple of kAdjBaseStep
// below the cell's entry depth; where it moves up between two cells, Psi and
// lambda~ are rescaled by the same factor (forward in the recompute, backward
// in the reverse pass), so that every scaled quantity stays in FP32 range
// however thick the dust of a segment.
//
// With separate line and dust source functions (a dust temperature field, or
// the literal level energies) J above is the dust's J_D, the line source
// function is J_L = J_D + H_n, and a window channel's step gains the term
// beta H (1 - e_n E), beta = tau_L / (tau_L + kD) the line's share of the
// depth. lambda's recurrence is unchanged; per cell two more window sums,
//   Hbar_n  = sum_k lambda beta (1 - e_n E)                       (dLoss/dH_n)
//   kDbar_n gains H sum_k lambda [beta - tau_L (1 - e_n E) / (tau_L + kD)^2],
// taubar gains lambda H [kD (1 - e_n E) / (tau_L + kD)^2 + beta e_n E], Q's
// recurrence subtracts H_n Hbar_n too, and the source functions get
// J_Lbar = Hbar_n, J_Dbar = Jbar_n - Hbar_n. In scaled form with
// h = H e^{P_{n-1} - base} (the forward's own term), lambda H = lambda~ h e^{kD}.
//
// The forward stores Delta and (C, D, P, a = C - J, B) every K cells. Each
// K-cell segment is recomputed from its checkpoint with the pre-update Psi of
// every window pass kept on an LDS tape; a segment whose passes exceed the
// tape is split into sub-segments, each recomputed from the checkpoint (the
// last first). The deficit a_n follows the forward's recursion
// a_n e^{P_{n-1}} = a_{n-1} e^{P_{n-2}} + (J_{n-1} - J_n) e^{P_{n-1}} from the
// checkpointed a, so it never comes from a cancellation of C and J.
//
// A wavefront reverses G sightlines at once, W = 64/G lanes each: the per-cell
// quantities of a segment go to an LDS table per sightline, the window sums
// are group reductions, and the FP64 recurrences run group-uniform in every
// lane. Per-cell window sums are FP32; recurrences and gradients are FP64.

#include "cell_partials.h"
#include "cell_setup.h"

namespace iris {

// Floats per cell of a segment's tables (multiples of 4 for 16-byte rows).
constexpr int kAdjRow = 12;
constexpr int kAdjRes = 12;
// Row: profile (G, A, c0, lk), (1/(kappa_L log2 e), window, 1 - e^{-kD},
// e^{P_{n-1} - base}), deficit a_n (FP64), background B_{n-1}, and the factor
// e^{-(base_n - base_{n-1})} that moves the scaled state to the cell's base
// (1 where the base does not move).
enum : int { kArG = 0, kArA, kArC0, kArLk, kArEmlk, kArPacked, kArOmen, kArEPex, kArAn, kArBm = 10,
             kArRs = 11 };
// Inside a segment the scaled quantities of cell n refer to a base that is the
// dust depth above the segment start rounded down to a multiple of
// kAdjBaseStep, so that P - base stays below kAdjBaseStep + kRebaseTau (64,
// the forward march's range) however thick the segment. Segments thinner than
// kAdjBaseStep (every segment of the usual workloads) never move their base.
constexpr double kAdjBaseStep = 4.0;
// With separate line and dust source functions a row has four more floats:
// h (the line source function's excess over the dust's, scaled like G), kD
// and e^{kD}.
constexpr int kAdjRowGen = 16;
enum : int { kArH = 12, kArKd, kArEk };
// Result: the window sums of the reverse pass (lambda (E - 1), the
// taubar-weighted profile moments and, with separate source functions, the
// h and kD sums), then the cell's stored fields (ln n, T, X, T_dust) for the
// chain rule.
enum : int { kAsS1 = 0, kAsS3, kAsS4, kAsS5, kAsSH, kAsSK, kAsLnn = 8, kAsT, kAsX, kAsTd };

// 1 - 2^{-x} for x >= 0, with the formal step's series below kSeriesX.
__device__ __forceinline__ float one_minus_ex2_neg(float x) {
  float q = fmaf(x, 0.0555041087f, -0.2402265070f);  // (ln 2)^3/6, -(ln 2)^2/2
  q = fmaf(x, q, 0.6931471806f);                      // ln 2
  return x < kSeriesX ? x * q : 1.f - ex2(-x);
}

// The forward's step with separate source functions (x = tau_L log2 e): the
// formal step of the dust's source function plus beta h (e^{kD} - e^{-tau_L}),
// beta = tau_L / (tau_L + kD).
__device__ __forceinline__ float gen_formal_step(float ps, float g, float x, float h, float kd,
                                                 float ek) {
  const float nw = formal_line_step(ps, g, x);
  const float E = ex2(-x);
  const float tL = x * kLn2;
  const float beta = tL * __builtin_amdgcn_rcpf(fmaxf(tL + kd, 1e-30f));
  return fmaf(beta * h, ek - E, nw);
}

// Terms of one window channel's reverse step with separate source functions,
// per unit lambda~ (x = tau_L log2 e, E = e^{-tau_L}, s = tau_L + kD,
// q = (1 - e^{-s}) / s):
//   tb, taubar's extra part per unit h:  (1 - beta) e^{kD} q + beta E;
//   sh, the h sum:                        beta e^{kD} (1 - e^{-s});
//   sk, the kD sum:                       beta e^{kD} (1 - q).
// 1 - e^{-s} and 1 - q come from series at small s, so that neither is the
// small difference of two numbers near 1.
struct GenRev {
  float tb, sh, sk;
};
__device__ __forceinline__ GenRev gen_reverse(float x, float E, float kd, float ek) {
  const float tL = x * kLn2;
  const float sd = tL + kd;
  const float r = __builtin_amdgcn_rcpf(fmaxf(sd, 1e-30f));
  const float om = one_minus_ex2_neg(fmaf(kd, kLog2e, x));  // 1 - e^{-s}
  const float q = om * r;
  // 1 - q = s/2 - s^2/6 + s^3/24 - s^4/120 + s^5/720 - s^6/5040 ... below s = 1/2
  // (the first omitted term is under 1e-6 of the sum there).
  float p = fmaf(sd, -1.f / 5040.f, 1.f / 720.f);
  p = fmaf(sd, p, -1.f / 120.f);
  p = fmaf(sd, p, 1.f / 24.f);
  p = fmaf(sd, p, -1.f / 6.f);
  p = fmaf(sd, p, 0.5f);
  const float omq = sd < 0.5f ? sd * p : 1.f - q;
  const float beta = tL * r, bek = beta * ek;
  GenRev g;
  g.tb = fmaf(kd * r * q, ek, beta * E);
  g.sh = bek * om;
  g.sk = bek * omq;
  return g;
}

template <typename L>
struct AdjLoaderMaker;
template <typename FT>
struct AdjLoaderMaker<Loader<FT>> {
  static __device__ __forceinline__ Loader<FT> make(const AdjParams& P, int64_t pix) {
    return Loader<FT>(P.f, P.at.base(pix));
  }
};
template <>
struct AdjLoaderMaker<DynLoader> {
  static __device__ __forceinline__ DynLoader make(const AdjParams& P, int64_t pix) {
    return DynLoader(P.f, P.at.base(pix), P.dtype);
  }
};

// Reverse march of sightlines pix0 .. pix0+G-1 by one wavefront; `lw` is its
// LDS (adj_wave_floats floats, four more per cell of a segment with separate
// source functions).
template <typename LoaderT, int G, bool GEN>
__device__ __forceinline__ void adj_wave(const AdjParams& P, int64_t pix0, float* lw) {
  constexpr int W = 64 / G;
  constexpr int RW = GEN ? kAdjRowGen : kAdjRow;  // floats per row
  const int lane = threadIdx.x & 63;
  const int sub = lane / W, sl = lane % W;
  const int64_t pix = pix0 + sub;
  const bool live = pix < P.n_pix;
  const int64_t pixc = live ? pix : P.n_pix - 1;  // a dead group reads valid memory only
  const Folded& c = P.c;
  const int C = c.n_chan;
  const int K = P.ckpt_K;
  const int TP = P.tape_passes;
  const int CP = P.chan_stride;  // >= C + W, multiple of 4
  float* psi = lw + sub * CP;
  float* lam = lw + (G + sub) * CP;
  float* tape = lw + 2 * G * CP + sub * TP * W;
  float* rows = lw + 2 * G * CP + G * TP * W + sub * (K * RW + kAdjSkew);
  float* res =
      lw + 2 * G * CP + G * TP * W + G * (K * RW + kAdjSkew) + sub * (K * kAdjRes + kAdjSkew);
  const float slf = (float)sl;
  const LoaderT load = AdjLoaderMaker<LoaderT>::make(P, pixc);
  const bool has_td = GEN && P.f[4] != nullptr;  // a dust temperature field

  // Seeds: lambda_N = gT + gL; gamma_N = sum (gT + gC); delta_N = sum gD;
  // sum gB for the background, each times the output units per
  // Rayleigh-Jeans kelvin (the march runs in kelvin). A dead group gets zero
  // cotangents.
  double gam = 0.0, del = 0.0, bsum = 0.0;
  const int CO = c.n_out;  // channels of the cotangent rows
  const float* gT = live && P.cot[0] ? P.cot[0] + pix * CO : nullptr;
  const float* gC = live && P.cot[1] ? P.cot[1] + pix * CO : nullptr;
  const float* gD = live && P.cot[2] ? P.cot[2] + pix * CO : nullptr;
  const float* gL = live && P.cot[3] ? P.cot[3] + pix * CO : nullptr;
  const float* gB = live && P.cot[4] ? P.cot[4] + pix * CO : nullptr;
  if (c.simpson_f > 0) {
    // Velocity subsampling: the channel averages are linear in the marched
    // velocities, so a marched velocity's seed is the weighted sum of the
    // cotangents of the channels it belongs to (a shared edge belongs to
    // two); the continuum sums run over the channels.
    for (int k = sl; k < CO; k += W) {
      const float vT = gT ? gload(gT + k) : 0.f, vC = gC ? gload(gC + k) : 0.f;
      gam += (double)vT + (double)vC;
      del += gD ? (double)gload(gD + k) : 0.0;
      bsum += gB ? (double)gload(gB + k) : 0.0;
    }
    const int f2 = 2 * c.simpson_f;
    const float w1 = 1.f / (3.f * (float)f2), w4 = 4.f * w1, w2 = 2.f * w1;
    auto lin = [&](int k) {
      return (gT ? gload(gT + k) : 0.f) + (gL ? gload(gL + k) : 0.f);
    };
    for (int j = sl; j < CP; j += W) {
      float v = 0.f;
      if (j < C) {
        const int k = j / f2, i = j - f2 * k;
        if (k < CO) v = lin(k) * (i == 0 ? w1 : ((i & 1) ? w4 : w2));
        if (i == 0 && k > 0) v = fmaf(lin(k - 1), w1, v);
      }
      lam[j] = v * c.out_scale;
      psi[j] = 0.f;
    }
  } else {
    // Four channels per lane in flight at a time.
    constexpr int kB = 4;
    for (int k0 = sl; k0 < CP; k0 += kB * W) {
      float vT[kB], vC[kB], vD[kB], vL[kB], vB[kB];
#pragma unroll
      for (int b = 0; b < kB; ++b) {
        const int k = k0 + b * W;
        const bool in = k < C;
        vT[b] = in && gT ? gload(gT + k) : 0.f;
        vC[b] = in && gC ? gload(gC + k) : 0.f;
        vD[b] = in && gD ? gload(gD + k) : 0.f;
        vL[b] = in && gL ? gload(gL + k) : 0.f;
        vB[b] = in && gB ? gload(gB + k) : 0.f;
      }
#pragma unroll
      for (int b = 0; b < kB; ++b) {
        const int k = k0 + b * W;
        if (k < CP) {
          lam[k] = (vT[b] + vL[b]) * c.out_scale;
          psi[k] = 0.f;
          gam += (double)vT[b] + (double)vC[b];
          del += (double)vD[b];
          bsum += (double)vB[b];
        }
      }
    }
  }
  gam = group_sum<W>(gam) * (double)c.out_scale;
  del = group_sum<W>(del) * (double)c.out_scale;
  bsum = group_sum<W>(bsum) * (double)c.out_scale;
  const double Ptrue = gload(P.ck_scal + pixc * kCkScal + kCkPtrue);
  const double Bout = c.J_bg * exp(-Ptrue);
  double Qend = 0.0;  // sum of lambda~ Psi over the channels at a segment's end
  const int n_seg = (P.n_los + K - 1) / K;

  // With four sightlines per wavefront (whose register budget has room),
  // loads are issued one segment ahead (segments run last to first): the
  // stored fields of the next segment's first setup round and, up to 512
  // channels, its checkpointed line excess.
  constexpr bool kAhead = G == 4;
  constexpr int kPf = kAhead ? 512 / W : 1;
  const bool pf_ck = kAhead && C <= kPf * W;
  typename LoaderT::Raw pre_f;
  float pre_ck[kPf];
  auto fetch_segment = [&](int gg) {
    const int i = gg * K + sl;
    pre_f = load.fetch((int64_t)i * P.at.los, live && sl < min(K, P.n_los - gg * K));
    if (pf_ck) {
      const float* src = P.ck_state + ((int64_t)gg * P.n_pix + pixc) * C;
#pragma unroll
      for (int b = 0; b < kPf; ++b) {
        const int k = sl + b * W;
        pre_ck[b] = k < C ? gload(src + k) : 0.f;
      }
    }
  };
  if (kAhead) fetch_segment(n_seg - 1);

  for (int g = n_seg - 1; g >= 0; --g) {
    const int s0 = g * K;
    const int L = min(K, P.n_los - s0);
    const double* cs = P.ck_scal + ((int64_t)g * P.n_pix + pixc) * kCkScal;
    const double As = gload(cs + kCkA), Bs = gload(cs + kCkB);
    // The checkpointed line excess goes to the channel state now (the state
    // of the segment above is no longer needed); the first recompute below
    // starts from it.
    if (pf_ck) {
      wave_order();
#pragma unroll
      for (int b = 0; b < kPf; ++b) {
        const int k = sl + b * W;
        if (k < C) psi[k] = pre_ck[b];
      }
      wave_order();
    }
    const typename LoaderT::Raw cur_f = pre_f;
    if (kAhead && g > 0) fetch_segment(g - 1);

    // Per-cell setup of the segment in rounds of W cells (lane sl = cell
    // s0 + r W + sl), FP64 prefixes carried across rounds.
    double Pcar = 0.0;  // dust depth above the segment start before the round
    double Gcar = As;   // scaled deficit of the last cell set up, at its base
    double bcar = 0.0;  // that cell's base
    float Jcar = 0.f;   // its dust source function
    bool rebased = false;  // some cell of the segment (any group) moves the base
    for (int r = 0; r * W < L; ++r) {
      const int i = r * W + sl;
      const bool valid = live && i < L;
      const CellIn in =
          load.decode(kAhead && r == 0 ? cur_f : load.fetch((int64_t)(s0 + i) * P.at.los, valid),
                      valid);
      const CellOut o = cell_setup<GEN>(c, in, valid, false);
      const double kD = valid ? (double)o.kD : 0.0;
      const double Pin = Pcar + group_scan_dpp<W>(kD);
      const double Pex = Pin - kD;
      // The cell's base, and whether it lies above its predecessor's. The
      // running maximum keeps the bases non-decreasing where the prefix sums
      // of different lanes round differently.
      double bse = fmax(kAdjBaseStep * floor(Pex * (1.0 / kAdjBaseStep)), bcar);
      if (__any(bse > 0.0)) bse = group_scan_max<W>(bse);
      const double bup = dpp_f64_keep<kDppWaveShr1, 0xF>(bse, 0.0);
      const double bprev = sl == 0 ? bcar : bup;
      const bool moved = valid && bse > bprev;
      const bool round_moves = __any(moved);
      rebased = rebased || round_moves;
      // e^{+-(Pex - base)} in FP32 (Pex - base < kAdjBaseStep): the chain rule
      // needs them to about 1e-7 only.
      const float epf = ex2((float)(Pex - bse) * kLog2e), emf = ex2(-(float)(Pex - bse) * kLog2e);
      const float rsf = moved ? (float)exp(bprev - bse) : 1.f;
      const double ePex = (double)epf;
      const float Jup = lane_up1(o.JD);
      const float Jprev = sl == 0 ? (r == 0 ? o.JD : Jcar) : Jup;
      const double tJ = valid ? ((double)Jprev - (double)o.JD) * ePex : 0.0;
      // Scaled deficit G_n = a_n e^{P_{n-1} - base_n}: a prefix sum while the
      // base stays put, else a scan of the maps G <- rs G + tJ.
      double Gn;
      if (!round_moves) {
        Gn = Gcar + group_scan_dpp<W>(tJ);
      } else {
        double M = (double)rsf, Cc = tJ, Sd = 0.0;
        group_scan_affine<W>(M, Cc, Sd);
        Gn = fma(M, Gcar, Cc);
      }
      if (i < L) {
        const int np = valid ? window_passes(o.nwin, W) : 0;
        float* rw = rows + i * RW;
        rw[kArG] = (float)Gn;
        rw[kArA] = o.A;
        rw[kArC0] = o.c0;
        rw[kArLk] = np ? o.lk : -256.f;
        rw[kArEmlk] = ex2(-o.lk);  // 1 / (kappa_L log2 e) with the forward's floor
        rw[kArPacked] = __int_as_float(np ? (o.kstart | (np << 24)) : 0);
        rw[kArOmen] = valid ? one_minus_exp_neg(o.kD) : 0.f;
        rw[kArEPex] = epf;
        *(double*)(rw + kArAn) = Gn * (double)emf;  // a_n = C_{n-1} - J_n
        rw[kArBm] = (float)(Bs * (double)emf * (bse > 0.0 ? exp(-bse) : 1.0));  // B_{n-1}
        rw[kArRs] = rsf;
        if (GEN) {
          rw[kArH] = valid ? (float)((double)(o.JL - o.JD) * ePex) : 0.f;
          rw[kArKd] = valid ? o.kD : 0.f;
          rw[kArEk] = ex2((valid ? o.kD : 0.f) * kLog2e);
        }
        float* rr = res + i * kAdjRes;
        rr[kAsLnn] = in.lnn;
        rr[kAsT] = in.T;
        rr[kAsX] = in.X;
        if (GEN) rr[kAsTd] = in.Td;
      }
      const int last = sub * W + min(W, L - r * W) - 1;
      Pcar = __shfl(Pin, last, 64);
      Gcar = __shfl(Gn, last, 64);
      bcar = __shfl(bse, last, 64);
      Jcar = __shfl(o.JD, last, 64);
    }

    // Every cell of the segment (in every group) within one pass: the pass
    // loops then need no per-cell bound across groups.
    bool one_pass = true;
    for (int i = sl; i < L; i += W)
      if ((__float_as_int(rows[i * RW + kArPacked]) >> 24) > 1) one_pass = false;
    one_pass = !__any(!one_pass);
    // The two-cell loops below assume a base that does not move.
    const bool pair = one_pass && !rebased;

    // lambda~ from the base of the segment above (its start, P_{s1-1}) to the
    // base of this segment's last cell: times e^{-(P_{s1-1} - P_{s0-1} - base)}.
    wave_order();
    if (Pcar > bcar) {
      // Eight channels per lane in flight (a read-use wait per channel would
      // serialise the LDS latency C/W times).
      const float fsc = (float)exp(bcar - Pcar);
      constexpr int kB = 8;
      for (int k0 = sl; k0 < C; k0 += kB * W) {
        float v[kB];
#pragma unroll
        for (int b = 0; b < kB; ++b) v[b] = k0 + b * W < C ? lam[k0 + b * W] : 0.f;
#pragma unroll
        for (int b = 0; b < kB; ++b)
          if (k0 + b * W < C) lam[k0 + b * W] = v[b] * fsc;
      }
    }
    wave_order();

    int u1 = L;
    while (u1 > 0) {
      // Sub-segment [u0, u1): the longest suffix whose window passes fit
      // the tape in every group (one cell always fits).
      int u0 = u1;
      if (one_pass) {
        u0 = max(0, u1 - TP);  // at most one pass per cell
      } else {
        int tot = 0;
        while (u0 > 0) {
          const int np = __float_as_int(rows[(u0 - 1) * RW + kArPacked]) >> 24;
          if (groups_max<G>(tot + np > TP ? 1 : 0)) break;
          tot += np;
          --u0;
        }
        if (u0 == u1) u0 = u1 - 1;
      }
      // Recompute the forward from the checkpoint to u1, taping [u0, u1).
      if (pf_ck && u1 == L) {
        // Already in place from the prefetch.
      } else {
        // Eight loads in flight per lane before their LDS stores (a load-use
        // wait per element would serialise the HBM latency C/W times).
        const float* src = P.ck_state + ((int64_t)g * P.n_pix + pixc) * C;
        wave_order();
        constexpr int kB = 8;
        for (int k0 = sl; k0 < C; k0 += kB * W) {
          float v[kB];
#pragma unroll
          for (int b = 0; b < kB; ++b) {
            const int k = k0 + b * W;
            v[b] = k < C ? gload(src + k) : 0.f;
          }
#pragma unroll
          for (int b = 0; b < kB; ++b) {
            const int k = k0 + b * W;
            if (k < C) psi[k] = v[b];
          }
        }
        wave_order();
      }
      int toff = 0;
      int i0 = 0;
      if (pair) {
        // Two cells per iteration (at most one pass each): both rows and
        // exponentials ahead of the two state updates, which may touch the
        // same channels and stay in order.
        for (; i0 + 1 < u1; i0 += 2) {
          float x[2], g[2];
          float4 rg[2];  // h, kD, e^{kD} (separate source functions)
          int k[2], np[2];
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            const float* rw = rows + (i0 + u) * RW;
            const float4 ra = *(const float4*)rw;
            const int pk = __float_as_int(rw[kArPacked]);
            np[u] = pk >> 24;
            k[u] = (pk & 0xFFFFFF) + sl;
            const float t = fmaf(slf, ra.y, ra.z);
            x[u] = ex2(fmaf(-t, t, ra.w));  // tau_L log2 e
            g[u] = ra.x;
            if (GEN) rg[u] = *(const float4*)(rw + kArH);
          }
          wave_order();
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            const float ps = psi[k[u]];  // every lane: no branch around the read
            if (np[u]) {
              if (i0 + u >= u0) tape[toff + sl] = ps;
              psi[k[u]] = GEN ? gen_formal_step(ps, g[u], x[u], rg[u].x, rg[u].y, rg[u].z)
                              : formal_line_step(ps, g[u], x[u]);
            }
            if (i0 + u >= u0) toff += W * np[u];
            wave_order();
          }
        }
      }
      for (int i = i0; i < u1; ++i) {
        const float* rw = rows + i * RW;
        const float4 ra = *(const float4*)rw;
        const int pk = __float_as_int(rw[kArPacked]);
        const int np = pk >> 24, kstart = pk & 0xFFFFFF;
        if (rebased && rw[kArRs] != 1.f) {
          // The cell's base lies above its predecessor's: rescale the state.
          const float rs = rw[kArRs];
          wave_order();
          for (int k = sl; k < C; k += W) psi[k] *= rs;
          wave_order();
        }
        const int npm = one_pass ? (__any(np > 0) ? 1 : 0) : groups_max<G>(np);
        if (npm == 0) continue;
        const bool rec = i >= u0;
        const float4 rg = GEN ? *(const float4*)(rw + kArH) : make_float4(0.f, 0.f, 0.f, 0.f);
        wave_order();
        for (int q = 0; q < npm; ++q) {
          if (q < np) {
            const int k = kstart + W * q + sl;
            const float t = fmaf(slf + (float)(W * q), ra.y, ra.z);
            const float ps = psi[k];
            if (rec) tape[toff + W * q + sl] = ps;
            const float x = ex2(fmaf(-t, t, ra.w));
            psi[k] = GEN ? gen_formal_step(ps, ra.x, x, rg.x, rg.y, rg.z)
                         : formal_line_step(ps, ra.x, x);
          }
        }
        if (rec) toff += W * np;
        wave_order();
      }
      if (u1 == L) {
        // Q at the segment end over every channel.
        double qs = 0.0;
        wave_order();
        constexpr int kB = 8;
        for (int k0 = sl; k0 < C; k0 += kB * W) {
          float a[kB], b[kB];
#pragma unroll
          for (int j = 0; j < kB; ++j) {
            const bool in = k0 + j * W < C;
            a[j] = in ? lam[k0 + j * W] : 0.f;
            b[j] = in ? psi[k0 + j * W] : 0.f;
          }
#pragma unroll
          for (int j = 0; j < kB; ++j) qs = fma((double)a[j], (double)b[j], qs);
        }
        Qend = group_sum<W>(qs);
      }
      // Reverse over the sub-segment.
      int i1 = u1 - 1;
      if (pair) {
        // Two cells per iteration (cells i, i-1): rows, exponentials and tape
        // reads ahead of the two lambda updates, which stay in order.
        for (; i1 - 1 >= u0; i1 -= 2) {
          float E[2], tl[2], t[2], g[2], em[2], ps0[2];
          float4 rg[2];  // h, kD, e^{kD} (separate source functions)
          int k[2], np[2];
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            const float* rw = rows + (i1 - u) * RW;
            const float4 ra = *(const float4*)rw;
            const float4 rb = *(const float4*)(rw + 4);
            if (GEN) rg[u] = *(const float4*)(rw + kArH);
            const int pk = __float_as_int(rb.y);
            np[u] = pk >> 24;
            k[u] = (pk & 0xFFFFFF) + sl;
            t[u] = fmaf(slf, ra.y, ra.z);
            tl[u] = ex2(fmaf(-t[u], t[u], ra.w));
            E[u] = ex2(-tl[u]);
            g[u] = ra.x;
            em[u] = rb.x;
            toff -= W * np[u];
            // Read by every lane (a cell without passes reads LDS it ignores),
            // so that no branch holds the two cells' reads apart.
            const float tv = tape[toff + sl];
            ps0[u] = np[u] ? tv : 0.f;
          }
          wave_order();
          // The lambda updates stay in order; the window sums come after both,
          // as selects, off the chain.
          float s1[2], s3[2], s4[2], s5[2], sh[2], sk[2], lt[2];
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            lt[u] = lam[k[u]];
            if (np[u]) lam[k[u]] = lt[u] * E[u];
            wave_order();
          }
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            const bool on = np[u] != 0 && k[u] < C;
            float tg;  // taubar * g
            if (GEN) {
              const GenRev gr = gen_reverse(tl[u], E[u], rg[u].y, rg[u].z);
              tg = lt[u] * fmaf(rg[u].x, gr.tb, -E[u] * (ps0[u] + g[u])) * (tl[u] * em[u]);
              sh[u] = on ? lt[u] * gr.sh : 0.f;
              sk[u] = on ? lt[u] * gr.sk : 0.f;
            } else {
              tg = -E[u] * lt[u] * (ps0[u] + g[u]) * (tl[u] * em[u]);
            }
            s1[u] = on ? lt[u] * (E[u] - 1.f) : 0.f;
            s3[u] = on ? tg : 0.f;
            s4[u] = on ? tg * t[u] : 0.f;
            s5[u] = on ? tg * t[u] * t[u] : 0.f;
          }
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            s1[u] = group_allsum<W>(s1[u]);
            s3[u] = group_allsum<W>(s3[u]);
            s4[u] = group_allsum<W>(s4[u]);
            s5[u] = group_allsum<W>(s5[u]);
            if (GEN) {
              sh[u] = group_allsum<W>(sh[u]);
              sk[u] = group_allsum<W>(sk[u]);
            }
          }
          if (sl == 0) {
#pragma unroll
            for (int u = 0; u < 2; ++u) {
              float* rr = res + (i1 - u) * kAdjRes;
              rr[kAsS1] = s1[u];
              rr[kAsS3] = s3[u];
              rr[kAsS4] = s4[u];
              rr[kAsS5] = s5[u];
              if (GEN) {
                rr[kAsSH] = sh[u];
                rr[kAsSK] = sk[u];
              }
            }
          }
        }
      }
      for (int i = i1; i >= u0; --i) {
        const float* rw = rows + i * RW;
        const float4 ra = *(const float4*)rw;
        const float4 rb = *(const float4*)(rw + 4);
        const int pk = __float_as_int(rb.y);
        const int np = pk >> 24, kstart = pk & 0xFFFFFF;
        const int npm = one_pass ? (__any(np > 0) ? 1 : 0) : groups_max<G>(np);
        float s1 = 0.f, s3 = 0.f, s4 = 0.f, s5 = 0.f, sh = 0.f, sk = 0.f;
        if (npm > 0) {
          const float4 rg = GEN ? *(const float4*)(rw + kArH) : make_float4(0.f, 0.f, 0.f, 0.f);
          toff -= W * np;
          wave_order();
          for (int q = 0; q < npm; ++q) {
            if (q < np) {
              const int k = kstart + W * q + sl;
              const float t = fmaf(slf + (float)(W * q), ra.y, ra.z);
              const float tl = ex2(fmaf(-t, t, ra.w));
              const float E = ex2(-tl);
              const float lt = lam[k];
              const float ps0 = tape[toff + W * q + sl];
              if (k < C) {
                s1 = fmaf(lt, E - 1.f, s1);
                float tb = -E * lt * (ps0 + ra.x);
                if (GEN) {
                  const GenRev gr = gen_reverse(tl, E, rg.y, rg.z);
                  tb = lt * fmaf(rg.x, gr.tb, -E * (ps0 + ra.x));
                  sh = fmaf(lt, gr.sh, sh);
                  sk = fmaf(lt, gr.sk, sk);
                }
                const float tg = tb * (tl * rb.x);  // taubar * g
                s3 += tg;
                s4 = fmaf(tg, t, s4);
                s5 = fmaf(tg * t, t, s5);
              }
              lam[k] = lt * E;
            }
          }
          wave_order();
          s1 = group_allsum<W>(s1);
          s3 = group_allsum<W>(s3);
          s4 = group_allsum<W>(s4);
          s5 = group_allsum<W>(s5);
          if (GEN) {
            sh = group_allsum<W>(sh);
            sk = group_allsum<W>(sk);
          }
        }
        if (sl == 0) {
          float* rr = res + i * kAdjRes;
          rr[kAsS1] = s1;
          rr[kAsS3] = s3;
          rr[kAsS4] = s4;
          rr[kAsS5] = s5;
          if (GEN) {
            rr[kAsSH] = sh;
            rr[kAsSK] = sk;
          }
        }
        if (rebased && rw[kArRs] != 1.f) {
          // lambda~ down to the predecessor's base.
          const float rs = rw[kArRs];
          wave_order();
          for (int k = sl; k < C; k += W) lam[k] *= rs;
          wave_order();
        }
      }
      u1 = u0;
    }

    // Recurrences of the reverse march, then the chain rule to the stored
    // fields. Lanes take the cells in descending order (cell r W + W-1-sl),
    // last round first; per cell the updates are affine maps,
    //   gamma <- e gamma + abar,  delta <- e delta,  Q <- Q - a abar,
    // so one FP64 scan of the maps per round gives every cell the values it
    // sees (the composition of the maps of the cells above it).
    wave_order();
    double Qc = Qend;
    for (int r = (L - 1) / W; r >= 0; --r) {
      const int i = r * W + (W - 1 - sl);
      const bool vc = i < L;
      double M = 1.0, Cm = 0.0, S = 0.0, abar = 0.0, omen = 0.0, an = 0.0, Bm = 0.0;
      if (vc) {
        const float* rw = rows + i * RW;
        omen = (double)rw[kArOmen];
        an = *(const double*)(rw + kArAn);
        Bm = (double)rw[kArBm];
        abar = (double)rw[kArEPex] * (double)res[i * kAdjRes + kAsS1];
        M = 1.0 - omen;
        Cm = abar;
        S = an * abar;
        // H_n Hbar_n = h sum lambda~ beta (e^{kD} - E) (separate source functions).
        if (GEN) S = fma((double)rw[kArH], (double)res[i * kAdjRes + kAsSH], S);
      }
      group_scan_affine<W>(M, Cm, S);
      // Exclusive: the maps of the cells above this one (identity in lane 0).
      double Mx = dpp_f64_keep<kDppWaveShr1, 0xF>(M, 1.0);
      double Cx = dpp_f64_keep<kDppWaveShr1, 0xF>(Cm, 0.0);
      double Sx = dpp_f64_keep<kDppWaveShr1, 0xF>(S, 0.0);
      if (sl == 0) {
        Mx = 1.0;
        Cx = 0.0;
        Sx = 0.0;
      }
      if (vc && live) {
        const double e_i = 1.0 - omen;
        const double gam_i = fma(Mx, gam, Cx), del_i = Mx * del, Q_i = Qc - Sx;
        const float* rr = res + i * kAdjRes;
        double kDbar_i = -Q_i - e_i * (gam_i * an + del_i * (an - Bm));
        double Jbar = (gam_i + del_i) * omen - abar;  // the dust's source function
        double Hbar = 0.0;                             // the line's excess over it
        if (GEN) {
          const float* rw = rows + i * RW;
          Hbar = (double)rw[kArEPex] * (double)rr[kAsSH];
          Jbar -= Hbar;
          kDbar_i = fma((double)rw[kArH], (double)rr[kAsSK], kDbar_i);
        }
        const int s = s0 + i;
        const double kLbar = (double)rr[kAsS3];
        const CellPartials cp =
            GEN && c.ot
                ? cell_partials_ot(c, (double)rr[kAsLnn], (double)rr[kAsT], (double)rr[kAsX])
                : cell_partials<GEN>(c, (double)rr[kAsLnn], (double)rr[kAsT], (double)rr[kAsX]);
        if (GEN && !cp.line_src) {
          // No line in the level grid's populations: J_L is J_D itself.
          Jbar += Hbar;
          Hbar = 0.0;
        }
        const double fac = 2.0 * cp.kL / cp.b;
        const double vbar = fac * (double)rr[kAsS4] * (1.0 / (double)kSqrtLog2e);
        const double bbar = fac * (double)rr[kAsS5] * (1.0 / (double)kLog2e);
        const double kDbar = cp.kD_clamped ? 0.0 : kDbar_i;
        double glnn = kLbar * cp.kL + kDbar * cp.kD - bsum * Bout * cp.kD_free;
        if (GEN) glnn += kLbar * cp.dkL_dlnn + Hbar * cp.dJL_dlnn;  // level grid's n_H2 slopes
        double gT = kLbar * cp.dkL_dT + bbar * cp.db_dT;
        double gTd = 0.0;
        if (GEN) {
          // J_L = J_D + H depends on T_kin; J_D on T_dust (T_kin without one).
          gT = fma(Hbar, cp.dJL_dT, gT);
          if (has_td) gTd = Jbar * planck_rj_dT(c, (double)rr[kAsTd]);
          else gT = fma(Jbar, cp.dJ_dT, gT);
        } else {
          gT = fma(Jbar, cp.dJ_dT, gT);
        }
        const double gX = kLbar * cp.dkL_dX;
        const int64_t off = P.gat.base(pix) + (int64_t)s * P.gat.los;
        gstore(P.grad[0] + off, glnn);
        gstore(P.grad[1] + off, gT);
        gstore(P.grad[2] + off, vbar);
        gstore(P.grad[3] + off, gX);
        if (GEN && has_td) gstore(P.grad[4] + off, gTd);
      }
      // Carry the composition of the whole round (the group's last lane).
      const int last = sub * W + W - 1;
      const double Ml = __shfl(M, last, 64), Cl = __shfl(Cm, last, 64), Sl = __shfl(S, last, 64);
      gam = fma(Ml, gam, Cl);
      del = Ml * del;
      Qc -= Sl;
    }
    wave_order();
  }
}

// Register caps: four sightlines per wavefront need LDS for only two
// wavefronts per SIMD, so their kernels may use up to 256 VGPRs; narrower
// packings keep three wavefronts per SIMD.
template <typename FT, int G, bool GEN>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(G == 4 || GEN ? 2 : 3))) void adj_kernel(
    const AdjParams P) {
  extern __shared__ float lds[];
  const int64_t pix0 = (int64_t)xcd_tile((int)blockIdx.x, (int)gridDim.x) * G;
  if (pix0 >= P.n_pix) return;
  adj_wave<Loader<FT>, G, GEN>(P, pix0, lds);
}

template <typename FT, int G>
static int launch_t(const AdjParams& p, void* stream) {
  const int blocks = (p.n_pix + G - 1) / G;
  const size_t lds = (size_t)p.lds_per_wave * sizeof(float);
  if (p.c.general)
    hipLaunchKernelGGL((adj_kernel<FT, G, true>), dim3(blocks), dim3(64), lds, (hipStream_t)stream,
                       p);
  else
    hipLaunchKernelGGL((adj_kernel<FT, G, false>), dim3(blocks), dim3(64), lds,
                       (hipStream_t)stream, p);
  return (int)hipGetLastError();
}

template <typename FT>
static int launch_g(const AdjParams& p, void* stream) {
  switch (p.groups) {
    case 1: return launch_t<FT, 1>(p, stream);
    case 2: return launch_t<FT, 2>(p, stream);
    case 4: return launch_t<FT, 4>(p, stream);
  }
  return (int)hipErrorInvalidValue;
}

int adjoint_waves_per_block() { return 1; }

int launch_adjoint(iris_dtype dt, const AdjParams& p, void* stream) {
  switch (dt) {
    case IRIS_F64: return launch_g<double>(p, stream);
    case IRIS_F32: return launch_g<float>(p, stream);
    case IRIS_BF16: return launch_g<bf16_t>(p, stream);
    case IRIS_F16: return launch_g<_Float16>(p, stream);
  }
  return (int)hipErrorInvalidValue;
}

// --- batched persistent launch -------------------------------------------------

// The batched kernel reads fields of any storage type (more registers): at
// three wavefronts per SIMD its narrower packings spilled, so every packing
// takes up to 256 VGPRs (64-cube batch, two sightlines per wavefront
// everywhere: 30.4 -> 21.6 ms).
template <int G, bool GEN>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void plan_adj_kernel(
    const PlanAdjParams Q) {
  extern __shared__ float lds[];
  ItemClaim claim(1, 0, Q.static_rounds != 0);
  while (true) {
    const int idx = claim.next(Q.slice_begin, Q.counter);
    if (idx < 0) break;
    wave_order();  // the previous item's LDS reads come first
    // Item and cube parameters are uniform and read-only for the launch:
    // scalar loads through the constant address space.
    const WorkItem wi = Q.items[idx];
    const int cube = __builtin_amdgcn_readfirstlane(wi.cube);
    const int64_t pix0 = __builtin_amdgcn_readfirstlane(wi.pix0);
    const AdjParams& P =
        *(const AdjParams*)((const __attribute__((address_space(4))) AdjParams*)Q.cubes + cube);
    adj_wave<DynLoader, G, GEN>(P, pix0, lds);
  }
}

template <int G, bool GEN>
static int launch_plan_adj(const PlanAdjParams& q, int blocks, void* stream) {
  const size_t lds = (size_t)q.wave_floats * sizeof(float);
  hipLaunchKernelGGL((plan_adj_kernel<G, GEN>), dim3(blocks), dim3(64), lds, (hipStream_t)stream,
                     q);
  return (int)hipGetLastError();
}

int launch_plan_adjoint(const PlanAdjParams& q, int groups, bool general, int blocks,
                        void* stream) {
  switch (groups * 2 + (general ? 1 : 0)) {
    case 2: return launch_plan_adj<1, false>(q, blocks, stream);
    case 3: return launch_plan_adj<1, true>(q, blocks, stream);
    case 4: return launch_plan_adj<2, false>(q, blocks, stream);
    case 5: return launch_plan_adj<2, true>(q, blocks, stream);
    case 8: return launch_plan_adj<4, false>(q, blocks, stream);
    case 9: return launch_plan_adj<4, true>(q, blocks, stream);
  }
  return (int)hipErrorInvalidValue;
}

template <int G, bool GEN>
static hipError_t plan_adj_occupancy(int* nb, size_t lds) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, plan_adj_kernel<G, GEN>, 64, lds);
}

int plan_adjoint_occupancy(int wave_floats, int groups, bool general) {
  int nb = 0;
  const size_t lds = (size_t)wave_floats * sizeof(float);
  hipError_t e = hipErrorInvalidValue;
  switch (groups * 2 + (general ? 1 : 0)) {
    case 2: e = plan_adj_occupancy<1, false>(&nb, lds); break;
    case 3: e = plan_adj_occupancy<1, true>(&nb, lds); break;
    case 4: e = plan_adj_occupancy<2, false>(&nb, lds); break;
    case 5: e = plan_adj_occupancy<2, true>(&nb, lds); break;
    case 8: e = plan_adj_occupancy<4, false>(&nb, lds); break;
    case 9: e = plan_adj_occupancy<4, true>(&nb, lds); break;
  }
  if (e != hipSuccess) return 1;
  return nb > 0 ? nb : 1;
}

}  // namespace iris
