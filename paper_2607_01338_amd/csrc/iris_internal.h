// Internal structures shared by the host library and the HIP kernels.
#pragma once

#include <cstddef>
#include <cstdint>

#include "iris_rt.h"

namespace iris {

// Largest channel count: each sightline keeps its channel state in LDS.
constexpr int kMaxChannels = 4000;
// Sightlines (wavefronts) per workgroup of the march kernels.
constexpr int kWavesPerBlock = 4;
// Cells handled per wavefront pass of the per-cell setup (one per lane).
constexpr int kChunk = 64;
// Dust optical depth allowed between two rebasings of the scaled state.
constexpr float kRebaseTau = 60.0f;

// Temperature tables (poptable.hip): kTabPerOctave intervals per octave of T
// over [2^kTabOct0, 2^kTabOct1) K, three float4 tables of kTabN intervals.
constexpr int kTabPerOctave = 128;
constexpr int kTabOct0 = 0;
constexpr int kTabOct1 = 16;
constexpr int kTabN = (kTabOct1 - kTabOct0) * kTabPerOctave;
constexpr size_t kTabBytes = (size_t)3 * kTabN * 16;

struct TabParams {
  double theta;  // E_J / k = theta J (J+1), K
  double dE;     // (E_u - E_l)/k, K
  double T0;     // h nu0 / k, K
  double g_l;
  int32_t j_max, j_l;
};

// Constants of one launch, folded on the host in double precision.
//
// Units inside the kernels: temperatures and intensities in Rayleigh-Jeans
// kelvin at the rest frequency; velocities in km/s; optical depths per cell.
struct Folded {
  // LTE partition sum: term_J = (2J+1) 2^(-th2 J(J+1) / T).
  double th2;      // (E_J/k) / (J (J+1)) * log2(e), K
  int32_t j_max;
  int32_t j_l;     // lower rotational level
  float g_l;       // statistical weight of the lower level
  float dE;        // (E_u - E_l) / k, K
  float T0;        // h nu0 / k, K (Rayleigh-Jeans scale of the Planck function)
  float kL;        // line-centre optical depth = kL * X * n_H2 * f_l * (1 - e^{-dE/T}) / b
  float bT, bt2;   // b^2 = bT * T + bt2, (km/s)^2
  float kD;        // dust optical depth of one cell = kD * n_H2
  float t_inf;     // no line above this kinetic temperature
  float xw2min;    // window half-width in Doppler units: x_w^2 = xw2min + ln(max(kappa_L, 1))
  float kL_min;    // forward: cells with kappa_L below this carry no line
  int32_t general; // 1 when the line source function can differ from the dust one
  double J_bg;     // background, RJ kelvin
  double v_lo;     // channel grid: centre of channel k = v_lo + (k + 1/2) dv
  double dv;
  double inv_dv;
  int32_t n_chan;   // velocities marched (2 f n_out + 1 when subsampled)
  int32_t n_out;    // output channels
  int32_t simpson_f; // Simpson panels per channel, 2f fine steps (0: channel centres)
  int32_t units;    // iris_units of the outputs
  float out_scale;  // output units per Rayleigh-Jeans kelvin (intensity units), else 1
  int32_t pad_;
  const void* tab;  // temperature tables (float4 [3][kTabN]) in the workspace
  // Non-LTE populations (null: LTE): the (FU, FL) grid [nc][nt][nn] of the
  // observed transition over ln n_H2 (nodes ot_n0 + i / ot_dn_inv), ln T
  // (ot_t0 + i / ot_dt_inv) and the molecular fraction, whose interval ot_ic
  // and local coordinate ot_tc are the same for every cell.
  const void* ot;
  float ot_n0, ot_dn_inv, ot_t0, ot_dt_inv, ot_tc;
  int32_t ot_nn, ot_nt, ot_nc, ot_ic;
};

// Checkpoint scalars per (checkpoint, sightline), entering cell ck*K, FP64:
// continuum C_{s-1}, dust emission D_{s-1}, dust depth P_{s-1} (absolute,
// clamped cells), continuum deficit C_{s-1} - J_s, background B_{s-1}
// attenuated by the clamped column; the unclamped column of the whole
// sightline (for [B]) in checkpoint 0 only.
enum : int { kCkC = 0, kCkD, kCkP, kCkA, kCkB, kCkPtrue, kCkScal };

// Element type tags of the stored fields.
struct bf16_t {
  uint16_t bits;
};

// Element offset of cell s of sightline pix in a field array:
//   (pix / div) * hi + (pix % div) * lo + s * los.
// Sightline-major copies: div = n_pix, lo = n_los, los = 1. Native
// [nx][ny][nz] arrays: axis 2 as above with lo = nz; axis 1: div = nz,
// hi = ny nz, lo = 1, los = nz; axis 0: div = n_pix, lo = 1, los = ny nz.
struct SightAddr {
  int64_t div, hi, lo, los;
  __host__ __device__ int64_t base(int64_t pix) const {
    return (pix / div) * hi + (pix % div) * lo;
  }
};

struct FwdParams {
  const void* f[5];       // ln n, T, v, X, T_dust, addressed by `at`
  SightAddr at;
  int32_t n_pix;
  int32_t n_los;
  Folded c;
  float* out[5];          // T, C, D, L, B: [n_pix][n_chan]
  int32_t ckpt_K;         // 0 = no checkpoints
  int32_t lds_per_wave;   // floats of channel state per sightline (multiple of 4)
  int32_t groups;         // sightlines per wavefront: 1, 2 or 4
  int32_t dtype;          // iris_dtype of the fields (used by batched launches)
  float* ck_state;        // [n_ck][n_pix][n_chan] line excess entering cell ck*K
  double* ck_scal;        // [n_ck][n_pix][kCkScal]: see kCk* below
};

// Work item of a batched launch: G sightlines of one cube.
struct WorkItem {
  int32_t cube;
  int32_t pix0;
};

// Work queues of a persistent launch: 8 slices, one per XCD (workgroup b
// serves slice b mod 8 first, then steals from the others). Slice x holds the
// x-th contiguous share of every cube's sightlines, so neighbouring
// sightlines, which share cache lines of the native field layout, are
// handled under one L2.
constexpr int kSlices = 8;

struct PlanFwdParams {
  const FwdParams* cubes;  // device array, one per cube
  const WorkItem* items;   // device array: the slices back to back
  int32_t slice_begin[kSlices + 1];
  int32_t wave_floats;     // LDS floats per wavefront (max over the cubes)
  int32_t static_rounds;   // 1: the launch runs alone with every workgroup resident
  int* counter;            // kSlices queue heads, zeroed before each launch
};

struct AdjParams {
  const void* f[5];
  SightAddr at;           // fields
  int32_t n_pix;
  int32_t n_los;
  Folded c;
  const float* cot[5];    // gT, gC, gD, gL, gB: [n_pix][n_chan]
  int32_t ckpt_K;
  int32_t lds_per_wave;   // floats per wavefront (adj_wave_floats)
  int32_t chan_stride;    // floats of channel state per sightline (adj_chan_stride)
  int32_t tape_passes;    // W-lane passes the LDS tape holds per sightline
  const float* ck_state;
  const double* ck_scal;
  double* grad[5];        // per stored field, addressed by `gat`
  SightAddr gat;
  int32_t dtype;          // iris_dtype of the fields (used by batched launches)
  int32_t groups;         // sightlines per wavefront: 1, 2 or 4
};

// LDS of the adjoint per wavefront of G sightlines (W = 64/G lanes each):
// channel state and lambda [G][chan_stride], the tape [G][tape_passes][W],
// and per segment of K cells a 12-float row and a 12-float result per cell.
__host__ __device__ inline int adj_chan_stride(int n_chan, int groups) {
  return (n_chan + 64 / groups + 3) & ~3;
}
// With 16 lanes per sightline, two sightlines share each half-wavefront; an
// odd pass count puts their tapes 16 banks apart.
__host__ __device__ inline int adj_tape_passes(int n_chan, int groups) {
  const int w = 64 / groups;
  const int widest = (n_chan + w - 1) / w + 1;  // passes of the widest window of one cell
  const int tp = widest > 16 ? widest : 16;
  return groups == 4 ? (tp | 1) : tp;
}
// The per-cell row and result tables of the G sightlines start kAdjSkew
// floats apart beyond their length, so that rows read together (one per
// sightline, broadcast to its lanes) sit in different LDS banks.
constexpr int kAdjSkew = 4;
__host__ __device__ inline int adj_wave_floats(int n_chan, int K, int groups) {
  return 2 * groups * adj_chan_stride(n_chan, groups) +
         groups * adj_tape_passes(n_chan, groups) * (64 / groups) +
         groups * (K * (12 + 12) + 2 * kAdjSkew);
}

struct PlanAdjParams {
  const AdjParams* cubes;
  const WorkItem* items;   // one sightline per item (pix0), in slices
  int32_t slice_begin[kSlices + 1];
  int32_t wave_floats;
  int32_t static_rounds;   // 1: the launch runs alone with every workgroup resident
  int* counter;            // kSlices queue heads
};

struct LayoutParams {
  const void* src[5];
  void* dst[5];
  int32_t n_fields;
  int32_t elem;           // bytes per element: 2, 4 or 8
  int64_t rows, cols;     // per batch: src [rows][cols] -> dst [cols][rows]
  int64_t batch;
};

// One cube's transpose (all of its fields) inside a batched layout launch.
struct TransposeJob {
  const void* src[5];
  void* dst[5];
  int32_t n_fields;
  int32_t elem;            // bytes per element: 2, 4 or 8
  int64_t rows, cols;      // per batch: src [rows][cols] -> dst [cols][rows]
  int64_t batch;
  int64_t tile_begin;      // first global tile of this job
  int32_t tiles_r, tiles_c;
};

// Launchers (return a hipError_t value as int).
int launch_forward(iris_dtype dt, const FwdParams& p, void* stream);
// Smooth (TR then BDF2) forward of one cube; p.groups is ignored.
int launch_smooth(iris_dtype dt, const FwdParams& p, void* stream);
int smooth_max_channels();
int fwd_state_floats(int n_chan, int groups);
size_t fwd_lds_bytes(int n_chan, int groups, bool general);
int launch_plan_forward(const PlanFwdParams& q, int groups, bool ckpt, int blocks, void* stream);
int plan_forward_occupancy(int wave_floats, int groups, bool ckpt);
int launch_adjoint(iris_dtype dt, const AdjParams& p, void* stream);
int adjoint_waves_per_block();
// `general`: separate line and dust source functions.
int launch_plan_adjoint(const PlanAdjParams& q, int groups, bool general, int blocks,
                        void* stream);
int plan_adjoint_occupancy(int wave_floats, int groups, bool general);
int launch_layout(const LayoutParams& p, void* stream);
int launch_batched_layout(const TransposeJob* jobs, int n_jobs, int64_t n_tiles, void* stream);
int launch_zero_ints(int* p, int n, void* stream);
int launch_pop_table(const TabParams& tp, void* tab, void* stream);

}  // namespace iris
