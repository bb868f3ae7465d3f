// C-ABI entry points: argument validation, constant folding (FP64) and
// workspace carving. Everything here runs on the host before any launch.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "iris_internal.h"

namespace {

// CODATA 2018, cgs.
constexpr double kPlanck = 6.62607015e-27;
constexpr double kBoltzmann = 1.380649e-16;
constexpr double kLight = 2.99792458e10;
constexpr double kAmu = 1.66053906660e-24;
constexpr double kPiD = 3.14159265358979323846;
constexpr double kLog2eD = 1.44269504088896340736;
// Window of the line: channels with Gaussian factor below kWindowEps (times
// max(kappa_L, 1)) are left untouched by a cell.
constexpr double kWindowEps = 1e-12;
// Forward pass: a cell whose line-centre optical depth is below this carries
// no line (changes every output by < 1e-10 of its source-function scale).
constexpr float kLineMin = 1e-10f;

thread_local std::string g_err;

iris_status fail(iris_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

bool finite(double x) { return std::isfinite(x); }

size_t elem_size(iris_dtype d) {
  switch (d) {
    case IRIS_F64: return 8;
    case IRIS_F32: return 4;
    case IRIS_BF16:
    case IRIS_F16: return 2;
  }
  return 0;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Geo {
  int64_t n_cells, n_los, n_pix;
  int n_fields;
};

iris_status check_fields(const iris_fields* f, Geo* g) {
  if (!f) return fail(IRIS_E_INVALID_ARG, "fields is NULL");
  if (f->nx < 1 || f->ny < 1 || f->nz < 1)
    return fail(IRIS_E_INVALID_ARG, "grid shape %d x %d x %d must be positive", f->nx, f->ny, f->nz);
  if (f->axis < 0 || f->axis > 2) return fail(IRIS_E_INVALID_ARG, "axis %d not in 0..2", f->axis);
  if (!(f->cell_cm > 0.0) || !finite(f->cell_cm))
    return fail(IRIS_E_INVALID_ARG, "cell_cm must be positive and finite");
  if (elem_size(f->dtype) == 0) return fail(IRIS_E_INVALID_ARG, "unknown dtype %d", (int)f->dtype);
  if (!f->ln_nh2 || !f->t_kin || !f->v_los || !f->x_tracer)
    return fail(IRIS_E_INVALID_ARG, "a field pointer is NULL");
  const int64_t n = (int64_t)f->nx * f->ny * f->nz;
  const int64_t los = f->axis == 0 ? f->nx : f->axis == 1 ? f->ny : f->nz;
  const int64_t pix = n / los;
  if (pix > INT32_MAX || los > (1 << 24))
    return fail(IRIS_E_UNSUPPORTED, "grid too large (%lld pixels, %lld cells per sightline)",
                (long long)pix, (long long)los);
  if (f->axis == 1 && f->nx > 65535)
    return fail(IRIS_E_UNSUPPORTED, "nx > 65535 with sightlines along y");
  if (f->axis == 0 && (f->nx + 63) / 64 > 65535)
    return fail(IRIS_E_UNSUPPORTED, "nx too large with sightlines along x");
  if (f->axis == 1 && (f->ny + 63) / 64 > 65535)
    return fail(IRIS_E_UNSUPPORTED, "ny too large with sightlines along y");
  g->n_cells = n;
  g->n_los = los;
  g->n_pix = pix;
  g->n_fields = f->t_dust ? 5 : 4;
  return IRIS_OK;
}

iris_status check_channels(const iris_channels* ch) {
  if (!ch) return fail(IRIS_E_INVALID_ARG, "channels is NULL");
  if (ch->n_chan < 1) return fail(IRIS_E_INVALID_ARG, "n_chan %d < 1", ch->n_chan);
  if (ch->n_chan > iris::kMaxChannels)
    return fail(IRIS_E_UNSUPPORTED, "n_chan %d above the maximum %d", ch->n_chan,
                iris::kMaxChannels);
  if (!(ch->dv_kms > 0.0) || !finite(ch->dv_kms) || !finite(ch->v_lo_kms))
    return fail(IRIS_E_INVALID_ARG, "channel grid needs finite v_lo and dv > 0");
  return IRIS_OK;
}

iris_status check_line(const iris_line* L) {
  if (!L) return fail(IRIS_E_INVALID_ARG, "line is NULL");
  if (!(L->nu0_hz > 0.0) || !finite(L->nu0_hz)) return fail(IRIS_E_INVALID_ARG, "nu0_hz must be > 0");
  if (!(L->a_ul > 0.0) || !finite(L->a_ul)) return fail(IRIS_E_INVALID_ARG, "a_ul must be > 0");
  if (L->j_u < 1 || L->j_max < L->j_u || L->j_max > 1000)
    return fail(IRIS_E_INVALID_ARG, "need 1 <= j_u <= j_max <= 1000");
  if (!(L->m_tracer_amu > 0.0)) return fail(IRIS_E_INVALID_ARG, "m_tracer_amu must be > 0");
  if (!(L->sigma_turb_kms >= 0.0) || !finite(L->sigma_turb_kms))
    return fail(IRIS_E_INVALID_ARG, "sigma_turb_kms must be >= 0");
  if (!(L->kappa_dust_cm2g >= 0.0) || !(L->dust_to_gas >= 0.0) || !finite(L->kappa_dust_cm2g) ||
      !finite(L->dust_to_gas))
    return fail(IRIS_E_INVALID_ARG, "dust opacity and dust-to-gas ratio must be >= 0");
  if (!(L->mu_amu_per_h2 > 0.0)) return fail(IRIS_E_INVALID_ARG, "mu_amu_per_h2 must be > 0");
  if (!(L->t_bg_k >= 0.0) || !finite(L->t_bg_k)) return fail(IRIS_E_INVALID_ARG, "t_bg_k must be >= 0");
  if (!(L->t_inf_k > 0.0)) return fail(IRIS_E_INVALID_ARG, "t_inf_k must be > 0");
  if (L->energy_mode != 0 && L->energy_mode != 1)
    return fail(IRIS_E_INVALID_ARG, "energy_mode must be 0 or 1");
  if (L->energy_mode == 1 && !(L->e_u_k > 0.0))
    return fail(IRIS_E_INVALID_ARG, "energy_mode 1 needs e_u_k > 0");
  return IRIS_OK;
}

iris::Folded fold(const iris_fields* f, const iris_channels* ch, const iris_line* L) {
  iris::Folded c{};
  const double nu = L->nu0_hz;
  const double T0 = kPlanck * nu / kBoltzmann;
  const double theta = L->energy_mode == 0 ? T0 / (2.0 * L->j_u)
                                           : L->e_u_k / (L->j_u * (L->j_u + 1.0));
  const int ju = L->j_u, jl = L->j_u - 1;
  const double gu = 2.0 * ju + 1.0, gl = 2.0 * jl + 1.0;
  const double Eu = theta * ju * (ju + 1.0), El = theta * jl * (jl + 1.0);
  const double Bul = kLight * kLight * L->a_ul / (2.0 * kPlanck * nu * nu * nu);
  const double Blu = gu / gl * Bul;
  c.th2 = theta * kLog2eD;
  c.j_max = L->j_max;
  c.j_l = jl;
  c.g_l = (float)gl;
  c.dE = (float)(Eu - El);
  c.T0 = (float)T0;
  // kappa_L = h_cell (h nu / 4 pi) n_l B_lu (1 - e^{-dE/T}) * c / (nu b sqrt(pi)),
  // with n_l = X n_H2 f_l and b in km/s.
  c.kL = (float)(f->cell_cm * (kPlanck * nu / (4.0 * kPiD)) * Blu * kLight /
                 (nu * 1e5 * std::sqrt(kPiD)));
  const double m = L->m_tracer_amu * kAmu;
  c.bT = (float)(2.0 * kBoltzmann / m / 1e10);
  c.bt2 = (float)(2.0 * L->sigma_turb_kms * L->sigma_turb_kms);
  c.kD = (float)(f->cell_cm * L->kappa_dust_cm2g * L->dust_to_gas * L->mu_amu_per_h2 * kAmu);
  c.t_inf = (float)L->t_inf_k;
  c.xw2min = (float)std::log(1.0 / kWindowEps);
  c.kL_min = kLineMin;
  c.general = (f->t_dust != nullptr || L->energy_mode == 1) ? 1 : 0;
  c.J_bg = L->t_bg_k > 0.0 ? T0 / std::expm1(T0 / L->t_bg_k) : 0.0;
  c.v_lo = ch->v_lo_kms;
  c.dv = ch->dv_kms;
  c.inv_dv = 1.0 / ch->dv_kms;
  c.n_chan = ch->n_chan;
  return c;
}

struct WsLayout {
  size_t soa = 0, ck_state = 0, ck_scal = 0, grad = 0, total = 0;
  int64_t n_ck = 0;
};

WsLayout ws_layout(const iris_fields* f, const Geo& g, int n_chan, int K) {
  WsLayout w;
  size_t off = 0;
  if (f->axis != 2) {
    w.soa = off;
    off += align256((size_t)g.n_fields * g.n_cells * elem_size(f->dtype));
  }
  if (K > 0) {
    w.n_ck = (g.n_los + K - 1) / K;
    w.ck_state = off;
    off += align256((size_t)w.n_ck * g.n_pix * n_chan * sizeof(float));
    w.ck_scal = off;
    off += align256((size_t)w.n_ck * g.n_pix * 4 * sizeof(double));
    if (f->axis != 2) {
      // Sightline-major FP64 gradients before they are laid back out.
      w.grad = off;
      off += align256((size_t)4 * g.n_cells * sizeof(double));
    }
  }
  w.total = off;
  return w;
}

bool valid_K(int K) { return K == 0 || K == 8 || K == 16 || K == 32 || K == 64; }

iris_status hip_status(int e, const char* what) {
  if (e != 0)
    return fail(IRIS_E_HIP, "%s: %s", what, hipGetErrorString((hipError_t)e));
  return IRIS_OK;
}

// Field pointers in sightline-major order: either the native arrays (axis 2)
// or the copies made by the layout kernel in the workspace.
iris_status prepare_fields(const iris_fields* f, const Geo& g, const WsLayout& w, void* ws,
                           const void* out[5], int64_t* pix_stride, void* stream) {
  const void* src[5] = {f->ln_nh2, f->t_kin, f->v_los, f->x_tracer, f->t_dust};
  if (f->axis == 2) {
    for (int i = 0; i < 5; ++i) out[i] = src[i];
    *pix_stride = g.n_los;
    return IRIS_OK;
  }
  iris::LayoutParams lp{};
  const size_t es = elem_size(f->dtype);
  for (int i = 0; i < g.n_fields; ++i) {
    lp.src[i] = src[i];
    lp.dst[i] = (char*)ws + w.soa + (size_t)i * g.n_cells * es;
    out[i] = lp.dst[i];
  }
  for (int i = g.n_fields; i < 5; ++i) out[i] = nullptr;
  lp.n_fields = g.n_fields;
  lp.elem = (int)es;
  if (f->axis == 1) {
    lp.batch = f->nx;
    lp.rows = f->ny;
    lp.cols = f->nz;
  } else {
    lp.batch = 1;
    lp.rows = f->nx;
    lp.cols = (int64_t)f->ny * f->nz;
  }
  *pix_stride = g.n_los;
  return hip_status(iris::launch_layout(lp, stream), "layout kernel");
}

}  // namespace

extern "C" {

const char* iris_version(void) { return "iris-rt-mi355x 0.1 (gfx950)"; }
int32_t iris_max_channels(void) { return iris::kMaxChannels; }

const char* iris_status_string(iris_status s) {
  switch (s) {
    case IRIS_OK: return "ok";
    case IRIS_E_INVALID_ARG: return "invalid argument";
    case IRIS_E_UNSUPPORTED: return "unsupported";
    case IRIS_E_WORKSPACE: return "workspace too small";
    case IRIS_E_HIP: return "HIP error";
  }
  return "unknown status";
}

const char* iris_last_error(void) { return g_err.c_str(); }

size_t iris_rt_layout_bytes(const iris_fields* fields) {
  Geo g;
  if (check_fields(fields, &g) != IRIS_OK) return 0;
  return (size_t)g.n_fields * g.n_cells * elem_size(fields->dtype);
}

iris_status iris_rt_layout(const iris_fields* f, void* dst, size_t dst_bytes, void* stream) {
  g_err.clear();
  Geo g;
  iris_status s = check_fields(f, &g);
  if (s != IRIS_OK) return s;
  const size_t need = (size_t)g.n_fields * g.n_cells * elem_size(f->dtype);
  if (!dst || dst_bytes < need)
    return fail(IRIS_E_WORKSPACE, "layout destination needs %zu bytes", need);
  if (f->axis == 2) {
    const void* src[5] = {f->ln_nh2, f->t_kin, f->v_los, f->x_tracer, f->t_dust};
    const size_t bytes = (size_t)g.n_cells * elem_size(f->dtype);
    for (int i = 0; i < g.n_fields; ++i) {
      const int e = (int)hipMemcpyAsync((char*)dst + i * bytes, src[i], bytes,
                                        hipMemcpyDeviceToDevice, (hipStream_t)stream);
      if (e) return hip_status(e, "hipMemcpyAsync");
    }
    return IRIS_OK;
  }
  WsLayout w;  // soa at offset 0 of dst
  const void* tmp[5];
  int64_t ps;
  return prepare_fields(f, g, w, dst, tmp, &ps, stream);
}

size_t iris_rt_workspace_bytes(const iris_fields* fields, const iris_channels* channels,
                               int32_t ckpt_K) {
  Geo g;
  if (check_fields(fields, &g) != IRIS_OK || check_channels(channels) != IRIS_OK ||
      !valid_K(ckpt_K))
    return 0;
  return ws_layout(fields, g, channels->n_chan, ckpt_K).total;
}

iris_status iris_rt_forward(const iris_fields* fields, const iris_channels* channels,
                            const iris_line* line, const iris_outputs* out, int32_t ckpt_K,
                            void* workspace, size_t workspace_bytes, void* stream) {
  g_err.clear();
  Geo g;
  iris_status s;
  if ((s = check_fields(fields, &g)) != IRIS_OK) return s;
  if ((s = check_channels(channels)) != IRIS_OK) return s;
  if ((s = check_line(line)) != IRIS_OK) return s;
  if (!out) return fail(IRIS_E_INVALID_ARG, "outputs is NULL");
  if (!valid_K(ckpt_K)) return fail(IRIS_E_INVALID_ARG, "ckpt_K %d not in {0,8,16,32,64}", ckpt_K);
  const WsLayout w = ws_layout(fields, g, channels->n_chan, ckpt_K);
  if (w.total > 0 && (!workspace || workspace_bytes < w.total))
    return fail(IRIS_E_WORKSPACE, "workspace needs %zu bytes, got %zu", w.total, workspace_bytes);

  iris::FwdParams p{};
  if ((s = prepare_fields(fields, g, w, workspace, p.f, &p.pix_stride, stream)) != IRIS_OK) return s;
  p.los_stride = 1;
  p.n_pix = (int32_t)g.n_pix;
  p.n_los = (int32_t)g.n_los;
  p.c = fold(fields, channels, line);
  p.out[0] = out->T;
  p.out[1] = out->C;
  p.out[2] = out->D;
  p.out[3] = out->L;
  p.out[4] = out->B;
  p.ckpt_K = ckpt_K;
  p.lds_per_wave = channels->n_chan + 64;
  if (ckpt_K > 0) {
    p.ck_state = (float*)((char*)workspace + w.ck_state);
    p.ck_scal = (double*)((char*)workspace + w.ck_scal);
  }
  return hip_status(iris::launch_forward(fields->dtype, p, stream), "forward kernel");
}

iris_status iris_rt_adjoint(const iris_fields* fields, const iris_channels* channels,
                            const iris_line* line, const iris_cotangents* cot, int32_t ckpt_K,
                            void* workspace, size_t workspace_bytes, const iris_gradients* grads,
                            void* stream) {
  g_err.clear();
  Geo g;
  iris_status s;
  if ((s = check_fields(fields, &g)) != IRIS_OK) return s;
  if ((s = check_channels(channels)) != IRIS_OK) return s;
  if ((s = check_line(line)) != IRIS_OK) return s;
  if (!cot) return fail(IRIS_E_INVALID_ARG, "cotangents is NULL");
  if (!grads || !grads->g_ln_nh2 || !grads->g_t_kin || !grads->g_v_los || !grads->g_x_tracer)
    return fail(IRIS_E_INVALID_ARG, "a gradient pointer is NULL");
  if (fields->t_dust && !grads->g_t_dust)
    return fail(IRIS_E_INVALID_ARG, "g_t_dust is NULL while t_dust is given");
  if (!valid_K(ckpt_K) || ckpt_K == 0)
    return fail(IRIS_E_INVALID_ARG, "adjoint needs ckpt_K in {8,16,32,64}");
  const WsLayout w = ws_layout(fields, g, channels->n_chan, ckpt_K);
  if (!workspace || workspace_bytes < w.total)
    return fail(IRIS_E_WORKSPACE, "workspace needs %zu bytes, got %zu", w.total, workspace_bytes);
  if (fields->t_dust || line->energy_mode != 0)
    return fail(IRIS_E_UNSUPPORTED,
                "adjoint is built for T_dust = T_kin and energy_mode 0 (line and dust share "
                "one source function)");

  iris::AdjParams p{};
  // The forward already laid the fields out in the workspace (axis 0/1).
  const void* src[5] = {fields->ln_nh2, fields->t_kin, fields->v_los, fields->x_tracer, nullptr};
  const size_t es = elem_size(fields->dtype);
  for (int i = 0; i < 4; ++i)
    p.f[i] = fields->axis == 2 ? src[i] : (const void*)((char*)workspace + w.soa + i * g.n_cells * es);
  p.f[4] = nullptr;
  p.pix_stride = g.n_los;
  p.los_stride = 1;
  p.n_pix = (int32_t)g.n_pix;
  p.n_los = (int32_t)g.n_los;
  p.c = fold(fields, channels, line);
  p.cot[0] = cot->gT;
  p.cot[1] = cot->gC;
  p.cot[2] = cot->gD;
  p.cot[3] = cot->gL;
  p.cot[4] = cot->gB;
  p.ckpt_K = ckpt_K;
  const int C = channels->n_chan;
  p.chan_stride = ((C + 64) + 1) & ~1;
  p.tape_passes = ckpt_K + (C + 63) / 64 + 1;
  p.lds_per_wave = 2 * p.chan_stride + 64 * p.tape_passes + 64 * 5 * 2;
  const size_t lds_block = (size_t)iris::adjoint_waves_per_block() * p.lds_per_wave * 4;
  if (lds_block > 65536)
    return fail(IRIS_E_UNSUPPORTED, "adjoint needs %zu bytes of LDS per workgroup (n_chan %d, K %d)",
                lds_block, C, ckpt_K);
  p.ck_state = (const float*)((char*)workspace + w.ck_state);
  p.ck_scal = (const double*)((char*)workspace + w.ck_scal);
  double* gsoa[4];
  if (fields->axis == 2) {
    gsoa[0] = grads->g_ln_nh2;
    gsoa[1] = grads->g_t_kin;
    gsoa[2] = grads->g_v_los;
    gsoa[3] = grads->g_x_tracer;
  } else {
    for (int i = 0; i < 4; ++i) gsoa[i] = (double*)((char*)workspace + w.grad) + i * g.n_cells;
  }
  for (int i = 0; i < 4; ++i) p.grad[i] = gsoa[i];
  p.grad[4] = nullptr;
  p.g_pix_stride = g.n_los;
  p.g_los_stride = 1;
  if ((s = hip_status(iris::launch_adjoint(fields->dtype, p, stream), "adjoint kernel")) != IRIS_OK)
    return s;
  if (fields->axis == 2) return IRIS_OK;
  // Sightline-major -> native layout: the inverse of the ingest transpose.
  iris::LayoutParams lp{};
  double* dst[4] = {grads->g_ln_nh2, grads->g_t_kin, grads->g_v_los, grads->g_x_tracer};
  for (int i = 0; i < 4; ++i) {
    lp.src[i] = gsoa[i];
    lp.dst[i] = dst[i];
  }
  lp.n_fields = 4;
  lp.elem = 8;
  if (fields->axis == 1) {
    lp.batch = fields->nx;
    lp.rows = fields->nz;
    lp.cols = fields->ny;
  } else {
    lp.batch = 1;
    lp.rows = (int64_t)fields->ny * fields->nz;
    lp.cols = fields->nx;
  }
  return hip_status(iris::launch_layout(lp, stream), "gradient layout kernel");
}

}  // extern "C"
