// C-ABI entry points of the single-cube path: validation, then the layout,
// forward march and adjoint launches on the caller's stream.

#include <hip/hip_runtime.h>

#include "host_common.h"

using namespace iris::host;

namespace iris {
namespace host {

// Reverse mode of optically thin transfer: no checkpoints (nothing is
// marched), so it rebuilds its tables in the workspace and reads the fields
// in place; `groups` 0 takes the forward's packing.
static iris_status thin_adjoint_impl(const iris_fields* fields, const Geo& g,
                                     const iris_channels* channels, const iris_line* line,
                                     const iris_cotangents* cot, int32_t ckpt_K, void* workspace,
                                     size_t workspace_bytes, const iris_gradients* grads,
                                     void* stream, int groups) {
  if (ckpt_K != 0)
    return fail(IRIS_E_INVALID_ARG, "optically thin transfer takes no checkpoints: ckpt_K must be 0");
  if (line->units == IRIS_UNITS_TB)
    return fail(IRIS_E_UNSUPPORTED, "adjoint is built for T_RJ and intensity units");
  const WsLayout w = ws_layout(fields, g, channels->n_chan, 0);
  if (!workspace || workspace_bytes < w.total)
    return fail(IRIS_E_WORKSPACE, "workspace needs %zu bytes, got %zu", w.total, workspace_bytes);
  AdjParams p{};
  p.c = fold(fields, channels, line);
  if (!groups) groups = thin_groups(p.c, channels->n_chan, false);
  while (groups > 1 && thin_adj_lds_bytes(channels->n_chan, groups) > 65536) groups /= 2;
  if (!groups || thin_adj_lds_bytes(channels->n_chan, groups) > 65536)
    return fail(IRIS_E_UNSUPPORTED, "n_chan %d needs more LDS than a workgroup has",
                channels->n_chan);
  void* tab = (char*)workspace + w.tab;
  iris_status s;
  if ((s = hip_status(launch_pop_table(tab_params(line), tab, stream), "table kernel")) != IRIS_OK)
    return s;
  p.c.tab = tab;
  const void* fsl[5] = {fields->ln_nh2, fields->t_kin, fields->v_los, fields->x_tracer,
                        fields->t_dust};
  for (int i = 0; i < 5; ++i) p.f[i] = fsl[i];
  p.at = native_addr(fields, g);
  p.gat = p.at;
  p.n_pix = (int32_t)g.n_pix;
  p.n_los = (int32_t)g.n_los;
  p.cot[0] = cot->gT;
  p.cot[1] = cot->gC;
  p.cot[2] = cot->gD;
  p.cot[3] = cot->gL;
  p.cot[4] = cot->gB;
  p.grad[0] = grads->g_ln_nh2;
  p.grad[1] = grads->g_t_kin;
  p.grad[2] = grads->g_v_los;
  p.grad[3] = grads->g_x_tracer;
  p.grad[4] = fields->t_dust ? grads->g_t_dust : nullptr;
  p.dtype = (int32_t)fields->dtype;
  p.groups = groups;
  return hip_status(launch_thin_adjoint(p, line->integrator == IRIS_INTEGRATOR_SMOOTH, groups,
                                        (char*)workspace + w.erfc, stream),
                    "thin adjoint kernel");
}

iris_status adjoint_impl(const iris_fields* fields, const iris_channels* channels,
                         const iris_line* line, const iris_cotangents* cot, int32_t ckpt_K,
                         void* workspace, size_t workspace_bytes, const iris_gradients* grads,
                         void* stream, int groups) {
  Geo g;
  iris_status s;
  if ((s = check_fields(fields, &g)) != IRIS_OK) return s;
  if ((s = check_channels(channels)) != IRIS_OK) return s;
  if ((s = check_line(line)) != IRIS_OK) return s;
  const iris_channels mg = march_channels(channels);
  channels = &mg;
  if (!cot) return fail(IRIS_E_INVALID_ARG, "cotangents is NULL");
  if (!grads || !grads->g_ln_nh2 || !grads->g_t_kin || !grads->g_v_los || !grads->g_x_tracer)
    return fail(IRIS_E_INVALID_ARG, "a gradient pointer is NULL");
  if (fields->t_dust && !grads->g_t_dust)
    return fail(IRIS_E_INVALID_ARG, "g_t_dust is NULL while t_dust is given");
  if (line->transfer == IRIS_TRANSFER_THIN)
    return thin_adjoint_impl(fields, g, channels, line, cot, ckpt_K, workspace, workspace_bytes,
                             grads, stream, groups);
  if (!valid_K(ckpt_K) || ckpt_K == 0)
    return fail(IRIS_E_INVALID_ARG, "adjoint needs ckpt_K in {8,16,32,64}");
  const WsLayout w = ws_layout(fields, g, channels->n_chan, ckpt_K);
  if (!workspace || workspace_bytes < w.total)
    return fail(IRIS_E_WORKSPACE, "workspace needs %zu bytes, got %zu", w.total, workspace_bytes);
  if (line->units == IRIS_UNITS_TB)
    return fail(IRIS_E_UNSUPPORTED, "adjoint is built for T_RJ and intensity units");
  if (line->integrator != IRIS_INTEGRATOR_FORMAL)
    return fail(IRIS_E_UNSUPPORTED, "adjoint is built for the formal step");
  if (line->transfer != IRIS_TRANSFER_THICK)
    return fail(IRIS_E_UNSUPPORTED, "adjoint is built for optically thick transfer");

  // The forward wrote the temperature tables and, unless the fields are read
  // in place, their sightline-major copy into the workspace.
  const size_t es = elem_size(fields->dtype);
  const bool in_place = reads_in_place(fields);
  const void* fsl[5] = {fields->ln_nh2, fields->t_kin, fields->v_los, fields->x_tracer,
                        fields->t_dust};
  if (!in_place)
    for (int i = 0; i < g.n_fields; ++i) fsl[i] = (char*)workspace + w.soa + i * g.n_cells * es;
  const iris::SightAddr at = in_place ? native_addr(fields, g) : sightline_major_addr(g);
  const int C = channels->n_chan;
  const iris::Folded fc = fold(fields, channels, line);
  const bool gen = fc.general != 0;  // separate line and dust source functions
  if (groups ? !adjoint_fits(C, ckpt_K, groups, gen)
             : adjoint_groups(fields, channels, line, fc, ckpt_K) == 0)
    return fail(IRIS_E_UNSUPPORTED, "adjoint needs %zu bytes of LDS per workgroup (n_chan %d, K %d)",
                (size_t)adj_lds_floats(C, ckpt_K, groups ? groups : 1, gen) * 4, C, ckpt_K);
  double* gsoa[5] = {grads->g_ln_nh2, grads->g_t_kin, grads->g_v_los, grads->g_x_tracer,
                     fields->t_dust ? grads->g_t_dust : nullptr};
  if (!in_place)
    for (int i = 0; i < g.n_fields; ++i)
      gsoa[i] = (double*)((char*)workspace + w.grad) + i * g.n_cells;
  const iris::AdjParams p =
      adj_params(fields, g, channels, line, cot, ckpt_K, fsl, at, (char*)workspace + w.tab,
                 (const float*)((char*)workspace + w.ck_state),
                 (const double*)((char*)workspace + w.ck_scal), gsoa, at, groups);
  if ((s = hip_status(iris::launch_adjoint(fields->dtype, p, stream), "adjoint kernel")) != IRIS_OK)
    return s;
  if (in_place) return IRIS_OK;
  // Sightline-major -> native layout: the inverse of the ingest transpose.
  double* dst[5] = {grads->g_ln_nh2, grads->g_t_kin, grads->g_v_los, grads->g_x_tracer,
                    fields->t_dust ? grads->g_t_dust : nullptr};
  return hip_status(iris::launch_layout(gradient_layout(fields, g, gsoa, dst), stream),
                    "gradient layout kernel");
}

}  // namespace host
}  // namespace iris

extern "C" {

const char* iris_version(void) { return "iris-rt-mi355x 0.1 (gfx950)"; }
int32_t iris_max_channels(void) { return iris::kMaxChannels; }
int32_t iris_smooth_max_channels(void) { return iris::smooth_max_channels(); }

const char* iris_status_string(iris_status s) {
  switch (s) {
    case IRIS_OK: return "ok";
    case IRIS_E_INVALID_ARG: return "invalid argument";
    case IRIS_E_UNSUPPORTED: return "unsupported";
    case IRIS_E_WORKSPACE: return "workspace too small";
    case IRIS_E_HIP: return "HIP error";
    case IRIS_E_NONFINITE: return "non-finite or out-of-range field values";
  }
  return "unknown status";
}

const char* iris_last_error(void) { return last_error(); }

size_t iris_rt_layout_bytes(const iris_fields* fields) {
  Geo g;
  if (check_fields(fields, &g) != IRIS_OK) return 0;
  return (size_t)g.n_fields * g.n_cells * elem_size(fields->dtype);
}

iris_status iris_rt_layout(const iris_fields* f, void* dst, size_t dst_bytes, void* stream) {
  clear_error();
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
  return hip_status(iris::launch_layout(field_layout(f, g, dst), stream), "layout kernel");
}

size_t iris_rt_workspace_bytes(const iris_fields* fields, const iris_channels* channels,
                               int32_t ckpt_K) {
  Geo g;
  if (check_fields(fields, &g) != IRIS_OK || check_channels(channels) != IRIS_OK ||
      !valid_K(ckpt_K))
    return 0;
  return ws_layout(fields, g, march_channels(channels).n_chan, ckpt_K).total;
}

iris_status iris_rt_forward(const iris_fields* fields, const iris_channels* channels,
                            const iris_line* line, const iris_outputs* out, int32_t ckpt_K,
                            void* workspace, size_t workspace_bytes, void* stream) {
  clear_error();
  return forward_impl(fields, channels, line, out, ckpt_K, workspace, workspace_bytes, stream, 0);
}

iris_status iris_rt_adjoint(const iris_fields* fields, const iris_channels* channels,
                            const iris_line* line, const iris_cotangents* cot, int32_t ckpt_K,
                            void* workspace, size_t workspace_bytes, const iris_gradients* grads,
                            void* stream) {
  clear_error();
  return adjoint_impl(fields, channels, line, cot, ckpt_K, workspace, workspace_bytes, grads,
                      stream, 0);
}

iris_status iris_rt_autotune_adjoint(const iris_fields* fields, const iris_channels* channels,
                                     const iris_line* line, const iris_cotangents* cot,
                                     int32_t ckpt_K, void* workspace, size_t workspace_bytes,
                                     const iris_gradients* grads, void* stream, int32_t* groups) {
  clear_error();
  if (!groups) return fail(IRIS_E_INVALID_ARG, "groups is NULL");
  // Validation (and the class's LDS limits) by one call with the current choice.
  iris_status s = adjoint_impl(fields, channels, line, cot, ckpt_K, workspace, workspace_bytes,
                               grads, stream, 0);
  if (s != IRIS_OK) return s;
  const iris_channels mg = march_channels(channels);
  const iris::Folded c = fold(fields, &mg, line);
  const hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  s = hip_status(hipEventCreate(&e0), "hipEventCreate");
  if (s == IRIS_OK) s = hip_status(hipEventCreate(&e1), "hipEventCreate");
  float best_ms = 1e30f;
  int best = 0;
  constexpr int kReps = 3;
  for (int g : {1, 2, 4}) {
    if (s != IRIS_OK) break;
    if (!adjoint_fits(mg.n_chan, ckpt_K, g, c.general != 0)) continue;
    s = adjoint_impl(fields, channels, line, cot, ckpt_K, workspace, workspace_bytes, grads,
                     stream, g);  // untimed
    if (s == IRIS_OK) s = hip_status(hipEventRecord(e0, st), "hipEventRecord");
    for (int r = 0; r < kReps && s == IRIS_OK; ++r)
      s = adjoint_impl(fields, channels, line, cot, ckpt_K, workspace, workspace_bytes, grads,
                       stream, g);
    if (s == IRIS_OK) s = hip_status(hipEventRecord(e1, st), "hipEventRecord");
    if (s == IRIS_OK) s = hip_status(hipEventSynchronize(e1), "hipEventSynchronize");
    float ms = 0.f;
    if (s == IRIS_OK) s = hip_status(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
    if (s == IRIS_OK && ms < best_ms) {
      best_ms = ms;
      best = g;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s != IRIS_OK) return s;
  record_adjoint_groups(fields, &mg, line, c, ckpt_K, best);
  s = adjoint_impl(fields, channels, line, cot, ckpt_K, workspace, workspace_bytes, grads, stream,
                   best);
  if (s == IRIS_OK) s = hip_status(hipStreamSynchronize(st), "hipStreamSynchronize");
  if (s == IRIS_OK) *groups = best;
  return s;
}

}  // extern "C"
