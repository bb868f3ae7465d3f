// Batched plans and the sightline-packing autotuner.
//
// A plan turns a list of cubes of uneven shape, sightline axis, storage type
// and channel grid into one persistent launch per phase. The work is a queue
// of items (one wavefront's sightlines of one cube) ordered by decreasing
// estimated cost, so the longest sightlines start first and the tail of the
// launch is made of short ones. Each phase is captured once in a hipGraph:
//   forward: reset queue head -> batched field transpose -> persistent march
//   adjoint: reset queue heads -> persistent reverse marches, one after
//            another -> batched gradient transpose
// The queue heads are cleared by a one-wave kernel, not a memset node.
//
// The smooth integrator and the thin transfer modes have no persistent
// variant: their plans capture the single-cube forward of every cube, in
// order, into the forward graph (forward only, no autotuning).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <limits>
#include <vector>

#include "host_common.h"

using namespace iris;
using namespace iris::host;

namespace {

// Time the forward march with 1, 2 and 4 sightlines per wavefront on this
// cube and keep the fastest. Leaves the outputs of the chosen variant.
iris_status tune_cube(const iris_fields* f, const iris_channels* ch, const iris_line* L,
                      const iris_outputs* out, void* ws, size_t ws_bytes, hipStream_t stream,
                      int* best) {
  const iris_channels mg = march_channels(ch);  // `ch` itself goes to forward_impl
  const Folded c = fold(f, &mg, L);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  iris_status s = hip_status(hipEventCreate(&e0), "hipEventCreate");
  if (s == IRIS_OK) s = hip_status(hipEventCreate(&e1), "hipEventCreate");
  float best_ms = std::numeric_limits<float>::infinity();
  int bg = 0;
  constexpr int kReps = 3;
  for (int g : {1, 2, 4}) {
    if (s != IRIS_OK) break;
    if (!groups_fit(mg.n_chan, g, c.general != 0)) continue;
    // One untimed call (first-touch and instruction-cache warm-up).
    s = forward_impl(f, ch, L, out, 0, ws, ws_bytes, stream, g);
    if (s == IRIS_OK) s = hip_status(hipEventRecord(e0, stream), "hipEventRecord");
    for (int r = 0; r < kReps && s == IRIS_OK; ++r)
      s = forward_impl(f, ch, L, out, 0, ws, ws_bytes, stream, g);
    if (s == IRIS_OK) s = hip_status(hipEventRecord(e1, stream), "hipEventRecord");
    if (s == IRIS_OK) s = hip_status(hipEventSynchronize(e1), "hipEventSynchronize");
    float ms = 0.f;
    if (s == IRIS_OK) s = hip_status(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
    if (s == IRIS_OK && ms < best_ms) {
      best_ms = ms;
      bg = g;
    }
  }
  if (s == IRIS_OK && bg == 0)
    s = fail(IRIS_E_UNSUPPORTED, "n_chan %d needs more LDS than a workgroup has", mg.n_chan);
  if (s == IRIS_OK) {
    record_groups(f, &mg, L, c, bg);
    s = forward_impl(f, ch, L, out, 0, ws, ws_bytes, stream, bg);
    if (s == IRIS_OK) s = hip_status(hipStreamSynchronize(stream), "hipStreamSynchronize");
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s == IRIS_OK) *best = bg;
  return s;
}

// Checkpoint interval of an adjoint plan chosen by timing: the forward with
// checkpoints and the adjoint, at K = 8, 16, 32 and 64, on the cube with the
// most cells (its outputs and gradients are written). Only intervals at which
// every cube's adjoint fits in LDS are tried.
iris_status tune_ckpt_K(const iris_cube* cubes, int n, const iris_line* L, hipStream_t stream,
                        int* best) {
  iris_status s;
  int big = 0;
  int64_t big_cells = -1;
  for (int i = 0; i < n; ++i) {
    Geo g;
    if ((s = check_fields(&cubes[i].fields, &g)) != IRIS_OK)
      return fail(s, "cube %d: %s", i, last_error());
    if ((s = check_channels(&cubes[i].channels)) != IRIS_OK)
      return fail(s, "cube %d: %s", i, last_error());
    if (g.n_cells > big_cells) {
      big_cells = g.n_cells;
      big = i;
    }
  }
  const iris_cube& cb = cubes[big];
  Geo gb;
  (void)check_fields(&cb.fields, &gb);
  const size_t ws_bytes = ws_layout(&cb.fields, gb, march_channels(&cb.channels).n_chan, 8).total;
  void* ws = nullptr;
  if ((s = hip_status(hipMalloc(&ws, ws_bytes), "hipMalloc (checkpoint tuning)")) != IRIS_OK)
    return s;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  s = hip_status(hipEventCreate(&e0), "hipEventCreate");
  if (s == IRIS_OK) s = hip_status(hipEventCreate(&e1), "hipEventCreate");
  float best_ms = std::numeric_limits<float>::infinity();
  int bk = 0;
  for (int K : {8, 16, 32, 64}) {
    if (s != IRIS_OK) break;
    bool fits = true;
    for (int i = 0; i < n && fits; ++i) {
      const iris_channels mg = march_channels(&cubes[i].channels);
      fits = adjoint_groups(&cubes[i].fields, &mg, L, fold(&cubes[i].fields, &mg, L), K) > 0;
    }
    if (!fits) continue;
    auto step = [&]() {
      iris_status r = forward_impl(&cb.fields, &cb.channels, L, &cb.out, K, ws, ws_bytes,
                                   stream, 0);
      if (r == IRIS_OK)
        r = adjoint_impl(&cb.fields, &cb.channels, L, &cb.cot, K, ws, ws_bytes, &cb.grads,
                         stream, 0);
      return r;
    };
    s = step();  // untimed
    if (s == IRIS_OK) s = hip_status(hipEventRecord(e0, stream), "hipEventRecord");
    for (int r = 0; r < 2 && s == IRIS_OK; ++r) s = step();
    if (s == IRIS_OK) s = hip_status(hipEventRecord(e1, stream), "hipEventRecord");
    if (s == IRIS_OK) s = hip_status(hipEventSynchronize(e1), "hipEventSynchronize");
    float ms = 0.f;
    if (s == IRIS_OK) s = hip_status(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
    if (s == IRIS_OK && ms < best_ms) {
      best_ms = ms;
      bk = K;
    }
  }
  (void)hipStreamSynchronize(stream);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(ws);
  if (s == IRIS_OK && bk == 0)
    s = fail(IRIS_E_UNSUPPORTED, "no checkpoint interval fits every cube's adjoint in LDS");
  if (s != IRIS_OK) return fail(s, "checkpoint tuning on cube %d: %s", big, last_error());
  *best = bk;
  return IRIS_OK;
}

// Work estimate of one item: per cell, the setup and the channel passes.
double item_cost(const Geo& g, int n_chan, int lanes) {
  return (double)g.n_los * (8.0 + (double)n_chan / lanes);
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

}  // namespace

struct iris_plan {
  int device = 0;
  int flags = 0;
  int K = 0;
  std::vector<int> groups;
  std::vector<int> adj_groups;  // adjoint packing per cube (empty without IRIS_PLAN_ADJOINT)
  void* mem = nullptr;
  hipStream_t cap = nullptr;        // capture stream
  hipStream_t side[2] = {nullptr, nullptr};  // concurrent branches of the forward graph
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
  hipGraph_t graph_fwd = nullptr, graph_adj = nullptr;
  hipGraphExec_t exec_fwd = nullptr, exec_adj = nullptr;
  iris_plan_info info{};

  ~iris_plan() {
    if (exec_fwd) (void)hipGraphExecDestroy(exec_fwd);
    if (exec_adj) (void)hipGraphExecDestroy(exec_adj);
    if (graph_fwd) (void)hipGraphDestroy(graph_fwd);
    if (graph_adj) (void)hipGraphDestroy(graph_adj);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    for (hipStream_t st : side)
      if (st) (void)hipStreamDestroy(st);
    if (cap) (void)hipStreamDestroy(cap);
    if (mem) {
      (void)hipDeviceSynchronize();
      (void)hipFree(mem);
    }
  }
};

namespace {

// Region bookkeeping for the plan's single allocation.
struct Carver {
  size_t off = 0;
  size_t take(size_t bytes) {
    const size_t o = off;
    off += align256(bytes);
    return o;
  }
};

// A persistent launch's queue: the items of the cubes `ids` (sightlines
// per item `per`), in kSlices slices; slice x holds the x-th contiguous
// share of every cube's items, cubes in decreasing per-item cost.
struct Queue {
  std::vector<WorkItem> items;
  int32_t begin[kSlices + 1] = {};
  double work = 0.0;  // estimated cost of all items
};

Queue build_queue(std::vector<int> ids, const std::vector<Geo>& geo,
                  const std::vector<double>& item_cost_of, int per) {
  std::stable_sort(ids.begin(), ids.end(),
                   [&](int a, int b) { return item_cost_of[a] > item_cost_of[b]; });
  Queue q;
  for (int x = 0; x < kSlices; ++x) {
    q.begin[x] = (int32_t)q.items.size();
    for (int i : ids) {
      const int64_t n = (geo[i].n_pix + per - 1) / per;
      const int64_t lo = n * x / kSlices, hi = n * (x + 1) / kSlices;
      for (int64_t k = lo; k < hi; ++k) q.items.push_back({i, (int32_t)(k * per)});
    }
  }
  q.begin[kSlices] = (int32_t)q.items.size();
  for (int i : ids) q.work += item_cost_of[i] * (double)((geo[i].n_pix + per - 1) / per);
  return q;
}

// Grid of a persistent launch: a multiple of kSlices workgroups (so that
// each slice has the same number of home workgroups), at most what stays
// resident (`cap`) and what the queue can use.
int persistent_grid(int64_t cap, int64_t items, int waves_per_block) {
  const int64_t need = (items + waves_per_block - 1) / waves_per_block;
  int64_t g = std::min(cap, need);
  g = std::max<int64_t>(kSlices, (g + kSlices - 1) / kSlices * kSlices);
  return (int)g;
}

iris_status build_plan(const iris_cube* cubes, int n, const iris_line* L, int flags, int K,
                       hipStream_t user_stream, iris_plan* P) {
  iris_status s;
  const bool adj = (flags & IRIS_PLAN_ADJOINT) != 0;
  P->flags = flags;
  if (adj && K == 0) {
    for (int i = 0; i < n; ++i)
      if (!cubes[i].grads.g_ln_nh2 || !cubes[i].grads.g_t_kin || !cubes[i].grads.g_v_los ||
          !cubes[i].grads.g_x_tracer)
        return fail(IRIS_E_INVALID_ARG, "cube %d: a gradient pointer is NULL", i);
    if ((s = tune_ckpt_K(cubes, n, L, user_stream, &K)) != IRIS_OK) return s;
  }
  P->K = adj ? K : 0;
  // 1. Validate every cube; choose its sightline packing.
  std::vector<Geo> geo(n);
  std::vector<WsLayout> wl(n);
  std::vector<Folded> folded(n);
  std::vector<iris_channels> mch(n);  // the grids the marches run on
  P->groups.assign(n, 1);
  for (int i = 0; i < n; ++i) {
    const iris_cube& cb = cubes[i];
    if ((s = check_fields(&cb.fields, &geo[i])) != IRIS_OK)
      return fail(s, "cube %d: %s", i, last_error());
    if ((s = check_channels(&cb.channels)) != IRIS_OK)
      return fail(s, "cube %d: %s", i, last_error());
    mch[i] = march_channels(&cb.channels);
    folded[i] = fold(&cb.fields, &mch[i], L);
    if (adj) {
      const iris_gradients& gr = cb.grads;
      if (!gr.g_ln_nh2 || !gr.g_t_kin || !gr.g_v_los || !gr.g_x_tracer)
        return fail(IRIS_E_INVALID_ARG, "cube %d: a gradient pointer is NULL", i);
      if (cb.fields.t_dust && !gr.g_t_dust)
        return fail(IRIS_E_INVALID_ARG, "cube %d: g_t_dust is NULL while t_dust is given", i);
      if (L->units == IRIS_UNITS_TB)
        return fail(IRIS_E_UNSUPPORTED, "adjoint is built for T_RJ and intensity units");
      if (adjoint_groups(&cb.fields, &mch[i], L, folded[i], K, true) == 0)
        return fail(IRIS_E_UNSUPPORTED, "cube %d: adjoint needs %zu bytes of LDS (n_chan %d, K %d)",
                    i,
                    (size_t)adj_lds_floats(mch[i].n_chan, K, 1, folded[i].general != 0) *
                        sizeof(float),
                    mch[i].n_chan, K);
    }
    P->groups[i] = choose_groups(&cb.fields, &mch[i], L, folded[i]);
    if (!groups_fit(mch[i].n_chan, P->groups[i], folded[i].general != 0))
      return fail(IRIS_E_UNSUPPORTED, "cube %d: n_chan %d needs more LDS than a workgroup has", i,
                  mch[i].n_chan);
    wl[i] = ws_layout(&cb.fields, geo[i], mch[i].n_chan, P->K);
  }

  if ((s = hip_status(hipGetDevice(&P->device), "hipGetDevice")) != IRIS_OK) return s;

  // 1b. Optional autotuning, one timing per class, in a temporary
  //     single-cube workspace (writes the cubes' outputs). The adjoint's
  //     packing is not tuned here: timed cube by cube it chose packings that
  //     ran slower together in the plan's launches than the plan rule's.
  if (flags & IRIS_PLAN_AUTOTUNE) {
    size_t ws_max = 0;
    for (int i = 0; i < n; ++i)
      ws_max = std::max(ws_max, ws_layout(&cubes[i].fields, geo[i], mch[i].n_chan, 0).total);
    void* tmp = nullptr;
    if ((s = hip_status(hipMalloc(&tmp, ws_max), "hipMalloc (autotune workspace)")) != IRIS_OK)
      return s;
    std::vector<int> tuned(n, 0);
    for (int i = 0; i < n && s == IRIS_OK; ++i) {
      int g = 0;
      for (int j = 0; j < i && !g; ++j)
        if (mch[j].n_chan == mch[i].n_chan && mch[j].dv_kms == mch[i].dv_kms &&
            cubes[j].fields.dtype == cubes[i].fields.dtype && geo[j].n_los == geo[i].n_los &&
            folded[j].general == folded[i].general)
          g = tuned[j];
      if (!g) {
        iris_outputs o = cubes[i].out;
        s = tune_cube(&cubes[i].fields, &cubes[i].channels, L, &o, tmp, ws_max, user_stream, &g);
        if (s != IRIS_OK) s = fail(s, "cube %d: autotune: %s", i, last_error());
      }
      tuned[i] = g;
      P->groups[i] = g;
    }
    (void)hipStreamSynchronize(user_stream);
    (void)hipFree(tmp);
    if (s != IRIS_OK) return s;
  }

  // 2. Queues: one forward launch per sightline packing present. The
  //    adjoint's LDS per wavefront grows with the channel count and sets how
  //    many wavefronts stay resident (its reverse march is latency-bound, so
  //    residency is its speed): one adjoint launch per (packing, resident
  //    wavefronts per CU) present, each sized for its own cubes rather than
  //    for the largest cube of its packing.
  static constexpr int kPackings[3] = {1, 2, 4};
  Queue fq[3];
  std::vector<int> agroups(n, 1);
  for (int i = 0; i < n; ++i)
    if (adj) agroups[i] = adjoint_groups(&cubes[i].fields, &mch[i], L, folded[i], K, true);
  if (adj) P->adj_groups = agroups;
  struct AdjClass {
    int groups, occupancy;
    bool general;  // separate line and dust source functions
    std::vector<int> ids;
    Queue q;
    int wave_floats = 0;
  };
  std::vector<AdjClass> acl;
  for (int i = 0; i < n && adj; ++i) {
    const bool gen = folded[i].general != 0;
    const int wf = adj_lds_floats(mch[i].n_chan, K, agroups[i], gen);
    const int occ = plan_adjoint_occupancy(wf, agroups[i], gen);
    auto it = std::find_if(acl.begin(), acl.end(), [&](const AdjClass& a) {
      return a.groups == agroups[i] && a.occupancy == occ && a.general == gen;
    });
    if (it == acl.end()) {
      acl.push_back({agroups[i], occ, gen, {}, {}, 0});
      it = acl.end() - 1;
    }
    it->ids.push_back(i);
    it->wave_floats = std::max(it->wave_floats, wf);
  }
  std::vector<double> cost_f(n), cost_a(n);
  for (int i = 0; i < n; ++i) {
    cost_f[i] = item_cost(geo[i], mch[i].n_chan, 64 / P->groups[i]);
    cost_a[i] = item_cost(geo[i], mch[i].n_chan, 64 / agroups[i]);
  }
  for (int c = 0; c < 3; ++c) {
    std::vector<int> ids;
    for (int i = 0; i < n; ++i)
      if (P->groups[i] == kPackings[c]) ids.push_back(i);
    fq[c] = build_queue(ids, geo, cost_f, kPackings[c]);
  }
  for (AdjClass& a : acl) a.q = build_queue(a.ids, geo, cost_a, a.groups);
  const int n_acl = (int)acl.size();
  size_t n_fwd_items = 0, n_adj_items = 0;
  for (const Queue& q : fq) n_fwd_items += q.items.size();
  for (const AdjClass& a : acl) n_adj_items += a.q.items.size();
  if (n_fwd_items > (size_t)INT32_MAX || n_adj_items > (size_t)INT32_MAX)
    return fail(IRIS_E_UNSUPPORTED, "batch too large for one launch");

  // 3. Transpose jobs (fields in, gradients out) for cubes whose fields are
  //    not read in place.
  std::vector<TransposeJob> fjobs, gjobs;

  // 4. One allocation: tables, queue heads, descriptors, queues, jobs, then
  //    a single-cube workspace per cube (checkpoints; sightline-major copies
  //    where used).
  Carver cv;
  const size_t o_tab = cv.take(kTabBytes);
  const size_t o_ctr = cv.take((3 + (size_t)n_acl) * kSlices * sizeof(int));
  const size_t o_fwd = cv.take((size_t)n * sizeof(FwdParams));
  const size_t o_adj = adj ? cv.take((size_t)n * sizeof(AdjParams)) : 0;
  size_t o_fq[3];
  for (int c = 0; c < 3; ++c) o_fq[c] = cv.take(fq[c].items.size() * sizeof(WorkItem));
  std::vector<size_t> o_aq(n_acl);
  for (int c = 0; c < n_acl; ++c) o_aq[c] = cv.take(acl[c].q.items.size() * sizeof(WorkItem));
  int n_moved = 0;
  for (int i = 0; i < n; ++i) n_moved += !reads_in_place(&cubes[i].fields);
  const size_t o_fj = cv.take((size_t)n_moved * sizeof(TransposeJob));
  const size_t o_gj = adj ? cv.take((size_t)n_moved * sizeof(TransposeJob)) : 0;
  std::vector<size_t> o_ws(n);
  for (int i = 0; i < n; ++i) o_ws[i] = cv.take(wl[i].total);
  const size_t total = cv.off;
  if ((s = hip_status(hipMalloc(&P->mem, total), "hipMalloc (plan scratch)")) != IRIS_OK) {
    P->mem = nullptr;
    return s;
  }
  char* base = (char*)P->mem;
  const void* tab = base + o_tab;
  // [3 + n_acl][kSlices]: forward packings 1, 2, 4, then the adjoint classes.
  int* counters = (int*)(base + o_ctr);

  // 5. Per-cube kernel parameters.
  std::vector<FwdParams> fp(n);
  std::vector<AdjParams> ap(adj ? n : 0);
  int fwd_wave_floats[3] = {0, 0, 0};
  int64_t ftiles = 0, gtiles = 0;
  int64_t samples = 0;
  for (int i = 0; i < n; ++i) {
    const iris_cube& cb = cubes[i];
    const Geo& g = geo[i];
    char* ws = base + o_ws[i];
    const void* fsl[5] = {cb.fields.ln_nh2, cb.fields.t_kin, cb.fields.v_los, cb.fields.x_tracer,
                          cb.fields.t_dust};
    const bool in_place = reads_in_place(&cb.fields);
    const SightAddr at = in_place ? native_addr(&cb.fields, g) : sightline_major_addr(g);
    if (!in_place) {
      const LayoutParams lp = field_layout(&cb.fields, g, ws + wl[i].soa);
      TransposeJob j{};
      for (int k = 0; k < 5; ++k) {
        j.src[k] = lp.src[k];
        j.dst[k] = lp.dst[k];
        fsl[k] = k < g.n_fields ? lp.dst[k] : nullptr;
      }
      j.n_fields = lp.n_fields;
      j.elem = lp.elem;
      j.rows = lp.rows;
      j.cols = lp.cols;
      j.batch = lp.batch;
      j.tiles_r = (int32_t)((lp.rows + 63) / 64);
      j.tiles_c = (int32_t)((lp.cols + 63) / 64);
      j.tile_begin = ftiles;
      ftiles += lp.batch * j.tiles_r * j.tiles_c;
      fjobs.push_back(j);
    }
    float* ck_state = P->K ? (float*)(ws + wl[i].ck_state) : nullptr;
    double* ck_scal = P->K ? (double*)(ws + wl[i].ck_scal) : nullptr;
    fp[i] = fwd_params(&cb.fields, g, &mch[i], L, &cb.out, P->K, fsl, at, tab, ck_state,
                       ck_scal, P->groups[i]);
    const int c = P->groups[i] == 1 ? 0 : P->groups[i] == 2 ? 1 : 2;
    fwd_wave_floats[c] = std::max<int>(
        fwd_wave_floats[c],
        (int)(fwd_lds_bytes(mch[i].n_chan, P->groups[i], folded[i].general != 0) /
              (sizeof(float) * kWavesPerBlock)));
    samples += g.n_cells * cb.channels.n_chan;
    if (adj) {
      double* const gtd = cb.fields.t_dust ? cb.grads.g_t_dust : nullptr;
      double* gsoa[5] = {cb.grads.g_ln_nh2, cb.grads.g_t_kin, cb.grads.g_v_los,
                         cb.grads.g_x_tracer, gtd};
      if (!in_place) {
        for (int k = 0; k < g.n_fields; ++k)
          gsoa[k] = (double*)(ws + wl[i].grad) + k * g.n_cells;
        double* dst[5] = {cb.grads.g_ln_nh2, cb.grads.g_t_kin, cb.grads.g_v_los,
                          cb.grads.g_x_tracer, gtd};
        const LayoutParams lp = gradient_layout(&cb.fields, g, gsoa, dst);
        TransposeJob j{};
        for (int k = 0; k < lp.n_fields; ++k) {
          j.src[k] = lp.src[k];
          j.dst[k] = lp.dst[k];
        }
        j.n_fields = lp.n_fields;
        j.elem = 8;
        j.rows = lp.rows;
        j.cols = lp.cols;
        j.batch = lp.batch;
        j.tiles_r = (int32_t)((lp.rows + 63) / 64);
        j.tiles_c = (int32_t)((lp.cols + 63) / 64);
        j.tile_begin = gtiles;
        gtiles += lp.batch * j.tiles_r * j.tiles_c;
        gjobs.push_back(j);
      }
      ap[i] = adj_params(&cb.fields, g, &mch[i], L, &cb.cot, P->K, fsl, at, tab, ck_state,
                         ck_scal, gsoa, at, agroups[i]);
    }
  }
  if (ftiles > INT32_MAX || gtiles > INT32_MAX)
    return fail(IRIS_E_UNSUPPORTED, "batch too large for one launch");

  // 6. Upload descriptors and queues; build the temperature tables once (the
  //    line is fixed for the plan).
  struct Up {
    size_t off;
    const void* src;
    size_t bytes;
  };
  std::vector<Up> ups = {{o_fwd, fp.data(), fp.size() * sizeof(FwdParams)},
                         {o_adj, ap.data(), ap.size() * sizeof(AdjParams)},
                         {o_fq[0], fq[0].items.data(), fq[0].items.size() * sizeof(WorkItem)},
                         {o_fq[1], fq[1].items.data(), fq[1].items.size() * sizeof(WorkItem)},
                         {o_fq[2], fq[2].items.data(), fq[2].items.size() * sizeof(WorkItem)},
                         {o_fj, fjobs.data(), fjobs.size() * sizeof(TransposeJob)},
                         {o_gj, gjobs.data(), gjobs.size() * sizeof(TransposeJob)}};
  for (int c = 0; c < n_acl; ++c)
    ups.push_back({o_aq[c], acl[c].q.items.data(), acl[c].q.items.size() * sizeof(WorkItem)});
  for (const Up& u : ups)
    if (u.bytes && (s = hip_status(hipMemcpy(base + u.off, u.src, u.bytes, hipMemcpyHostToDevice),
                                   "hipMemcpy (plan descriptors)")) != IRIS_OK)
      return s;
  if ((s = hip_status(launch_pop_table(tab_params(L), base + o_tab, user_stream), "table kernel")) !=
      IRIS_OK)
    return s;
  if ((s = hip_status(hipStreamSynchronize(user_stream), "hipStreamSynchronize")) != IRIS_OK)
    return s;

  // 7. Persistent grids. The forward packings run as concurrent launches;
  //    each gets a share of the resident workgroups in proportion to its
  //    estimated work, so that they finish together.
  int n_cu = 0;
  if ((s = hip_status(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount,
                                            P->device),
                      "hipDeviceGetAttribute")) != IRIS_OK)
    return s;
  const bool ck = P->K > 0;
  double fwork = 0.0;
  for (const Queue& q : fq) fwork += q.work;
  PlanFwdParams qf[3] = {};
  int fwd_blocks[3] = {0, 0, 0};
  for (int c = 0; c < 3; ++c) {
    if (fq[c].items.empty()) continue;
    qf[c].cubes = (const FwdParams*)(base + o_fwd);
    qf[c].items = (const WorkItem*)(base + o_fq[c]);
    for (int x = 0; x <= kSlices; ++x) qf[c].slice_begin[x] = fq[c].begin[x];
    qf[c].wave_floats = fwd_wave_floats[c];
    qf[c].counter = counters + c * kSlices;
    const int64_t resident =
        (int64_t)plan_forward_occupancy(fwd_wave_floats[c], kPackings[c], ck) * n_cu;
    const double share = fwork > 0.0 ? fq[c].work / fwork : 1.0;
    fwd_blocks[c] = persistent_grid((int64_t)std::ceil(resident * share),
                                    (int64_t)fq[c].items.size(), kWavesPerBlock);
    // Static rounds only for a launch that runs alone with every workgroup
    // resident; concurrent branches start their workgroups unevenly.
    qf[c].static_rounds = (share == 1.0 && fwd_blocks[c] <= resident) ? 1 : 0;
  }

  // The adjoint classes run one after another, each over the whole GPU: as
  // concurrent branches sized by estimated work, the packings finished
  // several milliseconds apart on the 64-cube batch (the estimate cannot
  // follow the latency-bound reverse march's speed per class).
  std::vector<PlanAdjParams> qa(n_acl);
  std::vector<int> adj_blocks(n_acl, 0);
  int adj_blocks_total = 0;
  for (int c = 0; c < n_acl; ++c) {
    qa[c] = PlanAdjParams{};
    qa[c].cubes = (const AdjParams*)(base + o_adj);
    qa[c].items = (const WorkItem*)(base + o_aq[c]);
    for (int x = 0; x <= kSlices; ++x) qa[c].slice_begin[x] = acl[c].q.begin[x];
    qa[c].wave_floats = acl[c].wave_floats;
    qa[c].counter = counters + (3 + c) * kSlices;
    const int64_t resident = (int64_t)acl[c].occupancy * n_cu;
    adj_blocks[c] = persistent_grid(resident, (int64_t)acl[c].q.items.size(), 1);
    // Items claimed one at a time: an adjoint item (a whole sightline's
    // reverse march) is long against the claim, and claiming does not depend
    // on every workgroup being resident as static rounds do.
    qa[c].static_rounds = 0;
    adj_blocks_total += adj_blocks[c];
  }

  // 8. Capture each phase once. Forward: clear the queue heads, lay out the
  //    fields that are not read in place, then the persistent launches, as
  //    parallel branches (fork/join through events on the side streams).
  if ((s = hip_status(hipStreamCreateWithFlags(&P->cap, hipStreamNonBlocking),
                      "hipStreamCreateWithFlags")) != IRIS_OK)
    return s;
  for (hipStream_t& st : P->side)
    if ((s = hip_status(hipStreamCreateWithFlags(&st, hipStreamNonBlocking),
                        "hipStreamCreateWithFlags")) != IRIS_OK)
      return s;
  for (hipEvent_t& e : P->ev)
    if ((s = hip_status(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate")) !=
        IRIS_OK)
      return s;
  auto capture = [&](bool forward, hipGraph_t* graph, hipGraphExec_t* exec) -> iris_status {
    iris_status r = hip_status(hipStreamBeginCapture(P->cap, hipStreamCaptureModeThreadLocal),
                               "hipStreamBeginCapture");
    if (r != IRIS_OK) return r;
    int e = 0;
    // The packings present run as branches: the first on the capture stream,
    // the others on the side streams, joined back before the capture ends.
    int used[3], nb = 0;
    for (int c = 0; c < 3 && forward; ++c)
      if (fwd_blocks[c]) used[nb++] = c;
    e = forward ? launch_zero_ints(counters, 3 * kSlices, P->cap)
                : launch_zero_ints(counters + 3 * kSlices, n_acl * kSlices, P->cap);
    if (forward && !e && ftiles)
      e = launch_batched_layout((const TransposeJob*)(base + o_fj), (int)fjobs.size(), ftiles,
                                P->cap);
    if (!e && nb > 1) e = (int)hipEventRecord(P->ev[0], P->cap);
    for (int b = 1; b < nb && !e; ++b) e = (int)hipStreamWaitEvent(P->side[b - 1], P->ev[0], 0);
    for (int b = 0; b < nb && !e; ++b) {
      const int c = used[b];
      hipStream_t st = b == 0 ? P->cap : P->side[b - 1];
      e = launch_plan_forward(qf[c], kPackings[c], ck, fwd_blocks[c], st);
    }
    for (int c = 0; c < n_acl && !forward && !e; ++c)
      e = launch_plan_adjoint(qa[c], acl[c].groups, acl[c].general, adj_blocks[c], P->cap);
    for (int b = 1; b < nb && !e; ++b) {
      e = (int)hipEventRecord(P->ev[b], P->side[b - 1]);
      if (!e) e = (int)hipStreamWaitEvent(P->cap, P->ev[b], 0);
    }
    if (!forward && !e && gtiles)
      e = launch_batched_layout((const TransposeJob*)(base + o_gj), (int)gjobs.size(), gtiles,
                                P->cap);
    hipGraph_t gph = nullptr;
    const int e2 = (int)hipStreamEndCapture(P->cap, &gph);
    if (e || e2) {
      if (gph) (void)hipGraphDestroy(gph);
      return hip_status(e ? e : e2, "graph capture");
    }
    *graph = gph;
    return hip_status(hipGraphInstantiate(exec, gph, nullptr, nullptr, 0), "hipGraphInstantiate");
  };
  if ((s = capture(true, &P->graph_fwd, &P->exec_fwd)) != IRIS_OK) return s;
  if (adj && (s = capture(false, &P->graph_adj, &P->exec_adj)) != IRIS_OK) return s;

  iris_plan_info& I = P->info;
  I.scratch_bytes = (int64_t)total;
  I.samples = samples;
  I.n_cubes = n;
  I.n_fwd_items = (int32_t)n_fwd_items;
  I.n_adj_items = (int32_t)n_adj_items;
  I.fwd_blocks = fwd_blocks[0] + fwd_blocks[1] + fwd_blocks[2];
  I.adj_blocks = adj_blocks_total;
  I.layout_tiles = (int32_t)ftiles;
  I.ckpt_K = P->K;
  return IRIS_OK;
}

// Forward-only plan of one launch per cube: every cube's single-cube forward
// (tables, field layout where needed, the march) on its own workspace carved
// from one allocation, captured once.
iris_status build_launch_plan(const iris_cube* cubes, int n, const iris_line* L, iris_plan* P) {
  iris_status s;
  P->flags = IRIS_PLAN_FORWARD;
  P->K = 0;
  P->groups.assign(n, 0);  // each cube's single-cube forward chooses its own packing
  std::vector<size_t> o_ws(n), ws_bytes(n);
  Carver cv;
  int64_t samples = 0;
  for (int i = 0; i < n; ++i) {
    const iris_cube& cb = cubes[i];
    Geo g;
    if ((s = check_fields(&cb.fields, &g)) != IRIS_OK)
      return fail(s, "cube %d: %s", i, last_error());
    if ((s = check_channels(&cb.channels)) != IRIS_OK)
      return fail(s, "cube %d: %s", i, last_error());
    ws_bytes[i] = ws_layout(&cb.fields, g, march_channels(&cb.channels).n_chan, 0).total;
    o_ws[i] = cv.take(ws_bytes[i]);
    samples += g.n_cells * cb.channels.n_chan;
  }
  if ((s = hip_status(hipGetDevice(&P->device), "hipGetDevice")) != IRIS_OK) return s;
  if ((s = hip_status(hipMalloc(&P->mem, cv.off), "hipMalloc (plan scratch)")) != IRIS_OK) {
    P->mem = nullptr;
    return s;
  }
  if ((s = hip_status(hipStreamCreateWithFlags(&P->cap, hipStreamNonBlocking),
                      "hipStreamCreateWithFlags")) != IRIS_OK)
    return s;
  if ((s = hip_status(hipStreamBeginCapture(P->cap, hipStreamCaptureModeThreadLocal),
                      "hipStreamBeginCapture")) != IRIS_OK)
    return s;
  char* base = (char*)P->mem;
  for (int i = 0; i < n && s == IRIS_OK; ++i) {
    const iris_cube& cb = cubes[i];
    s = forward_impl(&cb.fields, &cb.channels, L, &cb.out, 0, base + o_ws[i], ws_bytes[i], P->cap,
                     0);
    if (s != IRIS_OK) s = fail(s, "cube %d: %s", i, last_error());
  }
  hipGraph_t gph = nullptr;
  const int e2 = (int)hipStreamEndCapture(P->cap, &gph);
  if (s != IRIS_OK || e2) {
    if (gph) (void)hipGraphDestroy(gph);
    return s != IRIS_OK ? s : hip_status(e2, "graph capture");
  }
  P->graph_fwd = gph;
  if ((s = hip_status(hipGraphInstantiate(&P->exec_fwd, gph, nullptr, nullptr, 0),
                      "hipGraphInstantiate")) != IRIS_OK)
    return s;
  iris_plan_info& I = P->info;
  I.scratch_bytes = (int64_t)cv.off;
  I.samples = samples;
  I.n_cubes = n;
  I.n_fwd_items = n;  // one launch per cube
  return IRIS_OK;
}

}  // namespace

extern "C" {

iris_status iris_rt_autotune(const iris_fields* fields, const iris_channels* channels,
                             const iris_line* line, const iris_outputs* out, void* workspace,
                             size_t workspace_bytes, void* stream, int32_t* groups) {
  clear_error();
  if (!groups) return fail(IRIS_E_INVALID_ARG, "groups is NULL");
  Geo g;
  iris_status s;
  if ((s = check_fields(fields, &g)) != IRIS_OK) return s;
  if ((s = check_channels(channels)) != IRIS_OK) return s;
  if ((s = check_line(line)) != IRIS_OK) return s;
  if (line->integrator != IRIS_INTEGRATOR_FORMAL || line->transfer != IRIS_TRANSFER_THICK)
    return fail(IRIS_E_UNSUPPORTED, "autotuning chooses the packing of the formal thick march");
  if (!out) return fail(IRIS_E_INVALID_ARG, "outputs is NULL");
  const WsLayout w = ws_layout(fields, g, march_channels(channels).n_chan, 0);
  if (!workspace || workspace_bytes < w.total)
    return fail(IRIS_E_WORKSPACE, "workspace needs %zu bytes, got %zu", w.total, workspace_bytes);
  int best = 0;
  s = tune_cube(fields, channels, line, out, workspace, workspace_bytes, (hipStream_t)stream, &best);
  if (s == IRIS_OK) *groups = best;
  return s;
}

iris_status iris_plan_create(const iris_cube* cubes, int32_t n_cubes, const iris_line* line,
                             int32_t flags, int32_t ckpt_K, void* stream, iris_plan** plan) {
  clear_error();
  if (!plan) return fail(IRIS_E_INVALID_ARG, "plan is NULL");
  *plan = nullptr;
  if (!cubes || n_cubes < 1) return fail(IRIS_E_INVALID_ARG, "need at least one cube");
  iris_status s;
  if ((s = check_line(line)) != IRIS_OK) return s;
  if (flags & ~(IRIS_PLAN_FORWARD | IRIS_PLAN_ADJOINT | IRIS_PLAN_AUTOTUNE))
    return fail(IRIS_E_INVALID_ARG, "unknown plan flags 0x%x", flags);
  const bool persistent =
      line->integrator == IRIS_INTEGRATOR_FORMAL && line->transfer == IRIS_TRANSFER_THICK;
  if (!persistent && (flags & (IRIS_PLAN_ADJOINT | IRIS_PLAN_AUTOTUNE)))
    return fail(IRIS_E_UNSUPPORTED, "plans of the smooth integrator and the thin transfer modes "
                "are forward only, without autotuning");
  if ((flags & IRIS_PLAN_ADJOINT) && !valid_K(ckpt_K))
    return fail(IRIS_E_INVALID_ARG, "adjoint plans need ckpt_K in {8,16,32,64}");
  if ((flags & IRIS_PLAN_ADJOINT) && ckpt_K == 0 && !(flags & IRIS_PLAN_AUTOTUNE))
    return fail(IRIS_E_INVALID_ARG,
                "adjoint plans need ckpt_K in {8,16,32,64} (0 only with IRIS_PLAN_AUTOTUNE)");
  iris_plan* P = new iris_plan();
  s = persistent ? build_plan(cubes, n_cubes, line, flags, ckpt_K, (hipStream_t)stream, P)
                 : build_launch_plan(cubes, n_cubes, line, P);
  if (s != IRIS_OK) {
    const std::string why = last_error();
    delete P;
    return fail(s, "%s", why.c_str());
  }
  *plan = P;
  return IRIS_OK;
}

iris_status iris_plan_forward(iris_plan* plan, void* stream) {
  clear_error();
  if (!plan || !plan->exec_fwd) return fail(IRIS_E_INVALID_ARG, "plan is NULL");
  DeviceGuard dg(plan->device);
  return hip_status(hipGraphLaunch(plan->exec_fwd, (hipStream_t)stream), "hipGraphLaunch");
}

iris_status iris_plan_adjoint(iris_plan* plan, void* stream) {
  clear_error();
  if (!plan) return fail(IRIS_E_INVALID_ARG, "plan is NULL");
  if (!plan->exec_adj) return fail(IRIS_E_INVALID_ARG, "plan was created without IRIS_PLAN_ADJOINT");
  DeviceGuard dg(plan->device);
  return hip_status(hipGraphLaunch(plan->exec_adj, (hipStream_t)stream), "hipGraphLaunch");
}

iris_status iris_plan_get_info(const iris_plan* plan, iris_plan_info* info) {
  clear_error();
  if (!plan || !info) return fail(IRIS_E_INVALID_ARG, "plan or info is NULL");
  *info = plan->info;
  return IRIS_OK;
}

int32_t iris_plan_groups(const iris_plan* plan, int32_t cube) {
  if (!plan || cube < 0 || cube >= (int32_t)plan->groups.size()) return 0;
  return plan->groups[cube];
}

int32_t iris_plan_adjoint_groups(const iris_plan* plan, int32_t cube) {
  if (!plan || cube < 0 || cube >= (int32_t)plan->adj_groups.size()) return 0;
  return plan->adj_groups[cube];
}

void iris_plan_destroy(iris_plan* plan) {
  if (!plan) return;
  DeviceGuard dg(plan->device);
  delete plan;
}

}  // extern "C"
