// Host-side helpers shared by the single-cube entry points and the batched
// plans: argument validation, constant folding, workspace carving and the
// choice of sightlines per wavefront. Nothing here launches a kernel.
#pragma once

#include <cstddef>
#include <cstdint>

#include "iris_internal.h"

namespace iris {

// Optically thin forward of one cube (thin.hip); `smooth`: Simpson panels
// over the nodes instead of the midpoint sum; `selective`: selectively thin
// transfer (formal steps; the smooth steps are launch_smooth_selective)
// instead; `groups`: sightlines per wavefront (1 or 2); `table`:
// thin_table_bytes() of workspace for the erfc pieces, rebuilt by every call.
int launch_thin(const FwdParams& p, bool smooth, bool selective, int groups, void* table,
                void* stream);
size_t thin_lds_bytes(int n_chan, int groups, bool selective);
size_t thin_static_lds_bytes();
// Reverse mode of optically thin transfer (thin.hip); LDS of its workgroup.
int launch_thin_adjoint(const AdjParams& p, bool smooth, int groups, void* table, void* stream);
size_t thin_adj_lds_bytes(int n_chan, int groups);
size_t thin_table_bytes();
// Builds the erfc pieces (thin_table_bytes()) into `table` on `stream`.
void launch_erfc_table(void* table, void* stream);
// Selectively thin transfer under the smooth integrator (smooth.hip), the
// erfc pieces already built in `table` on the same stream.
int launch_smooth_selective(iris_dtype dt, const FwdParams& p, const void* table, void* stream);

namespace host {

iris_status fail(iris_status s, const char* fmt, ...);
void clear_error();
const char* last_error();
iris_status hip_status(int e, const char* what);

size_t elem_size(iris_dtype d);
inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Geo {
  int64_t n_cells, n_los, n_pix;
  int n_fields;
};

iris_status check_fields(const iris_fields* f, Geo* g);
iris_status check_channels(const iris_channels* ch);
// The grid the march runs on: the user's channels, or with simpson_f > 0
// the fine velocities v_lo + j dv / (2f) as channel centres (2 f n_chan + 1
// of them; simpson_f is kept so that fold() knows the output channels).
// Public entry points convert once; everything internal takes march grids.
iris_channels march_channels(const iris_channels* ch);
iris_status check_line(const iris_line* L);
// Non-LTE populations of a line (levels.hip): the grid's transition must be
// the line's; levels_fold sets the march's constants of the grid.
iris_status levels_check(const iris_line* L);
void levels_fold(const iris_line* L, Folded& c);
inline bool valid_K(int K) { return K == 0 || K == 8 || K == 16 || K == 32 || K == 64; }

// FP64 constant folding of the line, dust and channel constants for one cube.
Folded fold(const iris_fields* f, const iris_channels* ch, const iris_line* L);
TabParams tab_params(const iris_line* L);

// Addressing of a cube's fields: the native [nx][ny][nz] arrays read in
// place, or a sightline-major copy.
SightAddr native_addr(const iris_fields* f, const Geo& g);
SightAddr sightline_major_addr(const Geo& g);
// Whether the march reads the native arrays in place (no layout pass).
// IRIS_RT_FIELD_LAYOUT=transpose forces the sightline-major copy.
bool reads_in_place(const iris_fields* f);

// Byte offsets inside a single-cube workspace.
struct WsLayout {
  size_t tab = 0, erfc = 0, soa = 0, ck_state = 0, ck_scal = 0, grad = 0, total = 0;
  int64_t n_ck = 0;
};
WsLayout ws_layout(const iris_fields* f, const Geo& g, int n_chan, int K);

// Transpose descriptor that lays the fields of `f` out sightline-major at dst
// (n_fields arrays of n_cells elements), and its inverse for FP64 gradients.
LayoutParams field_layout(const iris_fields* f, const Geo& g, void* dst);
LayoutParams gradient_layout(const iris_fields* f, const Geo& g, double* const src[5],
                             double* const dst[5]);

// Sightlines per wavefront of the forward march for this cube: the override
// IRIS_RT_SIGHTLINES_PER_WAVE, else an autotuned choice recorded for the
// cube's class, else a rule from the Doppler width in channels.
int choose_groups(const iris_fields* f, const iris_channels* ch, const iris_line* L,
                  const Folded& c);
void record_groups(const iris_fields* f, const iris_channels* ch, const iris_line* L,
                   const Folded& c, int groups);
bool groups_fit(int n_chan, int groups, bool general);
// Sightlines per wavefront of the thin modes' kernels (0: none fits).
int thin_groups(const Folded& c, int n_chan, bool selective);

// Sightlines per wavefront of the adjoint: the override
// IRIS_RT_ADJOINT_SIGHTLINES_PER_WAVE, else (single-cube calls) a tuned choice
// recorded for the cube's class and checkpoint interval, else a rule on the
// line window's passes (plans and single cubes measured apart); reduced until
// its LDS fits a workgroup (0 if none).
int adjoint_groups(const iris_fields* f, const iris_channels* ch, const iris_line* L,
                   const Folded& c, int K, bool plan = false);
void record_adjoint_groups(const iris_fields* f, const iris_channels* ch, const iris_line* L,
                           const Folded& c, int K, int groups);
// LDS floats per wavefront of the adjoint: adj_wave_floats, whose rows of
// separate line and dust source functions (`general`) hold four more floats.
inline int adj_lds_floats(int n_chan, int K, int groups, bool general) {
  return adj_wave_floats(n_chan, K, groups) + (general ? groups * K * 4 : 0);
}
bool adjoint_fits(int n_chan, int K, int groups, bool general);
// The adjoint of one cube after the forward that wrote its checkpoints into
// `workspace`, with a fixed packing (0: adjoint_groups).
iris_status adjoint_impl(const iris_fields* fields, const iris_channels* channels,
                         const iris_line* line, const iris_cotangents* cot, int32_t ckpt_K,
                         void* workspace, size_t workspace_bytes, const iris_gradients* grads,
                         void* stream, int groups);

// Kernel parameters of one cube. `fsl` are the field arrays addressed by
// `at`, `tab` the temperature tables; the checkpoint pointers may be NULL
// when K = 0; gradients are written through `gat`.
FwdParams fwd_params(const iris_fields* f, const Geo& g, const iris_channels* ch,
                     const iris_line* L, const iris_outputs* out, int K, const void* const fsl[5],
                     const SightAddr& at, const void* tab, float* ck_state, double* ck_scal,
                     int groups);
AdjParams adj_params(const iris_fields* f, const Geo& g, const iris_channels* ch,
                     const iris_line* L, const iris_cotangents* cot, int K,
                     const void* const fsl[5], const SightAddr& at, const void* tab,
                     const float* ck_state, const double* ck_scal, double* const grad[5],
                     const SightAddr& gat, int groups = 0);

// Forward of one cube into a caller workspace with a fixed number of
// sightlines per wavefront (0: choose_groups).
iris_status forward_impl(const iris_fields* fields, const iris_channels* channels,
                         const iris_line* line, const iris_outputs* out, int32_t ckpt_K,
                         void* workspace, size_t workspace_bytes, void* stream, int groups);

}  // namespace host
}  // namespace iris
