// Host-side helpers shared by every entry point (see host_common.h).

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "host_common.h"

namespace iris {
namespace host {

namespace {

// CODATA 2018, cgs.
constexpr double kPlanck = 6.62607015e-27;
constexpr double kBoltzmann = 1.380649e-16;
constexpr double kLight = 2.99792458e10;
constexpr double kAmu = 1.66053906660e-24;
constexpr double kPiD = 3.14159265358979323846;
constexpr double kLog2eD = 1.44269504088896340736;
// Window of the line: channels where the line optical depth of a cell is
// below kWindowEps * max(kappa_L, 1) / kappa_L (i.e. both kappa_L g and g
// below 1e-9) are left untouched by that cell. A skipped step changes a
// channel by at most kWindowEps * |I - S| (< 1e-7 K per cell for S <= 100 K).
constexpr double kWindowEps = 1e-9;
// Forward pass: a cell whose line-centre optical depth is below this carries
// no line (changes every output by < 1e-10 of its source-function scale).
constexpr float kLineMin = 1e-10f;

thread_local std::string g_err;

bool finite(double x) { return std::isfinite(x); }

}  // namespace

iris_status fail(iris_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

void clear_error() { g_err.clear(); }
const char* last_error() { return g_err.c_str(); }

iris_status hip_status(int e, const char* what) {
  if (e != 0) return fail(IRIS_E_HIP, "%s: %s", what, hipGetErrorString((hipError_t)e));
  return IRIS_OK;
}

size_t elem_size(iris_dtype d) {
  switch (d) {
    case IRIS_F64: return 8;
    case IRIS_F32: return 4;
    case IRIS_BF16:
    case IRIS_F16: return 2;
  }
  return 0;
}

static_assert(sizeof(iris_dtype) == sizeof(int32_t), "iris_dtype is read as a 32-bit integer");

iris_status check_fields(const iris_fields* f, Geo* g) {
  if (!f) return fail(IRIS_E_INVALID_ARG, "fields is NULL");
  if (f->nx < 1 || f->ny < 1 || f->nz < 1)
    return fail(IRIS_E_INVALID_ARG, "grid shape %d x %d x %d must be positive", f->nx, f->ny, f->nz);
  if (f->axis < 0 || f->axis > 2) return fail(IRIS_E_INVALID_ARG, "axis %d not in 0..2", f->axis);
  if (!(f->cell_cm > 0.0) || !finite(f->cell_cm))
    return fail(IRIS_E_INVALID_ARG, "cell_cm must be positive and finite");
  // The caller's dtype may hold any 32-bit value: read it as an integer, since
  // an iris_dtype outside the enumeration would be undefined behaviour.
  int32_t dt;
  std::memcpy(&dt, &f->dtype, sizeof dt);
  if (dt < IRIS_F64 || dt > IRIS_F16) return fail(IRIS_E_INVALID_ARG, "unknown dtype %d", dt);
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
  if (ch->simpson_f < 0 || ch->simpson_f > 64)
    return fail(IRIS_E_INVALID_ARG, "simpson_f %d not in 0..64", ch->simpson_f);
  const int64_t marched = ch->simpson_f ? 2LL * ch->simpson_f * ch->n_chan + 1 : ch->n_chan;
  if (marched > kMaxChannels)
    return fail(IRIS_E_UNSUPPORTED, "%lld marched velocities (n_chan %d, simpson_f %d) above the "
                "maximum %d", (long long)marched, ch->n_chan, ch->simpson_f, kMaxChannels);
  if (!(ch->dv_kms > 0.0) || !finite(ch->dv_kms) || !finite(ch->v_lo_kms))
    return fail(IRIS_E_INVALID_ARG, "channel grid needs finite v_lo and dv > 0");
  return IRIS_OK;
}

iris_channels march_channels(const iris_channels* ch) {
  iris_channels m = *ch;
  if (ch->simpson_f > 0) {
    // Centres of the march grid at the fine velocities v_lo + j dv / (2f).
    const double dvf = ch->dv_kms / (2.0 * ch->simpson_f);
    m.n_chan = 2 * ch->simpson_f * ch->n_chan + 1;
    m.dv_kms = dvf;
    m.v_lo_kms = ch->v_lo_kms - 0.5 * dvf;
  }
  return m;
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
  if (L->units != IRIS_UNITS_TRJ && L->units != IRIS_UNITS_INTENSITY && L->units != IRIS_UNITS_TB)
    return fail(IRIS_E_INVALID_ARG, "units %d is not an iris_units value", L->units);
  if (L->integrator != IRIS_INTEGRATOR_FORMAL && L->integrator != IRIS_INTEGRATOR_SMOOTH)
    return fail(IRIS_E_INVALID_ARG, "integrator %d is not an iris_integrator value",
                L->integrator);
  if (L->transfer != IRIS_TRANSFER_THICK && L->transfer != IRIS_TRANSFER_THIN &&
      L->transfer != IRIS_TRANSFER_SELECTIVE)
    return fail(IRIS_E_INVALID_ARG, "transfer %d is not an iris_transfer value", L->transfer);
  return levels_check(L);
}

Folded fold(const iris_fields* f, const iris_channels* ch, const iris_line* L) {
  Folded c{};
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
  c.simpson_f = ch->simpson_f;
  c.n_out = ch->simpson_f ? (ch->n_chan - 1) / (2 * ch->simpson_f) : ch->n_chan;
  c.units = L->units;
  // Specific intensity per Rayleigh-Jeans kelvin at nu0: 2 k nu0^2 / c^2.
  c.out_scale = L->units == IRIS_UNITS_INTENSITY
                    ? (float)(2.0 * kBoltzmann * nu * nu / (kLight * kLight))
                    : 1.f;
  levels_fold(L, c);
  return c;
}

TabParams tab_params(const iris_line* L) {
  TabParams t{};
  const double T0 = kPlanck * L->nu0_hz / kBoltzmann;
  t.theta = L->energy_mode == 0 ? T0 / (2.0 * L->j_u) : L->e_u_k / (L->j_u * (L->j_u + 1.0));
  const int ju = L->j_u, jl = L->j_u - 1;
  t.dE = t.theta * (ju * (ju + 1.0) - jl * (jl + 1.0));
  t.T0 = T0;
  t.g_l = 2.0 * jl + 1.0;
  t.j_max = L->j_max;
  t.j_l = jl;
  return t;
}

SightAddr native_addr(const iris_fields* f, const Geo& g) {
  SightAddr a{};
  const int64_t ny = f->ny, nz = f->nz;
  if (f->axis == 2) {
    a.div = g.n_pix;
    a.lo = nz;
    a.los = 1;
  } else if (f->axis == 1) {
    a.div = nz;
    a.hi = ny * nz;
    a.lo = 1;
    a.los = nz;
  } else {
    a.div = g.n_pix;
    a.lo = 1;
    a.los = ny * nz;
  }
  return a;
}

SightAddr sightline_major_addr(const Geo& g) {
  SightAddr a{};
  a.div = g.n_pix;
  a.lo = g.n_los;
  a.los = 1;
  return a;
}

bool reads_in_place(const iris_fields* f) {
  if (f->axis == 2) return true;
  const char* e = std::getenv("IRIS_RT_FIELD_LAYOUT");
  return !(e && std::strcmp(e, "transpose") == 0);
}

WsLayout ws_layout(const iris_fields* f, const Geo& g, int n_chan, int K) {
  WsLayout w;
  size_t off = 0;
  w.tab = off;  // temperature tables, rebuilt by every forward call
  off += align256(kTabBytes);
  w.erfc = off;  // erfc pieces of the thin transfer modes, rebuilt by every such call
  off += align256(thin_table_bytes());
  const bool copy = !reads_in_place(f);
  if (copy) {
    w.soa = off;
    off += align256((size_t)g.n_fields * g.n_cells * elem_size(f->dtype));
  }
  if (K > 0) {
    w.n_ck = (g.n_los + K - 1) / K;
    w.ck_state = off;
    off += align256((size_t)w.n_ck * g.n_pix * n_chan * sizeof(float));
    w.ck_scal = off;
    off += align256((size_t)w.n_ck * g.n_pix * kCkScal * sizeof(double));
    if (copy) {
      // Sightline-major FP64 gradients before they are laid back out.
      w.grad = off;
      off += align256((size_t)g.n_fields * g.n_cells * sizeof(double));
    }
  }
  w.total = off;
  return w;
}

LayoutParams field_layout(const iris_fields* f, const Geo& g, void* dst) {
  LayoutParams lp{};
  const void* src[5] = {f->ln_nh2, f->t_kin, f->v_los, f->x_tracer, f->t_dust};
  const size_t es = elem_size(f->dtype);
  for (int i = 0; i < g.n_fields; ++i) {
    lp.src[i] = src[i];
    lp.dst[i] = (char*)dst + (size_t)i * g.n_cells * es;
  }
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
  return lp;
}

LayoutParams gradient_layout(const iris_fields* f, const Geo& g, double* const src[5],
                             double* const dst[5]) {
  LayoutParams lp{};
  for (int i = 0; i < g.n_fields; ++i) {
    lp.src[i] = src[i];
    lp.dst[i] = dst[i];
  }
  lp.n_fields = g.n_fields;
  lp.elem = 8;
  if (f->axis == 1) {
    lp.batch = f->nx;
    lp.rows = f->nz;
    lp.cols = f->ny;
  } else {
    lp.batch = 1;
    lp.rows = (int64_t)f->ny * f->nz;
    lp.cols = f->nx;
  }
  return lp;
}

bool adjoint_fits(int n_chan, int K, int groups, bool general) {
  return (size_t)adj_lds_floats(n_chan, K, groups, general) * sizeof(float) <= 65536;
}

// The most sightlines per wavefront (passes of 64/G - 1 channels) whose pass
// holds a line window at 100 K, about 2 x 4.55 Doppler widths plus the two
// edge channels; IRIS_RT_THIN_GROUPS=1|2|4 overrides. The forward's LDS
// decides whether a packing fits (the reverse mode's is smaller).
int thin_groups(const Folded& c, int n_chan, bool selective) {
  const double b100 = std::sqrt((double)c.bT * 100.0 + (double)c.bt2);
  const double width = 2 * std::sqrt(std::log(1.0 / kWindowEps)) * b100 * c.inv_dv + 3.0;
  int groups = width <= 15.0 ? 4 : width <= 31.0 ? 2 : 1;
  if (const char* e = std::getenv("IRIS_RT_THIN_GROUPS")) {
    if (std::strcmp(e, "1") == 0) groups = 1;
    if (std::strcmp(e, "2") == 0) groups = 2;
    if (std::strcmp(e, "4") == 0) groups = 4;
  }
  while (groups > 1 && thin_lds_bytes(n_chan, groups, selective) + thin_static_lds_bytes() > 65536)
    groups = 1;
  return thin_lds_bytes(n_chan, groups, selective) + thin_static_lds_bytes() > 65536 ? 0 : groups;
}

bool groups_fit(int n_chan, int groups, bool general) {
  return fwd_lds_bytes(n_chan, groups, general) <= 65536;
}

// ---- choice of sightlines per wavefront ------------------------------------

namespace {

// Cubes of one class share the choice: what sets the cost of a cell is the
// channel count, the Doppler width in channels (dv and the broadening
// constants), the storage type, the sightline length and the source variant.
using TuneKey = std::tuple<int, double, double, double, int, int64_t, int>;

std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune;
// The adjoint's packing per class and checkpoint interval.
std::map<std::pair<TuneKey, int>, int> g_tune_adj;
bool g_tune_loaded = false;

TuneKey tune_key(const iris_fields* f, const iris_channels* ch, const iris_line* L,
                 const Folded& c) {
  const int64_t los = f->axis == 0 ? f->nx : f->axis == 1 ? f->ny : f->nz;
  return TuneKey(ch->n_chan, ch->dv_kms, L->sigma_turb_kms, L->m_tracer_amu, (int)f->dtype, los,
                 c.general);
}

// Lines of the cache file: "iris-tune n_chan dv sigma m dtype n_los general groups".
void load_tune_file_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = std::getenv("IRIS_RT_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* fp = std::fopen(path, "r");
  if (!fp) return;
  char line[256];
  while (std::fgets(line, sizeof line, fp)) {
    int nch, dt, gen, grp;
    double dv, sg, m;
    long long los;
    int kk;
    if (std::sscanf(line, "iris-tune %d %lf %lf %lf %d %lld %d %d", &nch, &dv, &sg, &m, &dt, &los,
                    &gen, &grp) == 8 &&
        (grp == 1 || grp == 2 || grp == 4))
      g_tune[TuneKey(nch, dv, sg, m, dt, (int64_t)los, gen)] = grp;
    else if (std::sscanf(line, "iris-tune-adjoint %d %lf %lf %lf %d %lld %d %d %d", &nch, &dv, &sg,
                         &m, &dt, &los, &gen, &kk, &grp) == 9 &&
             (grp == 1 || grp == 2 || grp == 4))
      g_tune_adj[{TuneKey(nch, dv, sg, m, dt, (int64_t)los, gen), kk}] = grp;
  }
  std::fclose(fp);
}

int rule_groups(const Folded& c) {
  // The smallest lane group (64, 32 or 16 lanes) that holds the line window
  // of a cell at 100 K in one pass.
  const double b = std::sqrt((double)c.bT * 100.0 + (double)c.bt2);
  const double width = 2.0 * std::sqrt((double)c.xw2min) * b * c.inv_dv + 1.0;
  if (width <= 15.0) return 4;
  if (width <= 30.0) return 2;
  return 1;
}

}  // namespace

int choose_groups(const iris_fields* f, const iris_channels* ch, const iris_line* L,
                  const Folded& c) {
  int g = 0;
  if (const char* e = std::getenv("IRIS_RT_SIGHTLINES_PER_WAVE")) {
    const int v = std::atoi(e);
    if (v == 1 || v == 2 || v == 4) g = v;
  }
  if (g == 0) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_file_locked();
    auto it = g_tune.find(tune_key(f, ch, L, c));
    if (it != g_tune.end()) g = it->second;
  }
  if (g == 0) g = rule_groups(c);
  while (g > 1 && !groups_fit(ch->n_chan, g, c.general != 0)) g /= 2;
  return g;
}

int adjoint_groups(const iris_fields* f, const iris_channels* ch, const iris_line* L,
                   const Folded& c, int K, bool plan) {
  int g = 0;
  if (const char* e = std::getenv("IRIS_RT_ADJOINT_SIGHTLINES_PER_WAVE")) {
    const int v = std::atoi(e);
    if (v == 1 || v == 2 || v == 4) g = v;
  }
  if (g == 0 && !plan) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_file_locked();
    auto it = g_tune_adj.find({tune_key(f, ch, L, c), K});
    if (it != g_tune_adj.end()) g = it->second;
  }
  if (g == 0) {
    // Passes of the line window at 100 K over the lanes of each packing.
    const double b = std::sqrt((double)c.bT * 100.0 + (double)c.bt2);
    const double width = 2.0 * std::sqrt((double)c.xw2min) * b * c.inv_dv + 1.0;
    if (plan) {
      // Plans: four sightlines per wavefront up to two passes of their 16
      // lanes (64-cube batch: every cube at four, 14.1 ms per adjoint phase,
      // against 15.1 ms with the single-cube rule below and 15.3 ms with the
      // single-cube tuner's choices).
      g = width <= 30.0 ? 4 : width <= 60.0 ? 2 : 1;
    } else {
      // The widest packing whose window fits one pass of its lanes. (Which
      // packing is fastest also depends on how many wavefronts the LDS of
      // each leaves resident, in ways no simple bound captured: at K = 16 two
      // sightlines per wavefront beat four at 512 channels, at K = 64 four
      // beat two at 256 with fewer resident. iris_rt_autotune_adjoint times
      // them.)
      g = width <= 15.0 ? 4 : width <= 30.0 ? 2 : 1;
    }
  }
  while (g >= 1 && !adjoint_fits(ch->n_chan, K, g, c.general != 0)) g /= 2;
  return g;
}

void record_adjoint_groups(const iris_fields* f, const iris_channels* ch, const iris_line* L,
                           const Folded& c, int K, int groups) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  load_tune_file_locked();
  const TuneKey k = tune_key(f, ch, L, c);
  auto it = g_tune_adj.find({k, K});
  if (it != g_tune_adj.end() && it->second == groups) return;
  g_tune_adj[{k, K}] = groups;
  const char* path = std::getenv("IRIS_RT_TUNE_CACHE");
  if (!path || !*path) return;
  if (FILE* fp = std::fopen(path, "a")) {
    std::fprintf(fp, "iris-tune-adjoint %d %.17g %.17g %.17g %d %lld %d %d %d\n",
                 std::get<0>(k), std::get<1>(k), std::get<2>(k), std::get<3>(k), std::get<4>(k),
                 (long long)std::get<5>(k), std::get<6>(k), K, groups);
    std::fclose(fp);
  }
}

void record_groups(const iris_fields* f, const iris_channels* ch, const iris_line* L,
                   const Folded& c, int groups) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  load_tune_file_locked();
  const TuneKey k = tune_key(f, ch, L, c);
  auto it = g_tune.find(k);
  if (it != g_tune.end() && it->second == groups) return;
  g_tune[k] = groups;
  const char* path = std::getenv("IRIS_RT_TUNE_CACHE");
  if (!path || !*path) return;
  if (FILE* fp = std::fopen(path, "a")) {
    std::fprintf(fp, "iris-tune %d %.17g %.17g %.17g %d %lld %d %d\n", std::get<0>(k),
                 std::get<1>(k), std::get<2>(k), std::get<3>(k), std::get<4>(k),
                 (long long)std::get<5>(k), std::get<6>(k), groups);
    std::fclose(fp);
  }
}

// ---- kernel parameters ------------------------------------------------------

FwdParams fwd_params(const iris_fields* f, const Geo& g, const iris_channels* ch,
                     const iris_line* L, const iris_outputs* out, int K, const void* const fsl[5],
                     const SightAddr& at, const void* tab, float* ck_state, double* ck_scal,
                     int groups) {
  FwdParams p{};
  for (int i = 0; i < 5; ++i) p.f[i] = fsl[i];
  p.at = at;
  p.n_pix = (int32_t)g.n_pix;
  p.n_los = (int32_t)g.n_los;
  p.c = fold(f, ch, L);
  p.c.tab = tab;
  p.out[0] = out->T;
  p.out[1] = out->C;
  p.out[2] = out->D;
  p.out[3] = out->L;
  p.out[4] = out->B;
  p.ckpt_K = K;
  p.groups = groups;
  p.dtype = (int32_t)f->dtype;
  p.lds_per_wave = fwd_state_floats(ch->n_chan, groups);
  p.ck_state = ck_state;
  p.ck_scal = ck_scal;
  return p;
}

AdjParams adj_params(const iris_fields* f, const Geo& g, const iris_channels* ch,
                     const iris_line* L, const iris_cotangents* cot, int K,
                     const void* const fsl[5], const SightAddr& at, const void* tab,
                     const float* ck_state, const double* ck_scal, double* const grad[5],
                     const SightAddr& gat, int groups) {
  AdjParams p{};
  for (int i = 0; i < 5; ++i) p.f[i] = fsl[i];
  p.at = at;
  p.n_pix = (int32_t)g.n_pix;
  p.n_los = (int32_t)g.n_los;
  p.c = fold(f, ch, L);
  p.c.tab = tab;
  p.cot[0] = cot->gT;
  p.cot[1] = cot->gC;
  p.cot[2] = cot->gD;
  p.cot[3] = cot->gL;
  p.cot[4] = cot->gB;
  p.ckpt_K = K;
  p.dtype = (int32_t)f->dtype;
  p.groups = groups > 0 ? groups : adjoint_groups(f, ch, L, p.c, K);
  const int G = p.groups > 0 ? p.groups : 1;
  p.chan_stride = adj_chan_stride(ch->n_chan, G);
  p.tape_passes = adj_tape_passes(ch->n_chan, G);
  p.lds_per_wave = adj_lds_floats(ch->n_chan, K, G, p.c.general != 0);
  p.ck_state = ck_state;
  p.ck_scal = ck_scal;
  for (int i = 0; i < 5; ++i) p.grad[i] = grad[i];
  p.gat = gat;
  return p;
}

// ---- single-cube forward -----------------------------------------------------

iris_status forward_impl(const iris_fields* fields, const iris_channels* channels,
                         const iris_line* line, const iris_outputs* out, int32_t ckpt_K,
                         void* workspace, size_t workspace_bytes, void* stream, int groups) {
  Geo g;
  iris_status s;
  if ((s = check_fields(fields, &g)) != IRIS_OK) return s;
  if ((s = check_channels(channels)) != IRIS_OK) return s;
  if ((s = check_line(line)) != IRIS_OK) return s;
  const bool selective = line->transfer == IRIS_TRANSFER_SELECTIVE;
  const bool thin = line->transfer == IRIS_TRANSFER_THIN || selective;
  if (thin && channels->simpson_f != 0)
    return fail(IRIS_E_INVALID_ARG, "thin transfer modes average the profile over each "
                "channel analytically: simpson_f must be 0");
  const iris_channels mg = march_channels(channels);
  channels = &mg;
  if (!out) return fail(IRIS_E_INVALID_ARG, "outputs is NULL");
  if (!valid_K(ckpt_K)) return fail(IRIS_E_INVALID_ARG, "ckpt_K %d not in {0,8,16,32,64}", ckpt_K);
  const WsLayout w = ws_layout(fields, g, channels->n_chan, ckpt_K);
  if (!workspace || workspace_bytes < w.total)
    return fail(IRIS_E_WORKSPACE, "workspace needs %zu bytes, got %zu", w.total, workspace_bytes);

  const Folded c = fold(fields, channels, line);
  const bool smooth = line->integrator == IRIS_INTEGRATOR_SMOOTH;
  if (thin) {
    if (ckpt_K)
      return fail(IRIS_E_UNSUPPORTED, "thin transfer modes have no adjoint: ckpt_K must be 0");
    if (selective && smooth) {
      // Smooth steps: the smooth integrator's kernel, one sightline per wavefront.
      if (channels->n_chan > smooth_max_channels())
        return fail(IRIS_E_UNSUPPORTED, "%d channels above the smooth integrator's %d",
                    channels->n_chan, smooth_max_channels());
      groups = 1;
    } else {
      groups = thin_groups(c, channels->n_chan, selective);
      if (!groups)
        return fail(IRIS_E_UNSUPPORTED, "n_chan %d needs more LDS than a workgroup has",
                    channels->n_chan);
    }
  } else if (smooth) {
    if (ckpt_K)
      return fail(IRIS_E_UNSUPPORTED, "smooth integration has no adjoint: ckpt_K must be 0");
    if (channels->n_chan > smooth_max_channels())
      return fail(IRIS_E_UNSUPPORTED, "%d marched velocities above the smooth integrator's %d",
                  channels->n_chan, smooth_max_channels());
    groups = 1;
  } else {
    if (!groups) groups = choose_groups(fields, channels, line, c);
    if (!groups_fit(channels->n_chan, groups, c.general != 0))
      return fail(IRIS_E_UNSUPPORTED, "n_chan %d needs more LDS than a workgroup has",
                  channels->n_chan);
  }
  void* tab = (char*)workspace + w.tab;
  if ((s = hip_status(launch_pop_table(tab_params(line), tab, stream), "table kernel")) != IRIS_OK)
    return s;
  const void* fsl[5] = {fields->ln_nh2, fields->t_kin, fields->v_los, fields->x_tracer,
                        fields->t_dust};
  SightAddr at = native_addr(fields, g);
  if (!reads_in_place(fields)) {
    const LayoutParams lp = field_layout(fields, g, (char*)workspace + w.soa);
    for (int i = 0; i < 5; ++i) fsl[i] = i < g.n_fields ? lp.dst[i] : nullptr;
    at = sightline_major_addr(g);
    if ((s = hip_status(launch_layout(lp, stream), "layout kernel")) != IRIS_OK) return s;
  }
  float* ck_state = ckpt_K ? (float*)((char*)workspace + w.ck_state) : nullptr;
  double* ck_scal = ckpt_K ? (double*)((char*)workspace + w.ck_scal) : nullptr;
  const FwdParams p = fwd_params(fields, g, channels, line, out, ckpt_K, fsl, at, tab, ck_state,
                                 ck_scal, groups);
  if (selective && smooth) {
    launch_erfc_table((char*)workspace + w.erfc, stream);
    return hip_status(
        launch_smooth_selective(fields->dtype, p, (char*)workspace + w.erfc, stream),
        "smooth kernel");
  }
  if (thin)
    return hip_status(
        launch_thin(p, smooth, selective, groups, (char*)workspace + w.erfc, stream),
        "thin kernel");
  if (smooth) return hip_status(launch_smooth(fields->dtype, p, stream), "smooth kernel");
  return hip_status(launch_forward(fields->dtype, p, stream), "forward kernel");
}

}  // namespace host
}  // namespace iris
