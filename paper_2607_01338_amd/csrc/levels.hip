// Non-LTE level populations: the optically thin level balance and its
// startup grid (paper: "Level Populations: Mathematical Solution", eq. OT
// Levels System; "Einstein Coefficients, Collisions, and the Detailed
// Balance"; "Spectral-Line Configuration"; "Grid Precomputation").
//
// Host side: a reader of molecular data in the LAMDA .dat convention.
// Device side: one wavefront per grid node (ln n_H2, chi, ln T) assembles the
// rate matrix of every level in LDS and solves the balance, with the ground
// state's equation replaced by the conservation row, by FP64 Gaussian
// elimination with partial pivoting (lane j holds column j, the right-hand
// side is column L). The node keeps the observed transition's population
// factors FU = (g_l/g_u) f_u and FL = f_l - FU as an FP32 pair.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "host_common.h"

using namespace iris::host;

struct iris_molecule {
  std::vector<double> energy_k;  // level energy / k, K
  std::vector<double> g;
  std::vector<int> rad_u, rad_l;  // 0-based
  std::vector<double> rad_a, rad_nu;  // s^-1, Hz
  struct Partner {
    int code;
    std::vector<double> temps;
    std::vector<int> u, l;
    std::vector<double> rates;  // [n_coll][n_temps]
  };
  std::vector<Partner> partners;
};

struct iris_levels {
  void* tables = nullptr;  // device copy of the molecule's tables
  float2* grid = nullptr;  // [n_chi][n_t][n_n] (FU, FL)
  iris_levels_config cfg{};
  double g_u = 0, g_l = 0, nu = 0, a = 0;  // observed transition
};

namespace iris {

constexpr int kMaxLevels = 63;   // + the right-hand side: one column per lane
constexpr int kMaxPartners = 8;
constexpr int kMaxTemps = 64;
constexpr double kHPlanck = 6.62607015e-27, kKBoltz = 1.380649e-16, kCLight = 2.99792458e10;

enum : int { kPH2 = 1, kPPara = 2, kPOrtho = 3, kPElectron = 4, kPH = 5, kPHe = 6, kPHplus = 7 };

struct LevelsParams {
  const double* E;      // [L] level energy / k
  const double* g;      // [L]
  const int* rad_u;
  const int* rad_l;
  const double* rad_a;
  const double* rad_nbar;  // photon occupation of the background at each line
  const int* coll_u;
  const int* coll_l;
  const double* temps;
  const double* rates;
  int n_rad, L, n_part, u_obs, l_obs;
  double dens_a[kMaxPartners], dens_b[kMaxPartners];  // n_s = n_H2 (a + b / chi)
  int coll_off[kMaxPartners], n_coll[kMaxPartners];
  int temp_off[kMaxPartners], n_temp[kMaxPartners];
  long rate_off[kMaxPartners];
  int n_n, n_c, n_t;
  double lnn0, dlnn, chi0, dchi, lnt0, dlnt;
  float2* grid;
};

__global__ __launch_bounds__(64) void ot_levels_kernel(const LevelsParams P) {
  __shared__ double M[kMaxLevels][64];
  const int lane = threadIdx.x;
  const int L = P.L;
  const int n_pts = P.n_n * P.n_c * P.n_t;
  for (int pt = blockIdx.x; pt < n_pts; pt += gridDim.x) {
    const int i_n = pt % P.n_n;
    const int i_t = (pt / P.n_n) % P.n_t;
    const int i_c = pt / (P.n_n * P.n_t);
    const double nh2 = exp(P.lnn0 + i_n * P.dlnn);
    const double chi = P.chi0 + i_c * P.dchi;
    const double T = exp(P.lnt0 + i_t * P.dlnt);
    __syncthreads();  // the previous node's reads of M are done
    for (int i = 0; i < L; ++i) M[i][lane] = 0.0;
    __syncthreads();
    // Radiative rates: M[i][j] = rate from level j into level i.
    for (int t = lane; t < P.n_rad; t += 64) {
      const int u = P.rad_u[t], l = P.rad_l[t];
      const double A = P.rad_a[t], nb = P.rad_nbar[t];
      M[l][u] += A * (1.0 + nb);
      M[u][l] += P.g[u] / P.g[l] * A * nb;
    }
    __syncthreads();
    // Collisions, partner by partner (a partner lists each pair once).
    for (int p = 0; p < P.n_part; ++p) {
      const double ns = nh2 * (P.dens_a[p] + P.dens_b[p] / chi);
      const double* tt = P.temps + P.temp_off[p];
      const int nt = P.n_temp[p];
      int k = 0;
      double w = 0.0;
      if (T >= tt[nt - 1]) {
        k = nt - 1;
      } else if (T > tt[0]) {
        while (tt[k + 1] <= T) ++k;
        w = (T - tt[k]) / (tt[k + 1] - tt[k]);
      }
      for (int c = lane; c < P.n_coll[p]; c += 64) {
        const int u = P.coll_u[P.coll_off[p] + c], l = P.coll_l[P.coll_off[p] + c];
        const double* r = P.rates + P.rate_off[p] + (long)c * nt;
        const double kul = w == 0.0 ? r[k] : r[k] + w * (r[k + 1] - r[k]);
        const double down = kul * ns;
        M[l][u] += down;
        M[u][l] += down * (P.g[u] / P.g[l]) * exp(-(P.E[u] - P.E[l]) / T);
      }
      __syncthreads();
    }
    // Diagonal: minus the total rate out of each level (its column's sum).
    if (lane < L) {
      double s = 0.0;
      for (int i = 0; i < L; ++i)
        if (i != lane) s += M[i][lane];
      M[lane][lane] = -s;
    }
    __syncthreads();
    // Conservation in place of the ground state's balance; right-hand side
    // e_0 in column L.
    if (lane < L) M[0][lane] = 1.0;
    if (lane < L) M[lane][L] = lane == 0 ? 1.0 : 0.0;
    __syncthreads();
    // Elimination with partial pivoting.
    for (int p = 0; p < L; ++p) {
      double v = (lane >= p && lane < L) ? fabs(M[lane][p]) : -1.0;
      int r = lane;
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1) {
        const double ov = __shfl_xor(v, d, 64);
        const int orr = __shfl_xor(r, d, 64);
        if (ov > v || (ov == v && orr < r)) {
          v = ov;
          r = orr;
        }
      }
      __syncthreads();
      if (r != p && lane <= L) {
        const double a = M[p][lane];
        M[p][lane] = M[r][lane];
        M[r][lane] = a;
      }
      __syncthreads();
      const double inv = 1.0 / M[p][p];
      const double rowp = lane <= L ? M[p][lane] : 0.0;
      for (int i = p + 1; i < L; ++i) {
        const double f = M[i][p] * inv;
        if (lane > p && lane <= L) M[i][lane] -= f * rowp;
      }
      __syncthreads();
    }
    // Back substitution; x_j in lane j.
    double x = 0.0;
    for (int i = L - 1; i >= 0; --i) {
      double s = (lane > i && lane < L) ? M[i][lane] * x : 0.0;
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
      const double xi = (M[i][L] - s) / M[i][i];
      if (lane == i) x = xi;
    }
    const double fu = __shfl(x, P.u_obs, 64), fl = __shfl(x, P.l_obs, 64);
    if (lane == 0) {
      const double FU = P.g[P.l_obs] / P.g[P.u_obs] * fu;
      P.grid[pt] = make_float2((float)FU, (float)(fl - FU));
    }
  }
}

}  // namespace iris

namespace {

// Data lines of the file (those not starting with '!'), with their numbers.
struct Lines {
  std::vector<std::string> text;
  std::vector<int> number;
  size_t pos = 0;
  bool next(std::string& s, int& n) {
    if (pos >= text.size()) return false;
    s = text[pos];
    n = number[pos];
    ++pos;
    return true;
  }
};

iris_status bad_file(const char* path, int line, const char* what) {
  return fail(IRIS_E_INVALID_ARG, "%s: line %d: %s", path, line, what);
}

template <typename T>
bool read_values(const std::string& s, std::vector<T>& out, size_t n) {
  std::istringstream is(s);
  out.clear();
  T v;
  while (out.size() < n && is >> v) out.push_back(v);
  return out.size() == n;
}

}  // namespace

extern "C" {

iris_status iris_molecule_read(const char* path, iris_molecule** mol) {
  clear_error();
  if (!path || !mol) return fail(IRIS_E_INVALID_ARG, "path or output pointer is NULL");
  *mol = nullptr;
  std::ifstream in(path);
  if (!in) return fail(IRIS_E_INVALID_ARG, "cannot open molecular data file %s", path);
  Lines ls;
  std::string s;
  int ln = 0;
  while (std::getline(in, s)) {
    ++ln;
    size_t a = s.find_first_not_of(" \t\r");
    if (a == std::string::npos || s[a] == '!') continue;
    ls.text.push_back(s.substr(a));
    ls.number.push_back(ln);
  }
  auto m = new iris_molecule();
  auto cleanup = [&](iris_status st) {
    delete m;
    return st;
  };
  std::vector<double> d;
  std::vector<long> k;
  int n;
  // Molecule name, molecular weight.
  if (!ls.next(s, n) || !ls.next(s, n)) return cleanup(bad_file(path, ln, "truncated header"));
  if (!ls.next(s, n) || !read_values(s, k, 1) || k[0] < 2 || k[0] > iris::kMaxLevels)
    return cleanup(bad_file(path, n, "number of levels must be 2..63"));
  const int L = (int)k[0];
  m->energy_k.assign(L, 0.0);
  m->g.assign(L, 0.0);
  std::vector<char> seen(L, 0);
  const double hck = iris::kHPlanck * iris::kCLight / iris::kKBoltz;  // cm^-1 -> K
  for (int i = 0; i < L; ++i) {
    if (!ls.next(s, n) || !read_values(s, d, 3)) return cleanup(bad_file(path, n, "bad level line"));
    const int idx = (int)d[0] - 1;
    if (idx < 0 || idx >= L || seen[idx] || !(d[2] > 0.0) || !std::isfinite(d[1]))
      return cleanup(bad_file(path, n, "bad level index, energy or weight"));
    seen[idx] = 1;
    m->energy_k[idx] = d[1] * hck;
    m->g[idx] = d[2];
  }
  if (!ls.next(s, n) || !read_values(s, k, 1) || k[0] < 1 || k[0] > 100000)
    return cleanup(bad_file(path, n, "bad number of radiative transitions"));
  const int nr = (int)k[0];
  std::vector<char> pair((size_t)L * L, 0);
  for (int t = 0; t < nr; ++t) {
    if (!ls.next(s, n) || !read_values(s, d, 5))
      return cleanup(bad_file(path, n, "bad radiative transition line"));
    const int u = (int)d[1] - 1, l = (int)d[2] - 1;
    if (u < 0 || u >= L || l < 0 || l >= L || u == l || !(d[3] >= 0.0) || !(d[4] > 0.0) ||
        pair[(size_t)u * L + l])
      return cleanup(bad_file(path, n, "bad or repeated radiative transition"));
    pair[(size_t)u * L + l] = 1;
    m->rad_u.push_back(u);
    m->rad_l.push_back(l);
    m->rad_a.push_back(d[3]);
    m->rad_nu.push_back(d[4] * 1e9);
  }
  if (!ls.next(s, n) || !read_values(s, k, 1) || k[0] < 0 || k[0] > iris::kMaxPartners)
    return cleanup(bad_file(path, n, "number of collision partners must be 0..8"));
  const int np = (int)k[0];
  for (int p = 0; p < np; ++p) {
    iris_molecule::Partner P;
    if (!ls.next(s, n) || !read_values(s, k, 1))
      return cleanup(bad_file(path, n, "bad collision-partner line"));
    P.code = (int)k[0];
    if (!ls.next(s, n) || !read_values(s, k, 1) || k[0] < 1 || k[0] > 100000)
      return cleanup(bad_file(path, n, "bad number of collisional transitions"));
    const int nc = (int)k[0];
    if (!ls.next(s, n) || !read_values(s, k, 1) || k[0] < 1 || k[0] > iris::kMaxTemps)
      return cleanup(bad_file(path, n, "number of collision temperatures must be 1..64"));
    const int nt = (int)k[0];
    while ((int)P.temps.size() < nt) {
      if (!ls.next(s, n)) return cleanup(bad_file(path, ln, "truncated temperature list"));
      std::istringstream is(s);
      double t;
      while ((int)P.temps.size() < nt && is >> t) P.temps.push_back(t);
    }
    for (int i = 0; i < nt; ++i)
      if (!(P.temps[i] > 0.0) || (i > 0 && !(P.temps[i] > P.temps[i - 1])))
        return cleanup(bad_file(path, n, "collision temperatures must increase and be > 0"));
    std::fill(pair.begin(), pair.end(), 0);
    for (int c = 0; c < nc; ++c) {
      if (!ls.next(s, n) || !read_values(s, d, 3 + (size_t)nt))
        return cleanup(bad_file(path, n, "bad collisional transition line"));
      const int u = (int)d[1] - 1, l = (int)d[2] - 1;
      if (u < 0 || u >= L || l < 0 || l >= L || u == l || pair[(size_t)u * L + l])
        return cleanup(bad_file(path, n, "bad or repeated collisional transition"));
      pair[(size_t)u * L + l] = 1;
      for (int i = 0; i < nt; ++i)
        if (!(d[3 + i] >= 0.0)) return cleanup(bad_file(path, n, "negative collision rate"));
      P.u.push_back(u);
      P.l.push_back(l);
      P.rates.insert(P.rates.end(), d.begin() + 3, d.end());
    }
    m->partners.push_back(std::move(P));
  }
  *mol = m;
  return IRIS_OK;
}

iris_status iris_molecule_get_info(const iris_molecule* mol, iris_molecule_info* info) {
  clear_error();
  if (!mol || !info) return fail(IRIS_E_INVALID_ARG, "molecule or info is NULL");
  std::memset(info, 0, sizeof(*info));
  info->n_levels = (int32_t)mol->g.size();
  info->n_transitions = (int32_t)mol->rad_a.size();
  info->n_partners = (int32_t)mol->partners.size();
  for (size_t p = 0; p < mol->partners.size(); ++p) {
    info->partner_code[p] = mol->partners[p].code;
    info->partner_transitions[p] = (int32_t)mol->partners[p].u.size();
    info->partner_temperatures[p] = (int32_t)mol->partners[p].temps.size();
  }
  return IRIS_OK;
}

void iris_molecule_destroy(iris_molecule* mol) { delete mol; }

iris_status iris_levels_create(const iris_molecule* mol, const iris_levels_config* cfg,
                               void* stream, iris_levels** levels) {
  clear_error();
  if (!mol || !cfg || !levels) return fail(IRIS_E_INVALID_ARG, "molecule, config or output is NULL");
  *levels = nullptr;
  const int L = (int)mol->g.size();
  const int nr = (int)mol->rad_a.size();
  if (cfg->transition < 1 || cfg->transition > nr)
    return fail(IRIS_E_INVALID_ARG, "transition %d not in 1..%d", cfg->transition, nr);
  if (!(cfg->t_bar_k >= 0.0) || !std::isfinite(cfg->t_bar_k))
    return fail(IRIS_E_INVALID_ARG, "t_bar_k must be >= 0");
  if (!(cfg->ortho_para > 0.0) || !(cfg->he_per_h >= 0.0))
    return fail(IRIS_E_INVALID_ARG, "need ortho_para > 0 and he_per_h >= 0");
  const int dims[3] = {cfg->n_n, cfg->n_chi, cfg->n_t};
  for (int d : dims)
    if (d < 1 || d > 4096) return fail(IRIS_E_INVALID_ARG, "grid sizes must be 1..4096");
  const long n_pts = (long)cfg->n_n * cfg->n_chi * cfg->n_t;
  if (n_pts > (1L << 24)) return fail(IRIS_E_INVALID_ARG, "grid of %ld nodes above 2^24", n_pts);
  if (!std::isfinite(cfg->ln_nh2_lo) || !std::isfinite(cfg->ln_nh2_hi) ||
      (cfg->n_n > 1 && !(cfg->ln_nh2_hi > cfg->ln_nh2_lo)))
    return fail(IRIS_E_INVALID_ARG, "density axis must be finite and increasing");
  if (!(cfg->chi_lo > 0.0) || !(cfg->chi_hi <= 1.0) ||
      (cfg->n_chi > 1 ? !(cfg->chi_hi > cfg->chi_lo) : !(cfg->chi_lo <= 1.0)))
    return fail(IRIS_E_INVALID_ARG, "molecular-fraction axis must lie in (0, 1] and increase");
  if (!(cfg->t_lo_k > 0.0) || !std::isfinite(cfg->t_hi_k) ||
      (cfg->n_t > 1 && !(cfg->t_hi_k > cfg->t_lo_k)))
    return fail(IRIS_E_INVALID_ARG, "temperature axis must be > 0 and increasing");

  // Partners of the balance: ortho and para H2 where the file has either,
  // else combined H2; atomic H; He. n_s = n_H2 (a + b / chi).
  iris::LevelsParams P{};
  bool has[8] = {};
  for (const auto& p : mol->partners)
    if (p.code >= 1 && p.code <= 7) has[p.code] = true;
  const bool sep = has[iris::kPPara] || has[iris::kPOrtho];
  std::vector<int> used;
  for (size_t i = 0; i < mol->partners.size(); ++i) {
    const int code = mol->partners[i].code;
    double a = 0.0, b = 0.0;
    if (code == iris::kPPara && sep) a = 1.0 / (1.0 + cfg->ortho_para);
    else if (code == iris::kPOrtho && sep) a = cfg->ortho_para / (1.0 + cfg->ortho_para);
    else if (code == iris::kPH2 && !sep) a = 1.0;
    else if (code == iris::kPH) { a = -2.0; b = 2.0; }
    else if (code == iris::kPHe) b = 2.0 * cfg->he_per_h;
    else continue;
    P.dens_a[used.size()] = a;
    P.dens_b[used.size()] = b;
    used.push_back((int)i);
  }
  // Device tables: E, g, radiative (u, l, A, nbar), collisions (u, l, temps, rates).
  std::vector<double> nbar(nr);
  for (int t = 0; t < nr; ++t)
    nbar[t] = cfg->t_bar_k > 0.0
                  ? 1.0 / std::expm1(iris::kHPlanck * mol->rad_nu[t] / (iris::kKBoltz * cfg->t_bar_k))
                  : 0.0;
  std::vector<int> cu, cl;
  std::vector<double> temps, rates;
  for (size_t j = 0; j < used.size(); ++j) {
    const auto& p = mol->partners[used[j]];
    P.coll_off[j] = (int)cu.size();
    P.n_coll[j] = (int)p.u.size();
    P.temp_off[j] = (int)temps.size();
    P.n_temp[j] = (int)p.temps.size();
    P.rate_off[j] = (long)rates.size();
    cu.insert(cu.end(), p.u.begin(), p.u.end());
    cl.insert(cl.end(), p.l.begin(), p.l.end());
    temps.insert(temps.end(), p.temps.begin(), p.temps.end());
    rates.insert(rates.end(), p.rates.begin(), p.rates.end());
  }
  P.n_part = (int)used.size();
  size_t off = 0;
  auto carve = [&](size_t bytes) {
    const size_t o = off;
    off += align256(bytes);
    return o;
  };
  const size_t oE = carve(L * 8), oG = carve(L * 8), oRu = carve(nr * 4), oRl = carve(nr * 4),
               oRa = carve(nr * 8), oRn = carve(nr * 8), oCu = carve(cu.size() * 4 + 4),
               oCl = carve(cl.size() * 4 + 4), oT = carve(temps.size() * 8 + 8),
               oR = carve(rates.size() * 8 + 8);
  std::vector<char> host(off, 0);
  std::memcpy(host.data() + oE, mol->energy_k.data(), L * 8);
  std::memcpy(host.data() + oG, mol->g.data(), L * 8);
  std::memcpy(host.data() + oRu, mol->rad_u.data(), nr * 4);
  std::memcpy(host.data() + oRl, mol->rad_l.data(), nr * 4);
  std::memcpy(host.data() + oRa, mol->rad_a.data(), nr * 8);
  std::memcpy(host.data() + oRn, nbar.data(), nr * 8);
  if (!cu.empty()) {
    std::memcpy(host.data() + oCu, cu.data(), cu.size() * 4);
    std::memcpy(host.data() + oCl, cl.data(), cl.size() * 4);
    std::memcpy(host.data() + oT, temps.data(), temps.size() * 8);
    std::memcpy(host.data() + oR, rates.data(), rates.size() * 8);
  }
  auto lv = new iris_levels();
  lv->cfg = *cfg;
  const int t_obs = cfg->transition - 1;
  const int u_obs = mol->rad_u[t_obs], l_obs = mol->rad_l[t_obs];
  lv->g_u = mol->g[u_obs];
  lv->g_l = mol->g[l_obs];
  lv->nu = mol->rad_nu[t_obs];
  lv->a = mol->rad_a[t_obs];
  int e = (int)hipMalloc(&lv->tables, off);
  if (!e) e = (int)hipMalloc((void**)&lv->grid, (size_t)n_pts * sizeof(float2));
  if (!e) e = (int)hipMemcpy(lv->tables, host.data(), off, hipMemcpyHostToDevice);
  if (e) {
    iris_levels_destroy(lv);
    return hip_status(e, "levels grid set-up");
  }
  char* base = (char*)lv->tables;
  P.E = (const double*)(base + oE);
  P.g = (const double*)(base + oG);
  P.rad_u = (const int*)(base + oRu);
  P.rad_l = (const int*)(base + oRl);
  P.rad_a = (const double*)(base + oRa);
  P.rad_nbar = (const double*)(base + oRn);
  P.coll_u = (const int*)(base + oCu);
  P.coll_l = (const int*)(base + oCl);
  P.temps = (const double*)(base + oT);
  P.rates = (const double*)(base + oR);
  P.n_rad = nr;
  P.L = L;
  P.u_obs = u_obs;
  P.l_obs = l_obs;
  P.n_n = cfg->n_n;
  P.n_c = cfg->n_chi;
  P.n_t = cfg->n_t;
  P.lnn0 = cfg->ln_nh2_lo;
  P.dlnn = cfg->n_n > 1 ? (cfg->ln_nh2_hi - cfg->ln_nh2_lo) / (cfg->n_n - 1) : 0.0;
  P.chi0 = cfg->chi_lo;
  P.dchi = cfg->n_chi > 1 ? (cfg->chi_hi - cfg->chi_lo) / (cfg->n_chi - 1) : 0.0;
  P.lnt0 = std::log(cfg->t_lo_k);
  P.dlnt = cfg->n_t > 1 ? (std::log(cfg->t_hi_k) - std::log(cfg->t_lo_k)) / (cfg->n_t - 1) : 0.0;
  P.grid = lv->grid;
  const int blocks = (int)std::min<long>(n_pts, 16384);
  hipLaunchKernelGGL(iris::ot_levels_kernel, dim3(blocks), dim3(64), 0, (hipStream_t)stream, P);
  e = (int)hipGetLastError();
  if (e) {
    iris_levels_destroy(lv);
    return hip_status(e, "levels kernel");
  }
  *levels = lv;
  return IRIS_OK;
}

iris_status iris_levels_copy_grid(const iris_levels* lv, float* host, size_t n_floats) {
  clear_error();
  if (!lv || !host) return fail(IRIS_E_INVALID_ARG, "levels or host buffer is NULL");
  const size_t n = (size_t)2 * lv->cfg.n_n * lv->cfg.n_chi * lv->cfg.n_t;
  if (n_floats != n) return fail(IRIS_E_INVALID_ARG, "the grid holds %zu floats, not %zu", n, n_floats);
  int e = (int)hipDeviceSynchronize();
  if (!e) e = (int)hipMemcpy(host, lv->grid, n * sizeof(float), hipMemcpyDeviceToHost);
  return e ? hip_status(e, "levels grid copy") : IRIS_OK;
}

void iris_levels_destroy(iris_levels* lv) {
  if (!lv) return;
  if (lv->grid) (void)hipFree(lv->grid);
  if (lv->tables) (void)hipFree(lv->tables);
  delete lv;
}

}  // extern "C"

namespace iris {
namespace host {

// A line with non-LTE populations: its grid's transition must be the line's.
iris_status levels_check(const iris_line* L) {
  const iris_levels* lv = L->levels;
  if (!lv) return IRIS_OK;
  const double gu = 2.0 * L->j_u + 1.0, gl = 2.0 * L->j_u - 1.0;
  if (lv->g_u != gu || lv->g_l != gl || std::fabs(lv->nu - L->nu0_hz) > 1e-6 * L->nu0_hz ||
      std::fabs(lv->a - L->a_ul) > 1e-6 * L->a_ul)
    return fail(IRIS_E_INVALID_ARG,
                "the levels grid's transition (nu %.9g Hz, A %.6g, g %g -> %g) is not the line's "
                "(nu %.9g Hz, A %.6g, g %g -> %g)",
                lv->nu, lv->a, lv->g_u, lv->g_l, L->nu0_hz, L->a_ul, gu, gl);
  if (!(L->h2_frac >= 0.0 && L->h2_frac <= 1.0))
    return fail(IRIS_E_INVALID_ARG, "h2_frac must lie in [0, 1]");
  return IRIS_OK;
}

// Constants of the march for a line with non-LTE populations (after
// levels_check).
void levels_fold(const iris_line* L, Folded& c) {
  const iris_levels* lv = L->levels;
  if (!lv) return;
  const double chi = L->h2_frac == 0.0 ? 1.0 : L->h2_frac;
  const iris_levels_config& g = lv->cfg;
  c.ot = lv->grid;
  c.ot_nn = g.n_n;
  c.ot_nt = g.n_t;
  c.ot_nc = g.n_chi;
  c.ot_n0 = (float)g.ln_nh2_lo;
  c.ot_dn_inv = g.n_n > 1 ? (float)((g.n_n - 1) / (g.ln_nh2_hi - g.ln_nh2_lo)) : 0.f;
  c.ot_t0 = (float)std::log(g.t_lo_k);
  c.ot_dt_inv = g.n_t > 1 ? (float)((g.n_t - 1) / (std::log(g.t_hi_k) - std::log(g.t_lo_k))) : 0.f;
  // The molecular fraction is the same in every cell: its interval and
  // weight are folded here.
  const double uc = g.n_chi > 1 ? (chi - g.chi_lo) * (g.n_chi - 1) / (g.chi_hi - g.chi_lo) : 0.0;
  const double ic =
      g.n_chi > 1 ? std::min(std::max(std::floor(uc), 0.0), (double)(g.n_chi - 2)) : 0.0;
  c.ot_ic = (int32_t)ic;
  c.ot_tc = (float)(uc - ic);
  c.general = 1;  // the line's source function is its own
}

}  // namespace host
}  // namespace iris
