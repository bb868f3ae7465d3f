"""FP64 oracle of the optically thin (OT) non-LTE level balance and of its
startup grid. TEST INFRASTRUCTURE ONLY: only the test suite, the smoke check
and the CPU-baseline leg of the benchmark use this module; it shares no code
with the HIP library and never imports it.

What it computes, in the paper's order:
  read_lamda      -- molecular data in the LAMDA .dat convention ("Spectral-Line
                     Configuration"): levels, radiative transitions, collision
                     partners with rate tables.
  partner_densities -- the collision partners from n_H2 and the molecular
                     fraction chi = 2 n_H2 / n_H, with all H in H or H2, He per H
                     nucleus and a fixed ortho:para ratio ("Grid Precomputation").
  rate_matrix     -- transition rates R[i, j] (from level i to level j):
                     A_ij + B_ij Jbar_ij + C_ij, with Jbar the Planck intensity
                     at the background temperature Tbar (eq. OT Levels System and
                     the Planck law after it), C_ij = sum_s K_ij^[s] N_s
                     ("Level Populations: Mathematical Solution"), the excitation
                     rates from detailed balance ("Einstein Coefficients,
                     Collisions, and the Detailed Balance").
  populations     -- the OT Levels System: the balance of every level with the
                     ground-state equation replaced by sum n_i = 1, solved
                     directly (numpy.linalg.solve).
  build_grid      -- the per-abundance line factors over a (ln n_H2, chi, ln T)
                     grid ("Grid Precomputation").
  interpolate     -- multilinear interpolation of that grid, linear beyond its
                     bounds ("Grid Precomputation", "Observability
                     Determination").
  adjoint         -- reverse mode of the march through that interpolation
                     ("differentiability modes" in "Synthetic Observation
                     Implementation and Algorithms"): the oracle's reverse
                     mode with the populations held fixed, plus the
                     interpolation's derivatives.

Readings (the paper is silent on these): collision rates are interpolated
linearly in T between the tabulated temperatures and held at the end values
beyond them; the grid axes are uniform in ln n_H2, chi and ln T; the grid holds,
per unit tracer density, FU = (g_l/g_u) f_u and FL = f_l - FU of the observed
transition (f the fractional populations), from which the line coefficients
per tracer are j/N = (h nu / 4 pi) A (g_u/g_l) FU and
alpha/N = (h nu / 4 pi) B_ul (g_u/g_l) FL, and the line source function in
Rayleigh-Jeans kelvin is (h nu / k) FU / FL; where the interpolated FL is not
positive (an inverted or extrapolated level pair) the cell carries no line.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

H = 6.62607015e-27
K = 1.380649e-16
C = 2.99792458e10
HC_K = H * C / K  # cm K: level energy in cm^-1 -> K

# Collision-partner codes of the LAMDA convention.
P_H2, P_PH2, P_OH2, P_E, P_H, P_HE, P_HP = 1, 2, 3, 4, 5, 6, 7


@dataclass
class Partner:
    code: int
    temps: np.ndarray   # [n_t] K
    up: np.ndarray      # [n_c] 0-based upper level
    low: np.ndarray     # [n_c] 0-based lower level
    rates: np.ndarray   # [n_c][n_t] de-excitation rates, cm^3 s^-1


@dataclass
class MolData:
    energy_k: np.ndarray  # [L] level energy / k, K
    g: np.ndarray         # [L]
    up: np.ndarray        # [n_rad] 0-based
    low: np.ndarray       # [n_rad] 0-based
    a: np.ndarray         # [n_rad] s^-1
    nu: np.ndarray        # [n_rad] Hz
    partners: list


def read_lamda(path: str) -> MolData:
    """Parse a LAMDA-convention file. Lines starting with '!' are labels; the
    data lines follow in the convention's fixed order."""
    with open(path) as fh:
        lines = [ln.strip() for ln in fh if ln.strip() and not ln.lstrip().startswith("!")]
    it = iter(lines)
    next(it)                      # molecule name
    float(next(it).split()[0])    # molecular weight
    n_lev = int(next(it).split()[0])
    e, g = np.empty(n_lev), np.empty(n_lev)
    for i in range(n_lev):
        tok = next(it).split()
        idx = int(tok[0]) - 1
        e[idx] = float(tok[1]) * HC_K
        g[idx] = float(tok[2])
    n_rad = int(next(it).split()[0])
    up, low = np.empty(n_rad, int), np.empty(n_rad, int)
    a, nu = np.empty(n_rad), np.empty(n_rad)
    for t in range(n_rad):
        tok = next(it).split()
        up[t], low[t] = int(tok[1]) - 1, int(tok[2]) - 1
        a[t], nu[t] = float(tok[3]), float(tok[4]) * 1e9
    n_part = int(next(it).split()[0])
    parts = []
    for _ in range(n_part):
        code = int(next(it).split()[0])
        n_c = int(next(it).split()[0])
        n_t = int(next(it).split()[0])
        temps = []
        while len(temps) < n_t:
            temps += [float(x) for x in next(it).split()]
        pu, pl = np.empty(n_c, int), np.empty(n_c, int)
        rates = np.empty((n_c, n_t))
        for c in range(n_c):
            tok = next(it).split()
            pu[c], pl[c] = int(tok[1]) - 1, int(tok[2]) - 1
            rates[c] = [float(x) for x in tok[3:3 + n_t]]
        parts.append(Partner(code, np.array(temps[:n_t]), pu, pl, rates))
    return MolData(e, g, up, low, a, nu, parts)


def partner_densities(mol: MolData, n_h2: float, chi: float, ortho_para: float = 3.0,
                      he_per_h: float = 0.1) -> dict:
    """Number density of each partner code the file lists and the path uses
    (H2, para-H2, ortho-H2, H, He; separate ortho/para rates take precedence
    over combined H2 rates; electrons and H+ are not used)."""
    n_h = 2.0 * n_h2 / chi
    codes = {p.code for p in mol.partners}
    dens = {}
    if P_PH2 in codes or P_OH2 in codes:
        if P_PH2 in codes:
            dens[P_PH2] = n_h2 / (1.0 + ortho_para)
        if P_OH2 in codes:
            dens[P_OH2] = n_h2 * ortho_para / (1.0 + ortho_para)
    elif P_H2 in codes:
        dens[P_H2] = n_h2
    if P_H in codes:
        dens[P_H] = (1.0 - chi) * n_h
    if P_HE in codes:
        dens[P_HE] = he_per_h * n_h
    return dens


def collision_rate(p: Partner, T: float) -> np.ndarray:
    """De-excitation rates of one partner at T: linear in T between the
    tabulated temperatures, the end values beyond them."""
    n = len(p.temps)
    if T <= p.temps[0]:
        return p.rates[:, 0].copy()
    if T >= p.temps[-1]:
        return p.rates[:, n - 1].copy()
    k = int(np.searchsorted(p.temps, T, side="right")) - 1
    w = (T - p.temps[k]) / (p.temps[k + 1] - p.temps[k])
    return p.rates[:, k] + w * (p.rates[:, k + 1] - p.rates[:, k])


def rate_matrix(mol: MolData, T: float, dens: dict, t_bar: float) -> np.ndarray:
    """R[i, j]: rate per tracer molecule from level i to level j (i != j)."""
    L = len(mol.g)
    R = np.zeros((L, L))
    u, l = mol.up, mol.low
    # B_ul Jbar = A / (e^{h nu / k Tbar} - 1); B_lu = (g_u/g_l) B_ul.
    nbar = np.zeros(len(mol.a)) if t_bar <= 0.0 else 1.0 / np.expm1(H * mol.nu / (K * t_bar))
    np.add.at(R, (u, l), mol.a * (1.0 + nbar))
    np.add.at(R, (l, u), mol.g[u] / mol.g[l] * mol.a * nbar)
    for p in mol.partners:
        if p.code not in dens:
            continue
        down = collision_rate(p, T) * dens[p.code]
        pu, pl = p.up, p.low
        np.add.at(R, (pu, pl), down)
        np.add.at(R, (pl, pu), down * mol.g[pu] / mol.g[pl]
                  * np.exp(-(mol.energy_k[pu] - mol.energy_k[pl]) / T))
    return R


def populations(mol: MolData, T: float, dens: dict, t_bar: float) -> np.ndarray:
    """Fractional level populations (sum 1) of the OT Levels System."""
    R = rate_matrix(mol, T, dens, t_bar)
    L = len(mol.g)
    # Row i: sum_j n_j R[j, i] - n_i sum_j R[i, j] = 0; row 0 -> sum n_i = 1.
    M = R.T - np.diag(R.sum(axis=1))
    M[0, :] = 1.0
    b = np.zeros(L)
    b[0] = 1.0
    return np.linalg.solve(M, b)


@dataclass
class Grid:
    lnn: np.ndarray   # [n_n] ln n_H2 nodes
    chi: np.ndarray   # [n_chi]
    lnt: np.ndarray   # [n_t] ln T nodes
    FU: np.ndarray    # [n_chi][n_t][n_n]
    FL: np.ndarray


def axis_nodes(lo: float, hi: float, n: int) -> np.ndarray:
    return np.array([lo]) if n == 1 else lo + (hi - lo) * np.arange(n) / (n - 1)


def transition_levels(mol: MolData, transition: int):
    """Upper and lower level (0-based) of the 1-based radiative transition."""
    return int(mol.up[transition - 1]), int(mol.low[transition - 1])


def build_grid(mol: MolData, transition: int, t_bar: float, lnn_range, chi_range, t_range,
               shape, ortho_para: float = 3.0, he_per_h: float = 0.1) -> Grid:
    """FU, FL of the transition at every node; shape = (n_n, n_chi, n_t)."""
    n_n, n_c, n_t = shape
    lnn = axis_nodes(*lnn_range, n_n)
    chi = axis_nodes(*chi_range, n_c)
    lnt = axis_nodes(np.log(t_range[0]), np.log(t_range[1]), n_t)
    u, l = transition_levels(mol, transition)
    FU = np.empty((n_c, n_t, n_n))
    FL = np.empty((n_c, n_t, n_n))
    for ic, x in enumerate(chi):
        for it, lt in enumerate(lnt):
            T = np.exp(lt)
            for i_n, ln in enumerate(lnn):
                f = populations(mol, T, partner_densities(mol, np.exp(ln), x, ortho_para,
                                                          he_per_h), t_bar)
                fu = mol.g[l] / mol.g[u] * f[u]
                FU[ic, it, i_n] = fu
                FL[ic, it, i_n] = f[l] - fu
    return Grid(lnn, chi, lnt, FU, FL)


def node_values(mol: MolData, transition: int, t_bar: float, lnn: float, chi: float, T: float,
                ortho_para: float = 3.0, he_per_h: float = 0.1):
    """(FU, FL) at one point, solved directly."""
    u, l = transition_levels(mol, transition)
    f = populations(mol, T, partner_densities(mol, np.exp(lnn), chi, ortho_para, he_per_h), t_bar)
    fu = mol.g[l] / mol.g[u] * f[u]
    return fu, f[l] - fu


def _coord(nodes: np.ndarray, x: np.ndarray):
    """Interval index (clamped to the grid) and local coordinate (not clamped)."""
    n = len(nodes)
    if n == 1:
        return np.zeros(np.shape(x), int), np.zeros(np.shape(x))
    d = (nodes[-1] - nodes[0]) / (n - 1)
    u = (np.asarray(x, dtype=float) - nodes[0]) / d
    i = np.clip(np.floor(u), 0, n - 2).astype(int)
    return i, u - i


def interpolate(grid: Grid, F: np.ndarray, lnn, chi, T) -> np.ndarray:
    """Multilinear interpolation of F over (ln n_H2, chi, ln T), extended
    linearly beyond the grid (the edge interval's formula)."""
    i_n, t_n = _coord(grid.lnn, lnn)
    i_c, t_c = _coord(grid.chi, chi)
    i_t, t_t = _coord(grid.lnt, np.log(T))
    n_c, n_t, n_n = F.shape
    out = np.zeros(np.broadcast(t_n, t_c, t_t).shape)
    for dc in (0, 1):
        wc = t_c if dc else 1.0 - t_c
        jc = np.minimum(i_c + dc, n_c - 1)
        for dt in (0, 1):
            wt = t_t if dt else 1.0 - t_t
            jt = np.minimum(i_t + dt, n_t - 1)
            for dn in (0, 1):
                wn = t_n if dn else 1.0 - t_n
                jn = np.minimum(i_n + dn, n_n - 1)
                out = out + wc * wt * wn * F[jc, jt, jn]
    return out


def cell_fractions(grid: Grid, lnn, T, chi: float = 1.0):
    """Per-cell (FU, FL) from the grid for fields ln n_H2 and T_kin (and a
    uniform molecular fraction chi)."""
    c = np.full(np.shape(lnn), float(chi))
    return interpolate(grid, grid.FU, lnn, c, T), interpolate(grid, grid.FL, lnn, c, T)


def interpolate_grad(grid: Grid, F: np.ndarray, lnn, chi, T):
    """Derivatives of ``interpolate`` with respect to ln n_H2 and T: the
    multilinear form's slopes in the interval the point falls in (the edge
    interval's beyond the grid), the T slope through d ln T / dT = 1/T."""
    i_n, t_n = _coord(grid.lnn, lnn)
    i_c, t_c = _coord(grid.chi, chi)
    i_t, t_t = _coord(grid.lnt, np.log(T))
    n_c, n_t, n_n = F.shape
    d_n = (grid.lnn[-1] - grid.lnn[0]) / (n_n - 1) if n_n > 1 else np.inf
    d_t = (grid.lnt[-1] - grid.lnt[0]) / (n_t - 1) if n_t > 1 else np.inf
    shape = np.broadcast(t_n, t_c, t_t).shape
    dn, dlt = np.zeros(shape), np.zeros(shape)
    for dc in (0, 1):
        wc = t_c if dc else 1.0 - t_c
        jc = np.minimum(i_c + dc, n_c - 1)
        for dt in (0, 1):
            wt = t_t if dt else 1.0 - t_t
            st = (1.0 if dt else -1.0) / d_t
            jt = np.minimum(i_t + dt, n_t - 1)
            for dnn in (0, 1):
                wn = t_n if dnn else 1.0 - t_n
                sn = (1.0 if dnn else -1.0) / d_n
                jn = np.minimum(i_n + dnn, n_n - 1)
                f = F[jc, jt, jn]
                dn = dn + wc * wt * sn * f
                dlt = dlt + wc * st * wn * f
    return dn, dlt / np.asarray(T, dtype=float)


def adjoint(prob, line, grid: Grid, cot: dict, chi: float = 1.0, threads: int = 0) -> dict:
    """Gradients of sum(cot[X] * [X]) with respect to the stored fields, the
    level populations interpolated in ``grid`` per cell at the fields'
    ln n_H2 and T_kin (and a uniform molecular fraction chi)."""
    import oracle

    fu, fl = cell_fractions(grid, prob.ln_nh2, prob.t_kin, chi)
    g = oracle.adjoint_ot(prob, line, fu, fl, cot, threads)
    c = np.full(np.shape(prob.ln_nh2), float(chi))
    dfu_n, dfu_t = interpolate_grad(grid, grid.FU, prob.ln_nh2, c, prob.t_kin)
    dfl_n, dfl_t = interpolate_grad(grid, grid.FL, prob.ln_nh2, c, prob.t_kin)
    gfu, gfl = g.pop("fu"), g.pop("fl")
    g["ln_nh2"] = g["ln_nh2"] + gfu * dfu_n + gfl * dfl_n
    g["t_kin"] = g["t_kin"] + gfu * dfu_t + gfl * dfl_t
    return g
