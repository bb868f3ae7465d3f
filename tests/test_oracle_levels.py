"""Pins of the FP64 oracle of the optically thin (OT) level balance and its
startup grid (oracle/levels.py) against what the mathematics fixes: closed
forms of two- and three-level systems, the Boltzmann limits, detailed balance,
conservation, exact reproduction of multilinear functions by the grid
interpolation, and the LTE march at collision-dominated densities.
Paper sections: "Level Populations: Mathematical Solution" (eq. OT Levels
System, the Planck background), "Einstein Coefficients, Collisions, and the
Detailed Balance", "Spectral-Line Configuration", "Grid Precomputation"."""

import math
import os

import numpy as np
import pytest

import oracle
from oracle import levels as Lv
from paper_2607_01338_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
H, K, C = 6.62607015e-27, 1.380649e-16, 2.99792458e10


def boltzmann(mol, T):
    w = mol.g * np.exp(-mol.energy_k / T)
    return w / w.sum()


@pytest.fixture(scope="module")
def rotor(tmp_path_factory):
    path = str(tmp_path_factory.mktemp("mol") / "rotor.dat")
    gen = W.synthetic_rotor_molecule()
    W.write_lamda(path, gen)
    return gen, Lv.read_lamda(path)


# --- reader --------------------------------------------------------------------

def test_reader_round_trip_of_a_written_molecule(rotor):
    gen, mol = rotor
    np.testing.assert_allclose(mol.energy_k, gen.energy_cm * W.HC_OVER_K_CM_K, rtol=1e-11,
                               atol=1e-12)
    np.testing.assert_array_equal(mol.g, gen.g)
    np.testing.assert_array_equal(mol.up, gen.rad_up)
    np.testing.assert_array_equal(mol.low, gen.rad_low)
    np.testing.assert_allclose(mol.a, gen.a_ul, rtol=1e-11)
    np.testing.assert_allclose(mol.nu, gen.freq_ghz * 1e9, rtol=1e-11)
    assert [p.code for p in mol.partners] == [p["code"] for p in gen.partners]
    for p, q in zip(mol.partners, gen.partners):
        np.testing.assert_allclose(p.temps, q["temps"], rtol=1e-6)
        np.testing.assert_array_equal(p.up, q["up"])
        np.testing.assert_array_equal(p.low, q["low"])
        np.testing.assert_allclose(p.rates, q["rates"], rtol=1e-6)


def test_reader_golden_toy_file():
    # Hand-written file: three levels, two partners, a temperature list broken
    # over two lines.
    mol = Lv.read_lamda(os.path.join(GOLDEN, "toy3_lamda.dat"))
    np.testing.assert_allclose(mol.energy_k, np.array([0.0, 4.0, 12.0]) * Lv.HC_K, rtol=1e-15)
    np.testing.assert_array_equal(mol.g, [1.0, 3.0, 5.0])
    np.testing.assert_array_equal(mol.up, [1, 2])
    np.testing.assert_array_equal(mol.low, [0, 1])
    np.testing.assert_allclose(mol.a, [1e-6, 8e-6])
    np.testing.assert_allclose(mol.nu, [119.916983e9, 239.833966e9])
    assert [p.code for p in mol.partners] == [Lv.P_H2, Lv.P_HE]
    np.testing.assert_allclose(mol.partners[0].temps, [10.0, 20.0, 50.0, 100.0])
    np.testing.assert_allclose(mol.partners[0].rates[2], [2e-11, 2e-11, 2.5e-11, 3e-11])
    np.testing.assert_allclose(mol.partners[1].temps, [10.0, 100.0])
    # Transition frequencies agree with the level energies: nu = c (E_u - E_l).
    np.testing.assert_allclose(mol.nu, C * np.array([4.0, 8.0]), rtol=1e-8)


# --- partners and collision rates ----------------------------------------------

def test_partner_densities(rotor):
    _, mol = rotor
    d = Lv.partner_densities(mol, 1e3, 0.8, ortho_para=3.0, he_per_h=0.1)
    n_h = 2e3 / 0.8
    assert d[Lv.P_OH2] == pytest.approx(750.0) and d[Lv.P_PH2] == pytest.approx(250.0)
    assert d[Lv.P_H] == pytest.approx(0.2 * n_h)
    assert d[Lv.P_HE] == pytest.approx(0.1 * n_h)
    # H nuclei: 2 n_H2 + n_H(atomic) = n_H.
    assert 2 * (d[Lv.P_OH2] + d[Lv.P_PH2]) + d[Lv.P_H] == pytest.approx(n_h)
    toy = Lv.read_lamda(os.path.join(GOLDEN, "toy3_lamda.dat"))
    d = Lv.partner_densities(toy, 1e3, 1.0)
    assert d == {Lv.P_H2: 1e3, Lv.P_HE: pytest.approx(200.0)}


def test_collision_rates_interpolate_linearly_in_T_and_hold_beyond_the_table():
    toy = Lv.read_lamda(os.path.join(GOLDEN, "toy3_lamda.dat"))
    p = toy.partners[0]
    np.testing.assert_allclose(Lv.collision_rate(p, 20.0), [2e-11, 6e-12, 2e-11])
    np.testing.assert_allclose(Lv.collision_rate(p, 35.0), [2.5e-11, 6.5e-12, 2.25e-11])
    np.testing.assert_allclose(Lv.collision_rate(p, 5.0), [1e-11, 5e-12, 2e-11])
    np.testing.assert_allclose(Lv.collision_rate(p, 500.0), [4e-11, 8e-12, 3e-11])


def test_excitation_rates_obey_detailed_balance(rotor):
    _, mol = rotor
    mol0 = Lv.MolData(mol.energy_k, mol.g, mol.up, mol.low, 0.0 * mol.a, mol.nu, mol.partners)
    T = 37.0
    R = Lv.rate_matrix(mol0, T, Lv.partner_densities(mol0, 5e3, 1.0), 0.0)
    for u, l in [(1, 0), (2, 1), (5, 2), (12, 3)]:
        expect = mol.g[u] / mol.g[l] * math.exp(-(mol.energy_k[u] - mol.energy_k[l]) / T)
        assert R[l, u] / R[u, l] == pytest.approx(expect, rel=1e-13)


# --- level populations -----------------------------------------------------------

def two_level_molecule(tmp_path, A=2e-5, k_ul=(1e-11, 3e-11), temps=(10.0, 100.0)):
    mol = W.Molecule(name="two-level", weight_amu=28.0, energy_cm=np.array([0.0, 3.0]),
                     g=np.array([1.0, 3.0]), qn=["0", "1"], rad_up=np.array([1]),
                     rad_low=np.array([0]), a_ul=np.array([A]),
                     freq_ghz=np.array([3.0 * C / 1e9]),
                     partners=[dict(code=W.PARTNER_H2, label="H2", temps=np.array(temps),
                                    up=np.array([1]), low=np.array([0]),
                                    rates=np.array([list(k_ul)]))])
    path = str(tmp_path / "two.dat")
    W.write_lamda(path, mol)
    return Lv.read_lamda(path)


@pytest.mark.parametrize("n_h2,T,tbar", [(1e2, 30.0, 2.725), (1e5, 70.0, 2.725),
                                         (3e3, 15.0, 0.0), (1e4, 45.0, 20.0)])
def test_two_level_closed_form(tmp_path, n_h2, T, tbar):
    mol = two_level_molecule(tmp_path)
    f = Lv.populations(mol, T, Lv.partner_densities(mol, n_h2, 1.0), tbar)
    A, nu = mol.a[0], mol.nu[0]
    k_ul = np.interp(T, [10.0, 100.0], [1e-11, 3e-11])
    C_ul = k_ul * n_h2
    C_lu = C_ul * 3.0 * math.exp(-(mol.energy_k[1] - mol.energy_k[0]) / T)
    nbar = 0.0 if tbar == 0 else 1.0 / math.expm1(H * nu / (K * tbar))
    ratio = (C_lu + 3.0 * A * nbar) / (C_ul + A * (1.0 + nbar))  # n_u / n_l
    assert f[1] / f[0] == pytest.approx(ratio, rel=1e-13)
    assert f.sum() == pytest.approx(1.0, abs=1e-15)


def test_three_level_brute_force():
    # The toy file's system written out level by level and solved by Cramer's rule.
    mol = Lv.read_lamda(os.path.join(GOLDEN, "toy3_lamda.dat"))
    T, n, tbar = 35.0, 2e3, 2.725
    d = Lv.partner_densities(mol, n, 1.0)
    R = np.zeros((3, 3))
    E, g = mol.energy_k, mol.g
    for t, (u, l) in enumerate([(1, 0), (2, 1)]):
        nb = 1.0 / math.expm1(H * mol.nu[t] / (K * tbar))
        R[u, l] += mol.a[t] * (1 + nb)
        R[l, u] += g[u] / g[l] * mol.a[t] * nb
    for p in mol.partners:
        for c, (u, l) in enumerate(zip(p.up, p.low)):
            k = np.interp(T, p.temps, p.rates[c]) * d[p.code]
            R[u, l] += k
            R[l, u] += k * g[u] / g[l] * math.exp(-(E[u] - E[l]) / T)
    # Level 1 and 2 balance, and conservation.
    rows = [[1.0, 1.0, 1.0],
            [R[0, 1], -(R[1, 0] + R[1, 2]), R[2, 1]],
            [R[0, 2], R[1, 2], -(R[2, 0] + R[2, 1])]]
    rhs = [1.0, 0.0, 0.0]
    D = np.linalg.det(rows)
    expect = []
    for j in range(3):
        m = [r[:] for r in rows]
        for i in range(3):
            m[i][j] = rhs[i]
        expect.append(np.linalg.det(m) / D)
    f = Lv.populations(mol, T, d, tbar)
    np.testing.assert_allclose(f, expect, rtol=1e-12)


@pytest.mark.parametrize("n_h2", [1e-2, 1e1, 1e3, 1e6, 1e9])
def test_background_at_the_kinetic_temperature_gives_boltzmann(rotor, n_h2):
    # Radiative and collisional rates both satisfy detailed balance at T: the
    # balance is the Boltzmann distribution at every density.
    _, mol = rotor
    T = 41.0
    f = Lv.populations(mol, T, Lv.partner_densities(mol, n_h2, 1.0), T)
    np.testing.assert_allclose(f, boltzmann(mol, T), rtol=1e-9, atol=1e-30)


def test_collision_dominated_limit_is_boltzmann_at_T_kin(rotor):
    _, mol = rotor
    T = 60.0
    f = Lv.populations(mol, T, Lv.partner_densities(mol, 1e13, 1.0), 2.725)
    b = boltzmann(mol, T)
    np.testing.assert_allclose(f[:12], b[:12], rtol=1e-6)


def test_collisionless_limit_is_boltzmann_at_the_background(rotor):
    _, mol = rotor
    tbar = 12.0
    f = Lv.populations(mol, 80.0, Lv.partner_densities(mol, 1e-9, 1.0), tbar)
    b = boltzmann(mol, tbar)
    np.testing.assert_allclose(f[:8], b[:8], rtol=1e-6)


def test_subthermal_excitation_between_the_limits(rotor):
    # At intermediate densities the J=2 excitation temperature lies between
    # the background and the kinetic temperature.
    _, mol = rotor
    T, tbar = 60.0, 2.725
    f = Lv.populations(mol, T, Lv.partner_densities(mol, 3e2, 1.0), tbar)
    dE = mol.energy_k[2] - mol.energy_k[1]
    tex = dE / math.log(f[1] * mol.g[2] / (f[2] * mol.g[1]))
    assert tbar < tex < T
    assert f.sum() == pytest.approx(1.0, abs=1e-14)
    assert np.all(f > 0)


# --- grid and interpolation --------------------------------------------------------

def test_interpolation_reproduces_multilinear_functions_inside_and_beyond():
    g = Lv.Grid(Lv.axis_nodes(0.0, 9.0, 7), Lv.axis_nodes(0.2, 1.0, 3),
                Lv.axis_nodes(math.log(5.0), math.log(500.0), 9), None, None)
    N, X, T = np.meshgrid(g.lnn, g.chi, g.lnt, indexing="ij")
    f = lambda n, c, lt: 1.5 + 0.3 * n - 2.0 * c + 0.7 * lt + 0.1 * n * c - 0.05 * c * lt \
        + 0.02 * n * lt + 0.01 * n * c * lt
    F = np.transpose(f(N, X, T), (1, 2, 0))  # [chi][T][n]
    rng = np.random.default_rng(3)
    n = rng.uniform(-2.0, 11.0, 200)
    c = rng.uniform(0.1, 1.1, 200)
    lt = rng.uniform(math.log(2.0), math.log(900.0), 200)
    np.testing.assert_allclose(Lv.interpolate(g, F, n, c, np.exp(lt)), f(n, c, lt), rtol=1e-12,
                               atol=1e-12)
    # Node values exactly.
    np.testing.assert_allclose(Lv.interpolate(g, F, g.lnn[3], g.chi[1], math.exp(g.lnt[4])),
                               F[1, 4, 3], rtol=1e-14)


def test_grid_nodes_are_the_direct_solution(rotor):
    _, mol = rotor
    grid = Lv.build_grid(mol, 2, 2.725, (math.log(10.0), math.log(1e5)), (0.5, 1.0),
                         (10.0, 200.0), (5, 2, 4))
    for (i_n, i_c, i_t) in [(0, 0, 0), (4, 1, 3), (2, 1, 1)]:
        fu, fl = Lv.node_values(mol, 2, 2.725, grid.lnn[i_n], grid.chi[i_c],
                                math.exp(grid.lnt[i_t]))
        assert grid.FU[i_c, i_t, i_n] == fu and grid.FL[i_c, i_t, i_n] == fl
    # Transition 2 is J = 2 -> 1 (0-based levels 2 and 1).
    assert Lv.transition_levels(mol, 2) == (2, 1)


# --- the march with non-LTE populations ---------------------------------------------

def _slab_problem(n, T, ln_n, X, ch=(60, -6.0, 0.2)):
    shape = (1, 1, n)
    return oracle.Problem(np.full(shape, ln_n), np.full(shape, T), np.zeros(shape),
                          np.full(shape, X), 2, 0.5 * W.PC_CM, *ch)


def test_ot_slab_closed_form(rotor):
    # A uniform slab without dust with populations FU, FL: [L] = (J_ex - J_bg)(1 - e^{-tau})
    # with J_ex = (h nu / k) FU / FL and tau from FL (pins the populations -> coefficients map).
    _, mol = rotor
    L = dict(W.LINE_13CO_21, kappa_dust_cm2g=0.0)
    T, ln_n, X, n = 35.0, math.log(2e3), 1.5e-6, 7
    fu, fl = Lv.node_values(mol, 2, 2.725, ln_n, 1.0, T)
    pr = _slab_problem(n, T, ln_n, X)
    out = oracle.forward_ot(pr, L, np.full(pr.shape, fu), np.full(pr.shape, fl))
    t0 = H * L["nu0_hz"] / K
    jex = t0 * fu / fl
    jbg = t0 / math.expm1(t0 / L["t_bg_k"])
    nu = L["nu0_hz"]
    bul = C * C * L["a_ul"] / (2 * H * nu ** 3)
    alpha0 = H * nu / (4 * math.pi) * X * math.exp(ln_n) * bul * (5.0 / 3.0) * fl  # per Hz-integrated
    b = math.sqrt(2 * K * T / (L["m_tracer_amu"] * 1.66053906660e-24) + 2 * 1e10)
    v = (-6.0 + (np.arange(60) + 0.5) * 0.2) * 1e5
    phi = (C / nu) * np.exp(-(v / b) ** 2) / (b * math.sqrt(math.pi))
    tau = n * 0.5 * W.PC_CM * alpha0 * phi
    np.testing.assert_allclose(out["L"][0], (jex - jbg) * -np.expm1(-tau), rtol=1e-10,
                               atol=1e-13 * jex)


def test_ot_march_at_collision_dominated_density_is_the_lte_march(rotor):
    _, mol = rotor
    L = dict(W.LINE_13CO_21)
    cube = W.make_cube((2, 2, 12), 2, W.Channels(48, -12.0, 0.5), seed=7, v_rms_kms=3.0)
    pr = oracle.Problem(cube.ln_nh2, cube.t_kin, cube.v_los, cube.x_tracer, 2, cube.cell_cm,
                        48, -12.0, 0.5)
    # Populations solved at 1e13 cm^-3 (collision-dominated) for each cell's T.
    fu = np.empty(pr.shape)
    fl = np.empty(pr.shape)
    for idx in np.ndindex(pr.shape):
        fu[idx], fl[idx] = Lv.node_values(mol, 2, 2.725, math.log(1e13), 1.0, pr.t_kin[idx])
    ot = oracle.forward_ot(pr, L, fu, fl)
    lte = oracle.forward(pr, L)
    for k in "TL":
        np.testing.assert_allclose(ot[k], lte[k], rtol=2e-6, atol=2e-6 * np.max(np.abs(lte[k])))
    np.testing.assert_allclose(ot["C"], lte["C"], rtol=1e-14)


def test_inverted_or_extrapolated_populations_carry_no_line():
    pr = _slab_problem(4, 30.0, math.log(1e3), 1e-6)
    L = dict(W.LINE_13CO_21)
    out = oracle.forward_ot(pr, L, np.full(pr.shape, 0.1), np.full(pr.shape, -0.01))
    assert np.max(np.abs(out["L"])) == 0.0


# --- reverse mode through the level grid ------------------------------------------

def test_interpolation_gradient_matches_differences():
    # A random grid; points inside intervals (away from the nodes) and beyond
    # the grid on both sides: the multilinear form is linear in ln n_H2 and
    # in ln T on each interval, so central differences within one interval
    # reproduce its slopes.
    rng = np.random.default_rng(5)
    grid = Lv.Grid(lnn=Lv.axis_nodes(0.0, 10.0, 6), chi=Lv.axis_nodes(0.5, 1.0, 3),
                   lnt=Lv.axis_nodes(math.log(10.0), math.log(200.0), 7),
                   FU=rng.standard_normal((3, 7, 6)), FL=rng.standard_normal((3, 7, 6)))
    d_n = 2.0
    d_t = (math.log(200.0) - math.log(10.0)) / 6
    lnn = np.array([0.3, 4.9, 7.1, -1.5, 11.7]) * 1.0 + 0.0
    lnn = np.concatenate([lnn, 2.0 * np.arange(5) + d_n * rng.uniform(0.2, 0.8, 5)])
    lt = math.log(10.0) + d_t * (np.array([0.4, 2.3, 5.6, -0.7, 6.8, 1.5, 3.3, 4.4, 0.6, 5.2]))
    T = np.exp(lt)
    chi = rng.uniform(0.5, 1.0, lnn.size)
    for F in (grid.FU, grid.FL):
        dn, dT = Lv.interpolate_grad(grid, F, lnn, chi, T)
        h = 1e-6
        fn = (Lv.interpolate(grid, F, lnn + h, chi, T) - Lv.interpolate(grid, F, lnn - h, chi, T)) / (2 * h)
        ht = 1e-7 * T
        ft = (Lv.interpolate(grid, F, lnn, chi, T + ht) - Lv.interpolate(grid, F, lnn, chi, T - ht)) / (2 * ht)
        np.testing.assert_allclose(dn, fn, rtol=1e-6, atol=1e-8)
        np.testing.assert_allclose(dT, ft, rtol=1e-5, atol=1e-9)


@pytest.mark.parametrize("t_dust", [False, True])
def test_reverse_mode_through_the_level_grid_matches_differences(rotor, t_dust):
    # Gradients of sum(cot * [X]) with the populations interpolated per cell
    # from a level grid, against central differences of the same loss (the
    # fields moved, the populations interpolated again).
    _, mol = rotor
    grid = Lv.build_grid(mol, 2, 2.725, (math.log(10.0), math.log(1e5)), (0.5, 1.0),
                         (8.0, 120.0), (7, 2, 6))
    cube = W.make_cube((2, 2, 6), 2, W.Channels(24, -12.0, 1.0), seed=21, v_rms_kms=4.0,
                       t_dust=t_dust)
    L = dict(W.LINE_13CO_21, kappa_dust_cm2g=300.0)
    chi = 0.8

    def problem_of(f):
        return oracle.Problem(f["ln_nh2"], f["t_kin"], f["v_los"], f["x_tracer"], 2,
                              cube.cell_cm, 24, -12.0, 1.0, f.get("t_dust"))

    fields = {k: v.copy() for k, v in cube.fields().items()}
    rng = np.random.default_rng(4)
    cot = {k: rng.standard_normal((cube.n_pix, 24)) for k in "TCDLB"}

    def loss(f):
        pr = problem_of(f)
        fu, fl = Lv.cell_fractions(grid, pr.ln_nh2, pr.t_kin, chi)
        out = oracle.forward_ot(pr, L, fu, fl)
        return sum(np.sum(cot[k] * out[k]) for k in "TCDLB")

    g = Lv.adjoint(problem_of(fields), L, grid, cot, chi)
    names = ["ln_nh2", "t_kin", "v_los", "x_tracer"] + (["t_dust"] if t_dust else [])
    for name in names:
        for cell in rng.choice(cube.ln_nh2.size, 5, replace=False):
            x0 = fields[name].ravel()[cell]
            h = 1e-6 * (max(abs(x0), 1.0) if name == "v_los" else abs(x0))
            vals = []
            for sgn in (1, -1):
                f = {k: v.copy() for k, v in fields.items()}
                f[name].ravel()[cell] = x0 + sgn * h
                vals.append(loss(f))
            fd = (vals[0] - vals[1]) / (2 * h)
            ref = g[name].ravel()[cell]
            scale = np.max(np.abs(g[name]))
            assert abs(ref - fd) <= 1e-5 * scale + 1e-6 * abs(fd), (name, cell, ref, fd)
