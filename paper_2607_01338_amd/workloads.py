"""Seeded synthetic inputs for the 13CO(2-1) PPV radiative-transfer path.

This module only *generates inputs*: line constants, channel grids and
per-cell fields with the statistics of the paper's workloads. It performs
none of the radiative-transfer arithmetic, and both the HIP path and the
FP64 oracle consume what it produces.

The paper's own inputs are AREPO snapshots interpolated onto an (r, l, b)
lattice ("Physical Tensors"; dataset table: (512, 512, 128) cells,
+-200 km/s). Those snapshots are not available, so seeded random fields of
the same shape and of the following statistics stand in for them:

  ln n_H2 = ln(1e3 cm^-3) + 1.5 * G       (lognormal, median 1e3, sigma_ln 1.5)
  T_kin   ~ U[20, 100] K, independent per cell
  v_los   = rms * G' (+ a rotating ring for the CMZ-scale cube)
  X(13CO) = 1.5e-6 everywhere

where G, G' are independent periodic Gaussian random fields with power
spectrum P(k) ~ k^-4 (k in grid units, k = 0 removed), normalised to zero
mean and unit standard deviation. Streams come from
``numpy.random.SeedSequence(seed).spawn``.
"""

from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

PC_CM = 3.0856775814913673e18  # parsec in cm (IAU 2015)

# 13CO J=2-1 and the dust/background constants of the benchmark workload.
LINE_13CO_21 = dict(
    nu0_hz=220.3987e9,
    a_ul=6.04e-7,
    e_u_k=15.87,
    j_u=2,
    j_max=40,
    m_tracer_amu=28.99827,        # 13C + 16O
    sigma_turb_kms=1.0,
    kappa_dust_cm2g=0.9,          # per gram of dust at 220 GHz
    dust_to_gas=0.01,
    mu_amu_per_h2=2.0 * (1.00794 + 0.1 * 4.002602),  # all H in H2, He/H = 0.1
    t_bg_k=2.725,
    t_inf_k=5.0e4,
    energy_mode=0,
)


@dataclass(frozen=True)
class Channels:
    n_chan: int
    v_lo_kms: float
    dv_kms: float


@dataclass
class Cube:
    """One synthetic cube: native [nx][ny][nz] fields plus geometry."""

    ln_nh2: np.ndarray
    t_kin: np.ndarray
    v_los: np.ndarray
    x_tracer: np.ndarray
    axis: int
    cell_cm: float
    channels: Channels
    t_dust: np.ndarray | None = None
    name: str = ""

    @property
    def shape(self):
        return self.ln_nh2.shape

    @property
    def n_los(self) -> int:
        return self.shape[self.axis]

    @property
    def n_pix(self) -> int:
        return int(np.prod(self.shape)) // self.n_los

    @property
    def samples(self) -> int:
        """cell x channel samples of one forward pass."""
        return int(np.prod(self.shape)) * self.channels.n_chan

    def fields(self):
        out = dict(ln_nh2=self.ln_nh2, t_kin=self.t_kin, v_los=self.v_los, x_tracer=self.x_tracer)
        if self.t_dust is not None:
            out["t_dust"] = self.t_dust
        return out

    def astype(self, dtype) -> "Cube":
        """Same cube with every field cast to ``dtype`` (a NumPy dtype)."""
        f = {k: np.ascontiguousarray(v, dtype=dtype) for k, v in self.fields().items()}
        return replace(self, **f)


def grf(shape, rng: np.random.Generator, slope: float = -4.0) -> np.ndarray:
    """Periodic Gaussian random field with P(k) ~ |k|^slope, zero mean, unit std."""
    white = rng.standard_normal(shape)
    try:
        import scipy.fft as sfft

        fk = sfft.rfftn(white, workers=-1)
    except Exception:  # pragma: no cover - scipy is present in the image
        sfft = None
        fk = np.fft.rfftn(white)
    kx = np.fft.fftfreq(shape[0])[:, None, None]
    ky = np.fft.fftfreq(shape[1])[None, :, None]
    kz = np.fft.rfftfreq(shape[2])[None, None, :]
    k2 = kx * kx + ky * ky + kz * kz
    amp = np.zeros_like(k2)
    nz = k2 > 0
    amp[nz] = k2[nz] ** (slope / 4.0)  # |k|^(slope/2) in amplitude
    fk *= amp
    g = sfft.irfftn(fk, s=shape, workers=-1) if sfft is not None else np.fft.irfftn(fk, s=shape)
    g -= g.mean()
    g /= g.std()
    return g


def ring_velocity(shape, cell_cm: float, v_ring_kms: float = 100.0, r_ring_pc: float = 100.0,
                  los_axis: int = 1) -> np.ndarray:
    """Line-of-sight component of a disk rotating about z through the grid centre.

    v_phi(R) = v_ring * min(R / r_ring, 1). The observer sits beyond the last
    cell along ``los_axis`` (0 = x or 1 = y), so the receding velocity is
    minus the velocity component along that axis.
    """
    nx, ny, _ = shape
    cell_pc = cell_cm / PC_CM
    x = (np.arange(nx) + 0.5 - nx / 2.0) * cell_pc
    y = (np.arange(ny) + 0.5 - ny / 2.0) * cell_pc
    X, Y = np.meshgrid(x, y, indexing="ij")
    R = np.hypot(X, Y)
    vphi = v_ring_kms * np.minimum(R / r_ring_pc, 1.0)
    with np.errstate(invalid="ignore", divide="ignore"):
        vx = np.where(R > 0, -vphi * Y / R, 0.0)
        vy = np.where(R > 0, vphi * X / R, 0.0)
    v_along = vx if los_axis == 0 else vy
    return np.broadcast_to(-v_along[:, :, None], shape).copy()


def make_cube(shape, axis: int, channels: Channels, seed: int = 0, v_rms_kms: float = 20.0,
              ring: bool = False, cell_pc: float = 0.5, dtype=np.float64, t_dust: bool = False,
              name: str = "") -> Cube:
    """Fields with the statistics listed in the module docstring."""
    ss = np.random.SeedSequence(seed).spawn(5)
    r_n, r_t, r_v, r_d = (np.random.default_rng(s) for s in ss[:4])
    cell_cm = cell_pc * PC_CM
    ln_nh2 = np.log(1e3) + 1.5 * grf(shape, r_n)
    t_kin = r_t.uniform(20.0, 100.0, size=shape)
    v_los = v_rms_kms * grf(shape, r_v)
    if ring:
        v_los = v_los + ring_velocity(shape, cell_cm, los_axis=axis)
    x_tracer = np.full(shape, 1.5e-6)
    td = r_d.uniform(10.0, 40.0, size=shape) if t_dust else None
    cube = Cube(ln_nh2, t_kin, v_los, x_tracer, axis, cell_cm, channels, td, name)
    return cube.astype(dtype)


# --- the benchmark workloads -------------------------------------------------

CH_C1 = Channels(64, -64.0, 2.0)
CH_C2 = Channels(800, -200.0, 0.5)
CH_C4 = Channels(256, -128.0, 1.0)


def config_small(seed: int = 0, dtype=np.float64) -> Cube:
    """32^3 cube, 0.5 pc cells, sightlines along z, 64 channels of 2 km/s."""
    return make_cube((32, 32, 32), 2, CH_C1, seed=seed, v_rms_kms=20.0, dtype=dtype,
                     name="32x32x32 FP64, 64 ch x 2 km/s")


def config_cmz(seed: int = 0, dtype=np.float32) -> Cube:
    """512x512x128 CMZ-scale cube: rms 60 km/s plus a 100 km/s ring at 100 pc,
    sightlines along y (512 cells), 800 channels of 0.5 km/s over +-200 km/s."""
    return make_cube((512, 512, 128), 1, CH_C2, seed=seed, v_rms_kms=60.0, ring=True,
                     dtype=dtype, name="512x512x128, 800 ch x 0.5 km/s")


def config_adjoint(seed: int = 0, dtype=np.float32) -> Cube:
    """256^3 cube along z, 256 channels of 1 km/s over +-128 km/s."""
    return make_cube((256, 256, 256), 2, CH_C4, seed=seed, v_rms_kms=20.0, dtype=dtype,
                     name="256^3, 256 ch x 1 km/s")


def config_batch(seed: int = 3):
    """64 cubes of uneven size: two dims from {64,128,256}, one = 64 (randomly
    permuted), random sightline axis, 64..512 channels over +-200 km/s, half
    stored FP32 and half BF16 (returned as float32 here; the caller casts)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(64):
        dims = [int(rng.choice([64, 128, 256])), int(rng.choice([64, 128, 256])), 64]
        rng.shuffle(dims)
        axis = int(rng.integers(0, 3))
        nch = int(rng.integers(64, 513))
        ch = Channels(nch, -200.0, 400.0 / nch)
        cube = make_cube(tuple(dims), axis, ch, seed=1000 + i, v_rms_kms=20.0, dtype=np.float32,
                         name=f"batch[{i}]")
        cube.storage = "bf16" if i % 2 else "f32"
        out.append(cube)
    return out


# --- molecular data in the LAMDA .dat convention -------------------------------
#
# The paper's non-LTE level model reads Einstein A coefficients, level
# energies and weights, and collision-rate tables from a molecular data file
# in the convention of the Leiden Atomic and Molecular Database ("Spectral-Line
# Configuration"). The real 13CO file (with its added atomic-H rates) is not
# available here, so the tests and the benchmark write synthetic molecules in
# that convention. Their rates are made up: smooth, positive, of the usual
# magnitude for CO, and not any database's values.

# Collision-partner codes of the convention.
PARTNER_H2, PARTNER_PH2, PARTNER_OH2, PARTNER_E, PARTNER_H, PARTNER_HE, PARTNER_HP = range(1, 8)
HC_OVER_K_CM_K = 6.62607015e-27 * 2.99792458e10 / 1.380649e-16  # level energy cm^-1 -> K


@dataclass
class Molecule:
    """Molecular data as a LAMDA file holds it (levels 1-based in the file,
    0-based here)."""

    name: str
    weight_amu: float
    energy_cm: np.ndarray        # [n_levels], cm^-1
    g: np.ndarray                # [n_levels] statistical weights
    qn: list                     # [n_levels] quantum-number labels
    rad_up: np.ndarray           # [n_rad] 0-based upper level
    rad_low: np.ndarray          # [n_rad] 0-based lower level
    a_ul: np.ndarray             # [n_rad] s^-1
    freq_ghz: np.ndarray         # [n_rad]
    partners: list = field(default_factory=list)  # dicts: code, label, temps, up, low, rates


def write_lamda(path: str, mol: Molecule) -> None:
    """Write ``mol`` as a LAMDA-convention text file."""
    L = []
    L += ["!MOLECULE", mol.name, "!MOLECULAR WEIGHT", f"{mol.weight_amu:.4f}",
          "!NUMBER OF ENERGY LEVELS", f"{len(mol.g)}",
          "!LEVEL + ENERGIES(cm^-1) + WEIGHT + J"]
    for i, (e, g, q) in enumerate(zip(mol.energy_cm, mol.g, mol.qn)):
        L.append(f"{i + 1:5d} {e:.12e} {g:6.1f}   {q}")
    L += ["!NUMBER OF RADIATIVE TRANSITIONS", f"{len(mol.a_ul)}",
          "!TRANS + UP + LOW + EINSTEINA(s^-1) + FREQ(GHz) + E_u(K)"]
    for t in range(len(mol.a_ul)):
        u, l = int(mol.rad_up[t]), int(mol.rad_low[t])
        L.append(f"{t + 1:5d} {u + 1:5d} {l + 1:5d} {mol.a_ul[t]:.12e} {mol.freq_ghz[t]:.12e} "
                 f"{mol.energy_cm[u] * HC_OVER_K_CM_K:.6f}")
    L += ["!NUMBER OF COLL PARTNERS", f"{len(mol.partners)}"]
    for p in mol.partners:
        temps = np.asarray(p["temps"], dtype=float)
        L += ["!COLLISIONS BETWEEN", f"{p['code']} {p['label']}",
              "!NUMBER OF COLL TRANS", f"{len(p['up'])}",
              "!NUMBER OF COLL TEMPS", f"{len(temps)}", "!COLL TEMPS",
              " ".join(f"{t:.4f}" for t in temps),
              "!TRANS + UP + LOW + COLLRATES(cm^3 s^-1)"]
        for t in range(len(p["up"])):
            rates = " ".join(f"{r:.6e}" for r in p["rates"][t])
            L.append(f"{t + 1:5d} {int(p['up'][t]) + 1:5d} {int(p['low'][t]) + 1:5d} {rates}")
    with open(path, "w") as fh:
        fh.write("\n".join(L) + "\n")


def synthetic_rotor_molecule(line: dict | None = None, n_levels: int = 41,
                             partners=(PARTNER_PH2, PARTNER_OH2, PARTNER_H, PARTNER_HE),
                             temps=(2.0, 5.0, 10.0, 20.0, 40.0, 70.0, 100.0, 150.0, 200.0, 300.0,
                                    500.0, 1000.0),
                             seed: int = 11) -> Molecule:
    """A linear rotor with the line's frequency and Einstein A for its J_u -> J_u - 1
    transition: levels J = 0 .. n_levels - 1 with E_J/k = (h nu0 / k) J (J + 1) / (2 J_u)
    (so that E_u - E_l = h nu0 exactly), weights 2J + 1, dipole transitions
    J -> J - 1 at J nu0 / J_u with A scaled as nu^3 J / (2J + 1); collisional
    de-excitation between every pair of levels from each partner, a smooth made-up law
    K_ul(T) = k_s (T / 100 K)^a_s exp(-(J_u - J_l - 1) / 3) / (1 + J_u / 20) with
    seeded k_s in [2, 8] x 1e-11 cm^3 s^-1 and a_s in [0, 0.4]."""
    line = line or LINE_13CO_21
    ju0 = int(line["j_u"])
    nu0 = float(line["nu0_hz"])
    a0 = float(line["a_ul"])
    J = np.arange(n_levels)
    t0 = 6.62607015e-27 * nu0 / 1.380649e-16
    e_k = t0 * J * (J + 1) / (2.0 * ju0)
    up = J[1:]
    low = J[:-1]
    freq = up * nu0 / ju0
    a = a0 * (freq / nu0) ** 3 * (up / (2.0 * up + 1.0)) / (ju0 / (2.0 * ju0 + 1.0))
    rng = np.random.default_rng(seed)
    plist = []
    labels = {PARTNER_H2: "H2", PARTNER_PH2: "pH2", PARTNER_OH2: "oH2", PARTNER_E: "e",
              PARTNER_H: "H", PARTNER_HE: "He", PARTNER_HP: "H+"}
    pu, pl = np.nonzero(J[:, None] > J[None, :])
    for code in partners:
        ks = rng.uniform(2.0, 8.0) * 1e-11
        ex = rng.uniform(0.0, 0.4)
        tt = np.asarray(temps, dtype=float)
        rates = (ks * (tt[None, :] / 100.0) ** ex * np.exp(-(pu - pl - 1)[:, None] / 3.0)
                 / (1.0 + pu[:, None] / 20.0))
        plist.append(dict(code=int(code), label=f"synthetic-{labels[code]} (made-up rates)",
                          temps=tt, up=pu.copy(), low=pl.copy(), rates=rates))
    return Molecule(name="synthetic rotor", weight_amu=float(line["m_tracer_amu"]),
                    energy_cm=e_k / HC_OVER_K_CM_K, g=2.0 * J + 1.0, qn=[str(j) for j in J],
                    rad_up=up.copy(), rad_low=low.copy(), a_ul=a, freq_ghz=freq / 1e9,
                    partners=plist)
