"""FP64 CPU oracle for the 13CO(2-1) PPV radiative-transfer path.

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package; the product path
(the HIP library and its Python binding) never does, and this package never
imports the product.

The arithmetic lives in ``iris_oracle.cpp`` (plain C++17, double precision,
one OpenMP thread per sightline); this module only marshals NumPy arrays.
Fields are native C-ordered ``[nx][ny][nz]`` float64 arrays; sightlines run
along ``axis`` with position 0 on the far side; pixels enumerate the other
two axes in C order. Outputs are ``[n_pix][n_chan]`` Rayleigh-Jeans kelvin.

Functions (each follows the paper section named in the C++ source):
  forward        -- the five component cubes [T], [C], [D], [L], [B], by formal
                    steps or by smooth integration (line["integrator"]), optically
                    thick or thin (line["transfer"])
  forward_ot     -- the same with non-LTE populations given per cell (the
                    optically thin level balance of ``oracle.levels``)
  adjoint        -- hand-written reverse-mode gradient of sum(g_X * [X])
  complex_step   -- complex-step derivative of the same loss (pins adjoint)
  cell           -- per-cell LTE coefficients (for pins of the populations)
  planck, rj_per_intensity
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "iris_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

_c_double_p = ctypes.POINTER(ctypes.c_double)


class _Line(ctypes.Structure):
    _fields_ = [
        ("nu0_hz", ctypes.c_double),
        ("a_ul", ctypes.c_double),
        ("e_u_k", ctypes.c_double),
        ("j_u", ctypes.c_int32),
        ("j_max", ctypes.c_int32),
        ("m_tracer_amu", ctypes.c_double),
        ("sigma_turb_kms", ctypes.c_double),
        ("kappa_dust", ctypes.c_double),
        ("dust_to_gas", ctypes.c_double),
        ("mu_amu", ctypes.c_double),
        ("t_bg_k", ctypes.c_double),
        ("t_inf_k", ctypes.c_double),
        ("energy_mode", ctypes.c_int32),
        ("units", ctypes.c_int32),
        ("integrator", ctypes.c_int32),
        ("transfer", ctypes.c_int32),
    ]


# Sanitizer flags of the checking build (AddressSanitizer and
# UndefinedBehaviorSanitizer; the process must preload gcc's libasan).
SANITIZE_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                  "-fno-sanitize-recover=undefined"]


def build(sanitize: bool = False, out: str | None = None) -> str:
    """Compile the oracle shared library with g++ (always rebuilds); with
    ``sanitize`` an AddressSanitizer/UBSan build, written to ``out``."""
    dst = out or _LIB
    tmp = dst + ".tmp"
    opt = SANITIZE_FLAGS if sanitize else ["-O2"]
    subprocess.check_call(
        ["g++", *opt, "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-Wall", _SRC, "-o", tmp]
    )
    os.replace(tmp, dst)
    return dst


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        path = os.environ.get("IRIS_ORACLE_LIB")  # a checking build (see build())
        if not path:
            path = _LIB
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
        lib = ctypes.CDLL(path)
        common = [_c_double_p] * 5 + [ctypes.c_int] * 4 + [ctypes.c_double, ctypes.c_int,
                                                            ctypes.c_double, ctypes.c_double,
                                                            ctypes.c_int, ctypes.POINTER(_Line)]
        lib.oracle_forward.argtypes = common + [ctypes.c_int64, ctypes.c_int64] + [_c_double_p] * 5 + [ctypes.c_int]
        lib.oracle_forward.restype = ctypes.c_int
        lib.oracle_forward_ot.argtypes = common + [_c_double_p] * 2 + [_c_double_p] * 5 + [ctypes.c_int]
        lib.oracle_forward_ot.restype = ctypes.c_int
        lib.oracle_adjoint.argtypes = common + [ctypes.c_int64, ctypes.c_int64] + [_c_double_p] * 5 + [_c_double_p] * 5 + [ctypes.c_int]
        lib.oracle_adjoint.restype = ctypes.c_int
        lib.oracle_adjoint_ot.argtypes = common + [_c_double_p] * 2 + [_c_double_p] * 5 + [_c_double_p] * 7 + [ctypes.c_int]
        lib.oracle_adjoint_ot.restype = ctypes.c_int
        lib.oracle_complex_step.argtypes = common + [_c_double_p] * 5 + [ctypes.c_int, ctypes.c_int64, ctypes.c_double]
        lib.oracle_complex_step.restype = ctypes.c_double
        lib.oracle_cell.argtypes = [ctypes.POINTER(_Line)] + [ctypes.c_double] * 5 + [_c_double_p]
        lib.oracle_cell.restype = ctypes.c_int
        lib.oracle_planck.argtypes = [ctypes.c_double, ctypes.c_double]
        lib.oracle_planck.restype = ctypes.c_double
        lib.oracle_rj_per_intensity.argtypes = [ctypes.c_double]
        lib.oracle_rj_per_intensity.restype = ctypes.c_double
        _lib_handle = lib
    return _lib_handle


UNITS = {"trj": 0, "intensity": 1, "tb": 2}


def _units(line) -> int:
    """Output units of ``line``: 0 Rayleigh-Jeans K (default), 1 specific
    intensity (cgs), 2 Planck brightness temperature of [T], [C], [B]."""
    u = line.get("units", 0) if isinstance(line, dict) else getattr(line, "units", 0)
    return UNITS[u.lower()] if isinstance(u, str) else int(u)


INTEGRATORS = {"formal": 0, "smooth": 1}


def _integrator(line) -> int:
    """Integrator of ``line``: 0 formal exponential steps (default), 1 smooth
    (trapezoidal first step, then BDF2, each clamped at zero)."""
    u = line.get("integrator", 0) if isinstance(line, dict) else getattr(line, "integrator", 0)
    return INTEGRATORS[u.lower()] if isinstance(u, str) else int(u)


TRANSFERS = {"thick": 0, "thin": 1, "selective": 2}


def _transfer(line) -> int:
    """Transfer mode of ``line``: 0 optically thick (default), 1 optically
    thin (no absorption, channel-averaged erf profile), 2 selectively thin
    (the line absorbs the continuum, not itself)."""
    u = line.get("transfer", 0) if isinstance(line, dict) else getattr(line, "transfer", 0)
    return TRANSFERS[u.lower()] if isinstance(u, str) else int(u)


def _line(line) -> _Line:
    """Accepts a mapping or an object with the line attributes."""
    get = (lambda k: line[k]) if isinstance(line, dict) else (lambda k: getattr(line, k))
    return _Line(
        float(get("nu0_hz")), float(get("a_ul")), float(get("e_u_k")), int(get("j_u")),
        int(get("j_max")), float(get("m_tracer_amu")), float(get("sigma_turb_kms")),
        float(get("kappa_dust_cm2g")), float(get("dust_to_gas")), float(get("mu_amu_per_h2")),
        float(get("t_bg_k")), float(get("t_inf_k")), int(get("energy_mode")), _units(line),
        _integrator(line), _transfer(line),
    )


def _ptr(a):
    if a is None:
        return ctypes.cast(None, _c_double_p)
    return a.ctypes.data_as(_c_double_p)


@dataclass
class Problem:
    """Fields of one cube plus geometry and channel grid, all float64."""

    ln_nh2: np.ndarray
    t_kin: np.ndarray
    v_los: np.ndarray
    x_tracer: np.ndarray
    axis: int
    cell_cm: float
    n_chan: int
    v_lo_kms: float
    dv_kms: float
    t_dust: np.ndarray | None = None
    simpson_f: int = 0  # Simpson panels per channel (0: profile at channel centres)

    def __post_init__(self):
        for name in ("ln_nh2", "t_kin", "v_los", "x_tracer", "t_dust"):
            a = getattr(self, name)
            if a is not None:
                setattr(self, name, np.ascontiguousarray(a, dtype=np.float64))
        if self.ln_nh2.ndim != 3:
            raise ValueError("fields must be 3-D [nx][ny][nz]")
        shape = self.ln_nh2.shape
        for name in ("t_kin", "v_los", "x_tracer", "t_dust"):
            a = getattr(self, name)
            if a is not None and a.shape != shape:
                raise ValueError(f"{name} shape {a.shape} != {shape}")

    @property
    def shape(self):
        return self.ln_nh2.shape

    @property
    def n_los(self) -> int:
        return self.shape[self.axis]

    @property
    def n_pix(self) -> int:
        nx, ny, nz = self.shape
        return nx * ny * nz // self.n_los

    def _args(self, line):
        nx, ny, nz = self.shape
        return [
            _ptr(self.ln_nh2), _ptr(self.t_kin), _ptr(self.v_los), _ptr(self.x_tracer),
            _ptr(self.t_dust), nx, ny, nz, int(self.axis), float(self.cell_cm),
            int(self.n_chan), float(self.v_lo_kms), float(self.dv_kms), int(self.simpson_f),
            ctypes.byref(_line(line)),
        ]


def forward(prob: Problem, line, pix=None, threads: int = 0) -> dict:
    """Five cubes for pixels ``pix`` (a range(start, stop) or None = all)."""
    p0, p1 = (0, prob.n_pix) if pix is None else (pix.start, pix.stop)
    n = p1 - p0
    out = {k: np.empty((n, prob.n_chan)) for k in "TCDLB"}
    rc = _lib().oracle_forward(*prob._args(line), p0, p1, *(_ptr(out[k]) for k in "TCDLB"),
                               int(threads))
    if rc != 0:
        raise ValueError("oracle_forward rejected its arguments")
    return out


def forward_ot(prob: Problem, line, fu: np.ndarray, fl: np.ndarray, threads: int = 0) -> dict:
    """Five cubes of every pixel with non-LTE populations of the observed
    transition given per cell: ``fu`` = (g_l/g_u) f_u and ``fl`` = f_l - fu,
    native layout (see ``oracle.levels``)."""
    fu = np.ascontiguousarray(fu, dtype=np.float64)
    fl = np.ascontiguousarray(fl, dtype=np.float64)
    if fu.shape != prob.shape or fl.shape != prob.shape:
        raise ValueError("per-cell populations must have the fields' shape")
    out = {k: np.empty((prob.n_pix, prob.n_chan)) for k in "TCDLB"}
    rc = _lib().oracle_forward_ot(*prob._args(line), _ptr(fu), _ptr(fl),
                                  *(_ptr(out[k]) for k in "TCDLB"), int(threads))
    if rc != 0:
        raise ValueError("oracle_forward_ot rejected its arguments")
    return out


def _cot(prob, cot: dict, k: str, n_pix=None):
    a = cot.get(k)
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    n = prob.n_pix if n_pix is None else n_pix
    if a.shape != (n, prob.n_chan):
        raise ValueError(f"cotangent g{k} must be [{n}][n_chan]")
    return a


def adjoint(prob: Problem, line, cot: dict, threads: int = 0, pix=None) -> dict:
    """Gradients of sum(cot[X] * [X]) with respect to the stored fields.

    ``cot`` maps component letters to [n][n_chan] arrays for the pixels
    ``pix`` (a range; None = all). Returns ``{"ln_nh2", "t_kin", "v_los",
    "x_tracer"[, "t_dust"]}`` in native layout; cells of other pixels are 0.
    """
    p0, p1 = (0, prob.n_pix) if pix is None else (pix.start, pix.stop)
    cots = [_cot(prob, cot, k, p1 - p0) for k in "TCDLB"]
    g = {k: np.zeros(prob.shape) for k in ("ln_nh2", "t_kin", "v_los", "x_tracer")}
    gtd = np.zeros(prob.shape) if prob.t_dust is not None else None
    rc = _lib().oracle_adjoint(*prob._args(line), p0, p1, *(_ptr(c) for c in cots),
                               _ptr(g["ln_nh2"]), _ptr(g["t_kin"]), _ptr(g["v_los"]),
                               _ptr(g["x_tracer"]), _ptr(gtd), int(threads))
    if rc != 0:
        raise ValueError("oracle_adjoint rejected its arguments")
    if gtd is not None:
        g["t_dust"] = gtd
    return g


def adjoint_ot(prob: Problem, line, fu: np.ndarray, fl: np.ndarray, cot: dict,
               threads: int = 0) -> dict:
    """Reverse mode with non-LTE populations given per cell (as ``forward_ot``):
    the field gradients of every path but the one through ``fu`` and ``fl``,
    plus ``"fu"`` and ``"fl"``, the gradients with respect to those two
    (``oracle.levels.adjoint`` chains them through the level grid)."""
    fu = np.ascontiguousarray(fu, dtype=np.float64)
    fl = np.ascontiguousarray(fl, dtype=np.float64)
    if fu.shape != prob.shape or fl.shape != prob.shape:
        raise ValueError("per-cell populations must have the fields' shape")
    cots = [_cot(prob, cot, k) for k in "TCDLB"]
    names = ("ln_nh2", "t_kin", "v_los", "x_tracer", "t_dust", "fu", "fl")
    g = {k: np.zeros(prob.shape) for k in names}
    if prob.t_dust is None:
        g["t_dust"] = None
    rc = _lib().oracle_adjoint_ot(*prob._args(line), _ptr(fu), _ptr(fl),
                                  *(_ptr(c) for c in cots), *(_ptr(g[k]) for k in names),
                                  int(threads))
    if rc != 0:
        raise ValueError("oracle_adjoint_ot rejected its arguments")
    if g["t_dust"] is None:
        del g["t_dust"]
    return g


FIELD_INDEX = {"ln_nh2": 0, "t_kin": 1, "v_los": 2, "x_tracer": 3, "t_dust": 4}


def complex_step(prob: Problem, line, cot: dict, field: str, cell: int, h: float = 1e-30) -> float:
    """d/d field[cell] of sum(cot[X] * [X]) by the complex-step method."""
    cots = [_cot(prob, cot, k) for k in "TCDLB"]
    return _lib().oracle_complex_step(*prob._args(line), *(_ptr(c) for c in cots),
                                      FIELD_INDEX[field], int(cell), float(h))


def cell(line, ln_nh2: float, t_kin: float, v_los: float, x_tracer: float, t_dust=None) -> dict:
    """Per-cell cgs coefficients {jL0, aL0, aD, jD, b_cms, Z, n_u, n_l, N}."""
    out = np.empty(9)
    td = t_kin if t_dust is None else t_dust
    _lib().oracle_cell(ctypes.byref(_line(line)), ln_nh2, t_kin, v_los, x_tracer, td, _ptr(out))
    return dict(zip(("jL0", "aL0", "aD", "jD", "b_cms", "Z", "n_u", "n_l", "N"), out))


def planck(nu: float, t: float) -> float:
    return _lib().oracle_planck(nu, t)


def rj_per_intensity(nu: float) -> float:
    return _lib().oracle_rj_per_intensity(nu)
