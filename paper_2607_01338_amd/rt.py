"""PyTorch-facing binding of the HIP library (``libiris_rt.so``).

Argument marshalling only: every step of the synthesis runs in the HIP
kernels behind the C ABI declared in ``include/iris_rt.h``; PyTorch supplies
device memory (the caching allocator) and the current stream. There is no
CPU fallback: if the library cannot be loaded, or a tensor is not on a GPU,
the call raises.

Entry points (same names as the C ABI):
  iris_rt_forward(...)   -> dict of output cubes
  iris_rt_adjoint(...)   -> dict of field gradients
  iris_rt_layout(...)    -> sightline-major copy of the fields
  iris_rt_autotune(...)  -> fastest sightlines-per-wavefront for a cube class
  iris_rt_autotune_adjoint(...) -> the same for the adjoint's reverse march
  Plan                   -> iris_plan_* batched persistent launches
  IrisRT                 -> torch.autograd.Function over the fields (T_dust optional)
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

from . import workloads

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libiris_rt.so")

IRIS_OK = 0
_DTYPES = {torch.float64: 0, torch.float32: 1, torch.bfloat16: 2, torch.float16: 3}
_STATUS = {0: "ok", 1: "invalid argument", 2: "unsupported", 3: "workspace", 4: "HIP error",
           5: "non-finite or out-of-range field values"}


class IrisError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"iris_rt: {_STATUS.get(status, status)}: {detail}")
        self.status = status


class Fields(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("axis", ctypes.c_int32), ("cell_cm", ctypes.c_double), ("dtype", ctypes.c_int32),
        ("ln_nh2", ctypes.c_void_p), ("t_kin", ctypes.c_void_p), ("v_los", ctypes.c_void_p),
        ("x_tracer", ctypes.c_void_p), ("t_dust", ctypes.c_void_p),
    ]


class ChannelsC(ctypes.Structure):
    _fields_ = [("n_chan", ctypes.c_int32), ("simpson_f", ctypes.c_int32),
                ("v_lo_kms", ctypes.c_double), ("dv_kms", ctypes.c_double)]

    def __init__(self, n_chan=0, v_lo_kms=0.0, dv_kms=0.0, simpson_f=0):
        super().__init__(int(n_chan), int(simpson_f), float(v_lo_kms), float(dv_kms))


class LineC(ctypes.Structure):
    _fields_ = [
        ("nu0_hz", ctypes.c_double), ("a_ul", ctypes.c_double), ("e_u_k", ctypes.c_double),
        ("j_u", ctypes.c_int32), ("j_max", ctypes.c_int32), ("m_tracer_amu", ctypes.c_double),
        ("sigma_turb_kms", ctypes.c_double), ("kappa_dust_cm2g", ctypes.c_double),
        ("dust_to_gas", ctypes.c_double), ("mu_amu_per_h2", ctypes.c_double),
        ("t_bg_k", ctypes.c_double), ("t_inf_k", ctypes.c_double),
        ("energy_mode", ctypes.c_int32), ("units", ctypes.c_int32),
        ("integrator", ctypes.c_int32), ("transfer", ctypes.c_int32),
        ("levels", ctypes.c_void_p), ("h2_frac", ctypes.c_double),
    ]


# Output units (iris_units): Rayleigh-Jeans kelvin, specific intensity (cgs),
# Planck brightness temperature of [T], [C], [B].
UNITS_TRJ, UNITS_INTENSITY, UNITS_TB = 0, 1, 2
_UNITS = {"trj": UNITS_TRJ, "intensity": UNITS_INTENSITY, "tb": UNITS_TB}


def units_code(u) -> int:
    """iris_units value of ``u`` (an int or one of "trj", "intensity", "tb")."""
    return _UNITS[u.lower()] if isinstance(u, str) else int(u)


# Integrators (iris_integrator): formal exponential steps, or smooth (the
# trapezoidal first step, then BDF2, each clamped at zero).
INTEGRATOR_FORMAL, INTEGRATOR_SMOOTH = 0, 1
_INTEGRATORS = {"formal": INTEGRATOR_FORMAL, "smooth": INTEGRATOR_SMOOTH}


def integrator_code(i) -> int:
    """iris_integrator value of ``i`` (an int, "formal" or "smooth")."""
    return _INTEGRATORS[i.lower()] if isinstance(i, str) else int(i)


# Transfer modes (iris_transfer): optically thick, optically thin (no
# absorption, channel-averaged erf profile), or selectively thin (the line
# absorbs the continuum, not itself).
TRANSFER_THICK, TRANSFER_THIN, TRANSFER_SELECTIVE = 0, 1, 2
_TRANSFERS = {"thick": TRANSFER_THICK, "thin": TRANSFER_THIN, "selective": TRANSFER_SELECTIVE}


def transfer_code(t) -> int:
    """iris_transfer value of ``t`` (an int, "thick", "thin" or "selective")."""
    return _TRANSFERS[t.lower()] if isinstance(t, str) else int(t)


class Outputs(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("T", "C", "D", "L", "B")]


class Cotangents(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("gT", "gC", "gD", "gL", "gB")]


class Gradients(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("g_ln_nh2", "g_t_kin", "g_v_los", "g_x_tracer",
                                                "g_t_dust")]


class Cube(ctypes.Structure):
    _fields_ = [("fields", Fields), ("channels", ChannelsC), ("out", Outputs),
                ("cot", Cotangents), ("grads", Gradients)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("scratch_bytes", ctypes.c_int64), ("samples", ctypes.c_int64),
                ("n_cubes", ctypes.c_int32), ("n_fwd_items", ctypes.c_int32),
                ("n_adj_items", ctypes.c_int32), ("fwd_blocks", ctypes.c_int32),
                ("adj_blocks", ctypes.c_int32), ("layout_tiles", ctypes.c_int32),
                ("ckpt_K", ctypes.c_int32)]


PLAN_FORWARD, PLAN_ADJOINT, PLAN_AUTOTUNE = 1, 2, 4

# Every symbol declared in include/iris_rt.h, with its ctypes signature.
_SIGNATURES = {
    "iris_version": ([], ctypes.c_char_p),
    "iris_max_channels": ([], ctypes.c_int32),
    "iris_smooth_max_channels": ([], ctypes.c_int32),
    "iris_status_string": ([ctypes.c_int], ctypes.c_char_p),
    "iris_last_error": ([], ctypes.c_char_p),
    "iris_rt_layout_bytes": ([ctypes.POINTER(Fields)], ctypes.c_size_t),
    "iris_rt_layout": ([ctypes.POINTER(Fields), ctypes.c_void_p, ctypes.c_size_t,
                        ctypes.c_void_p], ctypes.c_int),
    "iris_rt_workspace_bytes": ([ctypes.POINTER(Fields), ctypes.POINTER(ChannelsC),
                                 ctypes.c_int32], ctypes.c_size_t),
    "iris_rt_forward": ([ctypes.POINTER(Fields), ctypes.POINTER(ChannelsC), ctypes.POINTER(LineC),
                         ctypes.POINTER(Outputs), ctypes.c_int32, ctypes.c_void_p,
                         ctypes.c_size_t, ctypes.c_void_p], ctypes.c_int),
    "iris_rt_check_fields": ([ctypes.POINTER(Fields), ctypes.c_void_p, ctypes.c_size_t,
                              ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "iris_rt_forward_static_max_bytes": ([], ctypes.c_size_t),
    "iris_rt_forward_static": ([ctypes.POINTER(Fields), ctypes.POINTER(ChannelsC),
                                ctypes.POINTER(LineC), ctypes.POINTER(Outputs), ctypes.c_void_p],
                               ctypes.c_int),
    "iris_rt_adjoint": ([ctypes.POINTER(Fields), ctypes.POINTER(ChannelsC), ctypes.POINTER(LineC),
                         ctypes.POINTER(Cotangents), ctypes.c_int32, ctypes.c_void_p,
                         ctypes.c_size_t, ctypes.POINTER(Gradients), ctypes.c_void_p],
                        ctypes.c_int),
    "iris_rt_autotune": ([ctypes.POINTER(Fields), ctypes.POINTER(ChannelsC), ctypes.POINTER(LineC),
                          ctypes.POINTER(Outputs), ctypes.c_void_p, ctypes.c_size_t,
                          ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "iris_rt_autotune_adjoint": ([ctypes.POINTER(Fields), ctypes.POINTER(ChannelsC),
                                  ctypes.POINTER(LineC), ctypes.POINTER(Cotangents),
                                  ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t,
                                  ctypes.POINTER(Gradients), ctypes.c_void_p,
                                  ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "iris_plan_create": ([ctypes.POINTER(Cube), ctypes.c_int32, ctypes.POINTER(LineC),
                          ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                          ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "iris_plan_forward": ([ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "iris_plan_adjoint": ([ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "iris_plan_get_info": ([ctypes.c_void_p, ctypes.POINTER(PlanInfo)], ctypes.c_int),
    "iris_plan_groups": ([ctypes.c_void_p, ctypes.c_int32], ctypes.c_int32),
    "iris_plan_adjoint_groups": ([ctypes.c_void_p, ctypes.c_int32], ctypes.c_int32),
    "iris_plan_destroy": ([ctypes.c_void_p], None),
    "iris_beam_workspace_bytes": ([ctypes.c_int32] * 3, ctypes.c_size_t),
    "iris_beam_convolve": ([ctypes.c_void_p, ctypes.c_void_p] + [ctypes.c_int32] * 3
                           + [ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p],
                           ctypes.c_int),
    "iris_lv_mean": ([ctypes.c_void_p, ctypes.c_void_p] + [ctypes.c_int32] * 4 + [ctypes.c_void_p],
                     ctypes.c_int),
    "iris_molecule_read": ([ctypes.c_char_p, ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "iris_molecule_get_info": ([ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "iris_molecule_destroy": ([ctypes.c_void_p], None),
    "iris_levels_create": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                            ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "iris_levels_copy_grid": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t], ctypes.c_int),
    "iris_levels_destroy": ([ctypes.c_void_p], None),
    "iris_probe_issue_rates": ([ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)],
                               ctypes.c_int),
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libiris_rt.so, building it first only if it does not exist. The
    environment variable IRIS_RT_LIBRARY names another build to load instead
    (the sanitizer-checked build of the host code)."""
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("IRIS_RT_LIBRARY", path)
    if not os.path.exists(path):
        from . import build

        build.build()
    lib = ctypes.CDLL(path)
    for name, (args, res) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(status: int):
    if status != IRIS_OK:
        raise IrisError(status, load_library().iris_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


@dataclass
class Channels:
    n_chan: int
    v_lo_kms: float
    dv_kms: float
    simpson_f: int = 0  # Simpson panels per channel (0: profile at channel centres)

    def c(self) -> ChannelsC:
        return ChannelsC(self.n_chan, self.v_lo_kms, self.dv_kms, self.simpson_f)


def line_struct(line: dict | None = None) -> LineC:
    d = dict(workloads.LINE_13CO_21)
    if line:
        d.update(line)
    return LineC(d["nu0_hz"], d["a_ul"], d["e_u_k"], int(d["j_u"]), int(d["j_max"]),
                 d["m_tracer_amu"], d["sigma_turb_kms"], d["kappa_dust_cm2g"], d["dust_to_gas"],
                 d["mu_amu_per_h2"], d["t_bg_k"], d["t_inf_k"], int(d["energy_mode"]),
                 units_code(d.get("units", UNITS_TRJ)),
                 integrator_code(d.get("integrator", INTEGRATOR_FORMAL)),
                 transfer_code(d.get("transfer", TRANSFER_THICK)),
                 _levels_handle(d.get("levels")), float(d.get("h2_frac", 0.0)))


def _levels_handle(levels):
    """The C handle of a Levels grid (None: LTE populations)."""
    if levels is None:
        return None
    if not isinstance(levels, Levels) or not levels.handle:
        raise ValueError("line['levels'] must be an open Levels grid")
    return levels.handle


def _fields_struct(ln_nh2, t_kin, v_los, x_tracer, t_dust, axis: int, cell_cm: float) -> Fields:
    ts = [ln_nh2, t_kin, v_los, x_tracer] + ([t_dust] if t_dust is not None else [])
    shape, dtype, dev = ln_nh2.shape, ln_nh2.dtype, ln_nh2.device
    if len(shape) != 3:
        raise ValueError("fields must be 3-D [nx][ny][nz]")
    if dev.type != "cuda":
        raise ValueError("fields must be GPU tensors (no CPU path exists)")
    for t in ts:
        if t.shape != shape or t.dtype != dtype or t.device != dev:
            raise ValueError("all fields must share shape, dtype and device")
        if not t.is_contiguous():
            raise ValueError("fields must be contiguous")
    if dtype not in _DTYPES:
        raise ValueError(f"unsupported field dtype {dtype}")
    return Fields(shape[0], shape[1], shape[2], int(axis), float(cell_cm), _DTYPES[dtype],
                  _ptr(ln_nh2), _ptr(t_kin), _ptr(v_los), _ptr(x_tracer), _ptr(t_dust))


def geometry(shape, axis: int):
    n_los = shape[axis]
    n_pix = shape[0] * shape[1] * shape[2] // n_los
    return n_pix, n_los


def workspace_bytes(fields: Fields, ch: ChannelsC, ckpt_K: int) -> int:
    return load_library().iris_rt_workspace_bytes(ctypes.byref(fields), ctypes.byref(ch),
                                                  int(ckpt_K))


def iris_rt_layout(ln_nh2, t_kin, v_los, x_tracer, t_dust=None, *, axis: int, cell_cm: float = 1.0):
    """Sightline-major copy: tensor [n_fields][n_pix][n_los] of the storage dtype."""
    lib = load_library()
    f = _fields_struct(ln_nh2, t_kin, v_los, x_tracer, t_dust, axis, cell_cm)
    n_pix, n_los = geometry(ln_nh2.shape, axis)
    nf = 5 if t_dust is not None else 4
    dst = torch.empty((nf, n_pix, n_los), dtype=ln_nh2.dtype, device=ln_nh2.device)
    _check(lib.iris_rt_layout(ctypes.byref(f), _ptr(dst), dst.numel() * dst.element_size(),
                              _stream(ln_nh2.device)))
    return dst


def iris_rt_forward(ln_nh2, t_kin, v_los, x_tracer, t_dust=None, *, axis: int, cell_cm: float,
                    channels: Channels, line: dict | None = None, components="TCDLB",
                    ckpt_K: int = 0, workspace=None, out=None):
    """Forward synthesis. Returns {component: [n_pix, n_chan] float32 tensor}.

    ``workspace`` (a uint8 tensor) may be passed in to reuse memory; when
    ``ckpt_K > 0`` the returned dict also holds ``"_workspace"``, needed by
    :func:`iris_rt_adjoint`.
    """
    lib = load_library()
    f = _fields_struct(ln_nh2, t_kin, v_los, x_tracer, t_dust, axis, cell_cm)
    ch = channels.c() if isinstance(channels, Channels) else Channels(*channels).c()
    ln = line_struct(line)
    n_pix, _ = geometry(ln_nh2.shape, axis)
    dev = ln_nh2.device
    if out is None:
        out = {k: torch.empty((n_pix, ch.n_chan), dtype=torch.float32, device=dev)
               for k in components}
    outs = Outputs(*(_ptr(out.get(k)) for k in "TCDLB"))
    need = workspace_bytes(f, ch, ckpt_K)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    _check(lib.iris_rt_forward(ctypes.byref(f), ctypes.byref(ch), ctypes.byref(ln),
                               ctypes.byref(outs), int(ckpt_K), _ptr(workspace), workspace.numel(),
                               _stream(dev)))
    res = dict(out)
    if ckpt_K:
        res["_workspace"] = workspace
    return res


def iris_rt_check_fields(ln_nh2, t_kin, v_los, x_tracer, t_dust=None, *, axis: int = 2,
                         cell_cm: float = 1.0) -> int:
    """Number of field values the march cannot use (non-finite, T <= 0, X < 0);
    raises IrisError (status 5) when there are any. Synchronises."""
    lib = load_library()
    f = _fields_struct(ln_nh2, t_kin, v_los, x_tracer, t_dust, axis, cell_cm)
    scratch = torch.empty(256, dtype=torch.uint8, device=ln_nh2.device)
    bad = ctypes.c_int64(0)
    st = lib.iris_rt_check_fields(ctypes.byref(f), _ptr(scratch), scratch.numel(),
                                  _stream(ln_nh2.device), ctypes.byref(bad))
    if st == 5:
        raise IrisError(st, lib.iris_last_error().decode())
    _check(st)
    return bad.value


def iris_rt_forward_static(ln_nh2, t_kin, v_los, x_tracer, t_dust=None, *, axis: int,
                           cell_cm: float, channels: Channels, line: dict | None = None, out):
    """Forward synthesis with no allocation in the library (its scratch is a
    static device array): ``out`` maps components to preallocated float32
    [n_pix, n_chan] tensors (missing components are skipped). No checkpoints."""
    lib = load_library()
    f = _fields_struct(ln_nh2, t_kin, v_los, x_tracer, t_dust, axis, cell_cm)
    ch = channels.c() if isinstance(channels, Channels) else Channels(*channels).c()
    ln = line_struct(line)
    outs = Outputs(*(_ptr(out.get(k)) for k in "TCDLB"))
    _check(lib.iris_rt_forward_static(ctypes.byref(f), ctypes.byref(ch), ctypes.byref(ln),
                                      ctypes.byref(outs), _stream(ln_nh2.device)))
    return out


def iris_rt_adjoint(ln_nh2, t_kin, v_los, x_tracer, t_dust=None, *, axis: int, cell_cm: float,
                    channels: Channels, line: dict | None = None, cot: dict, ckpt_K: int,
                    workspace):
    """Gradients (float64, native layout) of sum(cot[X] * [X]) w.r.t. the fields.

    ``workspace`` must be the one returned by :func:`iris_rt_forward` with the
    same ``ckpt_K``; optically thin transfer (``ckpt_K`` 0) needs nothing from
    the forward, and None allocates its workspace.
    """
    return _adjoint_call(ln_nh2, t_kin, v_los, x_tracer, t_dust, axis, cell_cm, channels, line,
                         cot, ckpt_K, workspace, tune=False)


def iris_rt_autotune_adjoint(ln_nh2, t_kin, v_los, x_tracer, t_dust=None, *, axis: int,
                             cell_cm: float, channels: Channels, line: dict | None = None,
                             cot: dict, ckpt_K: int, workspace):
    """Time the adjoint at 1, 2 and 4 sightlines per wavefront (those whose
    tape fits), record the fastest for the cube's class and return
    (groups, gradients of that packing). Same preconditions as
    :func:`iris_rt_adjoint`."""
    return _adjoint_call(ln_nh2, t_kin, v_los, x_tracer, t_dust, axis, cell_cm, channels, line,
                         cot, ckpt_K, workspace, tune=True)


def _adjoint_call(ln_nh2, t_kin, v_los, x_tracer, t_dust, axis, cell_cm, channels, line, cot,
                  ckpt_K, workspace, tune):
    lib = load_library()
    f = _fields_struct(ln_nh2, t_kin, v_los, x_tracer, t_dust, axis, cell_cm)
    ch = channels.c() if isinstance(channels, Channels) else Channels(*channels).c()
    ln = line_struct(line)
    dev = ln_nh2.device
    n_pix, _ = geometry(ln_nh2.shape, axis)
    cots = {}
    for k in "TCDLB":
        t = cot.get(k)
        if t is not None:
            if t.shape != (n_pix, ch.n_chan) or t.dtype != torch.float32 or t.device != dev:
                raise ValueError(f"cotangent {k} must be float32 [{n_pix}, {ch.n_chan}] on {dev}")
            cots[k] = t.contiguous()
    cs = Cotangents(*(_ptr(cots.get(k)) for k in "TCDLB"))
    names = ["ln_nh2", "t_kin", "v_los", "x_tracer"] + (["t_dust"] if t_dust is not None else [])
    grads = {n: torch.empty(ln_nh2.shape, dtype=torch.float64, device=dev) for n in names}
    gs = Gradients(*(_ptr(grads.get(n)) for n in ("ln_nh2", "t_kin", "v_los", "x_tracer",
                                                   "t_dust")))
    if workspace is None:
        workspace = torch.empty(max(workspace_bytes(f, ch, ckpt_K), 1), dtype=torch.uint8,
                                device=dev)
    args = (ctypes.byref(f), ctypes.byref(ch), ctypes.byref(ln), ctypes.byref(cs), int(ckpt_K),
            _ptr(workspace), workspace.numel(), ctypes.byref(gs), _stream(dev))
    if not tune:
        _check(lib.iris_rt_adjoint(*args))
        return grads
    g = ctypes.c_int32(0)
    _check(lib.iris_rt_autotune_adjoint(*args, ctypes.byref(g)))
    return g.value, grads


def iris_rt_autotune(ln_nh2, t_kin, v_los, x_tracer, t_dust=None, *, axis: int, cell_cm: float,
                     channels: Channels, line: dict | None = None, workspace=None, out=None):
    """Time 1, 2 and 4 sightlines per wavefront on this cube, record the
    fastest for its class and return (groups, outputs of that variant)."""
    lib = load_library()
    f = _fields_struct(ln_nh2, t_kin, v_los, x_tracer, t_dust, axis, cell_cm)
    ch = channels.c() if isinstance(channels, Channels) else Channels(*channels).c()
    ln = line_struct(line)
    n_pix, _ = geometry(ln_nh2.shape, axis)
    dev = ln_nh2.device
    if out is None:
        out = {k: torch.empty((n_pix, ch.n_chan), dtype=torch.float32, device=dev) for k in "TCDLB"}
    outs = Outputs(*(_ptr(out.get(k)) for k in "TCDLB"))
    need = workspace_bytes(f, ch, 0)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    g = ctypes.c_int32(0)
    _check(lib.iris_rt_autotune(ctypes.byref(f), ctypes.byref(ch), ctypes.byref(ln),
                                ctypes.byref(outs), _ptr(workspace), workspace.numel(),
                                _stream(dev), ctypes.byref(g)))
    return g.value, out


class Plan:
    """Batched plan over many cubes: one persistent, graph-captured launch per
    phase (``iris_plan_create`` / ``iris_plan_forward`` / ``iris_plan_adjoint``);
    for the smooth integrator and the thin transfer modes, forward only, the
    graph holds one single-cube forward per cube.

    ``cubes`` is a list of dicts with keys ``fields`` (tuple of four 3-D GPU
    tensors of one dtype), ``axis``, ``cell_cm``, ``channels``; the plan
    allocates each cube's output cubes (``outputs[i]``), and with
    ``adjoint=True`` its cotangent buffers (``cotangents[i]``, zero, to be
    filled in place) and FP64 gradients (``gradients[i]``). New data is
    processed by writing it into the same tensors and replaying.
    """

    def __init__(self, cubes, *, line: dict | None = None, adjoint: bool = False, ckpt_K: int = 16,
                 autotune: bool = False, components="TCDLB"):
        lib = load_library()
        self._lib = lib
        self._handle = None
        n = len(cubes)
        arr = (Cube * n)()
        self.outputs, self.cotangents, self.gradients, self._keep = [], [], [], []
        dev = None
        for i, cb in enumerate(cubes):
            fl = cb["fields"]
            f = _fields_struct(*fl[:4], fl[4] if len(fl) > 4 else None, cb["axis"], cb["cell_cm"])
            chn = cb["channels"]
            ch = chn.c() if isinstance(chn, Channels) else Channels(*chn).c()
            dev = fl[0].device
            n_pix, _ = geometry(fl[0].shape, cb["axis"])
            out = {k: torch.empty((n_pix, ch.n_chan), dtype=torch.float32, device=dev)
                   for k in components}
            cot, grads = {}, {}
            if adjoint:
                cot = {k: torch.zeros((n_pix, ch.n_chan), dtype=torch.float32, device=dev)
                       for k in cb.get("cot_components", "T")}
                names = ("ln_nh2", "t_kin", "v_los", "x_tracer") + (("t_dust",) if len(fl) > 4
                                                                    else ())
                grads = {nm: torch.empty(fl[0].shape, dtype=torch.float64, device=dev)
                         for nm in names}
            arr[i].fields = f
            arr[i].channels = ch
            arr[i].out = Outputs(*(_ptr(out.get(k)) for k in "TCDLB"))
            arr[i].cot = Cotangents(*(_ptr(cot.get(k)) for k in "TCDLB"))
            arr[i].grads = Gradients(*(_ptr(grads.get(nm)) for nm in
                                       ("ln_nh2", "t_kin", "v_los", "x_tracer", "t_dust")))
            self.outputs.append(out)
            self.cotangents.append(cot)
            self.gradients.append(grads)
            self._keep.append(fl)
        flags = PLAN_FORWARD | (PLAN_ADJOINT if adjoint else 0) | (PLAN_AUTOTUNE if autotune else 0)
        h = ctypes.c_void_p()
        ln = line_struct(line)
        self.device = dev
        _check(lib.iris_plan_create(arr, n, ctypes.byref(ln), flags, int(ckpt_K) if adjoint else 0,
                                    _stream(dev), ctypes.byref(h)))
        self._handle = h

    def forward(self):
        _check(self._lib.iris_plan_forward(self._handle, _stream(self.device)))
        return self.outputs

    def adjoint(self):
        _check(self._lib.iris_plan_adjoint(self._handle, _stream(self.device)))
        return self.gradients

    def info(self) -> dict:
        inf = PlanInfo()
        _check(self._lib.iris_plan_get_info(self._handle, ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in PlanInfo._fields_}

    def groups(self, i: int) -> int:
        return self._lib.iris_plan_groups(self._handle, int(i))

    def adjoint_groups(self, i: int) -> int:
        return self._lib.iris_plan_adjoint_groups(self._handle, int(i))

    def close(self):
        if self._handle:
            self._lib.iris_plan_destroy(self._handle)
            self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MoleculeInfo(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int32), ("n_transitions", ctypes.c_int32),
                ("n_partners", ctypes.c_int32), ("partner_code", ctypes.c_int32 * 8),
                ("partner_transitions", ctypes.c_int32 * 8),
                ("partner_temperatures", ctypes.c_int32 * 8)]


class LevelsConfig(ctypes.Structure):
    _fields_ = [("transition", ctypes.c_int32), ("t_bar_k", ctypes.c_double),
                ("ortho_para", ctypes.c_double), ("he_per_h", ctypes.c_double),
                ("n_n", ctypes.c_int32), ("n_chi", ctypes.c_int32), ("n_t", ctypes.c_int32),
                ("ln_nh2_lo", ctypes.c_double), ("ln_nh2_hi", ctypes.c_double),
                ("chi_lo", ctypes.c_double), ("chi_hi", ctypes.c_double),
                ("t_lo_k", ctypes.c_double), ("t_hi_k", ctypes.c_double)]


class Molecule:
    """Molecular data read from a LAMDA-convention file (``iris_molecule_read``)."""

    def __init__(self, path: str):
        lib = load_library()
        self._lib = lib
        h = ctypes.c_void_p()
        _check(lib.iris_molecule_read(os.fsencode(path), ctypes.byref(h)))
        self.handle = h

    def info(self) -> dict:
        inf = MoleculeInfo()
        _check(self._lib.iris_molecule_get_info(self.handle, ctypes.byref(inf)))
        n = inf.n_partners
        return {"n_levels": inf.n_levels, "n_transitions": inf.n_transitions,
                "partners": [(inf.partner_code[i], inf.partner_transitions[i],
                              inf.partner_temperatures[i]) for i in range(n)]}

    def close(self):
        if self.handle:
            self._lib.iris_molecule_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# Grid of the paper's study: (n_rho, n_chi, n_T) = (128, 64, 64).
LEVELS_GRID_DEFAULT = dict(n_n=128, n_chi=64, n_t=64, ln_nh2_lo=-2.302585092994046,
                           ln_nh2_hi=18.420680743952367, chi_lo=0.05, chi_hi=1.0, t_lo_k=3.0,
                           t_hi_k=3.0e3)


class Levels:
    """Grid of optically thin level populations of one transition
    (``iris_levels_create``), to pass as ``line["levels"]``."""

    def __init__(self, molecule: Molecule, transition: int, *, t_bar_k: float = 2.725,
                 ortho_para: float = 3.0, he_per_h: float = 0.1, device=None, **grid):
        lib = load_library()
        self._lib = lib
        g = dict(LEVELS_GRID_DEFAULT)
        g.update(grid)
        self.config = dict(g, transition=int(transition), t_bar_k=float(t_bar_k),
                           ortho_para=float(ortho_para), he_per_h=float(he_per_h))
        cfg = LevelsConfig(int(transition), float(t_bar_k), float(ortho_para), float(he_per_h),
                           int(g["n_n"]), int(g["n_chi"]), int(g["n_t"]), float(g["ln_nh2_lo"]),
                           float(g["ln_nh2_hi"]), float(g["chi_lo"]), float(g["chi_hi"]),
                           float(g["t_lo_k"]), float(g["t_hi_k"]))
        dev = torch.device(device) if device is not None else torch.device("cuda",
                                                                          torch.cuda.current_device())
        h = ctypes.c_void_p()
        _check(lib.iris_levels_create(molecule.handle, ctypes.byref(cfg), _stream(dev),
                                      ctypes.byref(h)))
        self.handle = h

    @property
    def shape(self):
        c = self.config
        return (c["n_chi"], c["n_t"], c["n_n"])

    def grid(self):
        """(FU, FL) as two float32 NumPy arrays [n_chi][n_t][n_n]."""
        import numpy as np

        buf = np.empty(self.shape + (2,), dtype=np.float32)
        _check(self._lib.iris_levels_copy_grid(self.handle, buf.ctypes.data_as(ctypes.c_void_p),
                                               buf.size))
        return buf[..., 0].copy(), buf[..., 1].copy()

    def close(self):
        if self.handle:
            torch.cuda.synchronize()
            self._lib.iris_levels_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _sky_cube(cube):
    if not (isinstance(cube, torch.Tensor) and cube.is_cuda and cube.dtype == torch.float32
            and cube.dim() == 3 and cube.is_contiguous()):
        raise ValueError("expected a contiguous float32 GPU tensor [n1][n2][n_chan]")
    return cube.shape


def beam_convolve(cube, fwhm_pix: float, out=None, workspace=None):
    """Gaussian beam convolution of a cube [n1][n2][n_chan] over its two sky
    axes (FWHM in pixels); returns `out` (a new tensor unless given)."""
    n1, n2, c = _sky_cube(cube)
    lib = load_library()
    out = torch.empty_like(cube) if out is None else out
    need = lib.iris_beam_workspace_bytes(n1, n2, c)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=cube.device)
    _check(lib.iris_beam_convolve(_ptr(cube), _ptr(out), n1, n2, c, float(fwhm_pix),
                                  _ptr(workspace), workspace.numel(), _stream(cube.device)))
    return out


def lv_mean(cube, axis: int, out=None):
    """Mean of a cube [n1][n2][n_chan] over sky axis `axis` (0 or 1)."""
    n1, n2, c = _sky_cube(cube)
    lib = load_library()
    if out is None:
        out = torch.empty(((n2 if axis == 0 else n1), c), dtype=torch.float32, device=cube.device)
    _check(lib.iris_lv_mean(_ptr(cube), _ptr(out), n1, n2, c, int(axis), _stream(cube.device)))
    return out


def iris_probe_issue_rates() -> dict:
    """Measured v_exp_f32 and FP32 FMA issue rates of the current device (per second)."""
    e, f = ctypes.c_double(), ctypes.c_double()
    _check(load_library().iris_probe_issue_rates(ctypes.byref(e), ctypes.byref(f)))
    return {"exp_per_s": e.value, "fma_per_s": f.value}


class IrisRT(torch.autograd.Function):
    """Differentiable synthesis: (ln n_H2, T_kin, v_los, X[, T_dust]) -> ([T], [C], [D], [L], [B]).

    The backward pass runs the hand-written adjoint kernel, recomputing each
    checkpoint segment of ``ckpt_K`` cells; gradients are returned in the
    dtype of the fields. ``t_dust`` may be None (T_dust = T_kin).
    """

    @staticmethod
    def forward(ctx, ln_nh2, t_kin, v_los, x_tracer, t_dust, axis, cell_cm, channels, line,
                ckpt_K):
        need_grad = any(ctx.needs_input_grad[:5])
        # Optically thin transfer marches nothing and takes no checkpoints.
        thin = transfer_code((line or {}).get("transfer", TRANSFER_THICK)) == TRANSFER_THIN
        K = int(ckpt_K) if need_grad and not thin else 0
        res = iris_rt_forward(ln_nh2, t_kin, v_los, x_tracer, t_dust, axis=axis, cell_cm=cell_cm,
                              channels=channels, line=line, ckpt_K=K)
        ctx.save_for_backward(ln_nh2, t_kin, v_los, x_tracer, t_dust)
        ctx.meta = (axis, cell_cm, channels, line, K, res.get("_workspace"))
        return tuple(res[k] for k in "TCDLB")

    @staticmethod
    def backward(ctx, gT, gC, gD, gL, gB):
        ln_nh2, t_kin, v_los, x_tracer, t_dust = ctx.saved_tensors
        axis, cell_cm, channels, line, K, ws = ctx.meta
        cot = {k: (g.float().contiguous() if g is not None else None)
               for k, g in zip("TCDLB", (gT, gC, gD, gL, gB))}
        g = iris_rt_adjoint(ln_nh2, t_kin, v_los, x_tracer, t_dust, axis=axis, cell_cm=cell_cm,
                            channels=channels, line=line, cot=cot, ckpt_K=K, workspace=ws)
        dt = ln_nh2.dtype
        gtd = g["t_dust"].to(dt) if t_dust is not None else None
        return (g["ln_nh2"].to(dt), g["t_kin"].to(dt), g["v_los"].to(dt), g["x_tracer"].to(dt),
                gtd, None, None, None, None, None)


def synthesize(ln_nh2, t_kin, v_los, x_tracer, t_dust=None, *, axis, cell_cm, channels, line=None,
               ckpt_K=16):
    """Autograd-aware wrapper returning {component: cube}."""
    outs = IrisRT.apply(ln_nh2, t_kin, v_los, x_tracer, t_dust, axis, cell_cm, channels, line,
                        ckpt_K)
    return dict(zip("TCDLB", outs))
