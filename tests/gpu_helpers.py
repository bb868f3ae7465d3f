"""Shared helpers of the GPU parity tests: run one cube through the HIP path
and through the FP64 oracle on the identical (dequantised) field values."""

from __future__ import annotations

import sys

import numpy as np
import torch

import oracle
from paper_2607_01338_amd import rt
from paper_2607_01338_amd import workloads as W

TORCH_DT = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16,
            "f16": torch.float16}
# Parity gate: normwise max error relative to max |reference|, per component.
TOL_FWD = 1e-5


def say(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def to_device(cube: W.Cube, dt: str) -> dict:
    out = {}
    for k, v in cube.fields().items():
        t = torch.from_numpy(np.ascontiguousarray(v, dtype=np.float64))
        out[k] = t.to(TORCH_DT[dt]).cuda().contiguous()
    return out


def dequantised(dev_fields: dict) -> dict:
    return {k: v.double().cpu().numpy() for k, v in dev_fields.items()}


def channels_of(cube: W.Cube) -> rt.Channels:
    ch = cube.channels
    return rt.Channels(ch.n_chan, ch.v_lo_kms, ch.dv_kms)


def gpu_forward(cube: W.Cube, dev: dict, line=None, ckpt_K=0, components="TCDLB"):
    res = rt.iris_rt_forward(dev["ln_nh2"], dev["t_kin"], dev["v_los"], dev["x_tracer"],
                             dev.get("t_dust"), axis=cube.axis, cell_cm=cube.cell_cm,
                             channels=channels_of(cube), line=line, ckpt_K=ckpt_K,
                             components=components)
    torch.cuda.synchronize()
    return res


def problem(cube: W.Cube, deq: dict) -> oracle.Problem:
    ch = cube.channels
    return oracle.Problem(deq["ln_nh2"], deq["t_kin"], deq["v_los"], deq["x_tracer"], cube.axis,
                          cube.cell_cm, ch.n_chan, ch.v_lo_kms, ch.dv_kms, deq.get("t_dust"))


def line_dict(**kw) -> dict:
    d = dict(W.LINE_13CO_21)
    d.update(kw)
    return d


def pixel_cells(cube: W.Cube, pix: int):
    """Native flat indices of the cells of sightline `pix`, far side first."""
    nx, ny, nz = cube.shape
    s = np.arange(cube.n_los)
    if cube.axis == 0:
        y, z = divmod(pix, nz)
        return (s * ny + y) * nz + z
    if cube.axis == 1:
        x, z = divmod(pix, nz)
        return (x * ny + s) * nz + z
    x, y = divmod(pix, ny)
    return (x * ny + y) * nz + s
