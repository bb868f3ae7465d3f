"""Error metrics for comparing cubes.

``err_inf`` / ``err_2`` are normwise relative errors (the parity gates use
``err_inf``); ``tsre`` and ``tam`` are the paper's threshold-symmetric
relative error and threshold-active mean ("Error Metrics for Synthetic
Observation"), reported beside them.
"""

from __future__ import annotations

import numpy as np

T_MIN = 0.05  # K, activity threshold of TSRE and TAM


def err_inf(x, ref, floor: float = 0.0) -> float:
    """max|x - ref| / max(max|ref|, floor)."""
    x, ref = np.asarray(x, dtype=np.float64), np.asarray(ref, dtype=np.float64)
    scale = max(float(np.max(np.abs(ref))), floor)
    if scale == 0:
        return float(np.max(np.abs(x)))
    return float(np.max(np.abs(x - ref)) / scale)


def err_2(x, ref) -> float:
    x, ref = np.asarray(x, dtype=np.float64), np.asarray(ref, dtype=np.float64)
    scale = np.linalg.norm(ref)
    if scale == 0:
        return float(np.linalg.norm(x))
    return float(np.linalg.norm(x - ref) / scale)


def tsre(t1, t2, t_min: float = T_MIN) -> np.ndarray:
    """Elementwise 2|T1-T2|/(|T1|+|T2|) where min(|T1|,|T2|) > t_min, else 0."""
    a, b = np.abs(t1), np.abs(t2)
    active = np.minimum(a, b) > t_min
    out = np.zeros(np.broadcast(t1, t2).shape)
    out[active] = 2 * np.abs(t1 - t2)[active] / (a + b)[active]
    return out


def tam(t, t_min: float = T_MIN) -> float:
    """Mean over the voxels with |T| > t_min."""
    t = np.asarray(t)
    act = np.abs(t) > t_min
    return float(t[act].mean()) if act.any() else 0.0


def report(x, ref) -> dict:
    return {"err_inf": err_inf(x, ref), "err_2": err_2(x, ref),
            "tsre_mean": float(tsre(np.asarray(x, float), np.asarray(ref, float)).mean()),
            "tam": tam(x), "tam_ref": tam(ref)}
