"""Benchmark of the 13CO(2-1) PPV synthesis on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config cmz|small|adjoint]
                    [--dtype f32|bf16|f16] [--no-cpu-baseline]

One step = one forward synthesis of the whole cube (field ingest/layout,
per-cell LTE setup, line-window march, five output cubes) on fields already
resident in HBM. Prints one JSON line. Inputs are seeded synthetic fields with
the statistics of the paper's training workload (see
paper_2607_01338_amd/workloads.py); there is no dataset.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Transcendental (v_exp_f32) issue rate: 256 CUs x 4 SIMDs x 16 lanes/clk at
# half the FMA rate x 2.4 GHz (gfx950 issues v_exp_f32 in 8 cycles per wave64;
# the library's issue-rate probe measures it beside every run).
EXP_PEAK_GPS = 256 * 4 * 16 / 2 * 2.4
# Window of the line that no method can skip at the library's accuracy:
# |v_k - v| <= x_min b with x_min^2 = ln(1e9) (beyond it the profile is below
# 1e-9 of its peak, the threshold under which the march leaves a channel
# untouched).
X_MIN = math.sqrt(math.log(1e9))
# FP32 vector issue rate without packed math: 256 CUs x 4 SIMDs x 16 lanes/clk
# x 2.4 GHz, in 1e12 lane-operations per second.
FMA_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# The smooth integrator's step of one (cell, channel) sample outside the
# line window: a difference, two FMAs and the clamp.
SMOOTH_OPS_PER_SAMPLE = 4
# Sources whose hash keys a stored HBM-traffic measurement of the march.
KERNEL_SOURCES = ("forward.hip", "cell_setup.h", "device_util.h", "iris_internal.h",
                  "epilogue.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fwd_kernel__cmz_512x512x128_800ch_f32.traffic.json")
K_B = 1.380649e-16
AMU = 1.66053906660e-24


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=30,
                    help="untimed launches first (the GPU clock settles within tens of ms)")
    ap.add_argument("--config", default="cmz", choices=["cmz", "small", "adjoint"])
    ap.add_argument("--dtype", default=None, choices=["f64", "f32", "bf16", "f16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the forward+adjoint measurement on the 256^3 cube")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 64-cube batched plan measurement")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the BF16/FP16-storage march timings")
    ap.add_argument("--no-smooth", action="store_true",
                    help="skip the smooth-integrator leg (TR then BDF2, against the formal march)")
    ap.add_argument("--no-post", action="store_true",
                    help="skip the post-transfer leg (30 arcsec beam on [L], l,v mean)")
    ap.add_argument("--no-thin", action="store_true",
                    help="skip the optically and selectively thin transfer legs")
    ap.add_argument("--no-levels", action="store_true",
                    help="skip the non-LTE level-model leg (grid build and march with it)")
    ap.add_argument("--no-subsampling", action="store_true",
                    help="skip the velocity-subsampled (simpson_f = 1) march timing")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle sample")
    ap.add_argument("--groups", type=int, default=0, choices=[0, 1, 2, 4],
                    help="sightlines per wavefront of the march (0 = library heuristic)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a 1 GiB device copy per step (counter calibration)")
    return ap.parse_args()


def window_samples(cube, line) -> int:
    """Number of (cell, channel) pairs inside the unavoidable line window."""
    ch = cube.channels
    m = line["m_tracer_amu"] * AMU
    total = 0
    T = np.asarray(cube.t_kin, dtype=np.float64).ravel()
    v = np.asarray(cube.v_los, dtype=np.float64).ravel()
    for i in range(0, T.size, 1 << 22):
        t, vv = T[i:i + (1 << 22)], v[i:i + (1 << 22)]
        b = np.sqrt(2 * K_B * t / m / 1e10 + 2 * line["sigma_turb_kms"] ** 2)
        u = (vv - ch.v_lo_kms) / ch.dv_kms - 0.5
        hw = X_MIN * b / ch.dv_kms
        lo = np.maximum(np.ceil(u - hw), 0)
        hi = np.minimum(np.floor(u + hw), ch.n_chan - 1)
        total += int(np.sum(np.maximum(hi - lo + 1, 0)))
    return total


def kernel_source_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2607_01338_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def stored_traffic():
    """HBM bytes per launch of the march kernel from its rocprofv3 FETCH_SIZE /
    WRITE_SIZE passes, if they were taken on the current kernel sources."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


N_ACC = 32  # sightlines compared against the oracle for the accuracy report

# After the W warm-up launches of a leg, its launch keeps running until the
# GPU has been busy for SETTLE_S: the clock of an MI355X that was idle (data
# generation, host work) ramps over tens of milliseconds of continuous work,
# and a few short warm-up launches leave the first timed steps in that ramp.
SETTLE_S = 0.5


def settle(fn) -> int:
    """Untimed launches of `fn` for SETTLE_S of wall time, synchronising every
    eight so that the queue stays short; returns their number."""
    import torch

    torch.cuda.synchronize()
    n, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < SETTLE_S:
        for _ in range(8):
            fn()
        n += 8
        torch.cuda.synchronize()
    return n


def _dequantised(cube, torch_dtype):
    """The cube's four fields as stored on the GPU in `torch_dtype`, back in FP64."""
    import torch

    return [torch.from_numpy(np.ascontiguousarray(a)).to(torch_dtype).double().numpy()
            for a in (cube.ln_nh2, cube.t_kin, cube.v_los, cube.x_tracer)]


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cube, line, target_s: float, gpu_rows: dict, adj_cube=None) -> dict:
    """The FP64 oracle timed on a bounded sample of host-core work, and the
    accuracy of the GPU outputs: the first N_ACC sightlines of each storage
    type against the oracle on the same (dequantised) field values, plus the
    storage-quantisation effect alone (oracle on quantised vs FP32 fields)."""
    import oracle
    import torch

    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16,
           "f16": torch.float16}

    def problem(fields):
        return oracle.Problem(*fields, cube.axis, cube.cell_cm, cube.channels.n_chan,
                              cube.channels.v_lo_kms, cube.channels.dv_kms)

    pr = problem(_dequantised(cube, torch.float32))
    per_pix = cube.n_los * cube.channels.n_chan

    def sized(run, n_max, n0, seconds):
        """Time run(n) on a probe of n0 sightlines, then on as many as take
        about `seconds`; returns (n, elapsed, result)."""
        t = time.perf_counter()
        run(n0)
        dt = time.perf_counter() - t
        n = int(min(n_max, max(n0, n0 * seconds / max(dt, 1e-3))))
        t = time.perf_counter()
        res = run(n)
        return n, time.perf_counter() - t, res

    n, dt, ref32 = sized(lambda m: oracle.forward(pr, line, pix=range(0, m), threads=threads),
                         cube.n_pix, min(cube.n_pix, max(threads * 4, 64)), target_s)
    out = {"value": n * per_pix / dt, "unit": "cell*channel samples/s", "cores": threads,
           "kind": "oracle", "cpu_model": cpu_model(),
           "sample": f"first {n} of {cube.n_pix} sightlines ({n * per_pix:.3g} samples, "
                     f"{dt:.1f} s), FP64 C++ oracle, OpenMP over sightlines"}
    # One thread on a contiguous subset (rate per core; linear in the
    # sightlines, which are independent).
    n1, dt1, _ = sized(lambda m: oracle.forward(pr, line, pix=range(0, m), threads=1),
                       cube.n_pix, 4, target_s / 3)
    out["single_thread"] = {"value": n1 * per_pix / dt1, "cores": 1,
                            "sample": f"first {n1} sightlines ({dt1:.1f} s)"}
    # Reverse mode (forward march with its tape, then the hand-written
    # reverse pass) on the forward+adjoint workload: all threads and one.
    if adj_cube is not None:
        a = adj_cube
        deq = _dequantised(a, torch.float32)
        rows_per_slab = a.shape[1]  # sightlines along z: one x-slab is ny sightlines
        per_pix_a = a.n_los * a.channels.n_chan
        rng = np.random.default_rng(4)

        def rev(m, th):
            k = max(1, m // rows_per_slab)
            sub = oracle.Problem(*(f[:k] for f in deq), a.axis, a.cell_cm, a.channels.n_chan,
                                 a.channels.v_lo_kms, a.channels.dv_kms)
            cot = rng.standard_normal((sub.n_pix, a.channels.n_chan))
            oracle.adjoint(sub, line, {"T": cot}, threads=th)
            return sub.n_pix

        def rev_sized(th, seconds):
            t = time.perf_counter()
            m0 = rev(rows_per_slab, th)
            d0 = time.perf_counter() - t
            k = int(min(a.shape[0], max(1, seconds / max(d0, 1e-3))))
            t = time.perf_counter()
            m = rev(k * rows_per_slab, th)
            return m, time.perf_counter() - t

        m, dtr = rev_sized(threads, target_s * 2 / 3)
        out["reverse_mode"] = {
            "value": m * per_pix_a / dtr, "unit": "cell*channel samples/s", "cores": threads,
            "workload": a.name, "loss": "sum of a seeded normal cotangent times [T]",
            "sample": f"{m} sightlines ({m * per_pix_a:.3g} samples, {dtr:.1f} s), FP64 forward "
                      f"march + hand-written reverse pass, OpenMP over sightlines"}
        m1, dtr1 = rev_sized(1, target_s / 3)
        out["reverse_mode"]["single_thread"] = {"value": m1 * per_pix_a / dtr1, "cores": 1,
                                                "sample": f"{m1} sightlines ({dtr1:.1f} s)"}

    def errs(gpu, ref):
        scale = float(np.max(np.abs(ref["T"][:N_ACC])))
        e = {}
        for k in "TCDLB":
            r = ref[k][:N_ACC]
            e[k] = float(np.max(np.abs(gpu[k] - r)) / max(float(np.max(np.abs(r))),
                                                        1e-6 * scale))
        return e

    acc = {"sightlines": N_ACC, "definition": "max|x - x_ref| / max|x_ref| per component"}
    quant = {}
    for name, rows in gpu_rows.items():
        ref = ref32 if name == "f32" else oracle.forward(
            problem(_dequantised(cube, tdt[name])), line, pix=range(0, N_ACC), threads=threads)
        acc[name] = errs(rows, ref)
        if name != "f32":
            quant[name] = errs({k: ref[k][:N_ACC] for k in "TCDLB"}, ref32)
    acc["storage_quantisation_vs_f32_oracle"] = quant
    out["accuracy_vs_fp64_oracle"] = acc
    return out


def main():
    args = parse()
    if args.groups:
        os.environ["IRIS_RT_SIGHTLINES_PER_WAVE"] = str(args.groups)
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported by this build "
              "(sightlines are independent; multi-GPU sharding is not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2607_01338_amd import rt
    from paper_2607_01338_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    line = dict(W.LINE_13CO_21)
    if args.config == "cmz":
        cube = W.config_cmz()
        dtype = args.dtype or "f32"
    elif args.config == "small":
        cube = W.config_small()
        dtype = args.dtype or "f64"
    else:
        cube = W.config_adjoint()
        dtype = args.dtype or "f32"
    tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16,
           "f16": torch.float16}[dtype]
    print(f"# config {args.config}: {cube.name}, storage {dtype}", file=sys.stderr, flush=True)

    f = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev).to(tdt).contiguous()
         for k, v in cube.fields().items()}
    ch = rt.Channels(cube.channels.n_chan, cube.channels.v_lo_kms, cube.channels.dv_kms)
    n_pix, n_los, C = cube.n_pix, cube.n_los, cube.channels.n_chan
    outs = {k: torch.empty((n_pix, C), dtype=torch.float32, device=dev) for k in "TCDLB"}
    fs = rt._fields_struct(f["ln_nh2"], f["t_kin"], f["v_los"], f["x_tracer"], None, cube.axis,
                           cube.cell_cm)
    ws = torch.empty(max(rt.workspace_bytes(fs, ch.c(), 0), 1), dtype=torch.uint8, device=dev)
    calib = None
    if args.calib_copy:
        calib = (torch.empty(1 << 28, dtype=torch.float32, device=dev),
                 torch.empty(1 << 28, dtype=torch.float32, device=dev))

    stream = torch.cuda.current_stream(dev)
    settled = {"launches": 0}

    def timed_launches(fields, n_steps, out, workspace=None, channels=None, line_=None):
        """Warmup, then exactly n_steps launches bracketed by synchronisations;
        returns (ms per step over the bracket, mean of per-launch HIP event
        pairs recorded on the stream the library launches on)."""
        def launch():
            rt.iris_rt_forward(fields[0], fields[1], fields[2], fields[3], axis=cube.axis,
                               cell_cm=cube.cell_cm, channels=channels or ch, line=line_ or line,
                               out=out, workspace=workspace)

        for _ in range(args.warmup):
            launch()
        settled["launches"] += settle(launch)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(n_steps)]
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0.record(stream)
        for j in range(n_steps):
            ev[j][0].record(stream)
            launch()
            ev[j][1].record(stream)
            if calib is not None:
                calib[1].copy_(calib[0])
        t1.record(stream)
        torch.cuda.synchronize()
        return (t0.elapsed_time(t1) / n_steps,
                float(np.mean([a.elapsed_time(b) for a, b in ev])))

    fl = (f["ln_nh2"], f["t_kin"], f["v_los"], f["x_tracer"])
    # One step = the table kernel (microseconds) + the march over the fields
    # read in place.
    ms_step, k_ms = timed_launches(fl, args.steps, outs, ws)
    gpu_rows = {dtype: {k: outs[k][:N_ACC].double().cpu().numpy() for k in "TCDLB"}}
    print(f"# timed {args.steps} steps: {ms_step:.3f} ms/step; {k_ms:.3f} ms per launch "
          f"(table + march, fields read in place)", file=sys.stderr, flush=True)

    # For comparison: the same synthesis through a sightline-major copy made
    # by the layout kernel first.
    outs2 = {k: torch.empty((n_pix, C), dtype=torch.float32, device=dev) for k in "TCDLB"}
    layout_cmp = None
    if cube.axis != 2:
        os.environ["IRIS_RT_FIELD_LAYOUT"] = "transpose"
        try:
            ms_t, _ = timed_launches(fl, args.steps, outs2)
        finally:
            del os.environ["IRIS_RT_FIELD_LAYOUT"]
        same = all(torch.equal(outs[k], outs2[k]) for k in "TCDLB")
        layout_cmp = {"ms_per_step": ms_t, "outputs_identical": same}
        print(f"# with a layout pass first: {ms_t:.3f} ms/step (outputs identical: {same})",
              file=sys.stderr, flush=True)

    precision = None
    if not args.no_precision and dtype == "f32":
        precision = {"f32": {"kernel_ms": k_ms}}
        for pd, ptd in (("bf16", torch.bfloat16), ("f16", torch.float16)):
            q = tuple(t.to(ptd).contiguous() for t in fl)
            _, pms = timed_launches(q, args.steps, outs2)
            gpu_rows[pd] = {k: outs2[k][:N_ACC].double().cpu().numpy() for k in "TCDLB"}
            precision[pd] = {"kernel_ms": pms, "speedup_vs_f32": k_ms / pms}
            print(f"# {pd} storage: {pms:.3f} ms/step", file=sys.stderr, flush=True)
            del q

    # Velocity subsampling (one Simpson panel per channel: 2 C + 1 marched
    # velocities), the paper's production setting for optically thick lines.
    subsampled = None
    if not args.no_subsampling:
        chs = rt.Channels(C, cube.channels.v_lo_kms, cube.channels.dv_kms, 1)
        ms_s, _ = timed_launches(fl, args.steps, outs2, channels=chs)
        subsampled = {"simpson_f": 1, "marched_velocities": 2 * C + 1, "ms_per_step": ms_s,
                      "value": n_pix * n_los * C / (ms_s * 1e-3),
                      "marched_samples_per_s": n_pix * n_los * (2 * C + 1) / (ms_s * 1e-3)}
        print(f"# subsampled (simpson_f=1, {2 * C + 1} marched velocities): {ms_s:.3f} ms/step",
              file=sys.stderr, flush=True)

    n_cells = n_pix * n_los
    samples = n_cells * C

    # Smooth integration (trapezoidal first step, then BDF2, each clamped at
    # zero), the paper's preferred integrator, on the same cube: its time and
    # its difference from the formal march in the paper's metrics.
    smooth = None
    if not args.no_smooth and dtype == "f32":
        ms_sm, k_sm = timed_launches(fl, args.steps, outs2, ws,
                                     line_=dict(line, integrator="smooth"))
        a, b = outs["L"].double(), outs2["L"].double()
        act = torch.minimum(a.abs(), b.abs()) > 0.05
        tsre = torch.where(act, 2 * (a - b).abs() / (a.abs() + b.abs()).clamp_min(1e-300),
                           torch.zeros_like(a))
        tam = lambda t: float(t[t.abs() > 0.05].mean()) if bool((t.abs() > 0.05).any()) else 0.0
        ops = SMOOTH_OPS_PER_SAMPLE * samples
        smooth = {
            "integrator": "trapezoidal first step, BDF2 after, clamped at zero",
            "ms_per_step": ms_sm, "kernel_ms": k_sm, "value": samples / (ms_sm * 1e-3),
            "formal_over_smooth_time": ms_step / ms_sm,
            "vs_formal_L": {"err_2": float((b - a).norm() / a.norm()),
                            "tsre_mean": float(tsre.mean()), "tam_formal": tam(a),
                            "tam_smooth": tam(b)},
            "roofline": {"bound": "alu", "kernel": "smooth_kernel (dense TR/BDF2 march)",
                         "achieved": ops / (k_sm * 1e-3) / 1e12,
                         "peak": FMA_PEAK_TOPS, "unit": "T lane-op/s",
                         "frac": ops / (k_sm * 1e-3) / 1e12 / FMA_PEAK_TOPS,
                         "work_per_launch": {"samples": samples,
                                             "ops_per_sample": SMOOTH_OPS_PER_SAMPLE}},
        }
        print(f"# smooth integration: {ms_sm:.3f} ms/step ({ms_step / ms_sm:.2f}x the formal "
              f"march's speed); [L] vs formal err_2 {smooth['vs_formal_L']['err_2']:.4f}",
              file=sys.stderr, flush=True)
        del a, b, act, tsre

    # Optically thin transfer (no absorption, channel-averaged erf profile),
    # with each integrator, on the same cube.
    thin = None
    if not args.no_thin and dtype == "f32":
        thin = {}
        for integ in ("formal", "smooth"):
            ms_t, k_t = timed_launches(fl, args.steps, outs2, ws,
                                       line_=dict(line, transfer="thin", integrator=integ))
            thin[integ] = {"ms_per_step": ms_t, "kernel_ms": k_t,
                           "value": samples / (ms_t * 1e-3),
                           "L_sum_over_thick": float(outs2["L"].double().sum()
                                                     / outs["L"].double().sum())}
            print(f"# optically thin ({integ}): {ms_t:.3f} ms/step", file=sys.stderr, flush=True)
        # Its reverse mode (formal steps): gradients of sum(gL * [L]) with
        # respect to the four fields (FP64, written in place), no checkpoints.
        tl = dict(line, transfer="thin")
        cot_l = {"L": outs2["L"].clone()}

        def adj_thin():
            return rt.iris_rt_adjoint(*fl, axis=cube.axis, cell_cm=cube.cell_cm, channels=ch,
                                      line=tl, cot=cot_l, ckpt_K=0, workspace=ws)

        for _ in range(args.warmup):
            adj_thin()
        settle(adj_thin)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            adj_thin()
        e1.record(stream)
        torch.cuda.synchronize()
        ms_a = e0.elapsed_time(e1) / args.steps
        thin["adjoint_formal"] = {"ms_per_step": ms_a, "value": samples / (ms_a * 1e-3),
                                  "gradient_bytes": 4 * 8 * n_pix * n_los}
        print(f"# optically thin (formal) reverse mode: {ms_a:.3f} ms/step", file=sys.stderr,
              flush=True)
        del cot_l
        for integ, key in (("formal", "selective"), ("smooth", "selective_smooth")):
            ms_t, k_t = timed_launches(fl, args.steps, outs2, ws,
                                       line_=dict(line, transfer="selective", integrator=integ))
            thin[key] = {"ms_per_step": ms_t, "kernel_ms": k_t,
                         "value": samples / (ms_t * 1e-3),
                         "L_sum_over_thick": float(outs2["L"].double().sum()
                                                   / outs["L"].double().sum())}
            print(f"# selectively thin ({integ}): {ms_t:.3f} ms/step", file=sys.stderr,
                  flush=True)

    # The paper's non-LTE level model: the optically thin level balance solved
    # over its (n_rho, n_chi, n_T) = (128, 64, 64) startup grid for a synthetic
    # 41-level rotor with made-up collision rates (the real 13CO data file is not
    # available), then the march with populations interpolated in that grid.
    levels = None
    if not args.no_levels and dtype == "f32":
        import tempfile

        with tempfile.TemporaryDirectory() as td:
            path = os.path.join(td, "rotor.dat")
            W.write_lamda(path, W.synthetic_rotor_molecule(line))
            mol = rt.Molecule(path)
        torch.cuda.synchronize()
        t = time.perf_counter()
        lv = rt.Levels(mol, 2)
        torch.cuda.synchronize()
        build_s = time.perf_counter() - t
        ms_ot, k_ot = timed_launches(fl, args.steps, outs2, ws, line_=dict(line, levels=lv))
        levels = {"molecule": "synthetic 41-level rotor, 4 partners (made-up rates)",
                  "grid": [lv.config["n_n"], lv.config["n_chi"], lv.config["n_t"]],
                  "grid_build_s": build_s, "ms_per_step": ms_ot, "kernel_ms": k_ot,
                  "value": samples / (ms_ot * 1e-3),
                  "L_sum_over_lte": float(outs2["L"].double().sum() / outs["L"].double().sum())}
        print(f"# non-LTE levels: grid {levels['grid']} built in {build_s * 1e3:.1f} ms; "
              f"march {ms_ot:.3f} ms/step", file=sys.stderr, flush=True)
        lv.close()
        mol.close()

    # Post-transfer products on the line cube: the paper's 30 arcsec beam (at
    # 8.2 kpc, 1.19 pc: 2.39 cells of 0.5 pc) and the l,v mean over the axis
    # perpendicular to the disk (z).
    post = None
    if not args.no_post and dtype == "f32" and args.config == "cmz":
        nx, ny, nz = cube.shape
        sky = (nx, nz) if cube.axis == 1 else ((ny, nz) if cube.axis == 0 else (nx, ny))
        Lc = outs["L"].view(sky[0], sky[1], C)
        bo = torch.empty_like(Lc)
        bws = torch.empty(rt.load_library().iris_beam_workspace_bytes(sky[0], sky[1], C),
                          dtype=torch.uint8, device=dev)
        lv = torch.empty((sky[0], C), dtype=torch.float32, device=dev)
        fwhm = 30.0 / 206264.806 * 8200.0 / 0.5

        def post_ms(fn):
            for _ in range(args.warmup):
                fn()
            settle(fn)
            a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            a0.record(stream)
            for _ in range(args.steps):
                fn()
            a1.record(stream)
            torch.cuda.synchronize()
            return a0.elapsed_time(a1) / args.steps

        beam_ms = post_ms(lambda: rt.beam_convolve(Lc, fwhm, out=bo, workspace=bws))
        lv_ms = post_ms(lambda: rt.lv_mean(bo, 1, out=lv))
        cube_bytes = Lc.numel() * 4
        post = {"beam": {"fwhm_pix": fwhm, "ms": beam_ms,
                         "hbm_gbs": 4 * cube_bytes / (beam_ms * 1e-3) / 1e9,
                         "hbm_frac": 4 * cube_bytes / (beam_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "bytes": 4 * cube_bytes},
                "lv_mean": {"ms": lv_ms, "hbm_gbs": cube_bytes / (lv_ms * 1e-3) / 1e9,
                            "hbm_frac": cube_bytes / (lv_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}}
        print(f"# beam (FWHM {fwhm:.2f} px) on [L]: {beam_ms:.3f} ms; l,v mean: {lv_ms:.3f} ms",
              file=sys.stderr, flush=True)
        del bo, bws, lv

    esz = torch.empty(0, dtype=tdt).element_size()
    bytes_march = 4 * n_cells * esz + 5 * n_pix * C * 4
    win = window_samples(cube, line)
    exps = 2.0 * win
    achieved_exp = exps / (k_ms * 1e-3) / 1e9
    hbm_gbs = bytes_march / (k_ms * 1e-3) / 1e9

    result = {
        "metric": "cell*channel samples/s, forward synthesis (1 GPU)",
        "value": samples / (ms_step * 1e-3),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "settle": {"seconds_per_leg": SETTLE_S, "launches_main_legs": settled["launches"],
                   "note": "after the W warm-up steps each leg keeps launching, untimed, "
                           "until the GPU has been busy for this long (clock ramp)"},
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "storage_dtype": dtype,
        "data": "synthetic (seeded lognormal density, GRF velocity + ring, uniform T)",
        "config": {"workload": cube.name, "grid": list(cube.shape), "sightline_axis": cube.axis,
                   "n_pix": n_pix, "n_los": n_los, "n_chan": C, "samples": samples,
                   "parallelism": "none (1 GPU)"},
        "roofline": {"bound": "alu", "kernel": "fwd_kernel (line-window march) + table kernel",
                     "achieved": achieved_exp, "peak": EXP_PEAK_GPS, "unit": "Gexp/s",
                     "frac": achieved_exp / EXP_PEAK_GPS,
                     "traffic": stored_traffic() if (args.config == "cmz" and dtype == "f32")
                     else None,
                     "work_per_launch": {"window_samples": win, "exp_per_window_sample": 2},
                     "kernel_ms": k_ms,
                     "hbm": {"achieved_gbs": hbm_gbs, "peak_gbs": HBM_PEAK_GBS,
                             "frac": hbm_gbs / HBM_PEAK_GBS, "bytes_per_launch": bytes_march}},
    }
    if layout_cmp is not None:
        result["with_layout_pass"] = layout_cmp
    if precision is not None:
        result["storage_precision"] = precision
    if subsampled:
        result["velocity_subsampling"] = subsampled
    if smooth:
        result["smooth_integration"] = smooth
    if thin:
        result["optically_thin"] = thin
    if post:
        result["post_transfer"] = post
    if levels:
        result["levels_ot"] = levels
    rates = rt.iris_probe_issue_rates()
    result["roofline"]["peak_measured"] = {
        "exp_per_s": rates["exp_per_s"], "fma_per_s": rates["fma_per_s"],
        "note": "issue-rate probe: 8 independent chains per lane over a full grid"}
    print(f"# probe: v_exp_f32 {rates['exp_per_s'] / 1e12:.2f}e12/s, FMA "
          f"{rates['fma_per_s'] / 1e12:.2f}e12/s", file=sys.stderr, flush=True)
    del f, outs, outs2, ws
    torch.cuda.empty_cache()
    if not args.no_adjoint:
        result["fwd_adj"] = bench_fwd_adj(args, line)
        torch.cuda.empty_cache()
    if not args.no_batch:
        result["batch"] = bench_batch(args, line)
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        print("# timing the oracle on a host-core sample", file=sys.stderr, flush=True)
        adj_cube = W.config_adjoint(seed=0) if not args.no_adjoint else None
        result["cpu_baseline"] = cpu_baseline(cube, line, args.cpu_seconds, gpu_rows, adj_cube)
    print(json.dumps(result), flush=True)


def bench_fwd_adj(args, line) -> dict:
    """Forward + adjoint on the 256^3 x 256-channel cube: loss = mean squared
    difference of [T] against the cube of a second seed; checkpoints every K
    cells. One step = forward with checkpoints + loss cotangent + adjoint."""
    import torch

    from paper_2607_01338_amd import rt
    from paper_2607_01338_amd import workloads as W

    dev = torch.device("cuda:0")
    cube = W.config_adjoint(seed=0)
    target = W.config_adjoint(seed=1)
    print(f"# fwd+adj: {cube.name}", file=sys.stderr, flush=True)
    f = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev).float().contiguous()
         for k, v in cube.fields().items()}
    tf = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev).float().contiguous()
          for k, v in target.fields().items()}
    ch = rt.Channels(cube.channels.n_chan, cube.channels.v_lo_kms, cube.channels.dv_kms)
    tgt = rt.iris_rt_forward(tf["ln_nh2"], tf["t_kin"], tf["v_los"], tf["x_tracer"],
                             axis=cube.axis, cell_cm=cube.cell_cm, channels=ch, line=line,
                             components="T")["T"]
    del tf
    samples = int(np.prod(cube.shape)) * ch.n_chan
    out = {}
    for K in (16, 32, 64):
        fs = rt._fields_struct(f["ln_nh2"], f["t_kin"], f["v_los"], f["x_tracer"], None,
                               cube.axis, cube.cell_cm)
        ws = torch.empty(rt.workspace_bytes(fs, ch.c(), K), dtype=torch.uint8, device=dev)
        T = {"T": torch.empty((cube.n_pix, ch.n_chan), dtype=torch.float32, device=dev)}
        gT = torch.empty_like(T["T"])

        def step():
            rt.iris_rt_forward(f["ln_nh2"], f["t_kin"], f["v_los"], f["x_tracer"],
                               axis=cube.axis, cell_cm=cube.cell_cm, channels=ch, line=line,
                               ckpt_K=K, workspace=ws, out=T)
            torch.sub(T["T"], tgt, out=gT)
            gT.mul_(2.0 / gT.numel())
            return rt.iris_rt_adjoint(f["ln_nh2"], f["t_kin"], f["v_los"], f["x_tracer"],
                                      axis=cube.axis, cell_cm=cube.cell_cm, channels=ch,
                                      line=line, cot={"T": gT}, ckpt_K=K, workspace=ws)

        for _ in range(args.warmup):
            step()
        settle(step)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            step()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        # Algorithmic HBM bytes of one step: the four FP32 fields read by the
        # forward and again by the adjoint, [T] written, the loss cotangent
        # ([T] and the target read, the cotangent written, then read by the
        # adjoint), the checkpoints (line excess per channel plus six FP64
        # scalars per sightline) written and read, and four FP64 gradients.
        n_cells, n_pix, C = int(np.prod(cube.shape)), cube.n_pix, ch.n_chan
        n_ck = (cube.n_los + K - 1) // K
        ck = n_ck * n_pix * (C * 4 + 6 * 8)
        byt = 2 * 4 * n_cells * 4 + n_pix * C * 4 * 5 + 2 * ck + 4 * n_cells * 8
        out[f"K{K}"] = {"ms_per_step": ms, "value": samples / (ms * 1e-3),
                        "hbm_bytes_per_step": byt, "hbm_gbs": byt / (ms * 1e-3) / 1e9,
                        "hbm_frac": byt / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        print(f"# fwd+adj K={K}: {ms:.3f} ms/step", file=sys.stderr, flush=True)
        del ws
    return {"metric": "cell*channel samples/s, forward + adjoint (1 GPU)",
            "unit": "samples/s", "workload": cube.name, "samples": samples,
            "loss": "mean squared difference of [T] vs the seed-1 cube", "by_ckpt": out}


def bench_batch(args, line) -> dict:
    """The 64-cube batch (uneven sizes and sightline axes, 64..512 channels,
    half FP32 and half BF16 storage) as one plan: forward, and forward +
    adjoint (K = 16, cotangent on [T]), each one graph launch per phase.
    Compared with the same cubes launched one by one through iris_rt_forward.
    Then the forward with smooth steps, a plan of one launch per cube."""
    import torch

    from paper_2607_01338_amd import rt
    from paper_2607_01338_amd import workloads as W

    dev = torch.device("cuda:0")
    print("# batch: generating 64 cubes", file=sys.stderr, flush=True)
    cubes = W.config_batch()
    tdt = {"f32": torch.float32, "bf16": torch.bfloat16}
    devs = []
    for c in cubes:
        devs.append({k: torch.from_numpy(np.ascontiguousarray(v)).to(dev).to(tdt[c.storage])
                     .contiguous() for k, v in c.fields().items()})
    samples = int(sum(int(np.prod(c.shape)) * c.channels.n_chan for c in cubes))

    def spec(c, d):
        return dict(fields=(d["ln_nh2"], d["t_kin"], d["v_los"], d["x_tracer"]), axis=c.axis,
                    cell_cm=c.cell_cm,
                    channels=rt.Channels(c.channels.n_chan, c.channels.v_lo_kms,
                                         c.channels.dv_kms),
                    cot_components="T")

    def timed(fn, n_steps):
        for _ in range(args.warmup):
            fn()
        settle(fn)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n_steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n_steps

    out = {"workload": "64 cubes, 64^3..256x256x64, random axis, 64-512 channels, "
                       "32 FP32 + 32 BF16 storage",
           "samples": samples}
    t = time.perf_counter()
    plan = rt.Plan([spec(c, d) for c, d in zip(cubes, devs)], autotune=True)
    out["plan_create_s"] = time.perf_counter() - t
    gs = [plan.groups(i) for i in range(len(cubes))]
    out["autotuned_groups"] = {str(g): gs.count(g) for g in (1, 2, 4)}
    out["info_fwd"] = plan.info()
    ms = timed(plan.forward, args.steps)
    out["fwd"] = {"ms_per_step": ms, "value": samples / (ms * 1e-3)}
    print(f"# batch plan forward: {ms:.3f} ms/step", file=sys.stderr, flush=True)

    # The same cubes one launch each (plain entry point, default packing).
    singles = []
    for c, d in zip(cubes, devs):
        chn = rt.Channels(c.channels.n_chan, c.channels.v_lo_kms, c.channels.dv_kms)
        fs = rt._fields_struct(d["ln_nh2"], d["t_kin"], d["v_los"], d["x_tracer"], None, c.axis,
                               c.cell_cm)
        singles.append((chn, torch.empty(rt.workspace_bytes(fs, chn.c(), 0), dtype=torch.uint8,
                                         device=dev)))

    def one_by_one():
        for i, (c, d) in enumerate(zip(cubes, devs)):
            rt.iris_rt_forward(d["ln_nh2"], d["t_kin"], d["v_los"], d["x_tracer"], axis=c.axis,
                               cell_cm=c.cell_cm, channels=singles[i][0], line=line,
                               out=plan.outputs[i], workspace=singles[i][1])

    ms1 = timed(one_by_one, max(2, args.steps // 4))
    out["fwd_one_launch_per_cube"] = {"ms_per_step": ms1, "value": samples / (ms1 * 1e-3)}
    print(f"# batch one launch per cube: {ms1:.3f} ms/step", file=sys.stderr, flush=True)
    plan.close()
    del plan, singles
    torch.cuda.empty_cache()

    def adjoint_plan(tune):
        # Tuned: the forward's packings per class and the checkpoint interval
        # (ckpt_K = 0); the adjoint's packings follow the plan rule either way.
        p = rt.Plan([spec(c, d) for c, d in zip(cubes, devs)], adjoint=True,
                    ckpt_K=0 if tune else 16, autotune=tune)
        gen = torch.Generator(device=dev)
        gen.manual_seed(5)
        for i in range(len(cubes)):
            tt = p.cotangents[i]["T"]
            tt.copy_(torch.randn(tt.shape, generator=gen, device=dev))
        ags = [p.adjoint_groups(i) for i in range(len(cubes))]
        return p, {str(g): ags.count(g) for g in (1, 2, 4)}

    plan, out["adjoint_groups"] = adjoint_plan(False)
    out["info_fwd_adj"] = plan.info()

    def fwd_adj():
        plan.forward()
        plan.adjoint()

    ms2 = timed(fwd_adj, max(2, args.steps // 2))
    out["fwd_adj"] = {"ms_per_step": ms2, "value": samples / (ms2 * 1e-3), "ckpt_K": 16}
    print(f"# batch plan forward+adjoint: {ms2:.3f} ms/step", file=sys.stderr, flush=True)

    # The same forward + adjoint as one forward and one adjoint launch per cube
    # through the plain entry points (one workspace, sized for the largest cube).
    chs, need = [], 0
    for c, d in zip(cubes, devs):
        chn = rt.Channels(c.channels.n_chan, c.channels.v_lo_kms, c.channels.dv_kms)
        fs = rt._fields_struct(d["ln_nh2"], d["t_kin"], d["v_los"], d["x_tracer"], None, c.axis,
                               c.cell_cm)
        chs.append(chn)
        need = max(need, rt.workspace_bytes(fs, chn.c(), 16))
    wsa = torch.empty(need, dtype=torch.uint8, device=dev)

    def fwd_adj_one_by_one():
        for i, (c, d) in enumerate(zip(cubes, devs)):
            fl = (d["ln_nh2"], d["t_kin"], d["v_los"], d["x_tracer"])
            rt.iris_rt_forward(*fl, axis=c.axis, cell_cm=c.cell_cm, channels=chs[i], line=line,
                               ckpt_K=16, workspace=wsa, out=plan.outputs[i])
            rt.iris_rt_adjoint(*fl, axis=c.axis, cell_cm=c.cell_cm, channels=chs[i], line=line,
                               cot=plan.cotangents[i], ckpt_K=16, workspace=wsa)

    ms2b = timed(fwd_adj_one_by_one, max(2, args.steps // 4))
    out["fwd_adj_one_launch_per_cube"] = {"ms_per_step": ms2b, "value": samples / (ms2b * 1e-3),
                                          "ckpt_K": 16}
    print(f"# batch forward+adjoint, one launch pair per cube: {ms2b:.3f} ms/step",
          file=sys.stderr, flush=True)
    del wsa
    plan.close()
    del plan
    torch.cuda.empty_cache()

    # Forward packings per class and the checkpoint interval tuned at plan creation.
    t = time.perf_counter()
    plan, _ = adjoint_plan(True)
    out["plan_create_tuned_adjoint_s"] = time.perf_counter() - t
    ms2c = timed(fwd_adj, max(2, args.steps // 2))
    out["fwd_adj_tuned"] = {"ms_per_step": ms2c, "value": samples / (ms2c * 1e-3),
                            "ckpt_K": plan.info()["ckpt_K"]}
    print(f"# batch plan forward+adjoint, forward packing and K tuned (K = "
          f"{out['fwd_adj_tuned']['ckpt_K']}): {ms2c:.3f} ms/step",
          file=sys.stderr, flush=True)
    plan.close()
    del plan
    torch.cuda.empty_cache()

    # The paper's production setting, thick transfer with smooth steps: a plan
    # of one captured launch per cube.
    plan = rt.Plan([spec(c, d) for c, d in zip(cubes, devs)], line=dict(line, integrator="smooth"))
    ms3 = timed(plan.forward, max(2, args.steps // 4))
    out["fwd_smooth"] = {"ms_per_step": ms3, "value": samples / (ms3 * 1e-3)}
    print(f"# batch plan forward, smooth steps: {ms3:.3f} ms/step", file=sys.stderr, flush=True)
    plan.close()
    return out


if __name__ == "__main__":
    main()
