"""GPU parity of the batched plans (one persistent, graph-captured launch per
phase over many cubes) and of the autotuner: every cube of a plan against the
FP64 oracle on its dequantised fields, gate err_inf <= 1e-5 (forward) and
1e-4 (gradients); replays after the inputs change in place; and the 64-cube
batch workload at full size, sampled sightlines against the oracle."""

import numpy as np
import pytest
import torch

import oracle
from paper_2607_01338_amd import metrics as M
from paper_2607_01338_amd import rt
from paper_2607_01338_amd import workloads as W

from gpu_helpers import (TOL_FWD, channels_of, dequantised, pixel_cells, problem, say,
                         to_device)

pytestmark = pytest.mark.gpu

TOL_ADJ = 1e-4
FIELDS = ("ln_nh2", "t_kin", "v_los", "x_tracer")


def mixed_cubes():
    """Small cubes of every sightline axis and storage type, ragged sizes,
    different channel grids."""
    specs = [((5, 7, 70), 2, W.Channels(64, -32.0, 1.0), "f32"),
             ((90, 3, 4), 0, W.Channels(150, -60.0, 0.8), "bf16"),
             ((4, 130, 3), 1, W.Channels(40, -20.0, 1.0), "f16"),
             ((3, 3, 65), 2, W.Channels(200, -50.0, 0.5), "f64"),
             ((6, 33, 5), 1, W.Channels(97, -48.5, 1.0), "f32")]
    out = []
    for i, (shape, axis, ch, dt) in enumerate(specs):
        c = W.make_cube(shape, axis, ch, seed=300 + i, v_rms_kms=10.0)
        out.append((c, dt))
    # One cell, one channel (the random-field generator needs more than one
    # cell, so the cell is cut from a larger cube).
    big = W.make_cube((2, 2, 2), 2, W.Channels(1, -0.5, 1.0), seed=306, v_rms_kms=0.3)
    one = W.Cube(*(np.ascontiguousarray(a[:1, :1, :1]) for a in
                   (big.ln_nh2, big.t_kin, big.v_los, big.x_tracer)),
                 axis=2, cell_cm=big.cell_cm, channels=big.channels)
    out.append((one, "f32"))
    return out


def plan_spec(cube, dev):
    return dict(fields=(dev["ln_nh2"], dev["t_kin"], dev["v_los"], dev["x_tracer"]),
                axis=cube.axis, cell_cm=cube.cell_cm, channels=channels_of(cube))


def check_outputs(cube, dev, out, label, pix=None):
    ref = oracle.forward(problem(cube, dequantised(dev)), W.LINE_13CO_21)
    floor = 1e-6 * float(np.max(np.abs(ref["T"])))
    errs = {k: M.err_inf(out[k].double().cpu().numpy(), ref[k], floor) for k in "TCDLB"}
    say(f"      {label} err_inf {errs}")
    for k, e in errs.items():
        assert e <= TOL_FWD, (label, k, e)


def test_plan_forward_mixed_batch_and_replay():
    cubes = mixed_cubes()
    devs = [to_device(c, dt) for c, dt in cubes]
    say(f"[plan] forward plan over {len(cubes)} mixed cubes")
    plan = rt.Plan([plan_spec(c, d) for (c, _), d in zip(cubes, devs)])
    info = plan.info()
    say(f"      info {info}")
    assert info["n_cubes"] == len(cubes) and info["fwd_blocks"] >= 1
    plan.forward()
    torch.cuda.synchronize()
    for i, ((c, dt), d) in enumerate(zip(cubes, devs)):
        check_outputs(c, d, plan.outputs[i], f"cube {i} ({dt}, axis {c.axis}, G={plan.groups(i)})")
    # The same plan on new data written into the same buffers.
    # (A small velocity shift keeps the one-channel cube's line in its band.)
    for d in devs:
        d["v_los"].add_(0.7)
        d["t_kin"].mul_(1.25)
    plan.forward()
    plan.forward()
    torch.cuda.synchronize()
    for i, ((c, dt), d) in enumerate(zip(cubes, devs)):
        check_outputs(c, d, plan.outputs[i], f"replay cube {i}")
    plan.close()


def test_plan_matches_single_cube_launch():
    cubes = mixed_cubes()[:4]
    devs = [to_device(c, dt) for c, dt in cubes]
    say("[plan] plan vs single-cube launches")
    plan = rt.Plan([plan_spec(c, d) for (c, _), d in zip(cubes, devs)])
    plan.forward()
    for i, ((c, dt), d) in enumerate(zip(cubes, devs)):
        single = rt.iris_rt_forward(d["ln_nh2"], d["t_kin"], d["v_los"], d["x_tracer"],
                                    axis=c.axis, cell_cm=c.cell_cm, channels=channels_of(c))
        torch.cuda.synchronize()
        for k in "TCDLB":
            a = plan.outputs[i][k].double()
            b = single[k].double()
            e = float((a - b).abs().max() / b.abs().max().clamp_min(1e-30))
            assert e <= 1e-6, (i, k, e)
    plan.close()


def test_plan_separate_dust_temperature_forward():
    c = W.make_cube((4, 5, 80), 2, W.Channels(60, -30.0, 1.0), seed=333, v_rms_kms=8.0)
    d = to_device(c, "f32")
    d["t_dust"] = (d["t_kin"] * 0.7).contiguous()
    say("[plan] separate T_dust cube in a plan")
    spec = plan_spec(c, d)
    spec["fields"] = spec["fields"] + (d["t_dust"],)
    plan = rt.Plan([spec])
    plan.forward()
    torch.cuda.synchronize()
    deq = dequantised(d)
    ref = oracle.forward(problem(c, deq), W.LINE_13CO_21)
    for k in "TCDLB":
        e = M.err_inf(plan.outputs[0][k].double().cpu().numpy(), ref[k],
                      1e-6 * float(np.max(np.abs(ref["T"]))))
        assert e <= TOL_FWD, (k, e)
    plan.close()


@pytest.mark.parametrize("K", [16, 32])
def test_plan_adjoint_mixed_batch(K):
    cubes = [(c, dt) for c, dt in mixed_cubes() if dt in ("f32", "bf16", "f64")]
    devs = [to_device(c, dt) for c, dt in cubes]
    say(f"[plan] forward+adjoint plan over {len(cubes)} cubes, K={K}")
    plan = rt.Plan([dict(plan_spec(c, d), cot_components="TL") for (c, _), d in zip(cubes, devs)],
                   adjoint=True, ckpt_K=K)
    rng = np.random.default_rng(K)
    cots = []
    for i, (c, _) in enumerate(cubes):
        cot = {k: rng.standard_normal((c.n_pix, c.channels.n_chan)).astype(np.float32)
               for k in "TL"}
        for k, v in cot.items():
            plan.cotangents[i][k].copy_(torch.from_numpy(v))
        cots.append(cot)
    for rep in range(2):
        plan.forward()
        plan.adjoint()
        torch.cuda.synchronize()
        for i, ((c, dt), d) in enumerate(zip(cubes, devs)):
            ref = oracle.adjoint(problem(c, dequantised(d)), W.LINE_13CO_21,
                                 {k: v.astype(np.float64) for k, v in cots[i].items()})
            errs = {f: M.err_inf(plan.gradients[i][f].cpu().numpy(), ref[f]) for f in FIELDS}
            say(f"      rep {rep} cube {i} ({dt}, axis {c.axis}) err_inf {errs}")
            for f, e in errs.items():
                assert e <= TOL_ADJ, (rep, i, f, e)
    plan.close()


def test_plan_adjoint_separate_source_functions():
    # Cubes with a dust temperature field (separate line and dust source
    # functions, their own batched adjoint launch) beside cubes without one,
    # in one plan; gradients of every field, T_dust included, against the
    # oracle's reverse mode on two replays.
    specs = [((5, 7, 70), 2, W.Channels(64, -32.0, 1.0), "f32", True),
             ((90, 3, 4), 0, W.Channels(150, -60.0, 0.8), "bf16", True),
             ((4, 60, 3), 1, W.Channels(40, -20.0, 1.0), "f32", False),
             ((3, 3, 65), 2, W.Channels(200, -50.0, 0.5), "f64", True)]
    cubes = [(W.make_cube(sh, ax, ch, seed=340 + i, v_rms_kms=10.0, t_dust=td), dt)
             for i, (sh, ax, ch, dt, td) in enumerate(specs)]
    devs = [to_device(c, dt) for c, dt in cubes]
    line = dict(W.LINE_13CO_21, kappa_dust_cm2g=300.0)
    say(f"[plan] forward+adjoint plan, {len(cubes)} cubes, three with a dust temperature")
    plan_specs = []
    for (c, _), d in zip(cubes, devs):
        sp = dict(plan_spec(c, d), cot_components="TB")
        if "t_dust" in d:
            sp["fields"] = sp["fields"] + (d["t_dust"],)
        plan_specs.append(sp)
    plan = rt.Plan(plan_specs, line=line, adjoint=True, ckpt_K=16)
    rng = np.random.default_rng(41)
    cots = []
    for i, (c, _) in enumerate(cubes):
        cot = {k: rng.standard_normal((c.n_pix, c.channels.n_chan)).astype(np.float32)
               for k in "TB"}
        for k, v in cot.items():
            plan.cotangents[i][k].copy_(torch.from_numpy(v))
        cots.append(cot)
    for rep in range(2):
        plan.forward()
        plan.adjoint()
        torch.cuda.synchronize()
        for i, ((c, dt), d) in enumerate(zip(cubes, devs)):
            ref = oracle.adjoint(problem(c, dequantised(d)), line,
                                 {k: v.astype(np.float64) for k, v in cots[i].items()})
            fields = FIELDS + (("t_dust",) if "t_dust" in d else ())
            errs = {f: M.err_inf(plan.gradients[i][f].cpu().numpy(), ref[f]) for f in fields}
            say(f"      rep {rep} cube {i} ({dt}, axis {c.axis}) err_inf {errs}")
            for f, e in errs.items():
                assert e <= TOL_ADJ, (rep, i, f, e)
    plan.close()


def test_autotune_single_cube():
    c = W.make_cube((6, 8, 90), 1, W.Channels(128, -64.0, 1.0), seed=341, v_rms_kms=12.0)
    d = to_device(c, "f32")
    say("[tune] iris_rt_autotune on one cube")
    g, out = rt.iris_rt_autotune(d["ln_nh2"], d["t_kin"], d["v_los"], d["x_tracer"], axis=c.axis,
                                 cell_cm=c.cell_cm, channels=channels_of(c))
    torch.cuda.synchronize()
    say(f"      chose {g} sightlines per wavefront")
    assert g in (1, 2, 4)
    check_outputs(c, d, out, "autotuned")


def test_plan_autotune_flag():
    cubes = mixed_cubes()[:3]
    devs = [to_device(c, dt) for c, dt in cubes]
    say("[plan] plan with autotuning")
    plan = rt.Plan([plan_spec(c, d) for (c, _), d in zip(cubes, devs)], autotune=True)
    plan.forward()
    torch.cuda.synchronize()
    for i, ((c, dt), d) in enumerate(zip(cubes, devs)):
        assert plan.groups(i) in (1, 2, 4)
        check_outputs(c, d, plan.outputs[i], f"tuned cube {i} G={plan.groups(i)}")
    plan.close()


def test_plan_adjoint_autotune_flag():
    # An adjoint plan with autotuning: forward packings timed per class, the
    # adjoint's by the plan rule; the replayed gradients pass the oracle gate.
    cubes = [(c, dt) for c, dt in mixed_cubes() if dt in ("f32", "bf16")][:3]
    devs = [to_device(c, dt) for c, dt in cubes]
    say("[plan] forward+adjoint plan with autotuning, K=16")
    plan = rt.Plan([dict(plan_spec(c, d), cot_components="T") for (c, _), d in zip(cubes, devs)],
                   adjoint=True, ckpt_K=16, autotune=True)
    rng = np.random.default_rng(5)
    cots = []
    for i, (c, _) in enumerate(cubes):
        cot = rng.standard_normal((c.n_pix, c.channels.n_chan)).astype(np.float32)
        plan.cotangents[i]["T"].copy_(torch.from_numpy(cot))
        cots.append(cot)
    plan.forward()
    plan.adjoint()
    torch.cuda.synchronize()
    for i, ((c, dt), d) in enumerate(zip(cubes, devs)):
        assert plan.groups(i) in (1, 2, 4)
        assert plan.adjoint_groups(i) in (1, 2, 4)
        ref = oracle.adjoint(problem(c, dequantised(d)), W.LINE_13CO_21,
                             {"T": cots[i].astype(np.float64)})
        errs = {f: M.err_inf(plan.gradients[i][f].cpu().numpy(), ref[f]) for f in FIELDS}
        say(f"      cube {i} ({dt}) G={plan.groups(i)} adjoint G={plan.adjoint_groups(i)} "
            f"err_inf {errs}")
        for f, e in errs.items():
            assert e <= TOL_ADJ, (i, f, e)
    plan.close()


def test_plan_chooses_the_checkpoint_interval():
    # ckpt_K = 0 with autotuning: the plan times K = 8..64 and keeps one; the
    # replayed gradients pass the oracle gate at that interval.
    cubes = [(c, dt) for c, dt in mixed_cubes() if dt in ("f32", "bf16")][:2]
    devs = [to_device(c, dt) for c, dt in cubes]
    say("[plan] forward+adjoint plan choosing its checkpoint interval")
    plan = rt.Plan([dict(plan_spec(c, d), cot_components="T") for (c, _), d in zip(cubes, devs)],
                   adjoint=True, ckpt_K=0, autotune=True)
    K = plan.info()["ckpt_K"]
    say(f"      chose K = {K}")
    assert K in (8, 16, 32, 64)
    rng = np.random.default_rng(9)
    cots = []
    for i, (c, _) in enumerate(cubes):
        cot = rng.standard_normal((c.n_pix, c.channels.n_chan)).astype(np.float32)
        plan.cotangents[i]["T"].copy_(torch.from_numpy(cot))
        cots.append(cot)
    for _ in range(2):
        plan.forward()
        plan.adjoint()
    torch.cuda.synchronize()
    for i, ((c, dt), d) in enumerate(zip(cubes, devs)):
        ref = oracle.adjoint(problem(c, dequantised(d)), W.LINE_13CO_21,
                             {"T": cots[i].astype(np.float64)})
        for f in FIELDS:
            e = M.err_inf(plan.gradients[i][f].cpu().numpy(), ref[f])
            assert e <= TOL_ADJ, (i, f, e)
    plan.close()


# --- the 64-cube batch at full size -------------------------------------------

@pytest.fixture(scope="module")
def batch_cubes():
    say("[plan] generating the 64-cube batch")
    return W.config_batch()


def test_batch_64_full_size_forward_adjoint(batch_cubes):
    """Forward and forward+adjoint over all 64 cubes in one plan (K = 16);
    six sampled sightlines per cube against the oracle. Errors are normwise
    over each cube's sampled sightlines, as for the full-size CMZ cube; the
    worst single-sightline figure is printed for information."""
    K, NS = 16, 6
    devs = [to_device(c, c.storage) for c in batch_cubes]
    specs = [dict(plan_spec(c, d), cot_components="T") for c, d in zip(batch_cubes, devs)]
    say("[plan] creating the 64-cube forward+adjoint plan")
    plan = rt.Plan(specs, adjoint=True, ckpt_K=K)
    say(f"      info {plan.info()}")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(64)
    for i in range(len(batch_cubes)):
        t = plan.cotangents[i]["T"]
        t.copy_(torch.randn(t.shape, generator=gen, device="cuda"))
    plan.forward()
    plan.adjoint()
    torch.cuda.synchronize()
    rng = np.random.default_rng(65)
    worst_f = {k: 0.0 for k in "TCDLB"}
    worst_g = {f: 0.0 for f in FIELDS}
    worst_single = 0.0
    for i, (c, d) in enumerate(zip(batch_cubes, devs)):
        pr = problem(c, dequantised(d))
        pix = [int(p) for p in rng.choice(c.n_pix, NS, replace=False)]
        ref = {k: [] for k in "TCDLB"}
        gref = {f: [] for f in FIELDS}
        gpu_g = {f: [] for f in FIELDS}
        for p in pix:
            r = oracle.forward(pr, W.LINE_13CO_21, pix=range(p, p + 1))
            for k in "TCDLB":
                ref[k].append(r[k][0])
            cot = {"T": plan.cotangents[i]["T"][p:p + 1].double().cpu().numpy()}
            gr = oracle.adjoint(pr, W.LINE_13CO_21, cot, pix=range(p, p + 1))
            cells = pixel_cells(c, p)
            idx = torch.from_numpy(cells).cuda()
            for f in FIELDS:
                gref[f].append(gr[f].reshape(-1)[cells])
                gpu_g[f].append(plan.gradients[i][f].reshape(-1)[idx].cpu().numpy())
        sel = torch.tensor(pix, device="cuda")
        floor = 1e-6 * float(np.max(np.abs(ref["T"])))
        for k in "TCDLB":
            g = plan.outputs[i][k][sel].double().cpu().numpy()
            worst_f[k] = max(worst_f[k], M.err_inf(g, np.array(ref[k]), floor))
            if k == "T":
                for j in range(NS):
                    worst_single = max(worst_single, M.err_inf(g[j], ref[k][j]))
        for f in FIELDS:
            worst_g[f] = max(worst_g[f], M.err_inf(np.concatenate(gpu_g[f]),
                                                   np.concatenate(gref[f])))
    say(f"      forward worst err_inf {worst_f}")
    say(f"      (worst single-sightline [T] err_inf {worst_single:.3g})")
    say(f"      adjoint worst err_inf {worst_g}")
    for k, e in worst_f.items():
        assert e <= TOL_FWD, (k, e)
    for f, e in worst_g.items():
        assert e <= TOL_ADJ, (f, e)
    plan.close()


def test_graph_replays_with_eager_work_between():
    # Each phase is a captured graph; replay it several times with eager
    # library and torch work and synchronisations in between, and check every
    # replay against eager single-cube launches on the same data.
    cubes = mixed_cubes()[:4]
    cubes = [(c, dt) for c, dt in cubes if dt in ("f32", "bf16", "f64")]
    devs = [to_device(c, dt) for c, dt in cubes]
    say(f"[plan] graph replays with eager work between, {len(cubes)} cubes")
    plan = rt.Plan([dict(plan_spec(c, d), cot_components="T") for (c, _), d in zip(cubes, devs)],
                   adjoint=True, ckpt_K=16)
    rng = np.random.default_rng(7)
    for i, (c, _) in enumerate(cubes):
        plan.cotangents[i]["T"].copy_(torch.from_numpy(
            rng.standard_normal((c.n_pix, c.channels.n_chan)).astype(np.float32)))
    for rep in range(3):
        plan.forward()
        plan.adjoint()
        torch.cuda.synchronize()
        for i, ((c, dt), d) in enumerate(zip(cubes, devs)):
            # Eager reference through the single-cube entry points.
            res = rt.iris_rt_forward(d["ln_nh2"], d["t_kin"], d["v_los"], d["x_tracer"],
                                     axis=c.axis, cell_cm=c.cell_cm, channels=channels_of(c),
                                     ckpt_K=16)
            g = rt.iris_rt_adjoint(d["ln_nh2"], d["t_kin"], d["v_los"], d["x_tracer"],
                                   axis=c.axis, cell_cm=c.cell_cm, channels=channels_of(c),
                                   cot={"T": plan.cotangents[i]["T"]}, ckpt_K=16,
                                   workspace=res["_workspace"])
            torch.cuda.synchronize()
            for k in "TCDLB":
                a, b = plan.outputs[i][k].double(), res[k].double()
                e = float((a - b).abs().max() / b.abs().max().clamp_min(1e-30))
                assert e <= 1e-6, (rep, i, k, e)
            for f in FIELDS:
                a, b = plan.gradients[i][f], g[f]
                e = float((a - b).abs().max() / b.abs().max().clamp_min(1e-300))
                assert e <= 1e-6, (rep, i, f, e)
        # Eager work of the program between replays: new data in place.
        for d in devs:
            d["v_los"].mul_(0.9)
            d["t_kin"].add_(3.0)
        torch.cuda.synchronize()
    plan.close()


def test_plan_with_velocity_subsampling():
    # A subsampled cube beside a centre-sampled one in one plan, forward and
    # adjoint: outputs and gradients against the single-cube entry points.
    c1 = W.make_cube((4, 6, 40), 2, W.Channels(32, -16.0, 1.0), seed=310, v_rms_kms=6.0)
    c2 = W.make_cube((5, 30, 4), 1, W.Channels(40, -20.0, 1.0), seed=311, v_rms_kms=6.0)
    d1, d2 = to_device(c1, "f32"), to_device(c2, "bf16")
    ch1 = rt.Channels(c1.channels.n_chan, c1.channels.v_lo_kms, c1.channels.dv_kms, 2)
    say("[plan] subsampled cube in a batch")
    spec1 = dict(plan_spec(c1, d1), channels=ch1)
    plan = rt.Plan([spec1, plan_spec(c2, d2)], adjoint=True, ckpt_K=16)
    rng = np.random.default_rng(312)
    for i, c in enumerate((c1, c2)):
        for k, t in plan.cotangents[i].items():
            t.copy_(torch.from_numpy(rng.standard_normal(tuple(t.shape)).astype(np.float32)))
    plan.forward()
    plan.adjoint()
    torch.cuda.synchronize()
    for i, (c, d, ch) in enumerate(((c1, d1, ch1), (c2, d2, channels_of(c2)))):
        res = rt.iris_rt_forward(d["ln_nh2"], d["t_kin"], d["v_los"], d["x_tracer"], axis=c.axis,
                                 cell_cm=c.cell_cm, channels=ch, ckpt_K=16)
        g = rt.iris_rt_adjoint(d["ln_nh2"], d["t_kin"], d["v_los"], d["x_tracer"], axis=c.axis,
                               cell_cm=c.cell_cm, channels=ch, cot=plan.cotangents[i], ckpt_K=16,
                               workspace=res["_workspace"])
        torch.cuda.synchronize()
        for k in "TCDLB":
            a, b = plan.outputs[i][k].double(), res[k].double()
            e = float((a - b).abs().max() / b.abs().max().clamp_min(1e-30))
            assert e <= 1e-6, (i, k, e)
        for f in FIELDS:
            a, b = plan.gradients[i][f], g[f]
            e = float((a - b).abs().max() / b.abs().max().clamp_min(1e-300))
            assert e <= 1e-6, (i, f, e)
    plan.close()


MODES = [("smooth", "thick"), ("formal", "thin"), ("smooth", "thin"), ("formal", "selective"),
         ("smooth", "selective")]


@pytest.mark.parametrize("integrator,transfer", MODES)
def test_plan_of_other_modes_matches_single_cube_forward(integrator, transfer):
    # The smooth integrator and the thin modes plan one captured launch per cube: every replay
    # equals the single-cube forward on the same data bit for bit, with eager work and new
    # data between replays; the first replay is also checked against the oracle.
    line = dict(W.LINE_13CO_21, integrator=integrator, transfer=transfer)
    cubes = mixed_cubes()
    devs = [to_device(c, dt) for c, dt in cubes]
    say(f"[plan] {transfer} transfer, {integrator} steps, {len(cubes)} cubes")
    plan = rt.Plan([plan_spec(c, d) for (c, _), d in zip(cubes, devs)], line=line)
    info = plan.info()
    assert info["n_cubes"] == len(cubes) and info["n_fwd_items"] == len(cubes)
    # Each captured single-cube forward chooses its own packing: the plan reports none.
    assert all(plan.groups(i) == 0 for i in range(len(cubes)))
    for rep in range(3):
        plan.forward()
        torch.cuda.synchronize()
        for i, ((c, dt), d) in enumerate(zip(cubes, devs)):
            res = rt.iris_rt_forward(d["ln_nh2"], d["t_kin"], d["v_los"], d["x_tracer"],
                                     axis=c.axis, cell_cm=c.cell_cm, channels=channels_of(c),
                                     line=line)
            torch.cuda.synchronize()
            for k in "TCDLB":
                assert torch.equal(plan.outputs[i][k], res[k]), (rep, i, k)
            if rep == 0:
                ref = oracle.forward(problem(c, dequantised(d)), line)
                floor = 1e-6 * float(np.max(np.abs(ref["T"])))
                for k in "TCDLB":
                    e = M.err_inf(plan.outputs[i][k].double().cpu().numpy(), ref[k], floor)
                    assert e <= TOL_FWD, (i, k, e)
        for d in devs:
            d["v_los"].mul_(0.9)
            d["t_kin"].add_(3.0)
        torch.cuda.synchronize()
    plan.close()
