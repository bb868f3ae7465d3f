"""GPU parity of the smooth integrator (trapezoidal first step, BDF2 after it,
each step clamped at zero): the HIP kernel against the FP64 oracle's smooth
integration, element by element on the same seeded inputs (the oracle reads
the dequantised stored values), gate err_inf <= 1e-5 per component."""

import math

import numpy as np
import pytest
import torch

import oracle
from paper_2607_01338_amd import metrics as M
from paper_2607_01338_amd import rt
from paper_2607_01338_amd import workloads as W

from gpu_helpers import TOL_FWD, dequantised, line_dict, problem, say, to_device

pytestmark = pytest.mark.gpu

SMOOTH = dict(integrator="smooth")


def smooth_forward(cube, dev, line, f=0, components="TCDLB"):
    ch = cube.channels
    out = rt.iris_rt_forward(dev["ln_nh2"], dev["t_kin"], dev["v_los"], dev["x_tracer"],
                             dev.get("t_dust"), axis=cube.axis, cell_cm=cube.cell_cm,
                             channels=rt.Channels(ch.n_chan, ch.v_lo_kms, ch.dv_kms, f),
                             line=line, components=components)
    torch.cuda.synchronize()
    return out


def check_smooth(cube, dt, line=None, f=0, pix=None, label=""):
    line = dict(line or W.LINE_13CO_21, **SMOOTH)
    say(f"[smooth] {label or cube.name} shape={cube.shape} axis={cube.axis} dtype={dt} "
        f"C={cube.channels.n_chan} f={f}")
    dev = to_device(cube, dt)
    out = smooth_forward(cube, dev, line, f)
    pr = problem(cube, dequantised(dev))
    pr.simpson_f = f
    ref = oracle.forward(pr, line, pix=pix)
    floor = 1e-6 * float(np.max(np.abs(ref["T"])))
    errs = {}
    for k in "TCDLB":
        g = out[k].double().cpu().numpy()
        if pix is not None:
            g = g[pix.start:pix.stop]
        errs[k] = M.err_inf(g, ref[k], floor)
    say(f"      err_inf {errs}")
    for k, e in errs.items():
        assert e <= TOL_FWD, (k, e)
    return out, ref


def test_small_config_fp64_full():
    check_smooth(W.config_small(), "f64")


@pytest.mark.parametrize("dt", ["f32", "f64", "bf16", "f16"])
def test_ragged_along_y(dt):
    # 101 cells: a full 64-cell chunk, then 37 (an unpaired last step);
    # 150 channels: three slots, windows across slot boundaries.
    cube = W.make_cube((6, 101, 5), 1, W.Channels(150, -30.0, 0.4), seed=21, v_rms_kms=12.0)
    check_smooth(cube, dt)


@pytest.mark.parametrize("dt", ["f32", "bf16"])
def test_ragged_along_x(dt):
    cube = W.make_cube((130, 3, 4), 0, W.Channels(96, -48.0, 1.0), seed=22, v_rms_kms=20.0)
    check_smooth(cube, dt)


def test_long_sightlines_wide_band():
    # CMZ-like sightlines: 512 cells, 800 channels of 0.5 km/s over +-200 km/s
    # (13 slots of the 16-slot variant).
    cube = W.make_cube((3, 512, 5), 1, W.CH_C2, seed=23, v_rms_kms=90.0)
    check_smooth(cube, "f32")


def test_widest_channel_grid():
    # The largest marched grid, 2048 velocities: every slot of the 32-slot
    # variant in use, and 2049 refused on the host.
    cube = W.make_cube((2, 3, 70), 2, W.Channels(2048, -204.8, 0.2), seed=33, v_rms_kms=60.0)
    check_smooth(cube, "f32")
    assert rt.load_library().iris_smooth_max_channels() == 2048
    dev = to_device(cube, "f32")
    with pytest.raises(rt.IrisError):
        rt.iris_rt_forward(dev["ln_nh2"], dev["t_kin"], dev["v_los"], dev["x_tracer"],
                           axis=2, cell_cm=cube.cell_cm, channels=rt.Channels(2049, -204.8, 0.2),
                           line=SMOOTH)


def test_separate_dust_temperature_and_strong_dust():
    # Separate line and dust source functions; a continuum that outshines the
    # line, so [L] is a small difference of large intensities.
    cube = W.make_cube((4, 5, 70), 2, W.Channels(64, -32.0, 1.0), seed=24, t_dust=True)
    out, ref = check_smooth(cube, "f32", line_dict(kappa_dust_cm2g=300.0))
    assert np.max(np.abs(ref["C"])) > 2.0 * np.max(np.abs(ref["L"]))


def test_literal_upper_energy_mode():
    cube = W.make_cube((4, 5, 40), 2, W.Channels(48, -24.0, 1.0), seed=25)
    check_smooth(cube, "f32", line_dict(energy_mode=1))


def test_thick_dust():
    cube = W.make_cube((3, 4, 90), 2, W.Channels(40, -20.0, 1.0), seed=26)
    check_smooth(cube, "f32", line_dict(kappa_dust_cm2g=3e4))


@pytest.mark.parametrize("n_los", [1, 2, 3, 4, 63, 64, 65, 66])
def test_short_sightlines(n_los):
    # Background only (1 cell), the trapezoidal step alone (2), one BDF2 step
    # (3), and the chunk edges.
    cube = W.make_cube((3, 4, n_los), 2, W.Channels(70, -35.0, 1.0), seed=27 + n_los,
                       v_rms_kms=5.0)
    out, ref = check_smooth(cube, "f32", label=f"n_los={n_los}")
    if n_los == 1:
        jbg = ref["B"][0, 0]
        for k in "TCB":
            assert torch.all(out[k] == out[k][0, 0]), k
        assert float(out["L"].abs().max()) == 0.0 and float(out["D"].abs().max()) == 0.0
        assert float(out["T"][0, 0]) == pytest.approx(jbg, rel=1e-6)


def test_single_channel():
    cube = W.make_cube((2, 1, 9), 1, W.Channels(1, -0.5, 1.0), seed=28, v_rms_kms=0.3)
    check_smooth(cube, "f32")


def test_edge_cases_hot_empty_and_out_of_band():
    cube = W.make_cube((4, 4, 33), 2, W.Channels(64, -16.0, 0.5), seed=29, v_rms_kms=40.0)
    cube.t_kin[:, :, ::3] = 80.0            # above T_inf below
    cube.x_tracer[:, :, 1::5] = 0.0         # no tracer
    cube.v_los[0, :, :] = 500.0             # far outside the band
    check_smooth(cube, "f32", line_dict(t_inf_k=60.0, t_bg_k=0.0))


def test_clamp_at_zero():
    # A hot background behind thick cold line cells with empty cells after
    # them: the steps overshoot below zero and are clamped, in the kernel as
    # in the oracle.
    cube = W.make_cube((2, 3, 6), 2, W.Channels(9, -2.0, 0.5), seed=35, v_rms_kms=0.0)
    cube.t_kin[...] = 5.0
    cube.ln_nh2[...] = math.log(1e6)
    cube.x_tracer[...] = 0.0
    cube.x_tracer[:, :, 1] = 1e-4
    cube.x_tracer[1, :, 0] = 1e-4
    out, ref = check_smooth(cube, "f32", line_dict(kappa_dust_cm2g=0.0, t_bg_k=100.0))
    assert np.min(ref["T"]) == 0.0
    assert float(out["T"].min()) == 0.0


@pytest.mark.parametrize("units", ["intensity", "tb"])
def test_output_units(units):
    cube = W.make_cube((4, 5, 60), 2, W.Channels(96, -24.0, 0.5), seed=80, v_rms_kms=6.0)
    check_smooth(cube, "f32", line_dict(units=units, kappa_dust_cm2g=200.0), label=units)


@pytest.mark.parametrize("f", [1, 2])
@pytest.mark.parametrize("dt", ["f32", "bf16"])
def test_velocity_subsampling(f, dt):
    cube = W.make_cube((4, 5, 50), 2, W.Channels(48, -24.0, 1.0), seed=84, v_rms_kms=6.0)
    check_smooth(cube, dt, f=f)


def test_cmz_sightlines_subsampled():
    # 800 channels at f = 1: 1601 marched velocities, the 32-slot variant.
    cube = W.make_cube((2, 512, 3), 1, W.CH_C2, seed=36, v_rms_kms=90.0)
    check_smooth(cube, "f32", f=1)


def test_deterministic_and_skippable_outputs():
    cube = W.make_cube((5, 6, 77), 2, W.Channels(130, -40.0, 0.6), seed=30)
    dev = to_device(cube, "f32")
    a = smooth_forward(cube, dev, SMOOTH)
    b = smooth_forward(cube, dev, SMOOTH)
    part = smooth_forward(cube, dev, SMOOTH, components="L")
    for k in "TCDLB":
        assert torch.equal(a[k], b[k]), k
    assert set(part) == {"L"} and torch.equal(part["L"], a["L"])


def test_smooth_refuses_checkpoints_and_adjoint():
    cube = W.make_cube((2, 2, 8), 2, W.Channels(16, -8.0, 1.0), seed=37)
    dev = to_device(cube, "f32")
    with pytest.raises(rt.IrisError):
        rt.iris_rt_forward(dev["ln_nh2"], dev["t_kin"], dev["v_los"], dev["x_tracer"], axis=2,
                           cell_cm=cube.cell_cm, channels=rt.Channels(16, -8.0, 1.0),
                           line=SMOOTH, ckpt_K=16)


@pytest.fixture(scope="module")
def cmz_cube():
    say("[smooth] generating the 512x512x128 CMZ cube")
    return W.config_cmz()


@pytest.mark.parametrize("dt", ["f32", "bf16"])
def test_cmz_full_size_sampled(cmz_cube, dt):
    rng = np.random.default_rng(41)
    pix = np.sort(rng.choice(cmz_cube.n_pix, 24, replace=False))
    say(f"[smooth] CMZ 512x512x128 along y, 800 ch, dtype={dt}, 24 sampled sightlines")
    line = dict(W.LINE_13CO_21, **SMOOTH)
    dev = to_device(cmz_cube, dt)
    out = smooth_forward(cmz_cube, dev, line)
    deq = dequantised(dev)
    del dev
    pr = problem(cmz_cube, deq)
    refs = {k: [] for k in "TCDLB"}
    for p in pix:
        ref = oracle.forward(pr, line, pix=range(int(p), int(p) + 1))
        for k in "TCDLB":
            refs[k].append(ref[k][0])
    errs = {}
    for k in "TCDLB":
        g = out[k][torch.from_numpy(pix).cuda()].double().cpu().numpy()
        errs[k] = M.err_inf(g, np.array(refs[k]))
    say(f"      err_inf {errs}")
    for k, e in errs.items():
        assert e <= TOL_FWD, (k, e)
    assert float(out["T"].max()) > 5.0 and float(out["T"].min()) >= 0.0
