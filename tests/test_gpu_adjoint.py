"""GPU parity of the adjoint: hand-written reverse march vs the FP64 oracle's
reverse mode (itself pinned by complex-step derivatives) on the same
cotangents, gate err_inf <= 1e-4 per field; central finite differences of
the oracle on sampled cells of the 256^3 workload, gate 1e-3."""

import numpy as np
import pytest
import torch

import oracle
from paper_2607_01338_amd import metrics as M
from paper_2607_01338_amd import rt
from paper_2607_01338_amd import workloads as W

from gpu_helpers import (channels_of, dequantised, line_dict, pixel_cells, problem, say,
                         to_device)

pytestmark = pytest.mark.gpu

TOL_ADJ = 1e-4
FIELDS = ("ln_nh2", "t_kin", "v_los", "x_tracer")


def gpu_grad(cube, dev, cot: dict, K: int, line=None):
    res = rt.iris_rt_forward(dev["ln_nh2"], dev["t_kin"], dev["v_los"], dev["x_tracer"],
                             dev.get("t_dust"), axis=cube.axis, cell_cm=cube.cell_cm,
                             channels=channels_of(cube), line=line, ckpt_K=K)
    tc = {k: torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32)).cuda()
          for k, v in cot.items()}
    g = rt.iris_rt_adjoint(dev["ln_nh2"], dev["t_kin"], dev["v_los"], dev["x_tracer"],
                           dev.get("t_dust"), axis=cube.axis, cell_cm=cube.cell_cm,
                           channels=channels_of(cube), line=line, cot=tc, ckpt_K=K,
                           workspace=res["_workspace"])
    torch.cuda.synchronize()
    return res, {k: v.cpu().numpy() for k, v in g.items()}


def random_cot(n_pix, n_chan, seed, comps="TCDLB"):
    rng = np.random.default_rng(seed)
    return {k: rng.standard_normal((n_pix, n_chan)).astype(np.float32) for k in comps}


def check_adjoint(cube, dt, K, cot, line=None, label=""):
    line = line or dict(W.LINE_13CO_21)
    say(f"[adj] {label or cube.name} shape={cube.shape} axis={cube.axis} dtype={dt} K={K} "
        f"C={cube.channels.n_chan}")
    dev = to_device(cube, dt)
    _, g = gpu_grad(cube, dev, cot, K, line)
    ref = oracle.adjoint(problem(cube, dequantised(dev)), line,
                         {k: v.astype(np.float64) for k, v in cot.items()})
    fields = FIELDS + (("t_dust",) if "t_dust" in dev else ())
    errs = {f: M.err_inf(g[f], ref[f]) for f in fields}
    say(f"      err_inf {errs}")
    for f, e in errs.items():
        assert e <= TOL_ADJ, (f, e)
    return g, ref


@pytest.mark.parametrize("K", [8, 16, 32, 64])
def test_adjoint_all_components_along_z(K):
    cube = W.make_cube((3, 4, 100), 2, W.Channels(96, -24.0, 0.5), seed=51, v_rms_kms=8.0)
    check_adjoint(cube, "f32", K, random_cot(cube.n_pix, 96, 1))


@pytest.mark.parametrize("axis,dt", [(0, "f32"), (1, "bf16"), (1, "f64")])
def test_adjoint_other_axes_and_storage(axis, dt):
    shape = [5, 6, 7]
    shape[axis] = 77
    cube = W.make_cube(tuple(shape), axis, W.Channels(130, -40.0, 0.6), seed=52, v_rms_kms=15.0)
    check_adjoint(cube, dt, 16, random_cot(cube.n_pix, 130, 2))


def test_adjoint_tape_subsegments():
    # 0.05 km/s channels: each window spans ~5 passes of 64 lanes, so a 16-cell
    # segment overflows the tape and is split into recomputed sub-segments.
    cube = W.make_cube((2, 3, 40), 2, W.Channels(400, -10.0, 0.05), seed=53, v_rms_kms=3.0)
    check_adjoint(cube, "f32", 16, random_cot(cube.n_pix, 400, 3))


def test_adjoint_dusty_and_hot_cells():
    cube = W.make_cube((3, 3, 70), 2, W.Channels(64, -16.0, 0.5), seed=54, v_rms_kms=6.0)
    cube.t_kin[:, :, ::4] = 90.0
    check_adjoint(cube, "f32", 32, random_cot(cube.n_pix, 64, 4),
                  line_dict(kappa_dust_cm2g=400.0, t_inf_k=80.0))


def test_adjoint_zero_abundance_still_has_abundance_gradient():
    cube = W.make_cube((2, 2, 30), 2, W.Channels(48, -12.0, 0.5), seed=55, v_rms_kms=4.0)
    cube.x_tracer[:, :, 10:20] = 0.0
    g, ref = check_adjoint(cube, "f32", 8, random_cot(cube.n_pix, 48, 5, "T"))
    assert np.abs(ref["x_tracer"][:, :, 10:20]).max() > 0


# Separate line and dust source functions: a dust temperature field (its own
# gradient), the literal upper-level energy, or both; dust from faint to
# tens of optical depths per segment, all sightline packings.
@pytest.mark.parametrize("K", [8, 32])
def test_adjoint_separate_dust_temperature(K):
    cube = W.make_cube((3, 4, 75), 2, W.Channels(96, -24.0, 0.5), seed=56, v_rms_kms=8.0,
                       t_dust=True)
    g, ref = check_adjoint(cube, "f32", K, random_cot(cube.n_pix, 96, 21),
                           line_dict(kappa_dust_cm2g=400.0), label=f"t_dust K={K}")
    assert np.abs(ref["t_dust"]).max() > 0


def test_adjoint_literal_upper_energy():
    cube = W.make_cube((4, 3, 60), 1, W.Channels(80, -20.0, 0.5), seed=63, v_rms_kms=6.0)
    check_adjoint(cube, "f32", 16, random_cot(cube.n_pix, 80, 22),
                  line_dict(energy_mode=1, kappa_dust_cm2g=200.0), label="energy_mode 1")


@pytest.mark.parametrize("groups", [1, 2, 4])
def test_adjoint_separate_source_functions_every_packing(groups, monkeypatch):
    monkeypatch.setenv("IRIS_RT_ADJOINT_SIGHTLINES_PER_WAVE", str(groups))
    cube = W.make_cube((3, 5, 70), 2, W.Channels(80, -20.0, 0.5), seed=64 + groups,
                       v_rms_kms=6.0, t_dust=True)
    check_adjoint(cube, "f32", 16, random_cot(cube.n_pix, 80, 23 + groups),
                  line_dict(energy_mode=1, kappa_dust_cm2g=300.0),
                  label=f"t_dust + energy_mode 1, G={groups}")


@pytest.mark.parametrize("dt", ["bf16", "f64"])
def test_adjoint_separate_source_functions_other_storage_and_axis(dt):
    cube = W.make_cube((50, 4, 5), 0, W.Channels(64, -16.0, 0.5), seed=67, v_rms_kms=5.0,
                       t_dust=True)
    check_adjoint(cube, dt, 8, random_cot(cube.n_pix, 64, 27),
                  line_dict(kappa_dust_cm2g=200.0), label=f"t_dust axis 0 {dt}")


def test_adjoint_separate_source_functions_thick_dust_and_subsegments():
    # Dust tens of optical depths per segment (the reverse march moves its
    # base) and narrow channels whose windows overflow the tape.
    cube = W.make_cube((2, 3, 48), 2, W.Channels(300, -7.5, 0.05), seed=68, v_rms_kms=3.0,
                       t_dust=True)
    g, ref = check_adjoint(cube, "f32", 16, random_cot(cube.n_pix, 300, 28),
                           line_dict(kappa_dust_cm2g=3.0e4, energy_mode=1),
                           label="t_dust thick dust, sub-segments")
    for f in FIELDS + ("t_dust",):
        assert np.all(np.isfinite(g[f])), f


def test_autograd_function_mse_loss():
    cube = W.make_cube((4, 3, 50), 1, W.Channels(80, -20.0, 0.5), seed=57, v_rms_kms=6.0)
    target = W.make_cube((4, 3, 50), 1, W.Channels(80, -20.0, 0.5), seed=58, v_rms_kms=6.0)
    say("[adj] autograd MSE loss")
    dev = to_device(cube, "f32")
    tdev = to_device(target, "f32")
    ch = channels_of(cube)
    with torch.no_grad():
        tgt = rt.synthesize(tdev["ln_nh2"], tdev["t_kin"], tdev["v_los"], tdev["x_tracer"],
                            axis=1, cell_cm=cube.cell_cm, channels=ch)["T"]
    leaves = {k: dev[k].clone().requires_grad_(True) for k in FIELDS}
    out = rt.synthesize(*(leaves[k] for k in FIELDS), axis=1, cell_cm=cube.cell_cm, channels=ch,
                        ckpt_K=16)
    loss = ((out["T"] - tgt) ** 2).mean()
    loss.backward()
    gT = (2.0 * (out["T"] - tgt) / out["T"].numel()).detach().double().cpu().numpy()
    ref = oracle.adjoint(problem(cube, dequantised(dev)), W.LINE_13CO_21, {"T": gT})
    for f in FIELDS:
        e = M.err_inf(leaves[f].grad.double().cpu().numpy(), ref[f])
        say(f"      {f}: err_inf {e:.2e}")
        assert e <= TOL_ADJ, (f, e)


def test_autograd_function_with_dust_temperature():
    # The dust temperature field is a differentiable input too; a field
    # without requires_grad gets no gradient.
    cube = W.make_cube((3, 4, 40), 2, W.Channels(64, -16.0, 0.5), seed=69, v_rms_kms=5.0,
                       t_dust=True)
    say("[adj] autograd with a dust temperature field")
    dev = to_device(cube, "f32")
    ch = channels_of(cube)
    line = line_dict(kappa_dust_cm2g=300.0)
    names = FIELDS + ("t_dust",)
    leaves = {k: dev[k].clone().requires_grad_(k != "v_los") for k in names}
    out = rt.synthesize(*(leaves[k] for k in names), axis=2, cell_cm=cube.cell_cm, channels=ch,
                        line=line, ckpt_K=8)
    cot = random_cot(cube.n_pix, 64, 31, comps="TB")
    loss = sum((out[k] * torch.from_numpy(cot[k]).cuda()).sum() for k in "TB")
    loss.backward()
    ref = oracle.adjoint(problem(cube, dequantised(dev)), line,
                         {k: v.astype(np.float64) for k, v in cot.items()})
    assert leaves["v_los"].grad is None
    for f in ("ln_nh2", "t_kin", "x_tracer", "t_dust"):
        e = M.err_inf(leaves[f].grad.double().cpu().numpy(), ref[f])
        say(f"      {f}: err_inf {e:.2e}")
        assert e <= TOL_ADJ, (f, e)


# --- the 256^3 forward + adjoint workload ----------------------------------------

N_FD_CELLS = 1000   # central differences on this many random cells (seed 2)
N_FD_SIGHT = 64     # ... drawn from this many random sightlines


@pytest.fixture(scope="module")
def adj_problem():
    """The 256^3 x 256-channel cube, the cotangent of the MSE of [T] against the
    seed-1 cube, and everything of the oracle that does not depend on the
    checkpoint interval: its reverse-mode gradients on N_FD_SIGHT sampled
    sightlines and central differences on N_FD_CELLS cells of them."""
    say("[adj] generating the 256^3 cube and its seed-1 target")
    cube = W.config_adjoint(seed=0)
    target = W.config_adjoint(seed=1)
    dev = to_device(cube, "f32")
    tdev = to_device(target, "f32")
    ch = channels_of(cube)
    tgt = rt.iris_rt_forward(tdev["ln_nh2"], tdev["t_kin"], tdev["v_los"], tdev["x_tracer"],
                             axis=2, cell_cm=cube.cell_cm, channels=ch, components="T")["T"]
    del tdev
    T = rt.iris_rt_forward(dev["ln_nh2"], dev["t_kin"], dev["v_los"], dev["x_tracer"], axis=2,
                           cell_cm=cube.cell_cm, channels=ch, components="T")["T"]
    gT = (2.0 * (T - tgt) / T.numel()).contiguous()
    torch.cuda.synchronize()
    gT_np = gT.double().cpu().numpy()
    deq = {k: v.double().cpu().numpy() for k, v in dev.items()}
    rng = np.random.default_rng(2)
    pix = rng.choice(cube.n_pix, N_FD_SIGHT, replace=False)
    # Sightline-major copies of the sampled sightlines: [N_FD_SIGHT][n_los].
    cells = np.stack([pixel_cells(cube, int(p)) for p in pix])
    sight = {k: deq[k].ravel()[cells] for k in FIELDS}
    chn = cube.channels

    def prob(fields):
        n = fields["ln_nh2"].shape[0]
        return oracle.Problem(*(fields[k].reshape(n, 1, -1) for k in FIELDS), 2, cube.cell_cm,
                              chn.n_chan, chn.v_lo_kms, chn.dv_kms)

    say(f"[adj] oracle reverse mode on {N_FD_SIGHT} sightlines")
    rev = oracle.adjoint(prob(sight), W.LINE_13CO_21, {"T": gT_np[pix]})
    rev = {f: rev[f].reshape(N_FD_SIGHT, -1) for f in FIELDS}
    # Central differences (step 1e-3 relative; velocity scaled by
    # max(|v|, 1.4 km/s)): every perturbed sightline is one pixel of a single
    # oracle call per field.
    which = rng.integers(0, N_FD_SIGHT, N_FD_CELLS)
    pos = rng.integers(0, cube.n_los, N_FD_CELLS)
    fd = {}
    say(f"[adj] oracle central differences on {N_FD_CELLS} cells x 4 fields")
    for f in FIELDS:
        rep = {k: np.repeat(sight[k][which], 2, axis=0) for k in FIELDS}
        x0 = sight[f][which, pos]
        h = 1e-3 * (np.maximum(np.abs(x0), 1.4) if f == "v_los" else np.abs(x0))
        rows = np.arange(N_FD_CELLS)
        rep[f][2 * rows, pos] = x0 + h
        rep[f][2 * rows + 1, pos] = x0 - h
        o = oracle.forward(prob(rep), W.LINE_13CO_21)["T"]
        Lval = np.sum(np.repeat(gT_np[pix[which]], 2, axis=0) * o, axis=1)
        fd[f] = (Lval[0::2] - Lval[1::2]) / (2 * h)
    flat = cells[which, pos]
    return dict(cube=cube, dev=dev, gT=gT, pix=pix, cells=cells, rev=rev, fd=fd, fd_flat=flat)


@pytest.mark.parametrize("K", [16, 32, 64])
def test_adjoint_256cube_sampled_and_finite_differences(adj_problem, K):
    A = adj_problem
    cube, dev = A["cube"], A["dev"]
    say(f"[adj] 256^3 x 256 ch, cotangent of the MSE of [T] vs the seed-1 cube, K={K}")
    ch = channels_of(cube)
    res = rt.iris_rt_forward(dev["ln_nh2"], dev["t_kin"], dev["v_los"], dev["x_tracer"], axis=2,
                             cell_cm=cube.cell_cm, channels=ch, ckpt_K=K, components="T")
    g = rt.iris_rt_adjoint(dev["ln_nh2"], dev["t_kin"], dev["v_los"], dev["x_tracer"], axis=2,
                           cell_cm=cube.cell_cm, channels=ch, cot={"T": A["gT"]}, ckpt_K=K,
                           workspace=res["_workspace"])
    torch.cuda.synchronize()
    cells = torch.from_numpy(A["cells"].ravel()).cuda()
    flat = torch.from_numpy(A["fd_flat"]).cuda()
    for f in FIELDS:
        gf = g[f].reshape(-1)
        assert bool(torch.isfinite(gf).all()), f
        # (i) the oracle's reverse mode on the sampled sightlines.
        gg = gf[cells].cpu().numpy().reshape(A["rev"][f].shape)
        e = M.err_inf(gg, A["rev"][f])
        say(f"      reverse {f} ({N_FD_SIGHT} sightlines): err_inf {e:.2e}")
        assert e <= TOL_ADJ, (f, e)
        # (ii) central differences of the oracle on the sampled cells.
        gpu_vals, fd_vals = gf[flat].cpu().numpy(), A["fd"][f]
        e = np.max(np.abs(gpu_vals - fd_vals)) / np.max(np.abs(fd_vals))
        say(f"      FD {f} ({N_FD_CELLS} cells): err_inf {e:.2e}")
        assert e <= 1e-3, (f, e)


@pytest.mark.parametrize("K,kappa,seed", [(16, 3.0e4, 61), (64, 1.0e4, 61), (8, 3.0e4, 62)])
def test_adjoint_dust_thicker_than_the_scaled_range_in_a_segment(K, kappa, seed):
    # Dust depths of tens to hundreds per segment (single cells up to the
    # clamp at 60): the reverse march moves the base of its scaled state
    # inside the segment; the gradients stay finite and match the oracle.
    cube = W.make_cube((3, 3, 70), 2, W.Channels(64, -16.0, 0.5), seed=seed, v_rms_kms=6.0)
    line = line_dict(kappa_dust_cm2g=kappa)
    cot = random_cot(cube.n_pix, 64, 9)
    g, ref = check_adjoint(cube, "f32", K, cot, line, label=f"thick dust kappa={kappa:g} K={K}")
    for f in FIELDS:
        assert np.all(np.isfinite(g[f])), f
    # The dust depth of some segment exceeds the scaled range of one base.
    from paper_2607_01338_amd.workloads import LINE_13CO_21 as L0
    kd = (kappa * L0["dust_to_gas"] * L0["mu_amu_per_h2"] * 1.66053906660e-24 *
          np.exp(cube.ln_nh2) * cube.cell_cm)
    seg = np.minimum(kd, 60.0).reshape(cube.n_pix, -1)[:, : (cube.n_los // K) * K]
    assert seg.reshape(cube.n_pix, -1, K).sum(axis=2).max() > 64.0


@pytest.mark.parametrize("axis", [0, 1])
def test_adjoint_in_place_matches_transposed_copy(axis, monkeypatch):
    # Gradients written in place (native layout) and through the
    # sightline-major buffer plus inverse transpose are the same numbers.
    shape = (40, 5, 33) if axis == 0 else (5, 40, 33)
    cube = W.make_cube(shape, axis, W.Channels(64, -16.0, 0.5), seed=78, v_rms_kms=5.0)
    dev = to_device(cube, "f32")
    cot = random_cot(cube.n_pix, 64, 7, comps="TL")
    say(f"[adj] in place vs transposed copy, axis={axis}")
    _, ga = gpu_grad(cube, dev, cot, 16)
    monkeypatch.setenv("IRIS_RT_FIELD_LAYOUT", "transpose")
    _, gb = gpu_grad(cube, dev, cot, 16)
    for f in FIELDS:
        assert np.array_equal(ga[f], gb[f]), f


@pytest.mark.parametrize("groups", [1, 2, 4])
@pytest.mark.parametrize("K", [8, 64])
def test_adjoint_every_sightline_packing(groups, K, monkeypatch):
    # 1, 2 or 4 sightlines per adjoint wavefront, forced: 3 x 5 = 15 sightlines
    # (a partly empty last wavefront), windows needing several passes at 16
    # lanes, a ragged last segment (70 cells) and dust.
    monkeypatch.setenv("IRIS_RT_ADJOINT_SIGHTLINES_PER_WAVE", str(groups))
    cube = W.make_cube((3, 5, 70), 2, W.Channels(80, -20.0, 0.5), seed=95 + groups,
                       v_rms_kms=6.0)
    check_adjoint(cube, "f32", K, random_cot(cube.n_pix, 80, 11 + groups),
                  line=line_dict(kappa_dust_cm2g=200.0), label=f"adjoint G={groups} K={K}")


def test_adjoint_autotune_records_its_choice(tmp_path, monkeypatch):
    # The adjoint tuner returns one of the packings, its gradients pass the
    # oracle gate, a plain adjoint of the same class afterwards reproduces
    # them bit for bit, and the choice is appended to the tuning cache file.
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("IRIS_RT_TUNE_CACHE", str(cache))
    cube = W.make_cube((4, 7, 83), 2, W.Channels(72, -18.0, 0.5), seed=131, v_rms_kms=6.0)
    dev = to_device(cube, "f32")
    cot = random_cot(cube.n_pix, 72, 19, comps="TCL")
    tc = {k: torch.from_numpy(v).cuda() for k, v in cot.items()}
    say("[adj] iris_rt_autotune_adjoint, K=16")
    kw = dict(axis=cube.axis, cell_cm=cube.cell_cm, channels=channels_of(cube),
              line=dict(W.LINE_13CO_21))
    fields = (dev["ln_nh2"], dev["t_kin"], dev["v_los"], dev["x_tracer"])
    res = rt.iris_rt_forward(*fields, ckpt_K=16, **kw)
    g, grads = rt.iris_rt_autotune_adjoint(*fields, cot=tc, ckpt_K=16,
                                           workspace=res["_workspace"], **kw)
    torch.cuda.synchronize()
    say(f"      chose {g} sightlines per wavefront")
    assert g in (1, 2, 4)
    ref = oracle.adjoint(problem(cube, dequantised(dev)), W.LINE_13CO_21,
                         {k: v.astype(np.float64) for k, v in cot.items()})
    for f in FIELDS:
        e = M.err_inf(grads[f].cpu().numpy(), ref[f])
        assert e <= TOL_ADJ, (f, e)
    again = rt.iris_rt_adjoint(*fields, cot=tc, ckpt_K=16, workspace=res["_workspace"], **kw)
    torch.cuda.synchronize()
    for f in FIELDS:
        assert torch.equal(again[f], grads[f]), f
    lines = [ln.split() for ln in cache.read_text().splitlines()
             if ln.startswith("iris-tune-adjoint")]
    assert lines and lines[-1][-2:] == ["16", str(g)], lines


def test_adjoint_in_intensity_units():
    # Cotangents with respect to intensity-unit cubes: the seeds carry the
    # units per Rayleigh-Jeans kelvin; against the oracle's reverse mode in
    # the same units.
    cube = W.make_cube((3, 3, 48), 2, W.Channels(64, -16.0, 0.5), seed=82, v_rms_kms=6.0)
    cot = random_cot(cube.n_pix, cube.channels.n_chan, 83)
    check_adjoint(cube, "f32", 16, cot, line_dict(units="intensity"), label="units=intensity")


def test_adjoint_with_velocity_subsampling():
    # Cotangents of the channel averages spread onto the marched velocities
    # with the Simpson weights; against the oracle's reverse mode on the same
    # subsampled grid.
    cube = W.make_cube((3, 3, 40), 2, W.Channels(32, -16.0, 1.0), seed=85, v_rms_kms=5.0)
    dev = to_device(cube, "f32")
    ch = cube.channels
    chs = rt.Channels(ch.n_chan, ch.v_lo_kms, ch.dv_kms, 1)
    say("[adj] subsampled f=1")
    cot = random_cot(cube.n_pix, ch.n_chan, 86)
    res = rt.iris_rt_forward(dev["ln_nh2"], dev["t_kin"], dev["v_los"], dev["x_tracer"],
                             axis=cube.axis, cell_cm=cube.cell_cm, channels=chs, ckpt_K=16)
    tc = {k: torch.from_numpy(v).cuda() for k, v in cot.items()}
    g = rt.iris_rt_adjoint(dev["ln_nh2"], dev["t_kin"], dev["v_los"], dev["x_tracer"],
                           axis=cube.axis, cell_cm=cube.cell_cm, channels=chs, cot=tc, ckpt_K=16,
                           workspace=res["_workspace"])
    torch.cuda.synchronize()
    deq = dequantised(dev)
    pr = oracle.Problem(deq["ln_nh2"], deq["t_kin"], deq["v_los"], deq["x_tracer"], cube.axis,
                        cube.cell_cm, ch.n_chan, ch.v_lo_kms, ch.dv_kms, simpson_f=1)
    ref = oracle.adjoint(pr, dict(W.LINE_13CO_21), {k: v.astype(np.float64) for k, v in cot.items()})
    errs = {f: M.err_inf(g[f].cpu().numpy(), ref[f]) for f in FIELDS}
    say(f"      err_inf {errs}")
    for f, e in errs.items():
        assert e <= TOL_ADJ, (f, e)


def test_adjoint_through_dust_opaque_sightlines():
    # Every cell 20 to 400 dust depths thick (many clamped at 60): the line
    # shares the dust's source function, so [L] and the gradients with respect
    # to density, velocity and abundance vanish below the FP64 rounding of the
    # oracle's own reverse mode; the temperature gradient (through the source
    # function of the cells nearest the observer) is what the cube measures.
    cube = W.make_cube((3, 3, 70), 2, W.Channels(64, -16.0, 0.5), seed=61, v_rms_kms=6.0)
    line = line_dict(kappa_dust_cm2g=3.0e5)
    say("[adj] dust-opaque sightlines, kappa 3e5, K=8")
    dev = to_device(cube, "f32")
    cot = random_cot(cube.n_pix, 64, 9)
    _, g = gpu_grad(cube, dev, cot, 8, line)
    ref = oracle.adjoint(problem(cube, dequantised(dev)), line,
                         {k: v.astype(np.float64) for k, v in cot.items()})
    for f in FIELDS:
        assert np.all(np.isfinite(g[f])), f
    e = M.err_inf(g["t_kin"], ref["t_kin"])
    say(f"      t_kin err_inf {e:.2e}")
    assert e <= TOL_ADJ
    # Both sides near zero (with less dust these gradients are of order 10 to
    # 1e5 in the same units).
    for f in ("ln_nh2", "v_los", "x_tracer"):
        say(f"      {f}: max |gpu| {np.max(np.abs(g[f])):.2e}, max |oracle| "
            f"{np.max(np.abs(ref[f])):.2e}")
        assert np.max(np.abs(g[f])) < 1e-6 and np.max(np.abs(ref[f])) < 1e-6, f
