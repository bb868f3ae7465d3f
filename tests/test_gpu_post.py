"""GPU parity of the post-transfer products (Gaussian beam convolution, l,v
mean) against the FP64 reference in oracle/post.py, gate err_inf <= 1e-5."""

import numpy as np
import pytest
import torch

from oracle import post
from paper_2607_01338_amd import metrics as M
from paper_2607_01338_amd import rt
from paper_2607_01338_amd import workloads as W

from gpu_helpers import TOL_FWD, say, to_device

pytestmark = pytest.mark.gpu


def _rand_cube(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape).astype(np.float32) + 2.0


@pytest.mark.parametrize("shape,fwhm", [((33, 47, 64), 2.39), ((20, 21, 7), 4.0),
                                        ((5, 3, 12), 6.0), ((64, 40, 1), 1.0),
                                        ((1, 30, 8), 3.0)])
def test_beam_against_reference(shape, fwhm):
    say(f"[beam] shape={shape} fwhm={fwhm}")
    a = _rand_cube(shape, 1)
    t = torch.from_numpy(a).cuda()
    out = rt.beam_convolve(t, fwhm)
    torch.cuda.synchronize()
    ref = post.beam_convolve(a.astype(np.float64), fwhm)
    err = M.err_inf(out.double().cpu().numpy(), ref)
    say(f"      err_inf {err:.2e}")
    assert err <= TOL_FWD


def test_beam_in_place_and_unaligned_match():
    a = _rand_cube((17, 19, 12), 2)
    t = torch.from_numpy(a).cuda()
    ref = rt.beam_convolve(t, 3.0).clone()
    flat = torch.empty(a.size + 1, device="cuda")
    view = flat[1:].view(a.shape)  # rows no longer 16-byte aligned: one channel per lane
    view.copy_(t)
    rt.beam_convolve(view, 3.0, out=view)  # in place
    torch.cuda.synchronize()
    assert torch.allclose(view, ref, rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("axis", [0, 1])
@pytest.mark.parametrize("shape", [(33, 47, 64), (9, 128, 5)])
def test_lv_mean_against_reference(shape, axis):
    a = _rand_cube(shape, 3)
    t = torch.from_numpy(a).cuda()
    out = rt.lv_mean(t, axis)
    torch.cuda.synchronize()
    ref = post.lv_mean(a.astype(np.float64), axis)
    assert M.err_inf(out.double().cpu().numpy(), ref) <= TOL_FWD


def test_beam_and_lv_of_a_synthesised_cube():
    # The paper's chain on a cube: synthesis, continuum-subtracted line, beam, l,v mean.
    cube = W.make_cube((24, 16, 20), 2, W.Channels(48, -24.0, 1.0), seed=60, v_rms_kms=6.0)
    dev = to_device(cube, "f32")
    ch = cube.channels
    res = rt.iris_rt_forward(dev["ln_nh2"], dev["t_kin"], dev["v_los"], dev["x_tracer"], axis=2,
                             cell_cm=cube.cell_cm,
                             channels=rt.Channels(ch.n_chan, ch.v_lo_kms, ch.dv_kms),
                             components="L")
    L = res["L"].view(24, 16, ch.n_chan)
    beam = rt.beam_convolve(L, 2.39)
    lv = rt.lv_mean(beam, 1)
    torch.cuda.synchronize()
    Lh = L.double().cpu().numpy()
    ref_beam = post.beam_convolve(Lh, 2.39)
    assert M.err_inf(beam.double().cpu().numpy(), ref_beam) <= TOL_FWD
    assert M.err_inf(lv.double().cpu().numpy(), post.lv_mean(ref_beam, 1)) <= TOL_FWD
