"""The forward entry point that allocates nothing (iris_rt_forward_static),
called through the C ABI, against iris_rt_forward with a caller workspace on
the same inputs: the same kernels, so the outputs must be bit-identical. Two
calls in a row on the same GPU, the second on a smaller cube, so that the
second reads scratch the first has left behind."""

import pytest
import torch

from paper_2607_01338_amd import rt
from paper_2607_01338_amd import workloads as W

from gpu_helpers import channels_of, line_dict, say, to_device

pytestmark = pytest.mark.gpu


def _outputs(cube):
    return {k: torch.full((cube.n_pix, cube.channels.n_chan), float("nan"), dtype=torch.float32,
                          device="cuda") for k in "TCDLB"}


def test_static_forward_matches_workspace_forward_twice():
    assert rt.load_library().iris_rt_forward_static_max_bytes() == 128 * 1024
    calls = [
        (W.make_cube((6, 40, 30), 1, W.Channels(160, -40.0, 0.5), seed=201, v_rms_kms=10.0),
         dict(W.LINE_13CO_21), "thick formal, 6x40x30 along y, 160 ch"),
        (W.make_cube((3, 4, 21), 2, W.Channels(48, -12.0, 0.5), seed=202, v_rms_kms=4.0),
         line_dict(transfer="selective", kappa_dust_cm2g=300.0),
         "selectively thin, 3x4x21 along z, 48 ch"),
    ]
    for cube, line, label in calls:
        say(f"[static forward] {label}")
        dev = to_device(cube, "f32")
        fl = (dev["ln_nh2"], dev["t_kin"], dev["v_los"], dev["x_tracer"])
        a = rt.iris_rt_forward_static(*fl, axis=cube.axis, cell_cm=cube.cell_cm,
                                      channels=channels_of(cube), line=line, out=_outputs(cube))
        b = rt.iris_rt_forward(*fl, axis=cube.axis, cell_cm=cube.cell_cm,
                               channels=channels_of(cube), line=line)
        torch.cuda.synchronize()
        for k in "TCDLB":
            assert bool(torch.isfinite(a[k]).all()), k
            assert torch.equal(a[k], b[k]), k


def test_static_forward_refuses_more_scratch_than_it_has(monkeypatch):
    # A sightline-major copy of the fields of a 64 x 32 x 32 cube (1 MiB) does
    # not fit the static scratch: refused on the host, nothing launched.
    cube = W.make_cube((64, 32, 32), 0, W.Channels(32, -8.0, 0.5), seed=203)
    dev = to_device(cube, "f32")
    monkeypatch.setenv("IRIS_RT_FIELD_LAYOUT", "transpose")
    say("[static forward] refused: copied layout above the static scratch")
    with pytest.raises(rt.IrisError) as e:
        rt.iris_rt_forward_static(dev["ln_nh2"], dev["t_kin"], dev["v_los"], dev["x_tracer"],
                                  axis=cube.axis, cell_cm=cube.cell_cm,
                                  channels=channels_of(cube), out=_outputs(cube))
    assert e.value.status == 3  # IRIS_E_WORKSPACE
