"""C-ABI library: loads on a CPU host, exports every symbol the header
declares, and rejects bad arguments on the host before launching anything."""

import ctypes
import os
import re

import pytest

from paper_2607_01338_amd import rt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "iris_rt.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(iris_\w+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_expected_api():
    names = declared_functions()
    for n in ("iris_rt_forward", "iris_rt_adjoint", "iris_rt_layout", "iris_rt_workspace_bytes",
              "iris_last_error", "iris_status_string"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = rt.load_library()
    for n in declared_functions():
        assert hasattr(lib, n), n
    assert set(declared_functions()) <= set(rt._SIGNATURES)


def test_version_and_limits():
    lib = rt.load_library()
    assert b"gfx950" in lib.iris_version()
    assert lib.iris_max_channels() >= 800
    assert 1601 <= lib.iris_smooth_max_channels() <= lib.iris_max_channels()
    assert lib.iris_status_string(1) == b"invalid argument"


def _fields(**kw):
    d = dict(nx=4, ny=5, nz=6, axis=2, cell_cm=1e18, dtype=1, ln_nh2=0x1000, t_kin=0x2000,
             v_los=0x3000, x_tracer=0x4000, t_dust=None)
    d.update(kw)
    return rt.Fields(d["nx"], d["ny"], d["nz"], d["axis"], d["cell_cm"], d["dtype"], d["ln_nh2"],
                     d["t_kin"], d["v_los"], d["x_tracer"], d["t_dust"])


@pytest.mark.parametrize("bad,status", [
    (dict(nx=0), 1), (dict(axis=3), 1), (dict(cell_cm=-1.0), 1), (dict(cell_cm=float("nan")), 1),
    (dict(dtype=7), 1), (dict(t_kin=None), 1),
])
def test_forward_rejects_bad_fields_on_host(bad, status):
    lib = rt.load_library()
    f = _fields(**bad)
    ch = rt.ChannelsC(16, -8.0, 1.0)
    ln = rt.line_struct()
    out = rt.Outputs(0x5000, None, None, None, None)
    s = lib.iris_rt_forward(ctypes.byref(f), ctypes.byref(ch), ctypes.byref(ln), ctypes.byref(out),
                            0, None, 0, None)
    assert s == status
    assert len(lib.iris_last_error()) > 0


@pytest.mark.parametrize("ch,status", [((0, -8.0, 1.0), 1), ((16, -8.0, 0.0), 1),
                                       ((100000, -8.0, 1.0), 2), ((16, float("inf"), 1.0), 1)])
def test_forward_rejects_bad_channels(ch, status):
    lib = rt.load_library()
    f = _fields()
    c = rt.ChannelsC(*ch)
    ln = rt.line_struct()
    out = rt.Outputs(0x5000, None, None, None, None)
    assert lib.iris_rt_forward(ctypes.byref(f), ctypes.byref(c), ctypes.byref(ln),
                               ctypes.byref(out), 0, None, 0, None) == status


@pytest.mark.parametrize("bad", [dict(nu0_hz=0.0), dict(j_u=0), dict(j_max=1), dict(t_bg_k=-1.0),
                                 dict(energy_mode=2), dict(mu_amu_per_h2=0.0),
                                 dict(sigma_turb_kms=-1.0), dict(units=7), dict(units=-1),
                                 dict(integrator=2), dict(integrator=-1), dict(transfer=3),
                                 dict(transfer=-1)])
def test_forward_rejects_bad_line(bad):
    lib = rt.load_library()
    f = _fields()
    c = rt.ChannelsC(16, -8.0, 1.0)
    ln = rt.line_struct(bad)
    out = rt.Outputs(0x5000, None, None, None, None)
    assert lib.iris_rt_forward(ctypes.byref(f), ctypes.byref(c), ctypes.byref(ln),
                               ctypes.byref(out), 0, None, 0, None) == 1


def test_workspace_sizes_and_checks(monkeypatch):
    lib = rt.load_library()
    c = rt.ChannelsC(16, -8.0, 1.0)
    f2 = _fields(axis=2)
    f1 = _fields(axis=1)
    n2 = lib.iris_rt_workspace_bytes(ctypes.byref(f2), ctypes.byref(c), 0)
    assert n2 > 0  # temperature tables only
    # Fields along x or y are read in place by default; the sightline-major
    # copy (and its room in the workspace) is only made on request.
    assert lib.iris_rt_workspace_bytes(ctypes.byref(f1), ctypes.byref(c), 0) == n2
    monkeypatch.setenv("IRIS_RT_FIELD_LAYOUT", "transpose")
    n1 = lib.iris_rt_workspace_bytes(ctypes.byref(f1), ctypes.byref(c), 0)
    assert n1 >= n2 + 4 * 4 * 5 * 6 * 4
    assert lib.iris_rt_workspace_bytes(ctypes.byref(f2), ctypes.byref(c), 0) == n2
    assert lib.iris_rt_workspace_bytes(ctypes.byref(f1), ctypes.byref(c), 5) == 0  # bad K
    k16 = lib.iris_rt_workspace_bytes(ctypes.byref(f2), ctypes.byref(c), 16)
    assert k16 >= 1 * 4 * 5 * 16 * 4
    # Too-small workspace is refused before any launch.
    ln = rt.line_struct()
    out = rt.Outputs(0x5000, None, None, None, None)
    assert lib.iris_rt_forward(ctypes.byref(f1), ctypes.byref(c), ctypes.byref(ln),
                               ctypes.byref(out), 0, ctypes.c_void_p(0x9000), 16, None) == 3
    assert lib.iris_rt_forward(ctypes.byref(f2), ctypes.byref(c), ctypes.byref(ln),
                               ctypes.byref(out), 7, None, 0, None) == 1
    assert lib.iris_rt_forward(ctypes.byref(f2), ctypes.byref(c), ctypes.byref(ln),
                               ctypes.byref(out), 0, None, 0, None) == 3


def test_adjoint_requires_checkpoints_and_gradients():
    lib = rt.load_library()
    f = _fields()
    c = rt.ChannelsC(16, -8.0, 1.0)
    ln = rt.line_struct()
    cot = rt.Cotangents(0x5000, None, None, None, None)
    g = rt.Gradients(0x6000, 0x7000, 0x8000, 0x9000, None)
    assert lib.iris_rt_adjoint(ctypes.byref(f), ctypes.byref(c), ctypes.byref(ln), ctypes.byref(cot),
                               0, None, 0, ctypes.byref(g), None) == 1
    g0 = rt.Gradients(None, 0x7000, 0x8000, 0x9000, None)
    assert lib.iris_rt_adjoint(ctypes.byref(f), ctypes.byref(c), ctypes.byref(ln), ctypes.byref(cot),
                               16, None, 0, ctypes.byref(g0), None) == 1
    assert lib.iris_rt_adjoint(ctypes.byref(f), ctypes.byref(c), ctypes.byref(ln), ctypes.byref(cot),
                               16, None, 0, ctypes.byref(g), None) == 3


def test_adjoint_refuses_brightness_temperature_units():
    # The reverse mode is built for the linear output units; Planck
    # brightness temperatures are refused on the host, before any launch.
    lib = rt.load_library()
    f = _fields()
    c = rt.ChannelsC(16, -8.0, 1.0)
    cot = rt.Cotangents(0x5000, None, None, None, None)
    g = rt.Gradients(0x6000, 0x7000, 0x8000, 0x9000, None)
    ws, ws_bytes = ctypes.c_void_p(0x9000), 1 << 40
    ln = rt.line_struct(dict(units="tb"))
    assert lib.iris_rt_adjoint(ctypes.byref(f), ctypes.byref(c), ctypes.byref(ln), ctypes.byref(cot),
                               16, ws, ws_bytes, ctypes.byref(g), None) == 2
    assert b"units" in lib.iris_last_error()


def test_adjoint_autotune_rejects_bad_arguments_on_host():
    # Every refusal comes from the host checks, before any timing launch.
    lib = rt.load_library()
    f = _fields()
    c = rt.ChannelsC(16, -8.0, 1.0)
    ln = rt.line_struct()
    cot = rt.Cotangents(0x5000, None, None, None, None)
    g = rt.Gradients(0x6000, 0x7000, 0x8000, 0x9000, None)
    grp = ctypes.c_int32(0)
    args = (ctypes.byref(f), ctypes.byref(c), ctypes.byref(ln), ctypes.byref(cot))
    assert lib.iris_rt_autotune_adjoint(*args, 16, None, 0, ctypes.byref(g), None, None) == 1
    assert b"groups" in lib.iris_last_error()
    assert lib.iris_rt_autotune_adjoint(*args, 0, None, 0, ctypes.byref(g), None,
                                        ctypes.byref(grp)) == 1
    assert lib.iris_rt_autotune_adjoint(*args, 16, None, 0, ctypes.byref(g), None,
                                        ctypes.byref(grp)) == 3
    tb = rt.line_struct(dict(units="tb"))
    assert lib.iris_rt_autotune_adjoint(ctypes.byref(f), ctypes.byref(c), ctypes.byref(tb),
                                        ctypes.byref(cot), 16, ctypes.c_void_p(0x9000), 1 << 40,
                                        ctypes.byref(g), None, ctypes.byref(grp)) == 2
    assert grp.value == 0


def test_python_binding_refuses_cpu_tensors():
    import torch

    x = torch.zeros(2, 2, 2)
    with pytest.raises(ValueError, match="GPU"):
        rt.iris_rt_forward(x, x, x, x, axis=2, cell_cm=1.0, channels=rt.Channels(8, -4, 1))


def _cube(**kw):
    c = rt.Cube()
    c.fields = _fields(**kw)
    c.channels = rt.ChannelsC(16, -8.0, 1.0)
    c.out = rt.Outputs(0x5000, None, None, None, None)
    c.cot = rt.Cotangents(0x5000, None, None, None, None)
    c.grads = rt.Gradients(0x6000, 0x7000, 0x8000, 0x9000, None)
    return c


def test_plan_rejects_bad_arguments_on_host():
    lib = rt.load_library()
    ln = rt.line_struct()
    h = ctypes.c_void_p()
    arr = (rt.Cube * 2)(_cube(), _cube(axis=1))
    # No cubes, unknown flags, adjoint without checkpoints, bad line.
    assert lib.iris_plan_create(arr, 0, ctypes.byref(ln), 1, 0, None, ctypes.byref(h)) == 1
    assert lib.iris_plan_create(arr, 2, ctypes.byref(ln), 64, 0, None, ctypes.byref(h)) == 1
    assert lib.iris_plan_create(arr, 2, ctypes.byref(ln), 3, 0, None, ctypes.byref(h)) == 1
    # Choosing the checkpoint interval (ckpt_K = 0 with autotuning) still checks
    # the gradients and the cubes on the host before any timing launch.
    nog = (rt.Cube * 2)(_cube(), _cube(axis=1))
    nog[1].grads = rt.Gradients(0x6000, None, 0x8000, 0x9000, None)
    assert lib.iris_plan_create(nog, 2, ctypes.byref(ln), 7, 0, None, ctypes.byref(h)) == 1
    assert b"gradient" in lib.iris_last_error()
    badc = (rt.Cube * 2)(_cube(), _cube(nx=0))
    assert lib.iris_plan_create(badc, 2, ctypes.byref(ln), 7, 0, None, ctypes.byref(h)) == 1
    bad_line = rt.line_struct(dict(j_u=0))
    assert lib.iris_plan_create(arr, 2, ctypes.byref(bad_line), 1, 0, None, ctypes.byref(h)) == 1
    # A bad cube is named in the message; nothing is allocated or launched.
    arr2 = (rt.Cube * 2)(_cube(), _cube(axis=5))
    assert lib.iris_plan_create(arr2, 2, ctypes.byref(ln), 1, 0, None, ctypes.byref(h)) == 1
    assert b"cube 1" in lib.iris_last_error()
    assert not h.value
    # Adjoint plans need every gradient pointer, g_t_dust too with a dust
    # temperature field.
    c = _cube()
    c.grads = rt.Gradients(None, 0x7000, 0x8000, 0x9000, None)
    arr3 = (rt.Cube * 1)(c)
    assert lib.iris_plan_create(arr3, 1, ctypes.byref(ln), 3, 16, None, ctypes.byref(h)) == 1
    gen = _cube(t_dust=0xA000)
    arr4 = (rt.Cube * 1)(gen)
    assert lib.iris_plan_create(arr4, 1, ctypes.byref(ln), 3, 16, None, ctypes.byref(h)) == 1
    assert b"g_t_dust" in lib.iris_last_error()
    # Null handles.
    assert lib.iris_plan_forward(None, None) == 1
    assert lib.iris_plan_adjoint(None, None) == 1
    assert lib.iris_plan_groups(None, 0) == 0
    assert lib.iris_plan_adjoint_groups(None, 0) == 0
    lib.iris_plan_destroy(None)
    info = rt.PlanInfo()
    assert lib.iris_plan_get_info(None, ctypes.byref(info)) == 1


def test_autotune_rejects_bad_arguments_on_host():
    lib = rt.load_library()
    f = _fields()
    c = rt.ChannelsC(16, -8.0, 1.0)
    ln = rt.line_struct()
    out = rt.Outputs(0x5000, None, None, None, None)
    g = ctypes.c_int32(0)
    assert lib.iris_rt_autotune(ctypes.byref(f), ctypes.byref(c), ctypes.byref(ln),
                                ctypes.byref(out), None, 0, None, None) == 1
    bad = _fields(nx=0)
    assert lib.iris_rt_autotune(ctypes.byref(bad), ctypes.byref(c), ctypes.byref(ln),
                                ctypes.byref(out), None, 0, None, ctypes.byref(g)) == 1
    assert lib.iris_rt_autotune(ctypes.byref(f), ctypes.byref(c), ctypes.byref(ln),
                                ctypes.byref(out), None, 0, None, ctypes.byref(g)) == 3
    assert g.value == 0


@pytest.mark.parametrize("f,n_chan,status", [(-1, 16, 1), (65, 16, 1), (2, 1000, 2)])
def test_forward_rejects_bad_subsampling(f, n_chan, status):
    # simpson_f outside 0..64, or more marched velocities (2 f n_chan + 1)
    # than the library holds, are refused before any launch.
    lib = rt.load_library()
    fl = _fields()
    c = rt.ChannelsC(n_chan, -8.0, 1.0, simpson_f=f)
    ln = rt.line_struct()
    out = rt.Outputs(0x5000, None, None, None, None)
    assert lib.iris_rt_forward(ctypes.byref(fl), ctypes.byref(c), ctypes.byref(ln),
                               ctypes.byref(out), 0, None, 0, None) == status


def test_workspace_counts_marched_velocities():
    # Checkpoints hold the marched (fine) velocities of a subsampled grid.
    lib = rt.load_library()
    fl = _fields(axis=2)
    a = lib.iris_rt_workspace_bytes(ctypes.byref(fl), ctypes.byref(rt.ChannelsC(16, -8.0, 1.0)), 16)
    b = lib.iris_rt_workspace_bytes(ctypes.byref(fl),
                                    ctypes.byref(rt.ChannelsC(16, -8.0, 1.0, simpson_f=1)), 16)
    assert b > a


def test_smooth_integrator_limits_on_host():
    # The smooth integrator is forward only: checkpoints, the adjoint, plans
    # and autotuning are refused, as is a marched grid beyond its limit, all
    # before any launch (the workspace pointer is never touched).
    lib = rt.load_library()
    f = _fields()
    c = rt.ChannelsC(16, -8.0, 1.0)
    ln = rt.line_struct(dict(integrator="smooth"))
    out = rt.Outputs(0x5000, None, None, None, None)
    ws, ws_bytes = ctypes.c_void_p(0x9000), 1 << 40
    assert lib.iris_rt_forward(ctypes.byref(f), ctypes.byref(c), ctypes.byref(ln),
                               ctypes.byref(out), 16, ws, ws_bytes, None) == 2
    assert b"smooth" in lib.iris_last_error()
    wide = rt.ChannelsC(lib.iris_smooth_max_channels() + 1, -8.0, 0.01)
    assert lib.iris_rt_forward(ctypes.byref(f), ctypes.byref(wide), ctypes.byref(ln),
                               ctypes.byref(out), 0, ws, ws_bytes, None) == 2
    sub = rt.ChannelsC(1024, -8.0, 0.01, simpson_f=1)  # 2049 marched velocities
    assert lib.iris_rt_forward(ctypes.byref(f), ctypes.byref(sub), ctypes.byref(ln),
                               ctypes.byref(out), 0, ws, ws_bytes, None) == 2
    cot = rt.Cotangents(0x5000, None, None, None, None)
    g = rt.Gradients(0x6000, 0x7000, 0x8000, 0x9000, None)
    assert lib.iris_rt_adjoint(ctypes.byref(f), ctypes.byref(c), ctypes.byref(ln), ctypes.byref(cot),
                               16, ws, ws_bytes, ctypes.byref(g), None) == 2
    # Plans of this mode are forward only, without autotuning (refused before any allocation).
    h = ctypes.c_void_p()
    arr = (rt.Cube * 1)(_cube())
    assert lib.iris_plan_create(arr, 1, ctypes.byref(ln), 3, 16, None, ctypes.byref(h)) == 2
    assert lib.iris_plan_create(arr, 1, ctypes.byref(ln), 5, 0, None, ctypes.byref(h)) == 2
    assert not h.value
    gr = ctypes.c_int32(0)
    assert lib.iris_rt_autotune(ctypes.byref(f), ctypes.byref(c), ctypes.byref(ln),
                                ctypes.byref(out), ws, ws_bytes, None, ctypes.byref(gr)) == 2


def test_thin_transfer_limits_on_host():
    # Optically thin transfer: no subsampling (invalid), no checkpoints (its
    # adjoint takes ckpt_K = 0), no adjoint plans or autotuning, refused before
    # any launch.
    lib = rt.load_library()
    f = _fields()
    c = rt.ChannelsC(16, -8.0, 1.0)
    out = rt.Outputs(0x5000, None, None, None, None)
    ws, ws_bytes = ctypes.c_void_p(0x9000), 1 << 40
    for integ in ("formal", "smooth"):
        ln = rt.line_struct(dict(transfer="thin", integrator=integ))
        sub = rt.ChannelsC(16, -8.0, 1.0, simpson_f=1)
        assert lib.iris_rt_forward(ctypes.byref(f), ctypes.byref(sub), ctypes.byref(ln),
                                   ctypes.byref(out), 0, ws, ws_bytes, None) == 1
        assert b"simpson_f" in lib.iris_last_error()
        assert lib.iris_rt_forward(ctypes.byref(f), ctypes.byref(c), ctypes.byref(ln),
                                   ctypes.byref(out), 16, ws, ws_bytes, None) == 2
        wide = rt.ChannelsC(lib.iris_max_channels(), -8.0, 0.01)
        assert lib.iris_rt_forward(ctypes.byref(f), ctypes.byref(wide), ctypes.byref(ln),
                                   ctypes.byref(out), 0, ws, ws_bytes, None) == 2
        cot = rt.Cotangents(0x5000, None, None, None, None)
        g = rt.Gradients(0x6000, 0x7000, 0x8000, 0x9000, None)
        assert lib.iris_rt_adjoint(ctypes.byref(f), ctypes.byref(c), ctypes.byref(ln),
                                   ctypes.byref(cot), 16, ws, ws_bytes, ctypes.byref(g), None) == 1
        assert b"ckpt_K must be 0" in lib.iris_last_error()
        tb = rt.line_struct(dict(transfer="thin", integrator=integ, units="tb"))
        assert lib.iris_rt_adjoint(ctypes.byref(f), ctypes.byref(c), ctypes.byref(tb),
                                   ctypes.byref(cot), 0, ws, ws_bytes, ctypes.byref(g), None) == 2
        h = ctypes.c_void_p()
        arr = (rt.Cube * 1)(_cube())
        assert lib.iris_plan_create(arr, 1, ctypes.byref(ln), 3, 16, None, ctypes.byref(h)) == 2
        assert lib.iris_plan_create(arr, 1, ctypes.byref(ln), 5, 0, None, ctypes.byref(h)) == 2
        assert not h.value
        gr = ctypes.c_int32(0)
        assert lib.iris_rt_autotune(ctypes.byref(f), ctypes.byref(c), ctypes.byref(ln),
                                    ctypes.byref(out), ws, ws_bytes, None, ctypes.byref(gr)) == 2


def test_post_transfer_products_reject_bad_arguments_on_host():
    lib = rt.load_library()
    a, b, ws = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000), ctypes.c_void_p(0x3000)
    assert lib.iris_beam_workspace_bytes(4, 5, 6) == 4 * 5 * 6 * 4
    assert lib.iris_beam_workspace_bytes(0, 5, 6) == 0
    big = 1 << 30
    assert lib.iris_beam_convolve(None, b, 4, 5, 6, 2.0, ws, big, None) == 1
    assert lib.iris_beam_convolve(a, b, 0, 5, 6, 2.0, ws, big, None) == 1
    assert lib.iris_beam_convolve(a, b, 4, 5, 6, 0.0, ws, big, None) == 1
    assert lib.iris_beam_convolve(a, b, 4, 5, 6, float("nan"), ws, big, None) == 1
    assert lib.iris_beam_convolve(a, b, 4, 5, 6, 100.0, ws, big, None) == 2  # radius 170 > 128
    assert lib.iris_beam_convolve(a, b, 4, 5, 6, 2.0, ws, 16, None) == 3
    assert lib.iris_lv_mean(a, b, 4, 5, 6, 2, None) == 1
    assert lib.iris_lv_mean(a, None, 4, 5, 6, 0, None) == 1


def test_selective_transfer_limits_on_host():
    lib = rt.load_library()
    f = _fields()
    c = rt.ChannelsC(16, -8.0, 1.0)
    out = rt.Outputs(0x5000, None, None, None, None)
    ws, ws_bytes = ctypes.c_void_p(0x9000), 1 << 40
    # Smooth steps: the smooth integrator's channel limit, and no adjoint.
    smooth = rt.line_struct(dict(transfer="selective", integrator="smooth"))
    wide = rt.ChannelsC(lib.iris_smooth_max_channels() + 1, -8.0, 0.01)
    assert lib.iris_rt_forward(ctypes.byref(f), ctypes.byref(wide), ctypes.byref(smooth),
                               ctypes.byref(out), 0, ws, ws_bytes, None) == 2
    assert lib.iris_rt_forward(ctypes.byref(f), ctypes.byref(c), ctypes.byref(smooth),
                               ctypes.byref(out), 16, ws, ws_bytes, None) == 2
    ln = rt.line_struct(dict(transfer="selective"))
    sub = rt.ChannelsC(16, -8.0, 1.0, simpson_f=1)
    assert lib.iris_rt_forward(ctypes.byref(f), ctypes.byref(sub), ctypes.byref(ln),
                               ctypes.byref(out), 0, ws, ws_bytes, None) == 1
    assert lib.iris_rt_forward(ctypes.byref(f), ctypes.byref(c), ctypes.byref(ln),
                               ctypes.byref(out), 16, ws, ws_bytes, None) == 2


# --- molecular data and the levels grid (host side) ------------------------------

def test_molecule_reader_matches_the_oracle_reader(tmp_path):
    # The library's LAMDA reader (host only) and the oracle's, on the golden
    # toy file and a written synthetic rotor: same counts, codes, tables.
    from oracle import levels as Lv
    from paper_2607_01338_amd import workloads as W

    golden = os.path.join(ROOT, "tests", "golden", "toy3_lamda.dat")
    path = str(tmp_path / "rotor.dat")
    W.write_lamda(path, W.synthetic_rotor_molecule())
    for p in (golden, path):
        ref = Lv.read_lamda(p)
        info = rt.Molecule(p).info()
        assert info["n_levels"] == len(ref.g)
        assert info["n_transitions"] == len(ref.a)
        assert info["partners"] == [(q.code, len(q.up), len(q.temps)) for q in ref.partners]


@pytest.mark.parametrize("mutate,what", [
    (lambda ls: ls[:6] + ["70"] + ls[7:], "number of levels"),
    (lambda ls: [l.replace("    3     2  8.000e-06", "    3     3  8.000e-06") for l in ls],
     "radiative transition"),
    (lambda ls: [l.replace("  50.0 100.0", "  50.0 40.0") for l in ls], "temperatures"),
    (lambda ls: ls[:30], "truncated"),
])
def test_molecule_reader_rejects_malformed_files(tmp_path, mutate, what):
    golden = os.path.join(ROOT, "tests", "golden", "toy3_lamda.dat")
    lines = open(golden).read().splitlines()
    p = tmp_path / "bad.dat"
    p.write_text("\n".join(mutate(lines)) + "\n")
    with pytest.raises(rt.IrisError) as e:
        rt.Molecule(str(p))
    assert e.value.status == 1
    assert "line" in str(e.value) or "truncated" in str(e.value)
    with pytest.raises(rt.IrisError):
        rt.Molecule(str(tmp_path / "missing.dat"))


def test_levels_create_rejects_bad_configs_on_host():
    lib = rt.load_library()
    mol = rt.Molecule(os.path.join(ROOT, "tests", "golden", "toy3_lamda.dat"))
    good = dict(transition=1, t_bar_k=2.725, ortho_para=3.0, he_per_h=0.1, n_n=4, n_chi=2, n_t=3,
                ln_nh2_lo=0.0, ln_nh2_hi=10.0, chi_lo=0.5, chi_hi=1.0, t_lo_k=5.0, t_hi_k=100.0)
    for bad in (dict(transition=0), dict(transition=3), dict(n_n=0), dict(t_lo_k=0.0),
                dict(chi_hi=1.5), dict(ln_nh2_hi=-1.0), dict(ortho_para=0.0),
                dict(n_n=4096, n_t=4096, n_chi=2)):
        d = dict(good, **bad)
        cfg = rt.LevelsConfig(*(d[k] for k, _ in rt.LevelsConfig._fields_))
        h = ctypes.c_void_p()
        assert lib.iris_levels_create(mol.handle, ctypes.byref(cfg), None, ctypes.byref(h)) == 1, bad
        assert not h.value


def test_line_levels_must_be_an_open_grid():
    class Closed(rt.Levels):
        def __init__(self):
            self.handle = None
    with pytest.raises(ValueError):
        rt.line_struct(dict(levels=Closed()))
    with pytest.raises(ValueError):
        rt.line_struct(dict(levels="not a grid"))


def test_field_scan_needs_scratch_and_has_a_status_string():
    lib = rt.load_library()
    f = _fields()
    bad = ctypes.c_int64(0)
    assert lib.iris_rt_check_fields(ctypes.byref(f), None, 0, None, ctypes.byref(bad)) == 3
    assert lib.iris_rt_check_fields(ctypes.byref(f), ctypes.c_void_p(0x1000), 256, None,
                                    None) == 1
    assert lib.iris_status_string(5) == b"non-finite or out-of-range field values"
