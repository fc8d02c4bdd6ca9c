"""Boundary checks that need no GPU: the library loads, exports every symbol
declared in include/neupig.h, the ctypes config matches the C struct layout,
and host-side validation rejects bad arguments before touching the device."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import paper_2602_22212_amd as npg
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "neupig.h")


def _lib():
    if not os.path.exists(npg.LIB_PATH):
        from paper_2602_22212_amd import build
        build.build()
    return npg.lib()


def test_library_exports_every_declared_symbol():
    L = _lib()
    src = open(HEADER).read()
    names = set(re.findall(r"\b(npg_[a-z_]+)\s*\(", src))
    assert len(names) >= 18
    for n in sorted(names):
        assert hasattr(L, n), f"missing export {n}"
    out = subprocess.run(["nm", "-D", "--defined-only", npg.LIB_PATH], capture_output=True, text=True).stdout
    for n in names:
        assert re.search(rf"\bT {n}$", out, re.M), n


def test_config_struct_layout_matches_c(tmp_path):
    prog = tmp_path / "layout.c"
    prog.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "neupig.h"\n'
                    "int main(){printf(\"%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n\", sizeof(npg_config),"
                    " offsetof(npg_config, lam), offsetof(npg_config, cg_rtol),"
                    " offsetof(npg_config, cg_maxit), offsetof(npg_config, precond),"
                    " offsetof(npg_config, rot_head), offsetof(npg_config, precision),"
                    " offsetof(npg_config, cg_mg), offsetof(npg_config, nn_search),"
                    " offsetof(npg_config, cg_one_stream));return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    vals = list(map(int, subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()))
    C = npg.npg_config
    assert vals == [ctypes.sizeof(C), C.lam.offset, C.cg_rtol.offset, C.cg_maxit.offset, C.precond.offset,
                    C.rot_head.offset, C.precision.offset, C.cg_mg.offset, C.nn_search.offset,
                    C.cg_one_stream.offset]


@pytest.mark.parametrize("name,head", [("c1", "expmap"), ("c2", "expmap"), ("c3", "expmap"), ("small", "expmap"),
                                       ("c1", "quat"), ("small", "quat")])
def test_param_count_matches_layout(name, head):
    _lib()
    cfg = dict(synth.config_by_name(name), rot_head=head)
    if cfg["mlp_width"] not in (32, 64, 128):
        cfg = dict(cfg, mlp_width=32)
    lay, total = npg.param_layout(cfg)
    assert npg.param_count(cfg) == total
    p = synth.init_params(cfg) if cfg["mlp_width"] == synth.config_by_name(name)["mlp_width"] else None
    if p is not None:
        flat = npg.pack_params(cfg, p)
        assert flat.size == total
        back = npg.unpack_params(cfg, flat)
        for a, b in zip(back["grid_p"], p["grid_p"]):
            np.testing.assert_array_equal(a, b)
        for (W1, b1), (W2, b2) in zip(back["mlp"], p["mlp"]):
            np.testing.assert_array_equal(W1, W2)
            np.testing.assert_array_equal(b1, b2)


@pytest.mark.parametrize("bad,msg", [
    (dict(levels=[]), "n_levels"),
    (dict(levels=[1, 4]), "nodes per axis"),
    (dict(feat_p=5), "feat_p"),
    (dict(mlp_width=48), "mlp_width"),
    (dict(mlp_hidden=0), "mlp_hidden"),
    (dict(time_freqs=9), "time_freqs"),
    (dict(eps=0.0), "eps"),
    (dict(cg_maxit=0), "cg_maxit"),
    (dict(w_iso=-1.0), "w_iso"),
    (dict(act="leaky", leaky_slope=1.5), "leaky_slope"),
    (dict(act="leaky", leaky_slope=0.0), "leaky_slope"),
    (dict(cg_mg=2), "cg_mg"),
])
def test_invalid_configs_are_rejected(bad, msg):
    _lib()
    cfg = synth.config_c1()
    cfg.update(bad)
    L = len(cfg["levels"])
    cfg["lr_grid"] = cfg["lr_grid"][:L] + [0.01] * max(0, L - len(cfg["lr_grid"]))
    cfg["lam"] = cfg["lam"][:L] + [0.4] * max(0, L - len(cfg["lam"]))
    with pytest.raises(npg.NpgError) as e:
        npg.param_count(cfg)
    assert e.value.status == npg.NPG_EINVAL and msg in str(e.value)


def test_invalid_nn_search_is_rejected():
    L = _lib()
    c = npg.make_config(synth.config_c1())
    c.nn_search = 7
    n = ctypes.c_int64()
    assert L.npg_param_count(ctypes.byref(c), ctypes.byref(n)) == npg.NPG_EINVAL
    assert "nn_search" in L.npg_last_error().decode()
    with pytest.raises(ValueError):
        npg.make_config(dict(synth.config_c1(), nn_search="kdtree"))


def test_invalid_cg_one_stream_is_rejected():
    L = _lib()
    c = npg.make_config(synth.config_c1())
    c.cg_one_stream = 2
    n = ctypes.c_int64()
    assert L.npg_param_count(ctypes.byref(c), ctypes.byref(n)) == npg.NPG_EINVAL
    assert "cg_one_stream" in L.npg_last_error().decode()


def _create_raw(cfg, V, T, off, xyz=1, nrm=1, pts=1):
    L = _lib()
    c = npg.make_config(cfg)
    h = ctypes.c_void_p()
    offa = np.asarray(off, np.int64)
    st = L.npg_plan_create(ctypes.byref(c), V, ctypes.c_void_p(xyz), ctypes.c_void_p(nrm), T,
                           ctypes.c_void_p(pts), offa.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                           None, ctypes.byref(h))
    return st, L.npg_last_error().decode(), h


def test_plan_create_validates_before_any_device_work():
    # These fail in host validation, before any HIP call, so they run here.
    cfg = synth.config_c1()
    assert _create_raw(cfg, 0, 1, [0, 5])[0] == npg.NPG_EINVAL
    st, msg, _ = _create_raw(cfg, 10, 2, [0, 5, 5])
    assert st == npg.NPG_EINVAL and "at least one point" in msg
    st, msg, _ = _create_raw(cfg, 10, 2, [1, 5, 9])
    assert st == npg.NPG_EINVAL and "frame_off[0]" in msg
    st, msg, _ = _create_raw(cfg, 10, 1, [0, 5], xyz=0)
    assert st == npg.NPG_EINVAL and "non-NULL" in msg
    st, msg, _ = _create_raw(dict(cfg, t_key=3), 10, 2, [0, 5, 9])
    assert st == npg.NPG_EINVAL and "t_key" in msg


def test_binding_refuses_host_tensors():
    import torch
    _lib()
    cfg = synth.config_small(mlp_width=32)
    with pytest.raises(ValueError):
        npg.Plan(cfg, torch.zeros(4, 3), torch.zeros(4, 3), torch.zeros(5, 3), [0, 5])
