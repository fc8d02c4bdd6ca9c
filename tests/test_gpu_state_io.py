"""Parameter import/export by block and the checkpoint pair (needs a GPU):
bitwise round trips against the flat layout, moments untouched by a
parameter import, bad arguments rejected."""
import numpy as np
import pytest

import synth
from gpu_util import gpu_plan, to_np

pytestmark = pytest.mark.gpu


def _blocks(cfg, p):
    out = list(p["grid_p"]) + [p["grid_n"]]
    for W, b in p["mlp"]:
        out += [W, b]
    return [np.ascontiguousarray(x, np.float32) for x in out]


@pytest.mark.parametrize("head", ["expmap", "quat"])
def test_block_import_export_round_trip(head):
    import torch

    import paper_2602_22212_amd as npg
    cfg = synth.config_small(name="io", levels=[8, 12, 16], feat_p=3, time_freqs=2, mlp_hidden=2, mlp_width=32,
                             act="leaky", V=300, T=3, N=[40, 50, 60], t_key=1, seed=41, rot_head=head)
    data = synth.make_workload(cfg)
    plan = gpu_plan(cfg, data)
    p = synth.random_state(cfg, 3)
    blocks = _blocks(cfg, p)
    n = plan.n_params
    m0 = torch.full((n,), 0.25, device="cuda")
    v0 = torch.full((n,), 0.5, device="cuda")
    plan.set_state(torch.zeros(n, device="cuda"), m0, v0, 7)
    plan.params_import([torch.from_numpy(b).cuda() for b in blocks])
    flat, m, v, k = plan.get_state()
    np.testing.assert_array_equal(to_np(flat), npg.pack_params(cfg, p))
    assert torch.equal(m, m0) and torch.equal(v, v0) and k == 7   # moments and count untouched
    for got, ref in zip(plan.params_export(), blocks):
        np.testing.assert_array_equal(to_np(got), ref)
    # checkpoint pair
    lib = npg.lib()
    import ctypes
    f2, m2, v2 = torch.randn(n, device="cuda"), torch.randn(n, device="cuda"), torch.rand(n, device="cuda")
    npg._check(lib.npg_state_import(plan._h, ctypes.c_void_p(f2.data_ptr()), ctypes.c_void_p(m2.data_ptr()),
                                    ctypes.c_void_p(v2.data_ptr()), 11))
    f3, m3, v3 = torch.empty_like(f2), torch.empty_like(f2), torch.empty_like(f2)
    k3 = ctypes.c_int64()
    npg._check(lib.npg_state_export(plan._h, ctypes.c_void_p(f3.data_ptr()), ctypes.c_void_p(m3.data_ptr()),
                                    ctypes.c_void_p(v3.data_ptr()), ctypes.byref(k3)))
    assert torch.equal(f3, f2) and torch.equal(m3, m2) and torch.equal(v3, v2) and k3.value == 11
    # a NULL block is rejected and leaves the parameters as they were
    arr = (ctypes.c_void_p * len(blocks))(*[ctypes.c_void_p(0)] * len(blocks))
    assert lib.npg_params_import(plan._h, arr) == npg.NPG_EINVAL
    assert torch.equal(plan.get_state()[0], f2)
    plan.close()
