"""Autotuner of the nearest-neighbour pass (npg_tune_nn; needs a GPU): every
work-group size gives bitwise the same indices, distances and frame sums;
the timed choice is one of the candidates; bad values are rejected."""
import numpy as np
import pytest

import synth
from gpu_util import flat_params, gpu_plan, to_np

pytestmark = pytest.mark.gpu


def _chamfer(plan, xh):
    import torch
    T, V = plan.T, plan.V
    out = (torch.empty(T * V, dtype=torch.int32, device="cuda"), torch.empty(T * V, device="cuda"),
           torch.empty(plan.Ntot, dtype=torch.int32, device="cuda"), torch.empty(plan.Ntot, device="cuda"),
           torch.empty(T, dtype=torch.float64, device="cuda"))
    plan.chamfer_fwd(xh, *out)
    torch.cuda.synchronize()
    return [to_np(x) for x in out]


@pytest.mark.parametrize("V,N", [(2100, [300, 2049, 1, 700, 1500]), (5, [7, 3, 1, 2, 9]), (5000, [4000] * 5)])
def test_every_workgroup_size_gives_the_same_result(V, N):
    import torch

    import paper_2602_22212_amd as npg
    cfg = synth.config_small(name="tune", levels=[16, 24], feat_p=4, time_freqs=4, mlp_hidden=2, mlp_width=64,
                             act="leaky", V=V, T=5, N=N, t_key=2, seed=31)
    data = synth.make_workload(cfg)
    plan = gpu_plan(cfg, data)
    flat = flat_params(cfg, synth.random_state(cfg, 7))
    plan.set_state(flat)
    z = torch.empty(V * plan.Fz, device="cuda")
    xh = torch.empty(5 * V * 4, device="cuda")
    plan.encode_fwd(flat, z)
    plan.decode_fwd(flat, z, xh)
    ref = None
    for kt in (128, 64, 256):
        assert plan.tune_nn(kt)[0] == kt
        got = _chamfer(plan, xh)
        if ref is None:
            ref = got
        else:
            for g, r in zip(got, ref):
                np.testing.assert_array_equal(g, r)
    chosen, ms = plan.tune_nn(0)
    assert chosen in (64, 128, 256) and all(m > 0 for m in ms), (chosen, ms)
    assert ms[(64, 128, 256).index(chosen)] == min(ms)
    for g, r in zip(_chamfer(plan, xh), ref):
        np.testing.assert_array_equal(g, r)
    with pytest.raises(npg.NpgError):
        plan.tune_nn(96)
    plan.close()
