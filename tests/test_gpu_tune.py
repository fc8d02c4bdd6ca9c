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


@pytest.mark.parametrize("zs", [32, 128])
def test_cg_tiles_give_the_exact_operator(zs):
    """Every z-tile depth of the CG kernels (grids of >= 100 nodes per axis,
    with partial tiles at 129 and 116) solves to the exact operator of the
    oracle within 1e-5, for both solves' residual bound; the timed choice is
    one of the candidates and a step runs after it."""
    import torch

    import oracle as O
    import paper_2602_22212_amd as npg
    from gpu_util import rel
    cfg = synth.config_small(levels=[16, 116, 129], feat_p=4, mlp_width=32, V=3000, T=1, N=10, t_key=0, seed=33,
                             precond="cg")
    data = synth.make_workload(cfg)
    plan = gpu_plan(cfg, data)
    assert plan.tune_cg(zs)[0] == zs
    rng = np.random.default_rng(12)
    gz = torch.from_numpy(rng.normal(size=(plan.V * plan.Fz)).astype(np.float32)).cuda()
    grad = torch.zeros(plan.n_params, dtype=torch.float32, device="cuda")
    plan.encode_bwd(gz, grad)
    g_in = npg.unpack_params(cfg, to_np(grad))
    its, st = plan.precond(grad)
    assert st == npg.NPG_OK, its
    got = npg.unpack_params(cfg, to_np(grad))
    errs = [rel(g, O.precond_dct(gi.astype(np.float64), R, lam))
            for g, gi, R, lam in zip(got["grid_p"], g_in["grid_p"], cfg["levels"], cfg["lam"])]
    print("zs", zs, "precond rel errors:", ["%.2e" % e for e in errs], "iterations:", its)
    assert max(errs) < 1e-5
    chosen, ms = plan.tune_cg(0)
    assert chosen in (32, 64, 128) and all(m > 0 for m in ms) and ms[(32, 64, 128).index(chosen)] == min(ms)
    plan.set_state(flat_params(cfg, synth.random_state(cfg, 2)), adam_steps=0)
    assert plan.step(0, 3) == npg.NPG_OK
    with pytest.raises(npg.NpgError):
        plan.tune_cg(48)
    plan.close()


def test_mlp_chunks_keep_the_step_on_the_oracle():
    """Teacher-forced icosphere steps with the decode backward split into the
    most frame chunks (one frame each) and with the timed choice: loss, cd and
    every MLP block after the update within 1e-5 of the oracle; a repeated
    step with the same chunking is bitwise the same."""
    import torch

    import oracle as O
    import paper_2602_22212_amd as npg
    from gpu_util import rel
    cfg = dict(synth.config_c1(), precond="dct")
    data = synth.make_workload(cfg)
    plan = gpu_plan(cfg, data)
    P = O.to64(synth.random_state(cfg, 8, grid_std=0.05))
    zero = O.zeros_like_params(P)
    Pn, _, _, d = O.step(P, zero, O.zeros_like_params(P), 1, data, cfg, 0, cfg["n_steps"], precond="dct")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    results = []
    for nch in (cfg["T"], 0, 0):
        chosen, cand, ms = plan.tune_mlp(nch)
        if nch == 0:
            assert chosen in cand and min(m for c, m in zip(cand, ms) if c) == ms[cand.index(chosen)]
        plan.set_state(flat_params(cfg, P), adam_steps=0)
        assert plan.step(0, cfg["n_steps"], loss) == npg.NPG_OK
        assert abs(loss.item() - d["ls"]["loss"]) <= 1e-5 * d["ls"]["loss"]
        got = npg.unpack_params(cfg, to_np(plan.get_state()[0]))
        for (W, b), (Wr, br) in zip(got["mlp"], Pn["mlp"]):
            assert rel(W, Wr) < 1e-5 and rel(b, br) < 1e-5, (nch, chosen)
        results.append((chosen, plan.get_state()[0]))
    for c, r in results[1:]:
        if c == results[0][0]:
            assert torch.equal(r, results[0][1])
    assert results[1][0] != results[2][0] or torch.equal(results[1][1], results[2][1])
    with pytest.raises(npg.NpgError):
        plan.tune_mlp(cfg["T"] + 1)
    plan.close()
