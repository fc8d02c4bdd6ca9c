"""The optimization step replayed as one captured HIP graph (npg_step_graph)
against the eager step (npg_step) and the oracle (needs a GPU).

Every replay is checked: the two plans alternate, each step is followed by a
synchronising read of the state, and the graph's parameters, Adam moments,
loss and per-frame Chamfer distances must equal the eager step's bitwise."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import flat_params, gpu_plan, rel, to_np

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _pair(cfg, data, state):
    eager, graph = gpu_plan(cfg, data), gpu_plan(cfg, data)
    for p in (eager, graph):
        p.set_state(*state)
    return eager, graph


def _same_state(a, b):
    sa, sb = a.get_state(), b.get_state()
    assert sa[3] == sb[3]
    for x, y in zip(sa[:3], sb[:3]):
        assert np.array_equal(to_np(x), to_np(y))


@pytest.mark.parametrize("variant", ["plain", "iso_quat", "bf16", "cg", "cg_plain"])
def test_graph_step_is_bitwise_the_eager_step(variant):
    """DCT form (plain, with the isometry term and the quaternion head, BF16)
    and CG form (V-cycle preconditioned and plain). The graph plan's first
    recording of the CG form takes 16 iterations per solve; plain CG needs
    more on the finer levels, so its first replays find a solve unfinished,
    leave the state untouched and record again with more iterations: the
    step's result is the eager one all the same."""
    import torch
    cfg = dict(synth.config_c1(), precond="dct")
    if variant == "iso_quat":
        cfg.update(w_iso=100.0, rot_head="quat")
    if variant == "bf16":
        cfg.update(precision="bf16")
    if variant.startswith("cg"):
        cfg.update(precond="cg", cg_mg=0 if variant == "cg_plain" else 1)
    data = synth.make_workload(cfg)
    P = synth.random_state(cfg, 7, grid_std=0.05)
    zeros = O.zeros_like_params(P)
    state = (flat_params(cfg, P), flat_params(cfg, zeros), flat_params(cfg, zeros), 0)
    eager, graph = _pair(cfg, data, state)
    T, E = data["T"], cfg["n_steps"]
    le, lg = (torch.empty(1, dtype=torch.float64, device="cuda") for _ in range(2))
    ce, cg = (torch.empty(T, dtype=torch.float64, device="cuda") for _ in range(2))
    for e in range(6):
        if e == 3:  # a new launch shape drops the recorded graph; the next call records again
            for p in (eager, graph):
                p.tune_nn(64)
        assert eager.step(e, E, le, ce) == 0
        graph.step_graph(e, E, lg, cg)
        assert to_np(le).tobytes() == to_np(lg).tobytes(), e
        assert to_np(ce).tobytes() == to_np(cg).tobytes(), e
        _same_state(eager, graph)
    eager.close()
    graph.close()


def test_graph_step_matches_the_oracle():
    """Teacher-forced steps through the graph: the state is set from the
    oracle's before each replay (the recorded graph reads the plan's buffers,
    so new contents are picked up)."""
    import torch

    import paper_2602_22212_amd as npg
    cfg = dict(synth.config_c1(), precond="dct")
    data = synth.make_workload(cfg)
    plan = gpu_plan(cfg, data)
    P = O.to64(synth.init_params(cfg))
    m, v = O.zeros_like_params(P), O.zeros_like_params(P)
    E = cfg["n_steps"]
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    cd = torch.empty(cfg["T"], dtype=torch.float64, device="cuda")
    for e in range(3):
        plan.set_state(flat_params(cfg, P), flat_params(cfg, m), flat_params(cfg, v), e)
        plan.step_graph(e, E, loss, cd)
        Pn, mn, vn, d = O.step(P, m, v, e + 1, data, cfg, e, E, precond="dct")
        assert abs(loss.item() - d["ls"]["loss"]) <= TOL * d["ls"]["loss"]
        assert rel(to_np(cd), d["ls"]["cd"]) < TOL
        got = npg.unpack_params(cfg, to_np(plan.get_state()[0]))
        for (W, b), (Wr, br) in zip(got["mlp"], Pn["mlp"]):
            assert rel(W, Wr) < TOL and rel(b, br) < TOL
        P, m, v = Pn, mn, vn
    plan.close()


def test_graph_step_cg_cap_is_reported():
    """A solve that reaches cg_maxit: the graph step completes like the eager
    one (the capped solve's result stands), reports NPG_ENOTCONV and leaves
    the same state, bitwise."""
    import paper_2602_22212_amd as npg
    cfg = synth.config_small(mlp_width=32, cg_maxit=3, cg_rtol=1e-12, levels=[6, 9], precond="cg")
    data = synth.make_workload(cfg)
    P = synth.random_state(cfg, 2)
    zeros = O.zeros_like_params(P)
    state = (flat_params(cfg, P), flat_params(cfg, zeros), flat_params(cfg, zeros), 0)
    eager, graph = _pair(cfg, data, state)
    for e in range(3):
        assert eager.step(e, 3) == npg.NPG_ENOTCONV
        assert graph.step_graph(e, 3) == npg.NPG_ENOTCONV
        _same_state(eager, graph)
    eager.close()
    graph.close()
