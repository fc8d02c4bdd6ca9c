"""Batched sequences (npg_plan_create_batched / npg_batch_step; survey
config 5) on the GPU: concurrency changes nothing, each sequence is the plain
step of its own plan, and errors name their sequence."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import flat_params, rel, to_np

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _small_batch():
    # C5-shaped sequences at a small scale, with smaller grids so the oracle
    # can follow; mixed kinds, ragged frames, both precisions, both rotation
    # heads and one sequence with the isometry term
    cfgs = synth.config_c5(n_seq=5, seed=7, scale=0.03)
    for k, c in enumerate(cfgs):
        c.update(levels=[8, 16, 24], lr_grid=[0.005 * 2.5 ** l for l in range(3)],
                 lam=[0.4 * 1.5 ** l for l in range(3)], mlp_width=64, mlp_hidden=2)
    cfgs[0]["precision"] = "fp32"
    cfgs[1]["rot_head"] = "quat"
    cfgs[2]["w_iso"] = 100.0
    cfgs[3]["precond"] = "dct"
    return cfgs, [synth.make_workload(c) for c in cfgs]


def test_batch_step_equals_individual_plans():
    import torch

    import paper_2602_22212_amd as npg
    cfgs, datas = _small_batch()
    states = [flat_params(c, synth.random_state(c, 40 + k, grid_std=0.05)) for k, c in enumerate(cfgs)]
    batch = npg.Batch(cfgs, datas)
    for p, s in zip(batch.plans, states):
        p.set_state(s, adam_steps=0)
    losses = [torch.empty(1, dtype=torch.float64, device="cuda") for _ in cfgs]
    for e in range(3):
        batch.step(e, 10, losses)
    got = [p.get_state()[0] for p in batch.plans]
    for k, (c, d, s) in enumerate(zip(cfgs, datas, states)):
        plan = npg.plan_from_workload(c, d)
        plan.set_state(s, adam_steps=0)
        l1 = torch.empty(1, dtype=torch.float64, device="cuda")
        for e in range(3):
            plan.step(e, 10, l1)
        assert torch.equal(plan.get_state()[0], got[k]), k
        assert l1.item() == losses[k].item(), k
        plan.close()
    print("sequences:", [(len(d["xyz"]), d["T"], int(d["frame_off"][-1])) for d in datas])
    batch.close()


@pytest.mark.parametrize("per_stream", [False, True])
def test_batch_graph_step_equals_eager_batch_step(per_stream):
    """npg_batch_step_graph (one HIP graph, the sequences' recorded steps as
    branches) against npg_batch_step, bitwise, step after step; a new launch
    shape of one sequence (autotuner) makes the next call rebuild the batch
    graph."""
    import torch

    import paper_2602_22212_amd as npg
    cfgs, datas = _small_batch()
    states = [flat_params(c, synth.random_state(c, 60 + k, grid_std=0.05)) for k, c in enumerate(cfgs)]
    eager, graph = npg.Batch(cfgs, datas), npg.Batch(cfgs, datas)
    graph.graph_mode(per_stream)
    for b in (eager, graph):
        for p, s in zip(b.plans, states):
            p.set_state(s, adam_steps=0)
    le = [torch.empty(1, dtype=torch.float64, device="cuda") for _ in cfgs]
    lg = [torch.empty(1, dtype=torch.float64, device="cuda") for _ in cfgs]
    for e in range(5):
        if e == 3:
            for b in (eager, graph):
                b.plans[1].tune_nn(64)
        assert eager.step(e, 10, le) == npg.NPG_OK
        assert graph.step_graph(e, 10, lg) == npg.NPG_OK
        for k in range(len(cfgs)):
            assert to_np(le[k]).tobytes() == to_np(lg[k]).tobytes(), (e, k)
            sa, sb = eager.plans[k].get_state(), graph.plans[k].get_state()
            assert sa[3] == sb[3] == e + 1
            for x, y in zip(sa[:3], sb[:3]):
                assert torch.equal(x, y), (e, k)
    eager.close()
    graph.close()


def test_batch_sequence_matches_the_oracle_step():
    import torch

    import paper_2602_22212_amd as npg
    cfgs, datas = _small_batch()
    batch = npg.Batch(cfgs, datas)
    k = 0  # the FP32 sequence with the CG preconditioner
    c, d = cfgs[k], datas[k]
    P = O.to64(synth.random_state(c, 3, grid_std=0.05))
    for j, p in enumerate(batch.plans):
        p.set_state(flat_params(cfgs[j], synth.random_state(cfgs[j], 3, grid_std=0.05)), adam_steps=0)
    losses = [torch.empty(1, dtype=torch.float64, device="cuda") for _ in cfgs]
    batch.step(0, 10, losses)
    Pn, _, _, diag = O.step(P, O.zeros_like_params(P), O.zeros_like_params(P), 1, d, c, 0, 10)
    assert abs(losses[k].item() - diag["ls"]["loss"]) <= TOL * diag["ls"]["loss"]
    got = npg.unpack_params(c, to_np(batch.plans[k].get_state()[0]))
    for (W, b), (Wr, br) in zip(got["mlp"], Pn["mlp"]):
        assert rel(W, Wr) < TOL and rel(b, br) < TOL
    batch.close()


def test_batch_reports_the_failing_sequence():
    import paper_2602_22212_amd as npg
    cfgs, datas = _small_batch()
    bad = dict(datas[2])
    bad["frame_off"] = np.concatenate([[0, 0], bad["frame_off"][1:]])  # an empty first frame
    datas[2] = bad
    with pytest.raises(npg.NpgError) as e:
        npg.Batch(cfgs, datas)
    assert e.value.status == npg.NPG_EINVAL and "sequence 2" in str(e.value)
