"""npg_metrics_noalloc (workspace in the library's fixed scratch array)
against npg_metrics (temporary allocations), through the C ABI (needs a GPU).

Two calls in a row on one GPU, the second with a smaller input: the human
workload (30 000 vertices, 100 frames: the frames are processed in several
chunks of the array) and then the icosphere workload (2562 vertices, 10
frames); each must equal npg_metrics bitwise. A plan whose single frame needs
more than the array is rejected on the host before any launch."""
import numpy as np
import pytest

import synth
from gpu_util import flat_params, gpu_plan, to_np

pytestmark = pytest.mark.gpu


def _inputs(cfg, data, seed):
    import torch
    plan = gpu_plan(cfg, data)
    T, V = data["T"], len(data["xyz"])
    plan.set_state(flat_params(cfg, synth.random_state(cfg, seed, grid_std=0.05)), adam_steps=0)
    xh = torch.empty(T * V * 4, device="cuda")
    nh = torch.empty(T * V * 4, device="cuda")
    plan.predict(xh, nh)
    gt = np.concatenate([data["truth"], np.zeros((T, V, 1))], -1).astype(np.float32)
    gn = np.concatenate([data["truth_nrm"], np.zeros((T, V, 1))], -1).astype(np.float32)
    tau = 0.005 * float(np.linalg.norm(data["xyz"].max(0) - data["xyz"].min(0)))
    return plan, xh, nh, torch.from_numpy(gt.ravel()).cuda(), torch.from_numpy(gn.ravel()).cuda(), tau


def test_metrics_noalloc_equals_metrics_two_calls():
    import torch
    runs = []
    c2 = synth.config_c2()
    runs.append((c2, synth.make_workload(c2, truth=True), 9))
    c1 = synth.config_c1()
    runs.append((c1, synth.make_workload(c1), 6))
    for cfg, data, seed in runs:
        plan, xh, nh, gt, gn, tau = _inputs(cfg, data, seed)
        T = data["T"]
        print(f"{cfg['name']}: V={len(data['xyz'])} T={T}", flush=True)
        ref = torch.full((T * 4,), -1.0, dtype=torch.float64, device="cuda")
        got = torch.full((T * 4,), -2.0, dtype=torch.float64, device="cuda")
        plan.metrics(xh, nh, gt, gn, tau, ref)
        plan.metrics_noalloc(xh, nh, gt, gn, tau, got)
        torch.cuda.synchronize()
        r, g = to_np(ref), to_np(got)
        assert np.all(np.isfinite(r)) and np.all(r[0::4] > 0)
        assert r.tobytes() == g.tobytes(), np.abs(r - g).max()
        plan.close()


def test_metrics_noalloc_rejects_a_frame_beyond_the_array():
    """100 000 vertices with 64-thread nearest-neighbour work-groups: one
    frame's workspace is about 80 MB, more than the 64 MiB array."""
    import torch

    import paper_2602_22212_amd as npg
    rng = np.random.default_rng(0)
    V, N = 100_000, 64
    X = rng.uniform(-0.5, 0.5, size=(V, 3)).astype(np.float32)
    Nr = X / np.linalg.norm(X, axis=1, keepdims=True)
    pts = rng.uniform(-0.5, 0.5, size=(N, 3)).astype(np.float32)
    cfg = synth.config_small(mlp_width=32, t_key=None)
    data = dict(xyz=X, nrm=Nr.astype(np.float32), pts=pts, frame_off=np.array([0, N], np.int64), T=1)
    plan = gpu_plan(cfg, data)
    plan.tune_nn(64)
    f = dict(device="cuda")
    xh = torch.zeros(V * 4, **f)
    out = torch.zeros(4, dtype=torch.float64, **f)
    with pytest.raises(npg.NpgError) as e:
        plan.metrics_noalloc(xh, xh, xh, xh, 0.01, out)
    assert e.value.status == npg.NPG_EINVAL and "scratch" in str(e.value)
    plan.close()
