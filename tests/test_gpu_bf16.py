"""BF16 form of the decoder MLP (bfloat16 matrix operands, float32
accumulation) against the oracle's emulation of the same rounding points,
and its trained quality against the FP32 form (needs a GPU).

Tolerances follow from bfloat16's 8-bit significand (relative spacing
2^-8): an activation whose float32 value (GPU) and float64 value (oracle)
round to neighbouring bfloat16 numbers differs by one spacing. About 1e-6 /
2^-8 ~ 3e-4 of the rounded values do, which moves the deformed vertices by
~1e-5 (norm-wise; bound 1e-4) and sums over many samples with cancelling
signs by ~1e-3 (bound 3e-3). A structural mistake (a transposed operand, a
dropped term) moves them by O(1)."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import flat_params, gpu_plan, rel, to_np

pytestmark = pytest.mark.gpu
TOL_X = 1e-4
TOL_G = 3e-3


def _mid_bf16(**kw):
    base = dict(name="mid", levels=[16, 24, 35], feat_p=4, time_freqs=4, mlp_hidden=3, mlp_width=128, act="leaky",
                V=2100, T=5, N=[300, 2049, 1, 700, 1500], t_key=2, seed=21, precision="bf16")
    base.update(kw)
    return synth.config_small(**base)


@pytest.mark.parametrize("width,hidden,head,shape", [(128, 3, "expmap", None), (64, 2, "quat", None),
                                                      (32, 1, "expmap", None), (128, 3, "expmap", "tiny")])
def test_bf16_stages(width, hidden, head, shape):
    import torch

    import paper_2602_22212_amd as npg
    cfg = _mid_bf16(mlp_width=width, mlp_hidden=hidden, rot_head=head)
    if shape == "tiny":
        # one frame (a single, half-empty frame pair) and 17 vertices (a second,
        # one-vertex block) for the forward's frame-pair items
        cfg = _mid_bf16(mlp_width=width, mlp_hidden=hidden, rot_head=head, V=17, T=1, N=[40], t_key=0)
    data = synth.make_workload(cfg)
    plan = gpu_plan(cfg, data)
    T, V = data["T"], len(data["xyz"])
    P = O.to64(synth.random_state(cfg, 100))
    flat = flat_params(cfg, P)
    z = torch.empty(V * plan.Fz, device="cuda")
    xh = torch.empty(T * V * 4, device="cuda")
    plan.encode_fwd(flat, z)
    plan.decode_fwd(flat, z, xh)
    fw = O.forward(P, data, cfg)
    assert rel(to_np(z).reshape(V, -1), fw["z"]) < 1e-5
    x = to_np(xh).reshape(T, V, 4)[..., :3]
    ex = [rel(x[t], fw["xhat"][t]) for t in range(T)]
    # the float32 form is genuinely different (the rounding is exercised)
    ff = O.forward(P, data, dict(cfg, precision="fp32"))
    d32 = [rel(fw["xhat"][t], ff["xhat"][t]) for t in range(T)]
    print("bf16 decode error per frame:", ["%.1e" % e for e in ex], "bf16 vs fp32 oracle:", ["%.1e" % e for e in d32])
    assert max(ex) < TOL_X
    if shape is None:  # at 17 samples the two forms differ by only ~10x the error; the larger cases check it
        assert min(d32) > 10 * max(ex)
    # decode backward with a fixed upstream gradient
    rng = np.random.default_rng(7)
    gx = rng.normal(size=(T, V, 3)).astype(np.float32)
    gx4 = np.concatenate([gx, np.zeros((T, V, 1), np.float32)], -1)
    grad = torch.zeros(plan.n_params, device="cuda")
    gz = torch.empty(V * plan.Fz, device="cuda")
    plan.decode_bwd(flat, z, torch.from_numpy(gx4.ravel()).cuda(), grad, gz)
    go = O.transform_backward(gx.reshape(-1, 3).astype(np.float64), fw["o"], fw["Xt"], fw["R"], fw["dh"],
                              cfg["alpha_t"], head)
    gmlp, gY = O.mlp_backward(P["mlp"], go, fw["pres"], fw["ins"], cfg["act"], cfg["leaky_slope"], bf16=True)
    got = npg.unpack_params(cfg, to_np(grad))
    errs = [(rel(gW, rW), rel(gb, rb)) for (gW, gb), (rW, rb) in zip(got["mlp"], gmlp)]
    Fz = cfg["feat_n"] + cfg["feat_p"]
    egz = rel(to_np(gz).reshape(V, -1), gY[:, :Fz].reshape(T, V, Fz).sum(0))
    print("bf16 decode backward errors:", errs, egz)
    assert max(max(e) for e in errs) < TOL_G and egz < TOL_G
    plan.close()


def test_bf16_training_reaches_the_fp32_quality():
    """Icosphere, 60 steps from the paper's identity start with the exact DCT
    preconditioner in both forms; the final Chamfer distance of each form's
    deformed vertices, evaluated by the oracle's float64 Chamfer, agrees
    within 5%, and falls by more than 10% from the start."""
    import torch
    res = {}
    for prec in ("fp32", "bf16"):
        cfg = dict(synth.config_c1(), precond="dct", precision=prec)
        data = synth.make_workload(cfg)
        plan = gpu_plan(cfg, data)
        plan.set_state(flat_params(cfg, synth.init_params(cfg)), adam_steps=0)
        for e in range(60):
            plan.step(e, 60)
        T, V = data["T"], len(data["xyz"])
        xh = torch.empty(T * V * 4, device="cuda")
        plan.predict(xh)
        x = to_np(xh).reshape(T, V, 4)[..., :3].astype(np.float64)
        off = data["frame_off"]
        cds = [O.chamfer(x[t], data["pts"][off[t]:off[t + 1]].astype(np.float64))[4] for t in range(T)]
        cd0 = [O.chamfer(data["xyz"].astype(np.float64), data["pts"][off[t]:off[t + 1]].astype(np.float64))[4]
               for t in range(T)]
        res[prec] = (np.mean(cds), np.mean(cd0))
        plan.close()
    print("mean CD after 60 steps (fp32, bf16) and at the start:", res["fp32"][0], res["bf16"][0], res["fp32"][1])
    assert res["fp32"][0] < 0.9 * res["fp32"][1]
    assert abs(res["bf16"][0] - res["fp32"][0]) <= 0.05 * res["fp32"][0]
