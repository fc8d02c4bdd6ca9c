"""Full optimization steps at the headline model and grids against the oracle
(needs a GPU).

Human workload: 30 000 reference vertices and 10 000 points per frame, 8
position-grid levels 16..256 x 4 features plus the 4^3 x 2 normal grid, decoder
14 -> 128 x 3 -> 6 with LeakyReLU and M = 4 time frequencies. The teacher-forced
steps use the workload's first three frames so that the float64 oracle (brute
force Chamfer) finishes in about a minute; the Chamfer of the full 100-frame
sequence is checked against k-d tree distances in float64 on the GPU's own
deformed vertices.
"""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import f32_hyper, flat_params, gpu_plan, rel, to_np, touched_nodes

pytestmark = pytest.mark.gpu
TOL = 1e-5
T_SUB = 3


@pytest.fixture(scope="module")
def headline_steps():
    """Two oracle steps from a non-degenerate state: k = 1 from zero Adam
    moments, then k = 2 from the oracle's own state after the first."""
    cfg = f32_hyper(synth.config_c2())
    data = synth.make_workload(cfg, T=T_SUB)
    P0 = O.to64(synth.random_state(cfg, 9, grid_std=0.05))
    m0, v0 = O.zeros_like_params(P0), O.zeros_like_params(P0)
    E = cfg["n_steps"]
    P1, m1, v1, d1 = O.step(P0, m0, v0, 1, data, cfg, 0, E)
    ls1 = d1["ls"]
    del d1
    P2, m2, v2, d2 = O.step(P1, m1, v1, 2, data, cfg, 1, E)
    ls2 = d2["ls"]
    del d2
    return dict(cfg=cfg, data=data, touched=touched_nodes(cfg, data),
                states=[(P0, m0, v0), (P1, m1, v1), (P2, m2, v2)], ls=[ls1, ls2])


def _blocks(cfg, s):
    P, m, v = s
    return (P["grid_p"] + [P["grid_n"]], m["grid_p"] + [m["grid_n"]], v["grid_p"] + [v["grid_n"]], P["mlp"],
            m["mlp"], v["mlp"])


@pytest.mark.parametrize("method", ["cg", "dct"])
def test_headline_teacher_forced_steps(headline_steps, method):
    """Each GPU step starts from the oracle's state (parameters and Adam
    moments; the oracle runs the library's float32 hyper-parameters).
    Compared at 1e-5 (norm-wise): the loss, every frame's Chamfer
    distance, every MLP block after the update, and, at the grid nodes a
    reference vertex reads, the updated parameters and both Adam moments
    (after step 1 the first moment is 0.1 times the preconditioned gradient,
    so it checks the preconditioner inside the step). The oracle
    preconditions exactly (cosine transform); the CG form solves to its
    residual bound. Step 1 from zero moments moves each entry by
    lr g~/(|g~| + eps), i.e. by lr times the sign of g~: entries whose
    oracle g~ lies within 1e-4 of the level's rms of zero (float32 noise can
    flip that sign) are compared only against the Adam bound |dtheta| <= lr.
    Nodes no vertex reads never influence the loss and are checked against
    the same bound."""
    import torch

    import paper_2602_22212_amd as npg
    H = headline_steps
    cfg = dict(H["cfg"], precond=method)
    data, touched = H["data"], H["touched"]
    plan = gpu_plan(cfg, data)
    lrs = list(cfg["lr_grid"]) + [cfg["lr_n"]]
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    cd = torch.empty(T_SUB, dtype=torch.float64, device="cuda")
    b1 = cfg["beta1"]
    bad = []
    for e in range(2):
        (P, m, v), (Pn, mn, vn), ls = H["states"][e], H["states"][e + 1], H["ls"][e]
        plan.set_state(flat_params(cfg, P), flat_params(cfg, m), flat_params(cfg, v), e)
        st = plan.step(e, cfg["n_steps"], loss, cd)
        assert st == npg.NPG_OK, st
        pg, mg, vg, k = plan.get_state()
        assert k == e + 1
        el, ec = abs(loss.item() - ls["loss"]) / ls["loss"], rel(to_np(cd), ls["cd"])
        print(f"{method} step {e + 1}: loss rel err {el:.2e}, cd rel err {ec:.2e}", flush=True)
        if not (el <= TOL and ec < TOL):
            bad.append((e, "loss/cd", el, ec))
        got = [npg.unpack_params(cfg, to_np(x)) for x in (pg, mg, vg)]
        gg, gm, gv, gW, gmW, gvW = _blocks(cfg, tuple(got))
        og, om, ov, oW, omW, ovW = _blocks(cfg, (Pn, mn, vn))
        for k_ in range(len(oW)):
            for j in range(2):
                errs = (rel(gW[k_][j], oW[k_][j]), rel(gmW[k_][j], omW[k_][j]), rel(gvW[k_][j], ovW[k_][j]))
                print(f"  layer {k_} {'Wb'[j]}: rel err params {errs[0]:.2e} m {errs[1]:.2e} v {errs[2]:.2e}",
                      flush=True)
                if max(errs) >= TOL:
                    bad.append((e, "mlp", k_, j, errs))
        g0 = P["grid_p"] + [P["grid_n"]]
        for l, tn in enumerate(touched):
            em, ev = rel(gm[l][tn], om[l][tn]), rel(gv[l][tn], ov[l][tn])
            new, ref = gg[l][tn], og[l][tn]
            step_bound = lrs[l] / (1 - b1) * 1.001 + 1e-6
            if e == 0:
                gt = om[l][tn] / (1 - b1)
                undecided = np.abs(gt) < 1e-4 * np.sqrt(np.mean(gt * gt))
                ep = rel(new[~undecided], ref[~undecided])
                if not np.all(np.abs(new[undecided] - g0[l][tn][undecided]) <= lrs[l] * 1.001):
                    bad.append((e, "undecided entries beyond lr", l))
                print(f"  grid {l}: touched nodes {len(tn)}, sign-undecided entries {int(undecided.sum())}, "
                      f"rel err params {ep:.2e} m {em:.2e} v {ev:.2e}", flush=True)
            else:
                ep = rel(new, ref)
                print(f"  grid {l}: rel err params {ep:.2e} m {em:.2e} v {ev:.2e}", flush=True)
            if not (ep < TOL and em < TOL and ev < TOL):
                bad.append((e, "grid", l, ep, em, ev))
            if not np.all(np.abs(gg[l] - g0[l]) <= step_bound):
                bad.append((e, "grid step bound", l))
        if method == "cg":
            res = plan.precond_residuals()
            print(f"  CG final relative residuals: max {max(res):.2e}", flush=True)
            if max(res) > cfg["cg_rtol"]:
                bad.append((e, "residual", max(res)))
    assert not bad, bad
    plan.close()


def test_headline_full_sequence_chamfer_against_kdtree():
    """All 100 frames of the headline workload at a non-degenerate state: per
    frame, the GPU's Chamfer distance and both directions' nearest distances
    against float64 k-d tree queries (scipy cKDTree, exact nearest
    neighbours) on the GPU's own float32 deformed vertices; the confidence
    weights and the loss of the GPU against the oracle's formulas on the
    k-d tree distances."""
    import torch
    from scipy.spatial import cKDTree

    cfg = f32_hyper(synth.config_c2())
    data = synth.make_workload(cfg)
    plan = gpu_plan(cfg, data)
    T, V = data["T"], len(data["xyz"])
    assert T == 100 and V == 30000
    P = O.to64(synth.random_state(cfg, 9, grid_std=0.05))
    flat = flat_params(cfg, P)
    z = torch.empty(V * plan.Fz, device="cuda")
    xh = torch.empty(T * V * 4, device="cuda")
    N = plan.Ntot
    a = torch.empty(T * V, dtype=torch.int32, device="cuda")
    da = torch.empty(T * V, device="cuda")
    b = torch.empty(N, dtype=torch.int32, device="cuda")
    db = torch.empty(N, device="cuda")
    cd = torch.empty(T, dtype=torch.float64, device="cuda")
    w = torch.empty(T, dtype=torch.float64, device="cuda")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    plan.encode_fwd(flat, z)
    plan.decode_fwd(flat, z, xh)
    plan.chamfer_fwd(xh, a, da, b, db, cd)
    plan.loss(cd, 3, cfg["n_steps"], w, loss)
    xha = to_np(xh).reshape(T, V, 4)[..., :3].astype(np.float64)
    off = data["frame_off"]
    pts = data["pts"].astype(np.float64)
    cd_g, da_g, db_g = to_np(cd), to_np(da).reshape(T, V), to_np(db)
    cd_k = np.empty(T)
    worst = 0.0
    for t in range(T):
        Pt = pts[off[t]:off[t + 1]]
        dA = cKDTree(Pt).query(xha[t], workers=-1)[0] ** 2
        dB = cKDTree(xha[t]).query(Pt, workers=-1)[0] ** 2
        cd_k[t] = dA.mean() + dB.mean()
        e = max(abs(cd_g[t] - cd_k[t]) / cd_k[t], rel(da_g[t], dA), rel(db_g[off[t]:off[t + 1]], dB))
        worst = max(worst, e)
        assert e < TOL, (t, e)
    t_key = (T - 1) // 2
    w_o = O.confidence(cd_k, t_key, 3, cfg["n_steps"])
    assert rel(to_np(w), w_o) < TOL
    assert abs(loss.item() - np.mean(w_o * cd_k)) <= TOL * np.mean(w_o * cd_k)
    print(f"100 frames: worst per-frame relative error {worst:.2e}")
    plan.close()
