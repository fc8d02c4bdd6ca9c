"""Per-stage parity of the HIP path against the FP64 oracle (needs a GPU).

Every stage runs through the C ABI on seeded inputs; the oracle evaluates
the same stage in float64 on the same inputs. Tolerance: norm-wise relative
difference <= 1e-5 per tensor (per frame for per-frame quantities);
nearest-neighbour indices bit-exact except documented float32 near-ties.
"""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import block_rel, flat_params, gpu_plan, nn_check, rel, to_np

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _mid():
    # Headline-shaped model (F=4, M=4, width 128, 3 hidden, LeakyReLU) at
    # oracle-friendly size: 2100 vertices span two Chamfer vertex blocks and a
    # ragged 64-vertex MLP block; frames are ragged down to a single point.
    return synth.config_small(name="mid", levels=[16, 24, 35], feat_p=4, time_freqs=4, mlp_hidden=3,
                              mlp_width=128, act="leaky", V=2100, T=5, N=[300, 2049, 1, 700, 1500], t_key=2,
                              seed=21)


def _c1():
    return synth.config_c1()


def _mid_quat():
    # the same model with the quaternion rotation head of Sec. 3.4 (7 outputs)
    return dict(_mid(), name="mid_quat", rot_head="quat")


CONFIGS = {"c1": _c1, "mid": _mid, "mid_quat": _mid_quat}


@pytest.fixture(scope="module", params=list(CONFIGS))
def case(request):
    import torch
    cfg = CONFIGS[request.param]()
    data = synth.make_workload(cfg)
    plan = gpu_plan(cfg, data)
    p = synth.random_state(cfg, 100)
    flat = flat_params(cfg, p)
    T, V = cfg["T"] if "T" in cfg else data["T"], len(data["xyz"])
    T = data["T"]
    st = dict(cfg=cfg, data=data, plan=plan, p=p, P=O.to64(p), flat=flat, T=T, V=V)
    # forward through the GPU stages once; later tests reuse the outputs
    z = torch.empty(V * plan.Fz, dtype=torch.float32, device="cuda")
    plan.encode_fwd(flat, z)
    xhat = torch.empty(T * V * 4, dtype=torch.float32, device="cuda")
    plan.decode_fwd(flat, z, xhat)
    torch.cuda.synchronize()
    st.update(z=z, xhat=xhat, fw=O.forward(st["P"], data, cfg))
    yield st
    plan.close()


def test_encode_forward(case):
    z = to_np(case["z"]).reshape(case["V"], -1)
    ref = O.encode(case["P"], case["data"]["xyz"].astype(np.float64), case["data"]["nrm"].astype(np.float64),
                   case["cfg"]["levels"], case["cfg"]["res_n"])
    assert rel(z, ref) < TOL


def test_decode_forward(case):
    xh = to_np(case["xhat"]).reshape(case["T"], case["V"], 4)
    assert np.all(xh[..., 3] == 0)
    for t in range(case["T"]):
        assert rel(xh[t, :, :3], case["fw"]["xhat"][t]) < TOL, t


def test_identity_start_is_exact(case):
    import torch
    cfg, data = case["cfg"], case["data"]
    flat = flat_params(cfg, synth.init_params(cfg))
    plan = case["plan"]
    z = torch.empty_like(case["z"])
    xhat = torch.empty_like(case["xhat"])
    plan.encode_fwd(flat, z)
    plan.decode_fwd(flat, z, xhat)
    xh = to_np(xhat).reshape(case["T"], case["V"], 4)
    for t in range(case["T"]):
        np.testing.assert_array_equal(xh[t, :, :3], data["xyz"])


def _chamfer(case):
    import torch
    plan, T, V = case["plan"], case["T"], case["V"]
    N = plan.Ntot
    a = torch.empty(T * V, dtype=torch.int32, device="cuda")
    da = torch.empty(T * V, dtype=torch.float32, device="cuda")
    b = torch.empty(N, dtype=torch.int32, device="cuda")
    db = torch.empty(N, dtype=torch.float32, device="cuda")
    cd = torch.empty(T, dtype=torch.float64, device="cuda")
    plan.chamfer_fwd(case["xhat"], a, da, b, db, cd)
    torch.cuda.synchronize()
    return a, da, b, db, cd


def test_chamfer_indices_and_distances(case):
    a, da, b, db, cd = _chamfer(case)
    T, V = case["T"], case["V"]
    off = case["data"]["frame_off"]
    P = case["data"]["pts"]
    xh = to_np(case["xhat"]).reshape(T, V, 4)[..., :3]
    a, da, b, db, cd = to_np(a).reshape(T, V), to_np(da).reshape(T, V), to_np(b), to_np(db), to_np(cd)
    ties = [0, 0]
    for t in range(T):
        Pt = P[off[t]:off[t + 1]]
        ta, tb = nn_check(xh[t], Pt, a[t], b[off[t]:off[t + 1]])
        ties[0] += ta
        ties[1] += tb
        ao, bo, dao, dbo, cdo = O.chamfer(xh[t].astype(np.float64), Pt.astype(np.float64))
        assert rel(da[t], dao) < TOL and rel(db[off[t]:off[t + 1]], dbo) < TOL
        assert abs(cd[t] - cdo) <= TOL * abs(cdo)
        # end to end against the oracle's own float64 forward
        assert abs(cd[t] - O.chamfer(case["fw"]["xhat"][t], Pt.astype(np.float64))[4]) <= TOL * cdo
    print("documented near-ties (rows, cols):", ties)


def test_chamfer_exact_ties_pick_lowest_index():
    import torch
    cfg = synth.config_small(mlp_width=32, V=5, T=1, N=6, t_key=0)
    data = synth.make_workload(cfg)
    X = np.array([[0, 0, 0], [0.5, 0, 0], [0, 0, 0], [0.5, 0, 0], [0.25, 0, 0]], np.float32)
    data["xyz"] = X
    # points equidistant from several vertices, and duplicated points
    data["pts"] = np.array([[0.25, 0.1, 0], [0.25, 0.1, 0], [0.1, 0, 0], [0.4, 0, 0], [0, 0, 0.3], [0.5, 0, 0]],
                           np.float32)
    data["frame_off"] = np.array([0, 6])
    plan = gpu_plan(cfg, data)
    flat = flat_params(cfg, synth.init_params(cfg))
    z = torch.empty(5 * plan.Fz, dtype=torch.float32, device="cuda")
    xh = torch.empty(20, dtype=torch.float32, device="cuda")
    plan.encode_fwd(flat, z)
    plan.decode_fwd(flat, z, xh)
    a = torch.empty(5, dtype=torch.int32, device="cuda")
    da = torch.empty(5, device="cuda")
    b = torch.empty(6, dtype=torch.int32, device="cuda")
    db = torch.empty(6, device="cuda")
    cd = torch.empty(1, dtype=torch.float64, device="cuda")
    plan.chamfer_fwd(xh, a, da, b, db, cd)
    ao, bo, *_ = O.chamfer(X.astype(np.float64), data["pts"].astype(np.float64))
    np.testing.assert_array_equal(to_np(a), ao)
    np.testing.assert_array_equal(to_np(b), bo)
    plan.close()


def test_loss_and_chamfer_backward(case):
    import torch
    a, da, b, db, cd = _chamfer(case)
    plan, T, V, cfg = case["plan"], case["T"], case["V"], case["cfg"]
    w = torch.empty(T, dtype=torch.float64, device="cuda")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    for epoch in (0, 3):
        plan.loss(cd, epoch, 7, w, loss)
        cdn = to_np(cd)
        tk = cfg["t_key"] if cfg["t_key"] is not None else (T - 1) // 2
        wo = O.confidence(cdn, tk, epoch, 7)
        assert rel(to_np(w), wo) < 1e-12
        assert abs(loss.item() - np.mean(wo * cdn)) < 1e-12 * abs(loss.item())
    gx = torch.empty(T * V * 4, dtype=torch.float32, device="cuda")
    plan.chamfer_bwd(case["xhat"], a, b, w, gx)
    xh = to_np(case["xhat"]).reshape(T, V, 4)[..., :3].astype(np.float64)
    off = case["data"]["frame_off"]
    ao = [to_np(a).reshape(T, V)[t] for t in range(T)]
    bo = [to_np(b)[off[t]:off[t + 1]] for t in range(T)]
    ref = O.chamfer_backward(xh, case["data"]["pts"].astype(np.float64), off, ao, bo, to_np(w))
    g = to_np(gx).reshape(T, V, 4)
    for t in range(T):
        assert rel(g[t, :, :3], ref[t]) < TOL, t
    assert np.all(g[..., 3] == 0)


def _oracle_decode_bwd(case, gx):
    cfg, fw = case["cfg"], case["fw"]
    T, V = case["T"], case["V"]
    go = O.transform_backward(gx.reshape(T * V, 3), fw["o"], fw["Xt"], fw["R"], fw["dh"], cfg["alpha_t"],
                              cfg.get("rot_head", "expmap"))
    gmlp, gY = O.mlp_backward(case["P"]["mlp"], go, fw["pres"], fw["ins"], cfg["act"], cfg["leaky_slope"])
    Fz = cfg["feat_n"] + cfg["feat_p"]
    return gmlp, gY[:, :Fz].reshape(T, V, Fz).sum(0)


def test_decode_backward(case):
    import torch
    plan, T, V, cfg = case["plan"], case["T"], case["V"], case["cfg"]
    rng = np.random.default_rng(7)
    gx = rng.normal(size=(T, V, 3)).astype(np.float32)
    gx4 = np.concatenate([gx, np.zeros((T, V, 1), np.float32)], -1)
    grad = torch.zeros(plan.n_params, dtype=torch.float32, device="cuda")
    gz = torch.empty(V * plan.Fz, dtype=torch.float32, device="cuda")
    plan.decode_bwd(case["flat"], case["z"], torch.from_numpy(gx4.ravel()).cuda(), grad, gz)
    gmlp, gz_ref = _oracle_decode_bwd(case, gx.astype(np.float64))
    import paper_2602_22212_amd as npg
    got = npg.unpack_params(cfg, to_np(grad))
    for k, ((gW, gb), (rW, rb)) in enumerate(zip(got["mlp"], gmlp)):
        assert rel(gW, rW) < TOL, ("W", k, rel(gW, rW))
        assert rel(gb, rb) < TOL, ("b", k, rel(gb, rb))
    assert rel(to_np(gz).reshape(V, -1), gz_ref) < TOL


def test_isometry_stage(case):
    """Sec. 3.5 isometry term on the GPU's deformed vertices: the loss value,
    the subgradient decisions (against float64 decisions on the same float32
    vertices; a difference is allowed only at a length tie within 1e-12
    relative) and the gradient evaluated with the kernel's decisions."""
    import torch
    cfg = dict(case["cfg"], w_iso=100.0)
    data, T, V = case["data"], case["T"], case["V"]
    plan = gpu_plan(cfg, data)
    E = data["edges"]
    t_key = cfg["t_key"] if cfg["t_key"] is not None else (T - 1) // 2
    gx = torch.zeros(T * V * 4, dtype=torch.float32, device="cuda")
    iso = torch.empty(1, dtype=torch.float64, device="cuda")
    sign = torch.empty(T * len(E), dtype=torch.int8, device="cuda")
    plan.iso(case["xhat"], iso, gx, sign)
    xh = to_np(case["xhat"]).reshape(T, V, 4)[..., :3].astype(np.float64)
    ref = O.iso_loss(xh, E, t_key)
    assert abs(iso.item() - ref) <= 1e-10 * ref
    sg = to_np(sign).reshape(T, len(E)).astype(np.float64)
    so = O.iso_signs(xh, E, t_key)
    ell = np.linalg.norm(xh[:, E[:, 0]] - xh[:, E[:, 1]], axis=-1)
    diff = sg != so
    assert np.all(np.abs(ell - ell[t_key][None])[diff] <= 1e-12 * ell[diff]), diff.sum()
    assert np.all(sg[t_key] == 0)
    g = to_np(gx).reshape(T, V, 4)
    gref = cfg["w_iso"] * O.iso_backward(xh, E, t_key, sg)
    for t in range(T):
        if t != t_key:
            assert rel(g[t, :, :3], gref[t]) < TOL, t
    assert np.all(g[t_key] == 0) and np.all(g[..., 3] == 0)
    print("decision differences:", int(diff.sum()), "of", diff.size)
    plan.close()


def test_encode_backward(case):
    import torch
    plan, V, cfg, data = case["plan"], case["V"], case["cfg"], case["data"]
    rng = np.random.default_rng(8)
    gz = rng.normal(size=(V, plan.Fz)).astype(np.float32)
    grad = torch.full((plan.n_params,), 7.0, dtype=torch.float32, device="cuda")
    plan.encode_bwd(torch.from_numpy(gz.ravel()).cuda(), grad)
    gp, gn = O.encode_backward(gz.astype(np.float64), data["xyz"].astype(np.float64),
                               data["nrm"].astype(np.float64), cfg["levels"], cfg["res_n"], cfg["feat_p"],
                               cfg["feat_n"])
    import paper_2602_22212_amd as npg
    got = npg.unpack_params(cfg, to_np(grad))
    for l, (g, r) in enumerate(zip(got["grid_p"], gp)):
        assert rel(g, r) < TOL, l
        assert np.all(g[np.abs(r).sum(1) == 0] == 0)   # untouched nodes are exactly zero
    assert rel(got["grid_n"], gn) < TOL
    assert np.all(got["mlp"][0][0] == 7.0)               # MLP block untouched


def test_encode_backward_is_deterministic(case):
    import torch
    plan, V = case["plan"], case["V"]
    gz = torch.randn(V * plan.Fz, device="cuda")
    g1 = torch.zeros(plan.n_params, device="cuda")
    g2 = torch.zeros(plan.n_params, device="cuda")
    plan.encode_bwd(gz, g1)
    plan.encode_bwd(gz, g2)
    assert torch.equal(g1, g2)


def test_preconditioner_matches_exact_operator(case):
    import torch
    plan, cfg, data = case["plan"], case["cfg"], case["data"]
    rng = np.random.default_rng(9)
    # a realistic input: the sparse, spiky grid gradient of a random vertex gradient
    gz = torch.from_numpy(rng.normal(size=(case["V"] * plan.Fz)).astype(np.float32)).cuda()
    grad = torch.zeros(plan.n_params, dtype=torch.float32, device="cuda")
    plan.encode_bwd(gz, grad)
    import paper_2602_22212_amd as npg
    g_in = npg.unpack_params(cfg, to_np(grad))
    its, st = plan.precond(grad)
    assert st == npg.NPG_OK, its
    got = npg.unpack_params(cfg, to_np(grad))
    errs = []
    for l, (g, gi) in enumerate(zip(got["grid_p"], g_in["grid_p"])):
        ref = O.precond_dct(gi.astype(np.float64), cfg["levels"][l], cfg["lam"][l])
        errs.append(rel(g, ref))
    refn = O.precond_dct(g_in["grid_n"].astype(np.float64), cfg["res_n"], cfg["lam_n"])
    errs.append(rel(got["grid_n"], refn))
    print("precond rel errors per grid:", ["%.2e" % e for e in errs], "iterations:", its)
    assert max(errs) < TOL
    rr = plan.precond_residuals()  # both CG solves of every grid stopped at the tolerance
    assert len(rr) == 2 * (len(cfg["levels"]) + 1)
    assert all(0 < r <= cfg["cg_rtol"] for r in rr), rr


def test_preconditioner_special_cases(case):
    import torch

    import paper_2602_22212_amd as npg
    cfg = dict(case["cfg"])
    # zero in -> exactly zero out, zero iterations
    plan = case["plan"]
    grad = torch.zeros(plan.n_params, dtype=torch.float32, device="cuda")
    its, st = plan.precond(grad)
    assert st == npg.NPG_OK and not grad.any() and max(its) == 0
    # lambda = 0 -> identity (one CG step solves I x = b exactly)
    cfg0 = dict(cfg, lam=[0.0] * len(cfg["levels"]), lam_n=0.0)
    p0 = gpu_plan(cfg0, case["data"])
    g = torch.randn(plan.n_params, device="cuda")
    h = g.clone()
    p0.precond(h)
    n_grid = dict((name, o) for name, o, _ in npg.param_layout(cfg)[0])["W0"]
    assert rel(to_np(h[:n_grid]), to_np(g[:n_grid])) < 1e-7
    assert torch.equal(h[n_grid:], g[n_grid:])
    p0.close()


def test_adam_matches_oracle(case):
    import torch

    import paper_2602_22212_amd as npg
    plan, cfg = case["plan"], case["cfg"]
    n = plan.n_params
    rng = np.random.default_rng(10)
    th, g = rng.normal(size=n).astype(np.float32), rng.normal(size=n).astype(np.float32)
    m, v = (rng.normal(size=n) * 0.1).astype(np.float32), rng.uniform(0, 0.1, n).astype(np.float32)
    T_ = [torch.from_numpy(x.copy()).cuda() for x in (th, g, m, v)]
    plan.adam(T_[0], T_[1], T_[2], T_[3], 3)
    lay, _ = npg.param_layout(cfg)
    L = len(cfg["levels"])
    for name, o, s in lay:
        k = int(np.prod(s))
        lr = (cfg["lr_grid"][int(name[6:])] if name.startswith("grid_p") else
              cfg["lr_n"] if name == "grid_n" else cfg["lr_mlp"])
        sl = slice(o, o + k)
        rt, rm, rv = O.adam(th[sl].astype(np.float64), g[sl].astype(np.float64), m[sl].astype(np.float64),
                            v[sl].astype(np.float64), 3, lr, cfg["beta1"], cfg["beta2"], cfg["eps"])
        assert rel(to_np(T_[0])[sl], rt) < TOL and rel(to_np(T_[2])[sl], rm) < TOL
        assert rel(to_np(T_[3])[sl], rv) < TOL
    assert L >= 1


@pytest.mark.parametrize("method", ["cg", "cg_plain", "dct"])
@pytest.mark.parametrize("levels,feat", [([100, 129, 20], 4), ([256], 4), ([7, 33, 50], 2), ([17, 24], 3),
                                         ([2, 3, 5, 9], 1), (list(range(2, 18)), 4)])
def test_preconditioner_large_grids(levels, feat, method):
    """Grids of >= 100 nodes per axis run the z-column CG kernels; 129 gives
    partial tiles in x, y and z; F = 2, 3 and odd sizes exercise the generic
    paths of both methods (odd sizes also give partial multigrid aggregates;
    2 and 3 nodes per axis give single-node coarse levels). Sixteen levels
    (2..17 nodes per axis, lambda up to 175) and the normal grid make 17
    systems, the most one V-cycle launch holds tasks for.
    cg: V-cycle preconditioned CG; cg_plain: plain CG. Sparse vertex-gradient
    input as in a step, plus a dense random component."""
    import torch

    import paper_2602_22212_amd as npg
    cfg = synth.config_small(levels=levels, feat_p=feat, mlp_width=32, V=3000, T=1, N=10, t_key=0, seed=33,
                             precond="dct" if method == "dct" else "cg", cg_mg=int(method == "cg"))
    data = synth.make_workload(cfg)
    plan = gpu_plan(cfg, data)
    rng = np.random.default_rng(12)
    gz = torch.from_numpy(rng.normal(size=(plan.V * plan.Fz)).astype(np.float32)).cuda()
    grad = torch.zeros(plan.n_params, dtype=torch.float32, device="cuda")
    plan.encode_bwd(gz, grad)
    n_grid = dict((name, o) for name, o, _ in npg.param_layout(cfg)[0])["W0"]
    grad[:n_grid] += 1e-3 * torch.randn(n_grid, device="cuda")
    g_in = npg.unpack_params(cfg, to_np(grad))
    its, st = plan.precond(grad)
    assert st == npg.NPG_OK, its
    got = npg.unpack_params(cfg, to_np(grad))
    errs = [rel(g, O.precond_dct(gi.astype(np.float64), R, lam))
            for g, gi, R, lam in zip(got["grid_p"], g_in["grid_p"], cfg["levels"], cfg["lam"])]
    errs.append(rel(got["grid_n"], O.precond_dct(g_in["grid_n"].astype(np.float64), cfg["res_n"], cfg["lam_n"])))
    print("precond rel errors:", ["%.2e" % e for e in errs], "iterations:", its)
    assert max(errs) < TOL
    plan.close()


@pytest.mark.parametrize("method", ["cg", "cg_plain"])
def test_preconditioner_early_stops_on_large_grids(method):
    """Solves that stop before their first odd iteration on the z-column
    grids: a zero right-hand side (no iteration: the result is exactly 0) and
    lambda = 0 (one iteration: the identity), next to a grid that iterates.
    The workspace and the gradient buffer hold a previous call's values, so a
    result that is not written in full shows up."""
    import torch

    import paper_2602_22212_amd as npg
    cfg = synth.config_small(levels=[100, 129, 20], lam=[0.0, 3.0, 1.0], feat_p=4, mlp_width=32, V=3000, T=1,
                             N=10, t_key=0, seed=34, precond="cg", cg_mg=int(method == "cg"))
    data = synth.make_workload(cfg)
    plan = gpu_plan(cfg, data)
    n_grid = dict((name, o) for name, o, _ in npg.param_layout(cfg)[0])["W0"]
    lay = dict((name, (o, int(np.prod(s)))) for name, o, s in npg.param_layout(cfg)[0])
    torch.manual_seed(5)
    warm = torch.randn(plan.n_params, device="cuda")
    assert plan.precond(warm)[1] == npg.NPG_OK
    grad = torch.randn(plan.n_params, device="cuda")
    o1, k1 = lay["grid_p1"]
    grad[o1:o1 + k1] = 0.0
    g_in = npg.unpack_params(cfg, to_np(grad))
    its, st = plan.precond(grad)
    assert st == npg.NPG_OK, its
    got = npg.unpack_params(cfg, to_np(grad))
    print("iterations per solve and system:", its)
    assert rel(got["grid_p"][0], g_in["grid_p"][0]) < 1e-7  # lambda = 0
    assert not np.any(got["grid_p"][1])                      # zero in, zero out
    assert rel(got["grid_p"][2], O.precond_dct(g_in["grid_p"][2].astype(np.float64), 20, 1.0)) < TOL
    assert rel(got["grid_n"], O.precond_dct(g_in["grid_n"].astype(np.float64), cfg["res_n"], cfg["lam_n"])) < TOL
    assert np.array_equal(to_np(grad[n_grid:]), npg.pack_params(cfg, g_in)[n_grid:])
    plan.close()


@pytest.mark.parametrize("method", ["cg", "cg_plain"])
@pytest.mark.parametrize("levels", [[100, 129, 20], [7, 33, 150, 50, 110]])
def test_preconditioner_streams_are_bitwise_equal(levels, method):
    """With the largest grid z-column tiled and other grids before it, the
    solves iterate the grids before it on a second stream, each group at its
    own pace; cg_one_stream = 1 runs the same launches on one stream, and
    with iteration profiling on the groups go in step. All three give the
    same result and iteration counts bit for bit (the systems are
    independent), on two calls in a row (the second starts from the first's
    iteration counts)."""
    import torch

    import paper_2602_22212_amd as npg
    out = []
    for one, prof in ((0, False), (1, False), (0, True)):
        cfg = synth.config_small(levels=levels, feat_p=4, mlp_width=32, V=3000, T=1, N=10, t_key=0, seed=35,
                                 precond="cg", cg_mg=int(method == "cg"), cg_one_stream=one)
        data = synth.make_workload(cfg)
        plan = gpu_plan(cfg, data)
        plan.profile(prof)
        torch.manual_seed(6)
        res = []
        for _ in range(2):
            grad = torch.randn(plan.n_params, device="cuda")
            its, st = plan.precond(grad)
            assert st == npg.NPG_OK, its
            res.append((to_np(grad), np.array(its)))
        out.append(res)
        plan.close()
    for (g0, i0), (g1, i1), (g2, i2) in zip(*out):
        print("iterations per solve and system:", i0.tolist())
        np.testing.assert_array_equal(i0, i1)
        np.testing.assert_array_equal(g0, g1)
        np.testing.assert_array_equal(i0, i2)
        np.testing.assert_array_equal(g0, g2)


def test_multigrid_preconditioned_cg_cuts_iterations():
    """The V-cycle preconditioned solves and plain CG reach the exact operator
    within the tolerance on the same input (smoothness up to the headline's
    finest 6.83), both stop at the residual tolerance, and the preconditioned
    solves need at most half the iterations on every grid with lambda >= 1."""
    import torch

    import paper_2602_22212_amd as npg
    lam = [0.4, 1.35, 6.834375]
    res = {}
    for mg in (0, 1):
        cfg = synth.config_small(levels=[16, 35, 64], lam=lam, feat_p=4, mlp_width=32, V=3000, T=1, N=10, t_key=0,
                                 seed=34, cg_mg=mg)
        data = synth.make_workload(cfg)
        plan = gpu_plan(cfg, data)
        rng = np.random.default_rng(13)
        grad = torch.zeros(plan.n_params, dtype=torch.float32, device="cuda")
        plan.encode_bwd(torch.from_numpy(rng.normal(size=(plan.V * plan.Fz)).astype(np.float32)).cuda(), grad)
        n_grid = dict((name, o) for name, o, _ in npg.param_layout(cfg)[0])["W0"]
        grad[:n_grid] += 1e-3 * torch.from_numpy(rng.normal(size=n_grid).astype(np.float32)).cuda()
        g_in = npg.unpack_params(cfg, to_np(grad))
        its, st = plan.precond(grad)
        assert st == npg.NPG_OK, its
        got = npg.unpack_params(cfg, to_np(grad))
        errs = [rel(g, O.precond_dct(gi.astype(np.float64), R, la))
                for g, gi, R, la in zip(got["grid_p"], g_in["grid_p"], cfg["levels"], lam)]
        errs.append(rel(got["grid_n"], O.precond_dct(g_in["grid_n"].astype(np.float64), cfg["res_n"], cfg["lam_n"])))
        rr = plan.precond_residuals()
        print("cg_mg", mg, "errors", ["%.2e" % e for e in errs], "iterations", its)
        assert max(errs) < TOL and all(0 < r <= cfg["cg_rtol"] for r in rr), (errs, rr)
        res[mg] = its
        plan.close()
    L = len(lam)
    for k in range(2 * (L + 1)):
        la = lam[k % (L + 1)] if k % (L + 1) < L else 0.4
        if la >= 1.0:
            assert 2 * res[1][k] <= res[0][k], (k, res)
