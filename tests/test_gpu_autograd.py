"""torch.autograd Functions over the stage entry points (needs a GPU).

The gradient that loss.backward() produces through EncodeFn, DecodeApplyFn,
ChamferLossFn and IsoFn is checked against the FP64 oracle's analytic
gradient (1e-5 norm-wise per block, teacher-forced on the kernel's nearest
neighbours and isometry decisions), against the library's own stage chain
(bitwise), against central differences of the GPU loss along the gradient,
and one optimizer step against npg_step (bitwise)."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import flat_params, gpu_plan, nn_check, rel, to_np

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _cfg(**kw):
    # the headline model shape (F=4, M=4, width 128, 3 hidden, LeakyReLU) with
    # ragged frames down to a single point
    c = synth.config_small(name="ag", levels=[16, 24, 35], feat_p=4, time_freqs=4, mlp_hidden=3, mlp_width=128,
                           act="leaky", V=2100, T=5, N=[300, 2049, 1, 700, 1500], t_key=2, seed=21)
    c.update(kw)
    return c


def _leaf(cfg, seed):
    return flat_params(cfg, synth.random_state(cfg, seed)).requires_grad_()


def _gpu_decisions(plan, cfg, data, flat):
    """Nearest neighbours and isometry decisions of the GPU's own deformed
    vertices (the same kernels on the same inputs as inside the Functions)."""
    import torch
    T, V = data["T"], len(data["xyz"])
    z = torch.empty(V * plan.Fz, device="cuda")
    xh = torch.empty(T * V * 4, device="cuda")
    plan.encode_fwd(flat, z)
    plan.decode_fwd(flat, z, xh)
    a = torch.empty(T * V, dtype=torch.int32, device="cuda")
    da = torch.empty(T * V, device="cuda")
    b = torch.empty(plan.Ntot, dtype=torch.int32, device="cuda")
    db = torch.empty(plan.Ntot, device="cuda")
    cd = torch.empty(T, dtype=torch.float64, device="cuda")
    plan.chamfer_fwd(xh, a, da, b, db, cd)
    sign = None
    if cfg.get("w_iso", 0.0) > 0:
        E = data["edges"]
        s = torch.empty(T * len(E), dtype=torch.int8, device="cuda")
        plan.iso(xh, torch.empty(1, dtype=torch.float64, device="cuda"), None, s)
        sign = to_np(s).reshape(T, len(E)).astype(np.float64)
    return to_np(xh).reshape(T, V, 4)[..., :3], to_np(a).reshape(T, V), to_np(b), sign


@pytest.mark.parametrize("w_iso", [0.0, 100.0])
def test_backward_matches_oracle_gradient(w_iso):
    import paper_2602_22212_amd as npg
    from paper_2602_22212_amd import autograd as AG
    cfg = _cfg(w_iso=w_iso)
    data = synth.make_workload(cfg)
    plan = gpu_plan(cfg, data)
    p = synth.random_state(cfg, 100)
    params = flat_params(cfg, p).requires_grad_()
    loss, cd = AG.objective(plan, params, 3, 7)
    loss.backward()
    T = data["T"]
    xh, a, b, sign = _gpu_decisions(plan, cfg, data, params.detach())
    off = data["frame_off"]
    for t in range(T):
        nn_check(xh[t], data["pts"][off[t]:off[t + 1]], a[t], b[off[t]:off[t + 1]])
    P = O.to64(p)
    fw = O.forward(P, data, cfg)
    ls = O.losses(fw, data, cfg, 3, 7)
    assert abs(loss.item() - ls["loss"]) <= TOL * ls["loss"]
    assert rel(to_np(cd), ls["cd"]) < TOL
    ls["a"] = [a[t] for t in range(T)]
    ls["b"] = [b[off[t]:off[t + 1]] for t in range(T)]
    if sign is not None:
        E = data["edges"]
        ell = np.linalg.norm(fw["xhat"][:, E[:, 0]] - fw["xhat"][:, E[:, 1]], axis=-1)
        diff = sign != O.iso_signs(fw["xhat"], E, ls["t_key"])
        assert np.all(np.abs(ell - ell[ls["t_key"]][None])[diff] <= 1e-5 * ell[diff]), diff.sum()
    g, _ = O.backward(P, data, cfg, fw, ls, iso_sign=sign)
    got = npg.unpack_params(cfg, to_np(params.grad))
    for k, ((gW, gb), (rW, rb)) in enumerate(zip(got["mlp"], g["mlp"])):
        assert rel(gW, rW) < TOL and rel(gb, rb) < TOL, (k, rel(gW, rW), rel(gb, rb))
    for l, (gg, rg) in enumerate(zip(got["grid_p"] + [got["grid_n"]], g["grid_p"] + [g["grid_n"]])):
        assert rel(gg, rg) < TOL, (l, rel(gg, rg))
    plan.close()


def test_backward_equals_stage_chain_and_recompute_form():
    """The Functions add nothing to the kernels' arithmetic: the gradient is
    bitwise the library's stage chain, and the form that decodes x^ again in
    backward gives bitwise the same gradient as the one that keeps x^."""
    import torch

    from paper_2602_22212_amd import autograd as AG
    cfg = _cfg()
    data = synth.make_workload(cfg)
    plan = gpu_plan(cfg, data)
    T, V = data["T"], len(data["xyz"])
    params = _leaf(cfg, 101)
    loss, _ = AG.objective(plan, params, 1, 7)
    loss.backward()
    # the same step through the entry points, one gradient vector
    flat = params.detach()
    z = torch.empty(V * plan.Fz, device="cuda")
    xh = torch.empty(T * V * 4, device="cuda")
    plan.encode_fwd(flat, z)
    plan.decode_fwd(flat, z, xh)
    a = torch.empty(T * V, dtype=torch.int32, device="cuda")
    da = torch.empty(T * V, device="cuda")
    b = torch.empty(plan.Ntot, dtype=torch.int32, device="cuda")
    db = torch.empty(plan.Ntot, device="cuda")
    cd = torch.empty(T, dtype=torch.float64, device="cuda")
    w = torch.empty(T, dtype=torch.float64, device="cuda")
    l2 = torch.empty(1, dtype=torch.float64, device="cuda")
    plan.chamfer_fwd(xh, a, da, b, db, cd)
    plan.loss(cd, 1, 7, w, l2)
    gx = torch.empty_like(xh)
    plan.chamfer_bwd(xh, a, b, w, gx)
    grad = torch.zeros(plan.n_params, device="cuda")
    gz = torch.empty_like(z)
    plan.decode_bwd(flat, z, gx, grad, gz)
    plan.encode_bwd(gz, grad)
    assert loss.item() == l2.item()
    assert torch.equal(params.grad, grad)
    # recompute form
    p2 = params.detach().clone().requires_grad_()
    z2 = AG.EncodeFn.apply(p2, plan)
    l3, cd3 = AG.DeformChamferLossFn.apply(p2, z2, plan, 1, 7)
    l3.backward()
    assert l3.item() == l2.item() and torch.equal(cd3, cd)
    assert torch.equal(p2.grad, grad)
    plan.close()


def test_upstream_gradient_scales_every_term():
    import torch

    from paper_2602_22212_amd import autograd as AG
    cfg = _cfg(w_iso=100.0)
    data = synth.make_workload(cfg)
    plan = gpu_plan(cfg, data)
    p1 = _leaf(cfg, 102)
    p2 = p1.detach().clone().requires_grad_()
    AG.objective(plan, p1, 2, 7)[0].backward()
    (AG.objective(plan, p2, 2, 7)[0] * -2.5).backward()
    assert rel(to_np(p2.grad), -2.5 * to_np(p1.grad)) < 1e-6
    # each Function alone under a non-unit upstream gradient
    x = AG.DecodeApplyFn.apply(p1.detach(), AG.EncodeFn.apply(p1.detach(), plan), plan).detach()
    x1, x2 = x.clone().requires_grad_(), x.clone().requires_grad_()
    AG.IsoFn.apply(x1, plan).backward()
    (3.0 * AG.IsoFn.apply(x2, plan)).backward()
    assert rel(to_np(x2.grad), 3.0 * to_np(x1.grad)) < 1e-6 and x1.grad.abs().sum() > 0
    x1.grad, x2.grad = None, None
    AG.ChamferLossFn.apply(x1, plan, 2, 7)[0].backward()
    (0.5 * AG.ChamferLossFn.apply(x2, plan, 2, 7)[0]).backward()
    assert torch.equal(x2.grad, 0.5 * x1.grad)   # a power of two is exact in the float64 weights
    plan.close()


def test_gradient_matches_central_differences_of_gpu_loss():
    """Directional derivative along the normalized gradient: the central
    difference of the GPU loss (confidence weights at delta = 0, i.e. all 1,
    so the loss has no stop-gradient) against |g|."""
    import torch

    from paper_2602_22212_amd import autograd as AG
    cfg = _cfg()
    data = synth.make_workload(cfg)
    plan = gpu_plan(cfg, data)
    params = _leaf(cfg, 103)
    E = 7
    loss, _ = AG.objective(plan, params, E, E)
    loss.backward()
    g = params.grad.double()
    gn = g.norm().item()
    d = (g / gn).float()
    with torch.no_grad():
        L0 = loss.item()
        errs = []
        for eps in (1e-3, 3e-4):
            # a step that moves the loss by eps of itself
            h = eps * L0 / gn
            lp = AG.objective(plan, params.detach() + h * d, E, E)[0].item()
            lm = AG.objective(plan, params.detach() - h * d, E, E)[0].item()
            fd = (lp - lm) / (2 * h)
            errs.append(abs(fd - gn) / gn)
    print("relative directional-derivative errors:", errs)
    assert min(errs) < 2e-2
    plan.close()


def test_optimizer_step_equals_npg_step():
    """Two steps through the Functions and NeuPigOptimizer (preconditioning,
    then Adam) give bitwise the parameters and moments of two npg_step calls,
    with and without the isometry term (the objective and its x^ gradient
    formed by the library: ObjectiveFn, DeformObjectiveFn)."""
    import torch

    import paper_2602_22212_amd as npg
    from paper_2602_22212_amd import autograd as AG
    for method, w_iso, recompute in (("cg", 0.0, False), ("dct", 0.0, True), ("dct", 100.0, False),
                                     ("cg", 100.0, True)):
        cfg = _cfg(precond=method, w_iso=w_iso)
        data = synth.make_workload(cfg)
        plan = gpu_plan(cfg, data)
        flat = flat_params(cfg, synth.random_state(cfg, 104))
        zero = torch.zeros_like(flat)
        plan.set_state(flat, zero, zero, 0)
        params = flat.clone().requires_grad_()
        opt = AG.NeuPigOptimizer(plan, params)
        loss = torch.empty(1, dtype=torch.float64, device="cuda")
        for e in range(2):
            assert plan.step(e, 9, loss) == npg.NPG_OK
            opt.zero_grad()
            l_ag, _ = AG.objective(plan, params, e, 9, recompute=recompute)
            l_ag.backward()
            assert opt.step() == npg.NPG_OK
            pg, mg, vg, k = plan.get_state()
            assert k == opt.k == e + 1
            assert l_ag.item() == loss.item(), (method, e)
            assert torch.equal(params.detach(), pg), (method, e)
            assert torch.equal(opt.m, mg) and torch.equal(opt.v, vg), (method, e)
        plan.close()


def test_isofn_needs_weight_and_edges():
    from paper_2602_22212_amd import autograd as AG
    cfg = _cfg()
    data = synth.make_workload(cfg)
    plan = gpu_plan(cfg, data)
    x = AG.DecodeApplyFn.apply(_leaf(cfg, 5).detach(), AG.EncodeFn.apply(_leaf(cfg, 5).detach(), plan), plan)
    with pytest.raises(ValueError):
        AG.IsoFn.apply(x, plan)
    plan.close()
