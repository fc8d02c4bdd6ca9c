"""torch.autograd Functions over the stage entry points of libneupig.so.

Every forward and backward below is a sequence of library calls (HIP
kernels); torch only allocates their outputs and, where two Functions
feed one tensor, sums the two gradients (the autograd engine's own
accumulation). The Functions take a Plan (static tables and workspace of one
sequence) and the flat float32 parameter vector of the plan's layout.

  EncodeFn          params -> z [V, F_n+F_p]                     (Sec. 3.2)
  DecodeApplyFn     params, z -> x^ [T, V, 4]                    (Sec. 3.3-3.4)
  ChamferLossFn     x^ -> L_def, cd [T]                          (Sec. 3.5)
  IsoFn             x^ -> L_iso                                  (Sec. 3.5)
  ObjectiveFn       x^ -> L_def + w_iso L_iso, cd [T]: the whole objective
                    and its x^ gradient formed by the library (Sec. 3.5)
  DeformChamferLossFn params, z -> L_def, cd: decode + Chamfer with x^
                    recomputed in backward instead of kept
  DeformObjectiveFn params, z -> L_def + w_iso L_iso, cd: decode + the
                    objective with x^ recomputed in backward
  NeuPigOptimizer   (I + lambda L)^-2 on the grid blocks of the gradient,
                    then Adam (Sec. 3.5)

The decoder's backward never stores MLP activations: the library recomputes
them per tile. The confidence weights of L_def are a stop-gradient, as in the
method. All tensors live on the plan's GPU and every call is issued on the
plan's stream, which must be torch's current stream while these run.
"""
import torch

_F32, _F64, _I32 = torch.float32, torch.float64, torch.int32


def _empty(plan, shape, dtype=_F32):
    return torch.empty(shape, dtype=dtype, device=plan.device)


def _zeros(plan, shape, dtype=_F32):
    return torch.zeros(shape, dtype=dtype, device=plan.device)


def _flat(t):
    return t.detach().contiguous().view(-1)


class EncodeFn(torch.autograd.Function):
    """z_i = (z_n(n_i), mean over levels of z_p^l(x_i)); the backward is the
    deterministic grid scatter (grid blocks of the returned gradient; its MLP
    block is zero)."""

    @staticmethod
    def forward(ctx, params, plan):
        z = _empty(plan, (plan.V, plan.Fz))
        plan.encode_fwd(_flat(params), z.view(-1))
        ctx.plan = plan
        return z

    @staticmethod
    def backward(ctx, gz):
        plan = ctx.plan
        grad = _zeros(plan, plan.n_params)
        plan.encode_bwd(_flat(gz), grad)
        return grad, None


class DecodeApplyFn(torch.autograd.Function):
    """Time-modulated MLP and the 6-DoF transform of every vertex in every
    frame; x^[..., 3] is 0. Saves only the parameters and z: the backward
    recomputes the decoder per tile. Returns (gradient with only the MLP
    block set, gz summed over frames)."""

    @staticmethod
    def forward(ctx, params, z, plan):
        xhat = _empty(plan, (plan.T, plan.V, 4))
        p, zf = _flat(params), _flat(z)
        plan.decode_fwd(p, zf, xhat.view(-1))
        ctx.save_for_backward(p, zf)
        ctx.plan = plan
        return xhat

    @staticmethod
    def backward(ctx, gx):
        plan = ctx.plan
        p, zf = ctx.saved_tensors
        grad = _zeros(plan, plan.n_params)
        gz = _empty(plan, (plan.V, plan.Fz))
        plan.decode_bwd(p, zf, _flat(gx), grad, gz.view(-1))
        return grad, gz, None


def _chamfer_forward(plan, xhat, epoch, n_epochs):
    a = _empty(plan, plan.T * plan.V, _I32)
    da = _empty(plan, plan.T * plan.V)
    b = _empty(plan, plan.Ntot, _I32)
    db = _empty(plan, plan.Ntot)
    cd = _empty(plan, plan.T, _F64)
    w = _empty(plan, plan.T, _F64)
    loss = _empty(plan, 1, _F64)
    plan.chamfer_fwd(xhat, a, da, b, db, cd)
    plan.loss(cd, epoch, n_epochs, w, loss)
    return a, b, cd, w, loss


def _chamfer_backward(plan, xhat, a, b, w, g_loss):
    # d L_def / d x^ with the per-frame weights (g w_t): the upstream factor
    # enters the kernel's float64 weights, not its float32 output
    wg = w.clone()
    plan.scale(g_loss.detach().reshape(1).to(_F64).contiguous(), wg)
    gx = _empty(plan, (plan.T, plan.V, 4))
    plan.chamfer_bwd(xhat, a, b, wg, gx.view(-1))
    return gx


class ChamferLossFn(torch.autograd.Function):
    """Bidirectional nearest-neighbour Chamfer distance per frame and the
    confidence-weighted mean L_def (0-d float64) at the given epoch. cd [T]
    is returned for reporting and is not differentiable (use L_def)."""

    @staticmethod
    def forward(ctx, xhat, plan, epoch, n_epochs):
        xf = _flat(xhat)
        a, b, cd, w, loss = _chamfer_forward(plan, xf, epoch, n_epochs)
        ctx.save_for_backward(xf, a, b, w)
        ctx.plan = plan
        ctx.mark_non_differentiable(cd)
        return loss.view(()), cd

    @staticmethod
    def backward(ctx, g_loss, g_cd):
        xf, a, b, w = ctx.saved_tensors
        return _chamfer_backward(ctx.plan, xf, a, b, w, g_loss), None, None, None


class DeformChamferLossFn(torch.autograd.Function):
    """DecodeApplyFn followed by ChamferLossFn without keeping x^: only the
    nearest-neighbour indices (4 B per vertex-frame and per point) and the
    frame weights are stored; the backward decodes x^ again."""

    @staticmethod
    def forward(ctx, params, z, plan, epoch, n_epochs):
        p, zf = _flat(params), _flat(z)
        xhat = _empty(plan, plan.T * plan.V * 4)
        plan.decode_fwd(p, zf, xhat)
        a, b, cd, w, loss = _chamfer_forward(plan, xhat, epoch, n_epochs)
        del xhat
        ctx.save_for_backward(p, zf, a, b, w)
        ctx.plan = plan
        ctx.mark_non_differentiable(cd)
        return loss.view(()), cd

    @staticmethod
    def backward(ctx, g_loss, g_cd):
        plan = ctx.plan
        p, zf, a, b, w = ctx.saved_tensors
        xhat = _empty(plan, plan.T * plan.V * 4)
        plan.decode_fwd(p, zf, xhat)
        gx = _chamfer_backward(plan, xhat, a, b, w, g_loss)
        del xhat
        grad = _zeros(plan, plan.n_params)
        gz = _empty(plan, (plan.V, plan.Fz))
        plan.decode_bwd(p, zf, gx.view(-1), grad, gz.view(-1))
        return grad, gz, None, None, None


class IsoFn(torch.autograd.Function):
    """Isometry loss L_iso (0-d float64) over the plan's mesh edges, key-frame
    lengths a stop-gradient. The library forms w_iso dL_iso/dx^ with the
    plan's w_iso, so the plan must have w_iso > 0 and edges set."""

    @staticmethod
    def forward(ctx, xhat, plan):
        w_iso = float(plan.cfg.get("w_iso", 0.0))
        if not w_iso > 0.0 or not getattr(plan, "n_edges", 0):
            raise ValueError("IsoFn needs a plan with w_iso > 0 and mesh edges (Plan.set_edges)")
        xf = _flat(xhat)
        iso = _empty(plan, 1, _F64)
        plan.iso(xf, iso)
        ctx.save_for_backward(xf)
        ctx.plan = plan
        return iso.view(())

    @staticmethod
    def backward(ctx, g):
        plan = ctx.plan
        (xf,) = ctx.saved_tensors
        gx = _zeros(plan, (plan.T, plan.V, 4))
        tmp = _empty(plan, 1, _F64)
        plan.iso(xf, tmp, gx.view(-1))
        plan.scale(g.detach().reshape(1).to(_F64).contiguous(), gx.view(-1), 1.0 / float(plan.cfg["w_iso"]))
        return gx, None


def _objective_forward(plan, xhat, epoch, n_epochs):
    a = _empty(plan, plan.T * plan.V, _I32)
    da = _empty(plan, plan.T * plan.V)
    b = _empty(plan, plan.Ntot, _I32)
    db = _empty(plan, plan.Ntot)
    cd = _empty(plan, plan.T, _F64)
    w = _empty(plan, plan.T, _F64)
    loss = _empty(plan, 1, _F64)
    plan.objective_fwd(xhat, epoch, n_epochs, a, da, b, db, cd, w, loss)
    return a, b, cd, w, loss


def _objective_backward(plan, xhat, a, b, w, g_loss):
    gx = _empty(plan, (plan.T, plan.V, 4))
    plan.objective_bwd(xhat, a, b, w, g_loss.detach().reshape(1).to(_F64).contiguous(), gx.view(-1))
    return gx


class ObjectiveFn(torch.autograd.Function):
    """The objective of Sec. 3.5, L_def + w_iso L_iso (0-d float64; the
    isometry term with the plan's w_iso and mesh edges when w_iso > 0), and
    cd [T] (not differentiable). Forward and backward are single library
    calls (npg_objective_fwd / npg_objective_bwd): the two terms and their x^
    gradients are summed by the library."""

    @staticmethod
    def forward(ctx, xhat, plan, epoch, n_epochs):
        xf = _flat(xhat)
        a, b, cd, w, loss = _objective_forward(plan, xf, epoch, n_epochs)
        ctx.save_for_backward(xf, a, b, w)
        ctx.plan = plan
        ctx.mark_non_differentiable(cd)
        return loss.view(()), cd

    @staticmethod
    def backward(ctx, g_loss, g_cd):
        xf, a, b, w = ctx.saved_tensors
        return _objective_backward(ctx.plan, xf, a, b, w, g_loss), None, None, None


class DeformObjectiveFn(torch.autograd.Function):
    """DecodeApplyFn followed by ObjectiveFn without keeping x^ (only the
    nearest-neighbour indices and the frame weights are stored; the backward
    decodes x^ again)."""

    @staticmethod
    def forward(ctx, params, z, plan, epoch, n_epochs):
        p, zf = _flat(params), _flat(z)
        xhat = _empty(plan, plan.T * plan.V * 4)
        plan.decode_fwd(p, zf, xhat)
        a, b, cd, w, loss = _objective_forward(plan, xhat, epoch, n_epochs)
        del xhat
        ctx.save_for_backward(p, zf, a, b, w)
        ctx.plan = plan
        ctx.mark_non_differentiable(cd)
        return loss.view(()), cd

    @staticmethod
    def backward(ctx, g_loss, g_cd):
        plan = ctx.plan
        p, zf, a, b, w = ctx.saved_tensors
        xhat = _empty(plan, plan.T * plan.V * 4)
        plan.decode_fwd(p, zf, xhat)
        gx = _objective_backward(plan, xhat, a, b, w, g_loss)
        del xhat
        grad = _zeros(plan, plan.n_params)
        gz = _empty(plan, (plan.V, plan.Fz))
        plan.decode_bwd(p, zf, gx.view(-1), grad, gz.view(-1))
        return grad, gz, None, None, None


def objective(plan, params, epoch, n_epochs, recompute=False):
    """The training objective of one step, L_def + w_iso L_iso (the isometry
    term only when the plan's w_iso > 0), and the per-frame Chamfer
    distances. recompute: x^ is decoded again in backward instead of kept.
    No arithmetic here: the library forms the objective and every gradient;
    the autograd engine only adds the grid-block gradient of EncodeFn to the
    MLP-block gradient of the decoder (disjoint blocks of params)."""
    z = EncodeFn.apply(params, plan)
    if recompute:
        return DeformObjectiveFn.apply(params, z, plan, epoch, n_epochs)
    xhat = DecodeApplyFn.apply(params, z, plan)
    return ObjectiveFn.apply(xhat, plan, epoch, n_epochs)


class NeuPigOptimizer:
    """Preconditioned Adam of Sec. 3.5 on a flat float32 parameter leaf:
    step() replaces every grid block of params.grad by (I + lambda L)^-2 g
    (in place; the MLP block is left as is), then applies bias-corrected Adam
    with the plan's per-block learning rates."""

    def __init__(self, plan, params):
        if params.dtype != _F32 or not params.is_contiguous() or params.numel() != plan.n_params:
            raise ValueError(f"params must be a contiguous float32 vector of {plan.n_params} elements")
        self.plan, self.params = plan, params
        self.m = torch.zeros_like(params, requires_grad=False)
        self.v = torch.zeros_like(params, requires_grad=False)
        self.k = 0
        self.last_iters = None

    def zero_grad(self):
        self.params.grad = None

    @torch.no_grad()
    def step(self):
        g = self.params.grad
        if g is None:
            raise RuntimeError("no gradient: call backward() first")
        if not g.is_contiguous():
            g = g.contiguous()
            self.params.grad = g
        self.last_iters, st = self.plan.precond(g)
        self.k += 1
        self.plan.adam(self.params.detach(), g, self.m, self.v, self.k)
        return st
