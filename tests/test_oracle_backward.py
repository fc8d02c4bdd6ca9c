"""Pins of the oracle's gradients, preconditioner and optimizer (no GPU)."""
import numpy as np
import pytest
import torch

import oracle as O
import synth


def _loss_fixed_w(p, data, cfg, w, ref, key_len=None):
    """Loss with the confidence weights frozen (stop-gradient of Sec. 3.5) and,
    with an isometry term, the key-frame edge lengths frozen too; also returns
    whether the NN assignments equal the reference ones."""
    fw = O.forward(p, data, cfg)
    P = np.asarray(data["pts"], np.float64)
    off = data["frame_off"]
    T = len(off) - 1
    tot, same = 0.0, True
    for t in range(T):
        a, b, _, _, cd = O.chamfer(fw["xhat"][t], P[off[t]:off[t + 1]])
        same &= np.array_equal(a, ref["a"][t]) and np.array_equal(b, ref["b"][t])
        tot += w[t] * cd
    tot /= T
    if key_len is not None:
        e = np.asarray(data["edges"])
        ell = np.linalg.norm(fw["xhat"][:, e[:, 0]] - fw["xhat"][:, e[:, 1]], axis=-1)
        tot += cfg["w_iso"] * np.abs(ell - key_len[None]).mean()
    return tot, same


def _perturb(p, flat_delta):
    out = O.zeros_like_params(p)
    i = 0
    for l, g in enumerate(p["grid_p"]):
        out["grid_p"][l] = g + flat_delta[i:i + g.size].reshape(g.shape)
        i += g.size
    out["grid_n"] = p["grid_n"] + flat_delta[i:i + p["grid_n"].size].reshape(p["grid_n"].shape)
    i += p["grid_n"].size
    mlp = []
    for W, b in p["mlp"]:
        W2 = W + flat_delta[i:i + W.size].reshape(W.shape)
        i += W.size
        b2 = b + flat_delta[i:i + b.size]
        i += b.size
        mlp.append((W2, b2))
    out["mlp"] = mlp
    return out


@pytest.mark.parametrize("act,M,head,w_iso", [("leaky", 2, "expmap", 0.0), ("relu", 0, "expmap", 0.0),
                                              ("leaky", 2, "quat", 0.0), ("leaky", 2, "expmap", 100.0)])
def test_full_loss_gradient_matches_central_differences(act, M, head, w_iso):
    cfg = synth.config_small(act=act, time_freqs=M, N=[50, 41, 47], rot_head=head, w_iso=w_iso)
    data = synth.make_workload(cfg)
    p = O.to64(synth.random_state(cfg, 3))
    fw = O.forward(p, data, cfg)
    ls = O.losses(fw, data, cfg, 1, 3)
    key_len = None
    if w_iso > 0:
        e = data["edges"]
        key_len = np.linalg.norm(fw["xhat"][ls["t_key"], e[:, 0]] - fw["xhat"][ls["t_key"], e[:, 1]], axis=-1)
    grads, _ = O.backward(p, data, cfg, fw, ls)
    g = O.flatten_params(grads)
    n = g.size
    rng = np.random.default_rng(0)
    h = 1e-6
    # every coordinate of a random subset covering all blocks
    idx = np.unique(np.concatenate([rng.choice(n, 150, replace=False),
                                    np.flatnonzero(np.abs(g) > 1e-8)[::7][:150]]))
    checked = 0
    for k in idx:
        e = np.zeros(n)
        e[k] = h
        fp, s1 = _loss_fixed_w(_perturb(p, e), data, cfg, ls["w"], ls, key_len)
        fm, s2 = _loss_fixed_w(_perturb(p, -e), data, cfg, ls["w"], ls, key_len)
        if not (s1 and s2):
            continue
        fd = (fp - fm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])) + 2e-9, (k, fd, g[k])
        checked += 1
    assert checked > 0.9 * len(idx)
    # directional derivative along a random direction
    d = rng.normal(size=n)
    d /= np.linalg.norm(d)
    fp, s1 = _loss_fixed_w(_perturb(p, h * d), data, cfg, ls["w"], ls, key_len)
    fm, s2 = _loss_fixed_w(_perturb(p, -h * d), data, cfg, ls["w"], ls, key_len)
    assert s1 and s2
    assert abs((fp - fm) / (2 * h) - g @ d) < 1e-7 * max(1, abs(g @ d))


def test_full_loss_gradient_matches_torch_autograd():
    # Independent derivative: the same forward written in torch float64 and
    # differentiated by autograd, with assignments and weights taken from the
    # oracle's forward.
    cfg = synth.config_small()
    data = synth.make_workload(cfg)
    p = O.to64(synth.random_state(cfg, 4))
    fw = O.forward(p, data, cfg)
    ls = O.losses(fw, data, cfg, 0, 3)
    grads, _ = O.backward(p, data, cfg, fw, ls)

    X = torch.tensor(data["xyz"], dtype=torch.float64)
    Nr = torch.tensor(data["nrm"], dtype=torch.float64)
    P = torch.tensor(data["pts"], dtype=torch.float64)
    off = data["frame_off"]
    T, V = len(off) - 1, len(X)
    gp = [torch.tensor(g, requires_grad=True) for g in p["grid_p"]]
    gn = torch.tensor(p["grid_n"], requires_grad=True)
    mlp = [(torch.tensor(W, requires_grad=True), torch.tensor(b, requires_grad=True)) for W, b in p["mlp"]]

    def tri(G, R, Q):
        u = (Q.clamp(-1, 1) + 1) * 0.5 * (R - 1)
        i0 = torch.clamp(torch.floor(u), max=R - 2)
        f = u - i0
        i0 = i0.long()
        out = 0
        for cz in (0, 1):
            for cy in (0, 1):
                for cx in (0, 1):
                    w = ((f[:, 0] if cx else 1 - f[:, 0]) * (f[:, 1] if cy else 1 - f[:, 1])
                         * (f[:, 2] if cz else 1 - f[:, 2]))
                    node = ((i0[:, 2] + cz) * R + i0[:, 1] + cy) * R + i0[:, 0] + cx
                    out = out + w[:, None] * G[node]
        return out

    zp = sum(tri(G, R, X) for G, R in zip(gp, cfg["levels"])) / len(gp)
    zn = tri(gn, cfg["res_n"], Nr)
    z = torch.cat([zn, zp], 1)
    gam = torch.tensor(O.time_code(T, cfg["time_freqs"]))
    Y = torch.cat([z.repeat(T, 1), gam.repeat_interleave(V, 0)], 1)
    h = Y
    for k, (W, b) in enumerate(mlp):
        h = h @ W.T + b
        if k < len(mlp) - 1:
            h = torch.nn.functional.leaky_relu(h, 0.01)
    w_, d_ = h[:, :3], h[:, 3:]
    th = w_.norm(dim=1, keepdim=True)
    k_ = w_ / th
    Xt = X.repeat(T, 1)
    # Rodrigues in axis-angle form (theta is far from 0 at this random state)
    rot = (Xt * torch.cos(th) + torch.cross(k_, Xt, dim=1) * torch.sin(th)
           + k_ * (k_ * Xt).sum(1, keepdim=True) * (1 - torch.cos(th)))
    xh = (rot + torch.tanh(cfg["alpha_t"] * d_)).reshape(T, V, 3)
    loss = 0
    for t in range(T):
        Pt = P[off[t]:off[t + 1]]
        a = torch.from_numpy(ls["a"][t])
        b = torch.from_numpy(ls["b"][t])
        cd = ((xh[t] - Pt[a]) ** 2).sum(1).mean() + ((xh[t][b] - Pt) ** 2).sum(1).mean()
        loss = loss + float(ls["w"][t]) * cd
    loss = loss / T
    assert abs(loss.item() - ls["loss"]) < 1e-13
    loss.backward()
    for G, g in zip(gp, grads["grid_p"]):
        np.testing.assert_allclose(G.grad.numpy(), g, rtol=1e-9, atol=1e-13)
    np.testing.assert_allclose(gn.grad.numpy(), grads["grid_n"], rtol=1e-9, atol=1e-13)
    for (W, b), (gW, gb) in zip(mlp, grads["mlp"]):
        np.testing.assert_allclose(W.grad.numpy(), gW, rtol=1e-9, atol=1e-13)
        np.testing.assert_allclose(b.grad.numpy(), gb, rtol=1e-9, atol=1e-13)


def test_first_step_grid_gradients_are_exactly_zero_at_paper_init():
    # Sec. 3.1: zero grids and a zero last layer -> only the last layer gets a
    # gradient on the first step.
    cfg = synth.config_c1()
    data = synth.make_workload(cfg)
    p = O.to64(synth.init_params(cfg))
    fw = O.forward(p, data, cfg)
    ls = O.losses(fw, data, cfg, 0, cfg["n_steps"])
    grads, _ = O.backward(p, data, cfg, fw, ls)
    for g in grads["grid_p"] + [grads["grid_n"]]:
        assert not g.any()
    for gW, gb in grads["mlp"][:-1]:
        assert not gW.any() and not gb.any()
    assert np.abs(grads["mlp"][-1][0]).max() > 0


def _dense_laplacian(R):
    # explicit edge loop over the 6-neighbour lattice (free boundary)
    n = R ** 3
    Lm = np.zeros((n, n))
    for iz in range(R):
        for iy in range(R):
            for ix in range(R):
                a = (iz * R + iy) * R + ix
                for dz, dy, dx in ((1, 0, 0), (0, 1, 0), (0, 0, 1)):
                    jz, jy, jx = iz + dz, iy + dy, ix + dx
                    if jz < R and jy < R and jx < R:
                        b = (jz * R + jy) * R + jx
                        Lm[a, a] += 1
                        Lm[b, b] += 1
                        Lm[a, b] -= 1
                        Lm[b, a] -= 1
    return Lm


@pytest.mark.parametrize("R,lam", [(2, 0.4), (3, 1.7), (5, 0.6), (6, 6.83)])
def test_preconditioner_matches_dense_solve(R, lam):
    rng = np.random.default_rng(R)
    g = rng.normal(size=(R ** 3, 3))
    A = np.eye(R ** 3) + lam * _dense_laplacian(R)
    ref = np.linalg.solve(A, np.linalg.solve(A, g))
    np.testing.assert_allclose(O.precond_dct(g, R, lam), ref, atol=1e-13)
    x, _ = O.precond_cg(g, R, lam)
    np.testing.assert_allclose(x, ref, atol=1e-11)
    np.testing.assert_allclose(O.laplacian_apply(g, R), _dense_laplacian(R) @ g, atol=1e-13)


def test_preconditioner_invariants():
    R, lam = 7, 2.5
    rng = np.random.default_rng(11)
    a = rng.normal(size=(R ** 3, 2))
    b = rng.normal(size=(R ** 3, 2))
    Pf = lambda g, l=lam: O.precond_dct(g, R, l)
    np.testing.assert_allclose(Pf(a, 0.0), a, atol=1e-14)                       # lambda=0: identity
    np.testing.assert_allclose(Pf(2 * a - 3 * b), 2 * Pf(a) - 3 * Pf(b), atol=1e-13)  # linear
    assert abs((Pf(a) * b).sum() - (a * Pf(b)).sum()) < 1e-12                   # symmetric
    np.testing.assert_allclose(Pf(np.ones((R ** 3, 1))), 1.0, atol=1e-13)        # L 1 = 0
    # a single DCT mode is scaled by (1 + lam mu_k)^-2
    k = (2, 5, 1)        # (kz, ky, kx)
    n = np.arange(R)
    vz, vy, vx = (np.cos(np.pi * kk * (n + 0.5) / R) for kk in k)
    mode = (vz[:, None, None] * vy[None, :, None] * vx[None, None, :]).reshape(-1, 1)
    mu = sum(2 - 2 * np.cos(np.pi * kk / R) for kk in k)
    np.testing.assert_allclose(Pf(mode), mode / (1 + lam * mu) ** 2, atol=1e-13)
    # zero in, zero out (CG path included)
    assert not O.precond_cg(np.zeros((R ** 3, 2)), R, lam)[0].any()


def test_adam_first_step_and_torch():
    rng = np.random.default_rng(12)
    th = rng.normal(size=20)
    g = rng.normal(size=20)
    new, m, v = O.adam(th, g, np.zeros(20), np.zeros(20), 1, 0.01, 0.9, 0.999, 1e-8)
    np.testing.assert_allclose(new, th - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    # several steps against torch.optim.Adam in float64
    x = torch.tensor(th, requires_grad=True)
    opt = torch.optim.Adam([x], lr=0.003)
    cur, m, v = th.copy(), np.zeros(20), np.zeros(20)
    for k in range(1, 6):
        gk = rng.normal(size=20)
        x.grad = torch.tensor(gk)
        opt.step()
        cur, m, v = O.adam(cur, gk, m, v, k, 0.003, 0.9, 0.999, 1e-8)
    np.testing.assert_allclose(cur, x.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_step_reduces_loss_on_sphere():
    # Oracle steps from the paper's identity start (Sec. 3.1) lower the mean
    # Chamfer distance on the icosphere workload at every step.
    cfg = synth.config_c1()
    data = synth.make_workload(cfg)
    p = O.to64(synth.init_params(cfg))
    m, v = O.zeros_like_params(p), O.zeros_like_params(p)
    losses = []
    for e in range(5):
        p, m, v, d = O.step(p, m, v, e + 1, data, cfg, e, cfg["n_steps"])
        losses.append(float(np.mean(d["ls"]["cd"])))
    assert np.all(np.diff(losses) < 0)


def test_isometry_loss_hand_worked_example():
    # two edges (0,1), (1,2); key frame 0 has lengths 1 and 1, frame 1 has
    # lengths 2 and 0.5: L = (|2-1| + |0.5-1|)/(T |E|) = 1.5/4. Frame 1's
    # gradient: edge (0,1) pulls with sign +1 along (x0-x1)/2, edge (1,2) with
    # sign -1 along (x1-x2)/0.5, each scaled by 1/(T |E|) = 1/4.
    x = np.array([[[0, 0, 0], [1, 0, 0], [1, 1, 0]],
                  [[0, 0, 0], [2, 0, 0], [2, 0.5, 0]]], np.float64)
    e = np.array([[0, 1], [1, 2]])
    assert O.iso_loss(x, e, 0) == 0.375
    g = O.iso_backward(x, e, 0)
    np.testing.assert_array_equal(g[0], 0.0)  # key frame: sign(0) = 0
    np.testing.assert_allclose(g[1], [[-0.25, 0, 0], [0.25, 0.25, 0], [0, -0.25, 0]], atol=1e-15)
    # with frame 1 as the key frame the roles swap
    assert O.iso_loss(x, e, 1) == 0.375


def test_isometry_loss_rigid_motions_and_finite_differences():
    from scipy.spatial.transform import Rotation
    X, _, E = synth.meshes.icosphere(2)
    rng = np.random.default_rng(2)
    T, t_key = 4, 1
    Rs = Rotation.random(T, random_state=3).as_matrix()
    rigid = np.stack([X @ Rs[t].T + rng.normal(size=3) for t in range(T)])
    assert O.iso_loss(rigid, E, t_key) < 1e-15
    # identical frames: every length difference is exactly 0, so is the gradient
    same = np.stack([X] * T)
    assert O.iso_loss(same, E, t_key) == 0.0
    assert np.all(O.iso_backward(same, E, t_key) == 0.0)
    # explicit decisions reproduce the float64 ones
    xs0 = rigid + rng.normal(scale=0.05, size=rigid.shape)
    np.testing.assert_array_equal(O.iso_backward(xs0, E, t_key, O.iso_signs(xs0, E, t_key)),
                                  O.iso_backward(xs0, E, t_key))
    # generic frames: gradient of every frame except the key frame against
    # central differences (the key-frame lengths are a stop-gradient, so only
    # perturbations of the other frames leave them fixed)
    xs = rigid + rng.normal(scale=0.05, size=rigid.shape)
    g = O.iso_backward(xs, E, t_key)
    h = 1e-7
    for t, i, c in zip(rng.choice([0, 2, 3], 40), rng.integers(0, len(X), 40), rng.integers(0, 3, 40)):
        d = np.zeros_like(xs)
        d[t, i, c] = h
        fd = (O.iso_loss(xs + d, E, t_key) - O.iso_loss(xs - d, E, t_key)) / (2 * h)
        assert abs(fd - g[t, i, c]) < 1e-7 * max(1e-3, abs(g[t, i, c])), (t, i, c, fd, g[t, i, c])
    assert np.all(g[t_key] == 0)


def test_bf16_backward_rounds_only_the_matrix_operands():
    # two layers, everything already bfloat16-representable: the BF16
    # backward equals the plain one exactly; a non-representable upstream
    # gradient is rounded for layer 2's products and kept for its bias
    rng = np.random.default_rng(3)
    W1 = O.bf16_round(rng.normal(size=(4, 3)))
    W2 = O.bf16_round(rng.normal(size=(2, 4)))
    mlp = [(W1, np.zeros(4)), (W2, np.zeros(2))]
    Y = O.bf16_round(rng.normal(size=(5, 3)))
    o, pres, ins = O.mlp_forward(mlp, Y, "relu", 0.0, bf16=True)
    go = O.bf16_round(rng.normal(size=(5, 2)))
    ref, gy = O.mlp_backward(mlp, go, pres, [Y, O.bf16_round(ins[1])], "relu", 0.0)
    got, gy2 = O.mlp_backward(mlp, go, pres, ins, "relu", 0.0, bf16=True)
    if np.array_equal(ins[1], O.bf16_round(ins[1])):
        for (a, b), (c, d) in zip(ref, got):
            np.testing.assert_array_equal(a, c)
            np.testing.assert_array_equal(b, d)
    go2 = rng.normal(size=(5, 2))
    got2, _ = O.mlp_backward(mlp, go2, pres, ins, "relu", 0.0, bf16=True)
    np.testing.assert_array_equal(got2[1][0], O.bf16_round(go2).T @ ins[1])
    np.testing.assert_array_equal(got2[1][1], go2.sum(0))


@pytest.mark.parametrize("method", ["dct", "cg"])
def test_step_composition_per_block(method):
    """How one step is put together (Sec. 3.5 "Preconditioning" and
    "Implementation Details"; Table 7 names the base smoothness 0.4): grid
    level l = 1..L (coarsest first) is preconditioned by (I + lam_l L)^-2 with
    lam_l = 0.4 * 1.5^(l-1) and updated with lr_l = 0.005 * 2.5^(l-1); the
    normal grid uses lam 0.4 and lr 0.005; the MLP gradient is not
    preconditioned and uses lr 1e-3. At Adam step 1 from zero moments every
    entry moves by -lr g~ / (|g~| + eps) and the moments are (1 - b1) g~ and
    (1 - b2) g~^2. The preconditioner is evaluated here by dense solves of the
    explicit edge-loop Laplacian (levels of 3, 4, 5 and 4 nodes per axis), so
    a swapped level order, a wrong level's lam or lr, or a preconditioned MLP
    gradient fails."""
    cfg = synth.config_small(precond=method)
    L = len(cfg["levels"])
    lam = [0.4 * 1.5 ** (l - 1) for l in range(1, L + 1)]
    lr = [0.005 * 2.5 ** (l - 1) for l in range(1, L + 1)]
    np.testing.assert_allclose(cfg["lam"], lam, rtol=1e-15)
    np.testing.assert_allclose(cfg["lr_grid"], lr, rtol=1e-15)
    assert cfg["lam_n"] == 0.4 and cfg["lr_n"] == 0.005 and cfg["lr_mlp"] == 1e-3
    data = synth.make_workload(cfg)
    p = O.to64(synth.random_state(cfg, 21))
    zero = O.zeros_like_params(p)
    fw = O.forward(p, data, cfg)
    ls = O.losses(fw, data, cfg, 0, cfg["n_steps"])
    g, _ = O.backward(p, data, cfg, fw, ls)
    p1, m1, v1, d = O.step(p, zero, O.zeros_like_params(p), 1, data, cfg, 0, cfg["n_steps"], precond=method)
    b1, b2, eps = cfg["beta1"], cfg["beta2"], cfg["eps"]
    tol = 1e-12 if method == "dct" else 1e-9

    def dense_precond(gl, R, lm):
        A = np.eye(R ** 3) + lm * _dense_laplacian(R)
        return np.linalg.solve(A, np.linalg.solve(A, gl))

    def check(th0, th1, mm, vv, gt, rate, name):
        np.testing.assert_allclose(mm, (1 - b1) * gt, rtol=tol, atol=1e-300, err_msg=name)
        np.testing.assert_allclose(vv, (1 - b2) * gt * gt, rtol=2 * tol, atol=1e-300, err_msg=name)
        np.testing.assert_allclose(th1, th0 - rate * gt / (np.abs(gt) + eps), rtol=tol, atol=tol * rate,
                                   err_msg=name)

    grids = list(zip(p["grid_p"], p1["grid_p"], m1["grid_p"], v1["grid_p"], g["grid_p"], cfg["levels"]))
    assert len(set(cfg["levels"])) == L  # distinct sizes: a level permutation cannot pass
    for l, (th0, th1, mm, vv, gl, R) in enumerate(grids):
        gt = dense_precond(gl, R, lam[l])
        assert np.abs(gt - gl).max() > 1e-3 * np.abs(gl).max()  # the preconditioner acts
        check(th0, th1, mm, vv, gt, lr[l], f"level {l + 1}")
    gt = dense_precond(g["grid_n"], cfg["res_n"], 0.4)
    check(p["grid_n"], p1["grid_n"], m1["grid_n"], v1["grid_n"], gt, 0.005, "normal grid")
    for k, ((W0, b0), (W1, b1_), (mW, mb), (vW, vb), (gW, gb)) in enumerate(
            zip(p["mlp"], p1["mlp"], m1["mlp"], v1["mlp"], g["mlp"])):
        check(W0, W1, mW, vW, gW, 1e-3, f"W{k}")
        check(b0, b1_, mb, vb, gb, 1e-3, f"b{k}")
    # the step reports the preconditioned gradients it fed to Adam
    for l, (gl, R) in enumerate(zip(g["grid_p"], cfg["levels"])):
        np.testing.assert_allclose(d["pgrads"]["grid_p"][l], dense_precond(gl, R, lam[l]), rtol=tol, atol=1e-14)
