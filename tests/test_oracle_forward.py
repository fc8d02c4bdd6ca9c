"""Pins of the oracle's forward stages against closed forms, invariants and
independent library routines (no GPU)."""
import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

import oracle as O
import synth


def _node_coords(R):
    # lattice positions of every node, row (iz*R+iy)*R+ix
    g = -1.0 + 2.0 * np.arange(R) / (R - 1)
    iz, iy, ix = np.meshgrid(g, g, g, indexing="ij")
    return np.stack([ix.ravel(), iy.ravel(), iz.ravel()], 1)


@pytest.mark.parametrize("R", [2, 3, 5, 8])
def test_trilinear_reproduces_affine_fields(R):
    # Sec. 3.2: trilinear interpolation is exact for affine fields; distinct
    # coefficients per axis catch swapped axes or a transposed node index.
    rng = np.random.default_rng(R)
    A = np.array([[1.0, -2.0, 0.5], [0.25, 3.0, -1.5]])
    c = np.array([0.3, -0.7])
    G = _node_coords(R) @ A.T + c
    X = rng.uniform(-1, 1, size=(200, 3))
    X[:6] = [[1, 1, 1], [-1, -1, -1], [0, 0, 1], [1, 0, -1], [-1, 1, 0], [0.999999, -1, 1]]
    np.testing.assert_allclose(O.trilinear(G, R, X), X @ A.T + c, atol=1e-12)
    # outside the box the coordinate is clamped
    Xo = rng.uniform(-2, 2, size=(50, 3))
    np.testing.assert_allclose(O.trilinear(G, R, Xo), np.clip(Xo, -1, 1) @ A.T + c, atol=1e-12)


def test_trilinear_node_values_and_partition_of_unity():
    R = 5
    rng = np.random.default_rng(0)
    G = rng.normal(size=(R ** 3, 3))
    X = _node_coords(R)
    np.testing.assert_allclose(O.trilinear(G, R, X), G, atol=1e-12)
    ones = np.ones((R ** 3, 1))
    np.testing.assert_allclose(O.trilinear(ones, R, rng.uniform(-1.5, 1.5, (100, 3))), 1.0, atol=1e-14)


def test_trilinear_backward_is_the_adjoint():
    # <T G, g> == <G, T^T g> for random G, g: a wrong node or weight in the
    # backward scatter breaks the identity.
    R = 6
    rng = np.random.default_rng(1)
    G = rng.normal(size=(R ** 3, 2))
    X = rng.uniform(-1.1, 1.1, size=(300, 3))
    g = rng.normal(size=(300, 2))
    lhs = (O.trilinear(G, R, X) * g).sum()
    rhs = (G * O.trilinear_backward(g, R, X, 2)).sum()
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)


def test_encode_level_average_and_order():
    # Sec. 3.2: z_p is the mean over levels; L identical single-level fields
    # give the single-level value. Output order is (z_n, z_p) (Sec. 3.3).
    cfg = synth.config_small(levels=[4, 4, 4], feat_p=3)
    rng = np.random.default_rng(2)
    G = rng.normal(size=(64, 3))
    Gn = rng.normal(size=(cfg["res_n"] ** 3, 2))
    X = rng.uniform(-1, 1, size=(40, 3))
    Nr = rng.normal(size=(40, 3))
    Nr /= np.linalg.norm(Nr, axis=1, keepdims=True)
    p = dict(grid_p=[G, G, G], grid_n=Gn, mlp=[])
    z = O.encode(p, X, Nr, [4, 4, 4], cfg["res_n"])
    np.testing.assert_allclose(z[:, 2:], O.trilinear(G, 4, X), atol=1e-13)
    np.testing.assert_allclose(z[:, :2], O.trilinear(Gn, 4, Nr), atol=1e-13)
    # different levels: average of the individual lookups
    G2 = rng.normal(size=(5 ** 3, 3))
    p2 = dict(grid_p=[G, G2], grid_n=Gn, mlp=[])
    z2 = O.encode(p2, X, Nr, [4, 5], cfg["res_n"])
    np.testing.assert_allclose(z2[:, 2:], 0.5 * (O.trilinear(G, 4, X) + O.trilinear(G2, 5, X)), atol=1e-13)


def test_time_code_closed_forms():
    # Sec. 3.3: t~ = 0 gives (0,1,0,1,...); t~ = 1 gives sin = 0 and
    # cos = (-1, 1, 1, 1); t~ = 1/2 gives sin(pi/2)=1, cos(pi/2)=0 at j = 1
    # and sin(pi)=0, cos(pi)=-1 at j = 2.
    g = O.time_code(3, 4)
    np.testing.assert_allclose(g[0], [0, 1, 0, 1, 0, 1, 0, 1], atol=1e-15)
    np.testing.assert_allclose(g[2], [0, -1, 0, 1, 0, 1, 0, 1], atol=1e-14)
    np.testing.assert_allclose(g[1][:4], [1, 0, 0, -1], atol=1e-15)
    np.testing.assert_allclose(O.time_code(5, 0)[:, 0], [0, 0.25, 0.5, 0.75, 1.0])
    np.testing.assert_allclose(O.time_code(1, 2), [[0, 1, 0, 1]])


def test_mlp_matches_torch_float64():
    rng = np.random.default_rng(3)
    dims = [7, 16, 16, 6]
    mlp = [(rng.normal(size=(dims[k + 1], dims[k])), rng.normal(size=dims[k + 1])) for k in range(3)]
    Y = rng.normal(size=(50, 7))
    for act in ("relu", "leaky"):
        out, pres, ins = O.mlp_forward(mlp, Y, act, 0.01)
        layers = []
        for k, (W, b) in enumerate(mlp):
            lin = torch.nn.Linear(W.shape[1], W.shape[0]).double()
            with torch.no_grad():
                lin.weight.copy_(torch.from_numpy(W))
                lin.bias.copy_(torch.from_numpy(b))
            layers.append(lin)
            if k < 2:
                layers.append(torch.nn.ReLU() if act == "relu" else torch.nn.LeakyReLU(0.01))
        net = torch.nn.Sequential(*layers)
        Yt = torch.from_numpy(Y).requires_grad_(True)
        ot = net(Yt)
        np.testing.assert_allclose(out, ot.detach().numpy(), rtol=1e-13, atol=1e-13)
        go = rng.normal(size=out.shape)
        ot.backward(torch.from_numpy(go))
        grads, gY = O.mlp_backward(mlp, go, pres, ins, act, 0.01)
        np.testing.assert_allclose(gY, Yt.grad.numpy(), rtol=1e-12, atol=1e-12)
        lins = [m for m in net if isinstance(m, torch.nn.Linear)]
        for (gW, gb), lin in zip(grads, lins):
            np.testing.assert_allclose(gW, lin.weight.grad.numpy(), rtol=1e-12, atol=1e-12)
            np.testing.assert_allclose(gb, lin.bias.grad.numpy(), rtol=1e-12, atol=1e-12)


def test_rodrigues_matches_scipy_and_is_a_rotation():
    rng = np.random.default_rng(4)
    w = rng.normal(size=(400, 3))
    scale = np.concatenate([np.full(100, 1e-7), np.full(50, 0.99e-4), np.full(50, 1.01e-4),
                            rng.uniform(0, np.pi, 200)])
    w = w / np.linalg.norm(w, axis=1, keepdims=True) * scale[:, None]
    R = O.rodrigues(w)
    np.testing.assert_allclose(R, Rotation.from_rotvec(w).as_matrix(), atol=2e-15)
    np.testing.assert_allclose(R @ np.swapaxes(R, 1, 2), np.broadcast_to(np.eye(3), R.shape), atol=1e-14)
    np.testing.assert_allclose(np.linalg.det(R), 1.0, atol=1e-14)
    np.testing.assert_array_equal(O.rodrigues(np.zeros((1, 3)))[0], np.eye(3))


def test_transform_backward_matches_finite_differences():
    rng = np.random.default_rng(5)
    o = rng.normal(size=(30, 6)) * 0.8
    o[:5, :3] *= 1e-6                      # exercise the series branch
    X = rng.normal(size=(30, 3))
    g = rng.normal(size=(30, 3))
    xh, R, dh = O.transform(o, X, 0.1)
    go = O.transform_backward(g, o, X, R, dh, 0.1)
    h = 1e-6
    fd = np.zeros_like(o)
    for k in range(6):
        e = np.zeros(6)
        e[k] = h
        fp = (O.transform(o + e, X, 0.1)[0] * g).sum(1)
        fm = (O.transform(o - e, X, 0.1)[0] * g).sum(1)
        fd[:, k] = (fp - fm) / (2 * h)
    np.testing.assert_allclose(go, fd, rtol=1e-6, atol=1e-8)
    # at omega = 0 the rotation Jacobian reduces to x cross g
    go0 = O.transform_backward(g, np.zeros((30, 6)), X, np.broadcast_to(np.eye(3), (30, 3, 3)),
                               np.zeros((30, 3)), 0.1)
    np.testing.assert_allclose(go0[:, :3], np.cross(X, g), atol=1e-15)


def test_quaternion_head_matches_scipy_and_is_a_rotation():
    # Sec. 3.4: u = (1 + q_w, q_x, q_y, q_z) / norm; R(u) against scipy's
    # quaternion -> matrix (scalar-last convention there).
    rng = np.random.default_rng(4)
    q = rng.normal(scale=0.6, size=(200, 4))
    u, n = O.quat_normalize(q)
    np.testing.assert_allclose(np.linalg.norm(u, axis=1), 1.0, atol=1e-15)
    R = O.quat_matrix(u)
    Rs = Rotation.from_quat(np.c_[u[:, 1:], u[:, 0]]).as_matrix()
    np.testing.assert_allclose(R, Rs, atol=1e-14)
    np.testing.assert_allclose(R @ np.swapaxes(R, 1, 2), np.broadcast_to(np.eye(3), R.shape), atol=1e-14)
    np.testing.assert_allclose(np.linalg.det(R), 1.0, atol=1e-14)
    # zero output is the identity; scaling (1 + q_w, q_v) leaves R unchanged
    np.testing.assert_array_equal(O.quat_matrix(O.quat_normalize(np.zeros((1, 4)))[0])[0], np.eye(3))
    a = q.copy()
    a[:, 0] += 1.0
    q2 = 2.5 * a
    q2[:, 0] -= 1.0
    np.testing.assert_allclose(O.quat_matrix(O.quat_normalize(q2)[0]), R, atol=1e-14)


def test_quaternion_head_agrees_with_the_exp_map_head():
    # the unit quaternion (cos(th/2), sin(th/2) k) and the rotation vector th k
    # are the same rotation, so both heads give the same deformed points
    rng = np.random.default_rng(5)
    w = rng.normal(scale=0.8, size=(100, 3))
    th = np.linalg.norm(w, axis=1, keepdims=True)
    q = np.c_[np.cos(th / 2) - 1.0, np.sin(th / 2) * w / th]
    d = rng.normal(size=(100, 3))
    X = rng.uniform(-1, 1, size=(100, 3))
    xq = O.transform(np.c_[q, d], X, 0.1, "quat")[0]
    xe = O.transform(np.c_[w, d], X, 0.1, "expmap")[0]
    np.testing.assert_allclose(xq, xe, atol=1e-14)


def test_quaternion_backward_matches_finite_differences():
    rng = np.random.default_rng(6)
    o = rng.normal(scale=0.5, size=(40, 7))
    X = rng.uniform(-1, 1, size=(40, 3))
    g = rng.normal(size=(40, 3))
    xh, R, dh = O.transform(o, X, 0.1, "quat")
    go = O.transform_backward(g, o, X, R, dh, 0.1, "quat")
    h = 1e-6
    fd = np.zeros_like(o)
    for k in range(7):
        e = np.zeros(7)
        e[k] = h
        fp = (O.transform(o + e, X, 0.1, "quat")[0] * g).sum(1)
        fm = (O.transform(o - e, X, 0.1, "quat")[0] * g).sum(1)
        fd[:, k] = (fp - fm) / (2 * h)
    np.testing.assert_allclose(go, fd, rtol=1e-6, atol=1e-8)
    # R depends only on the direction of (1 + q_w, q_v): no radial gradient
    a = o[:, :4].copy()
    a[:, 0] += 1.0
    np.testing.assert_allclose((go[:, :4] * a).sum(1), 0.0, atol=1e-13)


def test_identity_start_is_exact():
    # Sec. 3.1: zero last layer => o = 0 => R = I, d^ = 0, x^ = x exactly.
    cfg = synth.config_c1()
    data = synth.make_workload(cfg)
    p = O.to64(synth.init_params(cfg))
    fw = O.forward(p, data, cfg)
    for t in range(cfg["T"]):
        np.testing.assert_array_equal(fw["xhat"][t], data["xyz"].astype(np.float64))


def test_known_rigid_motion_gives_zero_loss_and_gradient():
    # Last layer weights 0 and bias (omega*, atanh(d*)/alpha): every frame is
    # the rigid motion R(omega*) x + d*, built here through scipy. Targets set
    # to exactly that motion give cd = 0 and a zero gradient everywhere.
    cfg = synth.config_small(V=40, T=2, N=40)
    data = synth.make_workload(cfg)
    p = O.to64(synth.random_state(cfg, 7))
    wstar = np.array([0.3, -0.2, 0.5])
    dstar = np.array([0.05, -0.02, 0.03])
    W, b = p["mlp"][-1]
    p["mlp"][-1] = (np.zeros_like(W), np.concatenate([wstar, np.arctanh(dstar) / cfg["alpha_t"]]))
    X = data["xyz"].astype(np.float64)
    target = X @ Rotation.from_rotvec(wstar).as_matrix().T + dstar
    data = dict(data, pts=np.concatenate([target, target]), frame_off=np.array([0, 40, 80]))
    fw = O.forward(p, data, cfg)
    np.testing.assert_allclose(fw["xhat"][0], target, atol=1e-14)
    ls = O.losses(fw, data, cfg, 0, 3)
    assert np.all(ls["cd"] < 1e-26)
    grads, _ = O.backward(p, data, cfg, fw, ls)
    assert np.abs(O.flatten_params(grads)).max() < 1e-12


def test_chamfer_against_double_loop_and_kdtree():
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(8)
    X = rng.normal(size=(23, 3))
    P = rng.normal(size=(17, 3))
    a, b, da, db, cd = O.chamfer(X, P, block=5)
    for i in range(23):
        best, bj = np.inf, -1
        for j in range(17):
            d = sum((X[i, k] - P[j, k]) ** 2 for k in range(3))
            if d < best:
                best, bj = d, j
        assert a[i] == bj and abs(da[i] - best) < 1e-15
    for j in range(17):
        best, bi = np.inf, -1
        for i in range(23):
            d = sum((X[i, k] - P[j, k]) ** 2 for k in range(3))
            if d < best:
                best, bi = d, i
        assert b[j] == bi and abs(db[j] - best) < 1e-15
    assert abs(cd - (da.mean() + db.mean())) < 1e-15
    # distances agree with a k-d tree on a larger set
    X = rng.normal(size=(500, 3))
    P = rng.normal(size=(300, 3))
    _, _, da, db, _ = O.chamfer(X, P, block=64)
    np.testing.assert_allclose(da, cKDTree(P).query(X)[0] ** 2, rtol=1e-12)
    np.testing.assert_allclose(db, cKDTree(X).query(P)[0] ** 2, rtol=1e-12)


def test_chamfer_closed_forms_and_ties():
    rng = np.random.default_rng(9)
    X = rng.normal(size=(30, 3))
    assert O.chamfer(X, X)[4] == 0.0
    perm = rng.permutation(30)
    P = rng.normal(size=(30, 3))
    assert abs(O.chamfer(X, P)[4] - O.chamfer(X, P[perm])[4]) < 1e-14
    c = np.array([0.3, -0.4, 1.2])
    assert abs(O.chamfer(X[:1], X[:1] + c)[4] - 2 * (c @ c)) < 1e-14
    # exact ties pick the lowest index in both directions
    Xt = np.array([[0.0, 0, 0], [2.0, 0, 0]])
    Pt = np.array([[1.0, 0, 0], [1.0, 0, 0], [-1.0, 0, 0]])
    a, b, *_ = O.chamfer(Xt, Pt)
    assert list(a) == [0, 0] and list(b) == [0, 0, 0]


def test_confidence_worked_example_and_invariants():
    # Hand-worked example (tests/golden/confidence_example.json).
    import json
    import os
    ex = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "confidence_example.json")))
    w = O.confidence(np.array(ex["cd"]), ex["t_key"], ex["epoch"], ex["n_epochs"])
    np.testing.assert_allclose(w, ex["w"], rtol=1e-6)
    rng = np.random.default_rng(10)
    cd = rng.uniform(0, 1, 9)
    for e in range(5):
        w = O.confidence(cd, 3, e, 5)
        assert w[3] == 1.0 and np.all(w > 0) and np.all(w <= 1)
        assert np.all(np.diff(w[3:]) <= 0) and np.all(np.diff(w[:4]) >= 0)
    np.testing.assert_array_equal(O.confidence(cd, 3, 5, 5), np.ones(9))   # delta = 0
    np.testing.assert_array_equal(O.confidence(cd, 3, 2, 5, enabled=False), np.ones(9))


def test_metrics_closed_forms():
    # Sec. 4 metrics (readings): identity, a small rigid shift, flipped and
    # perpendicular normals, and a hand-counted F-score
    X, _, _ = synth.meshes.icosphere(2)
    N = X.copy()
    gt, gn = X[None], N[None]
    m = O.metrics(gt, gn, gt, gn, 0.01)[0]
    np.testing.assert_allclose(m, [0.0, 1.0, 1.0, 0.0], atol=1e-15)
    spacing = min(np.linalg.norm(X[i] - X[j]) for i in range(10) for j in range(len(X)) if i != j)
    d = np.array([0.3, -0.2, 0.1]) * spacing / 10
    m = O.metrics(gt + d, -gn, gt, gn, np.linalg.norm(d) * 1.01)[0]
    np.testing.assert_allclose(m, [2 * (d @ d), 1.0, 1.0, np.linalg.norm(d)], rtol=1e-12)
    assert O.metrics(gt + d, gn, gt, gn, np.linalg.norm(d) * 0.99)[0][2] == 0.0
    perp = np.cross(gn[0], np.array([0.0, 0.0, 1.0]) + 0.3)
    perp /= np.linalg.norm(perp, axis=1, keepdims=True)
    assert O.metrics(gt, perp[None], gt, gn, 0.01)[0][1] < 1e-15
    # 4 predicted points at distances 0, 0.5, 0.5, 2 from 4 true ones on a line
    g = np.array([[0, 0, 0], [10, 0, 0], [20, 0, 0], [30, 0, 0]], float)
    x = g + np.array([[0, 0, 0], [0, 0.5, 0], [0, -0.5, 0], [0, 2, 0]], float)
    _, _, F, corr = O.metrics(x[None], np.ones((1, 4, 3)), g[None], np.ones((1, 4, 3)), 1.0)[0]
    assert F == 0.75 and corr == 0.75  # P = R = 3/4; mean distance (0 + .5 + .5 + 2)/4


def test_metrics_against_double_loops():
    rng = np.random.default_rng(9)
    x = rng.normal(size=(2, 30, 3))
    g = rng.normal(size=(2, 30, 3))
    nx = rng.normal(size=(2, 30, 3))
    ng = rng.normal(size=(2, 30, 3))
    tau = 0.4
    m = O.metrics(x, nx, g, ng, tau)
    for t in range(2):
        da = [min(((x[t, i] - g[t, j]) ** 2).sum() for j in range(30)) for i in range(30)]
        ai = [min(range(30), key=lambda j: ((x[t, i] - g[t, j]) ** 2).sum()) for i in range(30)]
        db = [min(((g[t, j] - x[t, i]) ** 2).sum() for i in range(30)) for j in range(30)]
        bj = [min(range(30), key=lambda i: ((g[t, j] - x[t, i]) ** 2).sum()) for j in range(30)]
        nc = 0.5 * (sum(abs(nx[t, i] @ ng[t, ai[i]]) for i in range(30)) / 30
                    + sum(abs(ng[t, j] @ nx[t, bj[j]]) for j in range(30)) / 30)
        P = sum(v < tau * tau for v in da) / 30
        R = sum(v < tau * tau for v in db) / 30
        np.testing.assert_allclose(m[t], [np.mean(da) + np.mean(db), nc, 2 * P * R / (P + R),
                                          np.mean(np.linalg.norm(x[t] - g[t], axis=1))], rtol=1e-12)


def test_deformed_normals_of_a_known_rotation():
    # last layer zero with bias omega*: every normal turns by R(omega*) (scipy)
    cfg = synth.config_small(V=40, T=2, N=40)
    data = synth.make_workload(cfg)
    p = O.to64(synth.init_params(cfg))
    np.testing.assert_array_equal(O.deformed_normals(O.forward(p, data, cfg), data["nrm"])[1],
                                  data["nrm"].astype(np.float64))
    wstar = np.array([0.3, -0.2, 0.5])
    W, b = p["mlp"][-1]
    p["mlp"][-1] = (np.zeros_like(W), np.concatenate([wstar, np.zeros(3)]))
    n = O.deformed_normals(O.forward(p, data, cfg), data["nrm"])
    np.testing.assert_allclose(n[0], data["nrm"] @ Rotation.from_rotvec(wstar).as_matrix().T, atol=1e-14)


def test_bf16_rounding_matches_torch_and_its_definition():
    # against torch's float32 -> bfloat16 cast (round to nearest even) on
    # float32 inputs, including ties and both signs
    rng = np.random.default_rng(8)
    x = np.concatenate([rng.normal(size=2000) * 10.0 ** rng.integers(-20, 20, 2000),
                        [1.0, -1.0, 1.00390625, 1.01171875, 1.0 + 2 ** -9, 1.0 + 3 * 2 ** -9, 0.0, 3.0e38,
                         1e-40, -5e-39, 1e-38, 2.0 ** -126]])
    x32 = x.astype(np.float32)
    ref = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(O.bf16_round(x32.astype(np.float64)), ref)
    # 8 significant bits: relative rounding error <= 2^-8 for normal numbers;
    # representable values are fixed points
    y = O.bf16_round(x)
    nz = np.abs(x) >= 2.0 ** -126
    assert np.all(np.abs(y[nz] - x[nz]) <= 2.0 ** -8 * np.abs(x[nz]))
    np.testing.assert_array_equal(O.bf16_round(y), y)


def test_bf16_forward_reduces_to_fp32_on_representable_operands():
    # with grids, decoder input and weights already bfloat16 values and
    # activations that stay representable, the BF16 form equals the plain one
    cfg = synth.config_small(act="relu", time_freqs=0)
    data = synth.make_workload(cfg)
    p = O.to64(synth.random_state(cfg, 3))
    p = dict(grid_p=[O.bf16_round(g) for g in p["grid_p"]], grid_n=O.bf16_round(p["grid_n"]),
             mlp=[(O.bf16_round(W), b) for W, b in p["mlp"]])
    a = O.forward(p, data, dict(cfg, precision="bf16"))
    b = O.forward(p, data, cfg)
    assert np.abs(a["xhat"] - b["xhat"]).max() < 1e-2          # activations were rounded
    np.testing.assert_array_equal(a["ins"][1], O.bf16_round(a["ins"][1]))
    # a single linear layer of bf16 values: exact agreement
    W = O.bf16_round(np.random.default_rng(1).normal(size=(6, 5)))
    Y = O.bf16_round(np.random.default_rng(2).normal(size=(7, 5)))
    o1 = O.mlp_forward([(W, np.zeros(6))], Y, "relu", 0.0, bf16=True)[0]
    np.testing.assert_array_equal(o1, Y @ W.T)
