"""Seeded workloads (reference mesh + per-frame target clouds) and parameter init.

Recipes (all seeded with numpy's default_rng):
  icosphere: 2562-vertex unit icosphere, exact normals; each frame warps the
      unit sphere by a sinusoidal radial bend y -> y (1 + 0.1 sin(2 pi y_z + phi_t)),
      then rotates it by up to 30 degrees about a random axis and translates it
      by up to 0.2 (uniform in a ball); targets are points drawn uniformly on
      the sphere and warped the same way.
  human / quadruped: capsule figures (14 / 13 capsules) sampled on their union
      surface; seeded smooth joint-angle trajectories (three sinusoids per
      joint axis, |angle| <= 45 deg) drive linear-blend skinning of a dense
      rest-surface sample set; each frame draws its target points from that
      set and adds Gaussian noise of 0.002 x the bounding-box diagonal.
      Everything is scaled into [-0.9, 0.9]^3 by the rest pose's bounding box.
"""
import numpy as np

from .meshes import icosphere, capsule_figure, FIGURES


def _rot_xyz(ax, ay, az):
    """Rotation matrices from intrinsic x-y-z Euler angles, batched over frames."""
    cx, sx = np.cos(ax), np.sin(ax)
    cy, sy = np.cos(ay), np.sin(ay)
    cz, sz = np.cos(az), np.sin(az)
    one, zero = np.ones_like(ax), np.zeros_like(ax)
    Rx = np.stack([np.stack([one, zero, zero], -1), np.stack([zero, cx, -sx], -1),
                   np.stack([zero, sx, cx], -1)], -2)
    Ry = np.stack([np.stack([cy, zero, sy], -1), np.stack([zero, one, zero], -1),
                   np.stack([-sy, zero, cy], -1)], -2)
    Rz = np.stack([np.stack([cz, -sz, zero], -1), np.stack([sz, cz, zero], -1),
                   np.stack([zero, zero, one], -1)], -2)
    return Rx @ Ry @ Rz


def _rot_axis_angle_quat(axis, ang):
    """Rotation matrix through the unit quaternion (cos a/2, sin a/2 * axis)."""
    w = np.cos(ang / 2)
    x, y, z = np.sin(ang / 2) * axis
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _sphere_workload(cfg, rng):
    V_, _, E = icosphere(4)
    T, N = cfg["T"], cfg["N"]
    pts, truth, truth_n = [], [], []
    for t in range(T):
        ang = np.deg2rad(rng.uniform(0, 30))
        axis = rng.normal(size=3)
        axis /= np.linalg.norm(axis)
        Rm = _rot_axis_angle_quat(axis, ang)
        d = rng.normal(size=3)
        d *= 0.2 * rng.random() ** (1 / 3) / np.linalg.norm(d)
        phi = rng.uniform(0, 2 * np.pi)

        def warp(Y):
            Y = Y * (1.0 + 0.1 * np.sin(2 * np.pi * Y[:, 2:3] + phi))
            return Y @ Rm.T + d

        def warp_normal(Y, Nn):
            # normals map by the inverse transpose of the bend's Jacobian
            # J = f I + y (df/dy_z) e_z^T, then rotate
            f = 1.0 + 0.1 * np.sin(2 * np.pi * Y[:, 2] + phi)
            df = 0.1 * 2 * np.pi * np.cos(2 * np.pi * Y[:, 2] + phi)
            J = f[:, None, None] * np.eye(3) + np.einsum("va,b->vab", Y * df[:, None], np.array([0.0, 0.0, 1.0]))
            n = np.linalg.solve(np.swapaxes(J, 1, 2), Nn[..., None])[..., 0]
            n /= np.linalg.norm(n, axis=1, keepdims=True)
            return n @ Rm.T

        S = rng.normal(size=(N, 3))
        S /= np.linalg.norm(S, axis=1, keepdims=True)
        pts.append(warp(S))
        truth.append(warp(V_))
        truth_n.append(warp_normal(V_, V_))
    return dict(xyz=V_, nrm=V_.copy(), pts_list=pts, truth=np.stack(truth), truth_nrm=np.stack(truth_n), edges=E)


def _figure_workload(cfg, rng, kind, want_truth=False):
    J, C = FIGURES[kind]()
    V, T = cfg["V"], cfg["T"]
    Ns = list(cfg["N"]) if isinstance(cfg["N"], (list, tuple)) else [cfg["N"]] * T
    X, Nrm, own = capsule_figure(kind, V, rng)
    dense, _, dense_own = capsule_figure(kind, max(200_000, 4 * max(Ns)), rng)
    lo, hi = X.min(0), X.max(0)
    c = 0.5 * (lo + hi)
    s = 0.9 / (0.5 * (hi - lo)).max()
    diag = np.linalg.norm((hi - lo) * s)

    # joint-angle trajectories: 3 sinusoids per joint axis, |angle| <= 45 deg
    nj = len(J)
    tt = np.arange(T) / max(T, 1)
    freqs = np.array([0.5, 1.0, 2.0])
    A = np.deg2rad(rng.uniform(0, 15, size=(nj, 3, 3)))
    ph = rng.uniform(0, 2 * np.pi, size=(nj, 3, 3))
    ang = (A[None] * np.sin(2 * np.pi * freqs[None, None, None] * tt[:, None, None, None]
                            + ph[None])).sum(-1)            # [T, nj, 3]
    root_shift = 0.1 * np.stack([np.sin(2 * np.pi * tt + rng.uniform(0, 6.3)) for _ in range(3)], -1)

    # forward kinematics in rest-pose coordinates
    Rg = np.zeros((T, nj, 3, 3))
    tg = np.zeros((T, nj, 3))
    for j, (_, p, cj) in enumerate(J):
        cj = np.asarray(cj, float)
        Rl = _rot_xyz(ang[:, j, 0], ang[:, j, 1], ang[:, j, 2])     # [T,3,3]
        tl = cj - np.einsum("tab,b->ta", Rl, cj)
        if p < 0:
            Rg[:, j] = Rl
            tg[:, j] = tl + root_shift
        else:
            Rg[:, j] = Rg[:, p] @ Rl
            tg[:, j] = np.einsum("tab,tb->ta", Rg[:, p], tl) + tg[:, p]

    # skinning weights of the dense set: softmax over the 4 nearest capsules
    dist = np.stack([_seg(dense, a, b) - r for a, b, r, _ in C], 1)     # [M, nc]
    top = np.argsort(dist, 1)[:, :4]
    dtop = np.take_along_axis(dist, top, 1)
    w = np.exp(-(dtop - dtop[:, :1]) / 0.02)
    w /= w.sum(1, keepdims=True)
    cap_joint = np.array([jj for *_, jj in C])
    jtop = cap_joint[top]                                                # [M,4]

    pts = []
    drop = cfg.get("drop", 0.0)
    for t in range(T):
        N = Ns[t]
        sel = rng.choice(len(dense), size=N, replace=False)
        if drop > 0:
            sel = sel[rng.random(N) >= drop]
        P = dense[sel]
        Q = np.zeros_like(P)
        for k in range(4):
            jk = jtop[sel, k]
            Q += w[sel, k:k + 1] * (np.einsum("nab,nb->na", Rg[t, jk], P) + tg[t, jk])
        Q = (Q - c) * s + rng.normal(scale=0.002 * diag, size=Q.shape)
        pts.append(Q)
    truth = truth_n = None
    if want_truth:
        # the reference vertices skinned like the dense set (no noise): true
        # positions and normals (weight-blended rotations, renormalised)
        dX = np.stack([_seg(X, a, b) - r for a, b, r, _ in C], 1)
        topX = np.argsort(dX, 1)[:, :4]
        dtX = np.take_along_axis(dX, topX, 1)
        wX = np.exp(-(dtX - dtX[:, :1]) / 0.02)
        wX /= wX.sum(1, keepdims=True)
        jX = cap_joint[topX]
        truth = np.zeros((T, len(X), 3))
        truth_n = np.zeros((T, len(X), 3))
        for t in range(T):
            for k in range(4):
                Rk = Rg[t, jX[:, k]]
                truth[t] += wX[:, k:k + 1] * (np.einsum("nab,nb->na", Rk, X) + tg[t, jX[:, k]])
                truth_n[t] += wX[:, k:k + 1] * np.einsum("nab,nb->na", Rk, Nrm)
            truth[t] = (truth[t] - c) * s
        truth_n /= np.linalg.norm(truth_n, axis=-1, keepdims=True)
    return dict(xyz=(X - c) * s, nrm=Nrm, pts_list=pts, truth=truth, truth_nrm=truth_n, edges=knn_edges((X - c) * s))


def knn_edges(X, k=6):
    """Undirected edge list [E, 2] (i < j, sorted, unique) of the symmetrised
    k-nearest-neighbour graph of the points X: the connectivity used for
    reference vertex sets that come without faces."""
    from scipy.spatial import cKDTree
    V = len(X)
    k = min(k, V - 1)
    if k < 1:
        return np.zeros((0, 2), np.int64)
    _, nb = cKDTree(X).query(X, k + 1)
    e = np.stack([np.repeat(np.arange(V), k), nb[:, 1:].ravel()], 1)
    e.sort(axis=1)
    return np.unique(e, axis=0).astype(np.int64)


def _seg(P, a, b):
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    ab = b - a
    t = np.clip(((P - a) @ ab) / (ab @ ab), 0.0, 1.0)
    return np.linalg.norm(P - (a + t[:, None] * ab), axis=1)


def make_workload(cfg, T=None, truth=False):
    """Build the seeded workload of a config.

    Returns a dict with float32 arrays xyz [V,3], nrm [V,3], pts [sum N_t,3],
    int64 frame_off [T+1], int64 mesh edges [E,2] (icosphere faces' edges, else
    a symmetrised 6-nearest-neighbour graph of the vertices) and the config's
    frame count T. ``T`` truncates
    the sequence to its first T frames (same seed, same frames).
    Ground truth (the true per-frame positions and unit normals of the
    reference vertices, truth [T,V,3] and truth_nrm [T,V,3]) comes with the
    icosphere workload always and with the capsule figures when ``truth``.
    """
    rng = np.random.default_rng(cfg["seed"])
    name = cfg["name"]
    if name.startswith("c1") or cfg.get("shape") == "sphere":
        w = _sphere_workload(cfg, rng)
    elif name.startswith("c3") or cfg.get("shape") == "quadruped":
        w = _figure_workload(cfg, rng, "quadruped", truth)
    elif name.startswith("c2") or cfg.get("shape") == "human":
        w = _figure_workload(cfg, rng, "human", truth)
    else:
        w = _small_workload(cfg, rng)
    plist = w.pop("pts_list")
    if T is not None:
        plist = plist[:T]
        for k in ("truth", "truth_nrm"):
            if w.get(k) is not None:
                w[k] = w[k][:T]
    off = np.zeros(len(plist) + 1, np.int64)
    off[1:] = np.cumsum([len(p) for p in plist])
    w["pts"] = np.ascontiguousarray(np.concatenate(plist), dtype=np.float32)
    w["frame_off"] = off
    w["xyz"] = np.ascontiguousarray(w["xyz"], dtype=np.float32)
    w["nrm"] = np.ascontiguousarray(w["nrm"], dtype=np.float32)
    w["T"] = len(plist)
    return w


def _small_workload(cfg, rng):
    """Random oriented points in [-0.8,0.8]^3 and jittered copies as targets.

    Frame sizes may be ragged (cfg["N"] may be a list)."""
    V, T = cfg["V"], cfg["T"]
    X = rng.uniform(-0.8, 0.8, size=(V, 3))
    Nrm = rng.normal(size=(V, 3))
    Nrm /= np.linalg.norm(Nrm, axis=1, keepdims=True)
    Ns = cfg["N"] if isinstance(cfg["N"], (list, tuple)) else [cfg["N"]] * T
    pts = []
    for t in range(T):
        P = rng.uniform(-0.9, 0.9, size=(Ns[t], 3))
        pts.append(P)
    return dict(xyz=X, nrm=Nrm, pts_list=pts, truth=None, truth_nrm=None, edges=knn_edges(X))


def _out_dim(cfg):
    """Network outputs: rotation parameters (3 for the exp map, 4 for the
    quaternion head) plus the 3 displacement components."""
    return 7 if cfg.get("rot_head", "expmap") == "quat" else 6


def _in_dim(cfg):
    M = cfg["time_freqs"]
    return cfg["feat_n"] + cfg["feat_p"] + (2 * M if M > 0 else 1)


def init_params(cfg, seed=None):
    """Initial parameters (Sec. 3.1): grids zero or N(0, std); hidden layers
    uniform +-1/sqrt(fan_in); last layer weights and bias zero.

    Returns dict(grid_p=[float32 [R^3, F] per level], grid_n=float32 [Rn^3, Fn],
    mlp=[(W [out,in], b [out]) float32 per layer]).
    """
    rng = np.random.default_rng(cfg["seed"] + 1000 if seed is None else seed)
    std = cfg["grid_init_std"]
    F, Fn, Rn = cfg["feat_p"], cfg["feat_n"], cfg["res_n"]
    gp = [(rng.normal(scale=std, size=(R ** 3, F)) if std > 0 else np.zeros((R ** 3, F)))
          .astype(np.float32) for R in cfg["levels"]]
    gn = (rng.normal(scale=std, size=(Rn ** 3, Fn)) if std > 0 else np.zeros((Rn ** 3, Fn))).astype(np.float32)
    dims = [_in_dim(cfg)] + [cfg["mlp_width"]] * cfg["mlp_hidden"] + [_out_dim(cfg)]
    mlp = []
    for k in range(len(dims) - 1):
        fi, fo = dims[k], dims[k + 1]
        if k == len(dims) - 2:
            W = np.zeros((fo, fi))
            b = np.zeros(fo)
        else:
            bound = 1.0 / np.sqrt(fi)
            W = rng.uniform(-bound, bound, size=(fo, fi))
            b = rng.uniform(-bound, bound, size=fo)
        mlp.append((W.astype(np.float32), b.astype(np.float32)))
    return dict(grid_p=gp, grid_n=gn, mlp=mlp)


def random_state(cfg, seed, grid_std=0.1, last_scale=0.3):
    """A non-degenerate parameter state: random grids and a random last layer,
    so that every gradient block is non-zero (used by gradient checks)."""
    rng = np.random.default_rng(seed)
    p = init_params(cfg, seed=seed)
    p["grid_p"] = [rng.normal(scale=grid_std, size=g.shape).astype(np.float32) for g in p["grid_p"]]
    p["grid_n"] = rng.normal(scale=grid_std, size=p["grid_n"].shape).astype(np.float32)
    W, b = p["mlp"][-1]
    bound = last_scale / np.sqrt(W.shape[1])
    p["mlp"][-1] = (rng.uniform(-bound, bound, size=W.shape).astype(np.float32),
                    rng.uniform(-0.05, 0.05, size=b.shape).astype(np.float32))
    return p
