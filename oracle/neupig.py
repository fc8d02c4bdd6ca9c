"""FP64 oracle of the Neu-PiG optimization step (test infrastructure only).

Section references are to the paper (Neu-PiG, arXiv 2602.22212):
  Sec. 3   problem statement (reference mesh with normals, per-frame clouds)
  Sec. 3.1 initialization
  Sec. 3.2 multi-resolution latent grids (level average, normal grid)
  Sec. 3.3 temporal deformation model (decoder input, Fourier time code, MLP)
  Sec. 3.4 transformation mapping (rotation head, tanh displacement, apply)
  Sec. 3.5 optimization objectives (preconditioned update, deformation loss,
           confidence weight, implementation details)
  Supp. "Rotation Modeling" / Table 11: exponential-map rotation head.
  Sec. 3.4 "Rotation Component": quaternion rotation head (rot_head "quat").
  Sec. 4 "Evaluation Metrics": CD, NC, F-score, correspondence error (the
           paper names them only; the definitions below are readings).

Parameter structure (float64 numpy):
  params = dict(grid_p=[G_l of shape [R_l^3, F] per level],
                grid_n=G_n of shape [Rn^3, Fn],
                mlp=[(W [out,in], b [out]) per layer])
Grid node (ix, iy, iz) of a level with R nodes per axis is row
(iz*R + iy)*R + ix; ix follows the first coordinate.
"""
import numpy as np
import scipy.fft

__all__ = [
    "grid_coords", "trilinear", "trilinear_backward", "encode", "encode_backward",
    "time_code", "decoder_input", "mlp_forward", "mlp_backward", "rodrigues",
    "transform", "transform_backward", "chamfer", "confidence", "forward",
    "backward", "laplacian_apply", "precond_dct", "precond_cg", "precondition",
    "adam", "step", "to64", "zeros_like_params", "flatten_params", "losses",
    "chamfer_backward", "quat_matrix", "quat_normalize", "n_outputs", "iso_loss", "iso_backward", "iso_signs",
    "deformed_normals", "metrics", "bf16_round",
]


def to64(params):
    return dict(grid_p=[np.asarray(g, np.float64) for g in params["grid_p"]],
                grid_n=np.asarray(params["grid_n"], np.float64),
                mlp=[(np.asarray(W, np.float64), np.asarray(b, np.float64)) for W, b in params["mlp"]])


def zeros_like_params(p):
    return dict(grid_p=[np.zeros_like(g) for g in p["grid_p"]], grid_n=np.zeros_like(p["grid_n"]),
                mlp=[(np.zeros_like(W), np.zeros_like(b)) for W, b in p["mlp"]])


def flatten_params(p):
    """Concatenate all blocks (levels, normal grid, then W_k, b_k per layer)."""
    parts = [g.ravel() for g in p["grid_p"]] + [p["grid_n"].ravel()]
    for W, b in p["mlp"]:
        parts += [W.ravel(), b.ravel()]
    return np.concatenate(parts)


# --------------------------------------------------------------------------
# Sec. 3.2: trilinear interpolation in a grid spanning [-1,1]^3 whose corner
# nodes sit on +-1. Coordinates outside are clamped to the box; the cell index
# is capped at R-2 so a coordinate on the upper face uses the last cell with
# fraction 1.
# --------------------------------------------------------------------------
def grid_coords(X, R):
    u = (np.clip(X, -1.0, 1.0) + 1.0) * 0.5 * (R - 1)
    i0 = np.minimum(np.floor(u).astype(np.int64), R - 2)
    return i0, u - i0


def _corners(X, R):
    """Yield (node index [n], weight [n]) for the 8 cell corners."""
    i0, f = grid_coords(X, R)
    for cz in (0, 1):
        for cy in (0, 1):
            for cx in (0, 1):
                w = ((f[:, 0] if cx else 1.0 - f[:, 0]) *
                     (f[:, 1] if cy else 1.0 - f[:, 1]) *
                     (f[:, 2] if cz else 1.0 - f[:, 2]))
                node = ((i0[:, 2] + cz) * R + (i0[:, 1] + cy)) * R + (i0[:, 0] + cx)
                yield node, w


def trilinear(G, R, X):
    out = np.zeros((len(X), G.shape[1]))
    for node, w in _corners(X, R):
        out += w[:, None] * G[node]
    return out


def trilinear_backward(gout, R, X, F):
    gG = np.zeros((R ** 3, F))
    for node, w in _corners(X, R):
        np.add.at(gG, node, w[:, None] * gout)
    return gG


# --------------------------------------------------------------------------
# Mixed-precision form (BF16): bfloat16 keeps 8 significant bits (7 stored)
# of a binary32 number with the same exponent range; rounding is to nearest,
# ties to even. The BF16 form rounds every MLP matrix operand (the gathered
# grid features, the decoder input, weights, hidden activations and the
# back-propagated gradients fed to the matrix products) and accumulates in
# full precision; biases, the first layer's sums and everything outside the
# MLP stay unrounded.
# --------------------------------------------------------------------------
def bf16_round(x):
    """Round to the nearest bfloat16 (8-bit significand, ties to even; below
    the smallest normal 2^-126 the spacing stays 2^-133, as in binary32)."""
    x = np.asarray(x, np.float64)
    _, e = np.frexp(x)                      # x = m 2^e, 0.5 <= |m| < 1
    q = np.maximum(e, -125) - 8             # spacing 2^q of the bfloat16 grid at x
    return np.ldexp(np.round(np.ldexp(x, -q)), q)


def encode(params, X, Nrm, levels, res_n, bf16=False):
    """Sec. 3.2: z_p = (1/L) sum_l trilinear(G_p^l, x); z_n = trilinear(G_n, n).
    With bf16 the gathered features are rounded to bfloat16.

    Returns z = [z_n, z_p] per vertex (normal part first, the decoder's
    input order of Sec. 3.3)."""
    L = len(levels)
    rd = bf16_round if bf16 else (lambda a: a)
    zp = sum(trilinear(rd(G), R, X) for G, R in zip(params["grid_p"], levels)) / L
    zn = trilinear(rd(params["grid_n"]), res_n, Nrm)
    return np.concatenate([zn, zp], axis=1)


def encode_backward(gz, X, Nrm, levels, res_n, Fp, Fn):
    L = len(levels)
    gzn, gzp = gz[:, :Fn], gz[:, Fn:]
    gp = [trilinear_backward(gzp / L, R, X, Fp) for R in levels]
    gn = trilinear_backward(gzn, res_n, Nrm, Fn)
    return gp, gn


# --------------------------------------------------------------------------
# Sec. 3.3: Fourier time code on 0-based frames, t~ = t/(T-1) (0 for T = 1),
# gamma = [sin(pi 2^(j-1) t~), cos(pi 2^(j-1) t~)] for j = 1..M, kept in that
# interleaved order. M = 0 selects the scalar code [t~].
# --------------------------------------------------------------------------
def time_code(T, M):
    tt = np.arange(T, dtype=np.float64) / (T - 1) if T > 1 else np.zeros(1)
    if M == 0:
        return tt[:, None]
    cols = []
    for j in range(1, M + 1):
        nu = 2.0 ** (j - 1)
        cols += [np.sin(np.pi * nu * tt), np.cos(np.pi * nu * tt)]
    return np.stack(cols, axis=1)


def decoder_input(z, gamma):
    """Sec. 3.3: y_{i,t} = (z_n, z_p, gamma(t)); rows ordered t-major
    (row t*V + i)."""
    T, V = len(gamma), len(z)
    return np.concatenate([np.tile(z, (T, 1)), np.repeat(gamma, V, axis=0)], axis=1)


def _act(x, kind, slope):
    if kind == "relu":
        return np.maximum(x, 0.0)
    return np.where(x > 0, x, slope * x)


def _act_grad(pre, kind, slope):
    if kind == "relu":
        return (pre > 0).astype(np.float64)
    return np.where(pre > 0, 1.0, slope)


def mlp_forward(mlp, Y, act, slope, bf16=False):
    """Sec. 3.3 "Network Architecture": hidden Linear+activation layers, then a
    linear output layer. Returns (output, list of pre-activations, list of
    layer inputs). With bf16 every layer input and weight is rounded to
    bfloat16 (biases are not)."""
    rd = bf16_round if bf16 else (lambda a: a)
    h = Y
    pres, ins = [], []
    for k, (W, b) in enumerate(mlp):
        h = rd(h)
        ins.append(h)
        pre = h @ rd(W).T + b
        if k < len(mlp) - 1:
            pres.append(pre)
            h = _act(pre, act, slope)
        else:
            h = pre
    return h, pres, ins


def mlp_backward(mlp, go, pres, ins, act, slope, bf16=False):
    """Reverse-mode derivative of mlp_forward. Returns ([(gW, gb)], gY).
    With bf16 the gradient entering each matrix product of layers 2.. is
    rounded to bfloat16 (weight gradient and back-propagation), as are the
    weights; bias gradients and the first layer's weight gradient (a sum
    over samples of the unrounded gradient times the rounded input) and its
    input gradient use the unrounded gradient."""
    rd = bf16_round if bf16 else (lambda a: a)
    grads = [None] * len(mlp)
    g = go
    for k in range(len(mlp) - 1, -1, -1):
        W, _ = mlp[k]
        gm = rd(g) if k > 0 else g
        grads[k] = (gm.T @ ins[k], g.sum(0))
        g = gm @ rd(W)
        if k > 0:
            g = g * _act_grad(pres[k - 1], act, slope)
    return grads, g


# --------------------------------------------------------------------------
# Sec. 3.4 with the exponential-map head of the rotation study (Table 11):
# R = exp([omega]_x) by Rodrigues' formula; d^ = tanh(alpha d);
# x^ = R x + d^. Below theta = 1e-4 the two Rodrigues coefficients use their
# Taylor series.
# --------------------------------------------------------------------------
def _coeffs(theta):
    small = theta < 1e-4
    th = np.where(small, 1.0, theta)
    A = np.where(small, 1.0 - theta ** 2 / 6.0, np.sin(th) / th)
    B = np.where(small, 0.5 - theta ** 2 / 24.0, (1.0 - np.cos(th)) / th ** 2)
    C = np.where(small, 1.0 / 6.0 - theta ** 2 / 120.0, (th - np.sin(th)) / th ** 3)
    return A, B, C


def _hat(w):
    z = np.zeros(w.shape[:-1])
    return np.stack([np.stack([z, -w[..., 2], w[..., 1]], -1),
                     np.stack([w[..., 2], z, -w[..., 0]], -1),
                     np.stack([-w[..., 1], w[..., 0], z], -1)], -2)


def rodrigues(omega):
    theta = np.linalg.norm(omega, axis=-1)
    A, B, _ = _coeffs(theta)
    K = _hat(omega)
    I = np.broadcast_to(np.eye(3), K.shape)
    return I + A[..., None, None] * K + B[..., None, None] * (K @ K)


def _transform_expmap(o, X, alpha):
    """o [..., 6] = (omega, d); X [..., 3] -> x^ = R(omega) X + tanh(alpha d)."""
    R = rodrigues(o[..., :3])
    dh = np.tanh(alpha * o[..., 3:])
    return np.einsum("...ab,...b->...a", R, X) + dh, R, dh


def _transform_expmap_backward(g, o, X, R, dh, alpha):
    """Derivative of the exp-map transform w.r.t. o. For the rotation part,
    d(R x) = -R [x]_x J_r(omega) d omega (right Jacobian of SO(3)), so the
    gradient is J_r^T (x cross (R^T g))."""
    omega = o[..., :3]
    theta = np.linalg.norm(omega, axis=-1)
    _, B, C = _coeffs(theta)
    u = np.einsum("...ba,...b->...a", R, g)            # R^T g
    c = np.cross(X, u)
    K = _hat(omega)
    Jr = np.broadcast_to(np.eye(3), K.shape) - B[..., None, None] * K + C[..., None, None] * (K @ K)
    gw = np.einsum("...ba,...b->...a", Jr, c)          # J_r^T c
    gd = alpha * (1.0 - dh ** 2) * g
    return np.concatenate([gw, gd], axis=-1)


# --------------------------------------------------------------------------
# Sec. 3.4 quaternion head (the paper's default): the network's first four
# outputs (q_w, q_x, q_y, q_z) become the unit quaternion
# u = (1 + q_w, q_x, q_y, q_z) / |(1 + q_w, q_x, q_y, q_z)| (zero output gives
# the identity), R(u) is the rotation matrix of u, d^ = tanh(alpha d) from the
# last three outputs, x^ = R(u) x + d^.
# --------------------------------------------------------------------------
def quat_normalize(q):
    """q [..., 4] raw outputs -> (u [..., 4] unit quaternion (w, x, y, z), norm)."""
    a = np.array(q, dtype=np.float64, copy=True)
    a[..., 0] += 1.0
    n = np.linalg.norm(a, axis=-1)
    return a / n[..., None], n


def quat_matrix(u):
    """Rotation matrix of the unit quaternion u = (w, x, y, z), entry by entry."""
    w, x, y, z = u[..., 0], u[..., 1], u[..., 2], u[..., 3]
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], -2)


def _quat_matrix_partials(u):
    """d quat_matrix / d (w, x, y, z) [..., 4, 3, 3]: the entry-wise partial
    derivatives of the polynomial matrix above."""
    w, x, y, z = u[..., 0], u[..., 1], u[..., 2], u[..., 3]
    o = np.zeros_like(w)
    m = lambda *rows: 2.0 * np.stack([np.stack(r, -1) for r in rows], -2)
    dw = m((o, -z, y), (z, o, -x), (-y, x, o))
    dx = m((o, y, z), (y, -2 * x, -w), (z, w, -2 * x))
    dy = m((-2 * y, x, w), (x, o, z), (-w, z, -2 * y))
    dz = m((-2 * z, -w, x), (w, -2 * z, y), (x, y, o))
    return np.stack([dw, dx, dy, dz], -3)


def _transform_quat(o, X, alpha):
    u, _ = quat_normalize(o[..., :4])
    R = quat_matrix(u)
    dh = np.tanh(alpha * o[..., 4:7])
    return np.einsum("...ab,...b->...a", R, X) + dh, R, dh


def _transform_quat_backward(g, o, X, R, dh, alpha):
    """Chain rule through the normalisation: with u = a/|a|, du/da =
    (I - u u^T)/|a|; d(g . R(u) x)/du_k = g^T (dR/du_k) x."""
    u, n = quat_normalize(o[..., :4])
    gu = np.einsum("...a,...kab,...b->...k", g, _quat_matrix_partials(u), X)
    gq = (gu - u * (u * gu).sum(-1, keepdims=True)) / n[..., None]
    gd = alpha * (1.0 - dh ** 2) * g
    return np.concatenate([gq, gd], axis=-1)


def n_outputs(head):
    """Network outputs of each rotation head: exp map (omega, d) or quaternion (q, d)."""
    return {"expmap": 6, "quat": 7}[head]


def transform(o, X, alpha, head="expmap"):
    """x^ = R X + tanh(alpha d) for either rotation head; returns (x^, R, d^)."""
    return (_transform_quat if head == "quat" else _transform_expmap)(o, X, alpha)


def transform_backward(g, o, X, R, dh, alpha, head="expmap"):
    """d (g . x^) / d o for either rotation head."""
    return (_transform_quat_backward if head == "quat" else _transform_expmap_backward)(g, o, X, R, dh, alpha)


# --------------------------------------------------------------------------
# Sec. 3.5 "Deformation Loss": bidirectional squared-L2 Chamfer distance per
# frame, mean over each direction, nearest neighbours chosen with the lowest
# index on exact ties.
# --------------------------------------------------------------------------
def chamfer(Xh, P, block=2048):
    V, N = len(Xh), len(P)
    a = np.empty(V, np.int64)
    da = np.empty(V)
    db = np.full(N, np.inf)
    b = np.zeros(N, np.int64)
    for s in range(0, V, block):
        D = ((Xh[s:s + block, None, :] - P[None, :, :]) ** 2).sum(-1)
        a[s:s + block] = D.argmin(1)
        da[s:s + block] = D[np.arange(len(D)), a[s:s + block]]
        j = D.argmin(0)
        m = D[j, np.arange(N)]
        upd = m < db
        db[upd] = m[upd]
        b[upd] = j[upd] + s
    cd = da.mean() + db.mean()
    return a, b, da, db, cd


def confidence(cd, t_key, epoch, n_epochs, enabled=True):
    """Sec. 3.5 confidence weight: omega(tau) = 1/(1 + max(0, cd_tau - cd_key)),
    w(t) = prod over tau between t_key and t (inclusive) of omega(tau)^delta,
    delta = 1 - sqrt(epoch / n_epochs), epoch 0-based."""
    T = len(cd)
    if not enabled:
        return np.ones(T)
    delta = 1.0 - np.sqrt(epoch / n_epochs)
    om = 1.0 / (1.0 + np.maximum(0.0, cd - cd[t_key]))
    w = np.empty(T)
    for t in range(T):
        lo, hi = min(t, t_key), max(t, t_key)
        w[t] = np.prod(om[lo:hi + 1] ** delta)
    return w


# --------------------------------------------------------------------------
# Sec. 3.5 "Isometry Loss": mean over frames and mesh edges of
# | |x^_i,t - x^_j,t| - sg(|x^_i,key - x^_j,key|) |, the key-frame lengths taken
# from the current deformed key frame under a stop-gradient. The total
# objective is L_def + w_iso L_iso. Subgradients: sign(0) = 0 (so the key
# frame's own terms contribute no gradient); a zero-length edge contributes 0.
# --------------------------------------------------------------------------
def _edge_lengths(xhat, edges):
    d = xhat[:, edges[:, 0]] - xhat[:, edges[:, 1]]          # [T, E, 3]
    return d, np.sqrt((d * d).sum(-1))


def iso_loss(xhat, edges, t_key):
    """xhat [T, V, 3], edges [E, 2] -> L_iso (float)."""
    T, E = xhat.shape[0], len(edges)
    _, ell = _edge_lengths(xhat, edges)
    return float(np.abs(ell - ell[t_key][None]).sum() / (T * E))


def iso_signs(xhat, edges, t_key):
    """sign(|e_t| - |e_key|) per frame and edge [T, E]: the subgradient
    decisions of the L1 isometry term."""
    _, ell = _edge_lengths(xhat, edges)
    return np.sign(ell - ell[t_key][None])


def iso_backward(xhat, edges, t_key, sign=None):
    """d L_iso / d x^ [T, V, 3] with the key-frame lengths held fixed. `sign`
    ([T, E], values -1/0/+1) replaces the float64 decisions of iso_signs, so a
    caller can evaluate the gradient with decisions taken in another
    precision."""
    T, E = xhat.shape[0], len(edges)
    d, ell = _edge_lengths(xhat, edges)
    s = iso_signs(xhat, edges, t_key) if sign is None else np.asarray(sign, np.float64)
    coef = np.where(ell > 0, s / np.where(ell > 0, ell, 1.0), 0.0) / (T * E)
    g = np.zeros_like(xhat)
    tt = np.repeat(np.arange(T), E)
    np.add.at(g, (tt, np.tile(edges[:, 0], T)), (coef[..., None] * d).reshape(-1, 3))
    np.add.at(g, (tt, np.tile(edges[:, 1], T)), -(coef[..., None] * d).reshape(-1, 3))
    return g


def forward(params, data, cfg):
    """Forward pass over all frames. data: xyz [V,3], nrm [V,3], pts [sum N,3],
    frame_off [T+1]."""
    X = np.asarray(data["xyz"], np.float64)
    Nrm = np.asarray(data["nrm"], np.float64)
    T = len(data["frame_off"]) - 1
    V = len(X)
    bf16 = cfg.get("precision", "fp32") == "bf16"
    z = encode(params, X, Nrm, cfg["levels"], cfg["res_n"], bf16)
    gamma = time_code(T, cfg["time_freqs"])
    Y = decoder_input(z, gamma)
    o, pres, ins = mlp_forward(params["mlp"], Y, cfg["act"], cfg["leaky_slope"], bf16)
    Xt = np.tile(X, (T, 1))
    xh, R, dh = transform(o, Xt, cfg["alpha_t"], cfg.get("rot_head", "expmap"))
    return dict(z=z, gamma=gamma, Y=Y, o=o, pres=pres, ins=ins, R=R, dh=dh,
                xhat=xh.reshape(T, V, 3), Xt=Xt)


def losses(fw, data, cfg, epoch, n_epochs):
    P = np.asarray(data["pts"], np.float64)
    off = data["frame_off"]
    T = len(off) - 1
    res = [chamfer(fw["xhat"][t], P[off[t]:off[t + 1]]) for t in range(T)]
    cd = np.array([r[4] for r in res])
    t_key = cfg["t_key"] if cfg["t_key"] is not None else (T - 1) // 2
    w = confidence(cd, t_key, epoch, n_epochs, bool(cfg["conf_weight"]))
    loss = float(np.mean(w * cd))
    iso = 0.0
    if cfg.get("w_iso", 0.0) > 0:
        iso = iso_loss(fw["xhat"], np.asarray(data["edges"]), t_key)
        loss += cfg["w_iso"] * iso
    return dict(a=[r[0] for r in res], b=[r[1] for r in res], da=[r[2] for r in res],
                db=[r[3] for r in res], cd=cd, w=w, loss=loss, iso=iso, t_key=t_key)


def chamfer_backward(xhat, P, off, a, b, w):
    """d loss / d x^ with the assignments and the weights held fixed:
    (w_t/T) [ (2/V)(x^_i - p_{a_i}) + (2/N_t) sum_{j: b_j = i} (x^_i - p_j) ]."""
    T, V, _ = xhat.shape
    g = np.zeros_like(xhat)
    for t in range(T):
        Pt = P[off[t]:off[t + 1]]
        Nt = len(Pt)
        gt = (2.0 / V) * (xhat[t] - Pt[a[t]])
        acc = np.zeros((V, 3))
        np.add.at(acc, b[t], xhat[t][b[t]] - Pt)
        g[t] = (w[t] / T) * (gt + (2.0 / Nt) * acc)
    return g


def backward(params, data, cfg, fw, ls, iso_sign=None):
    """Gradient of the loss w.r.t. every parameter block (Sec. 3.5 objective,
    derivative written out stage by stage); iso_sign as in iso_backward."""
    P = np.asarray(data["pts"], np.float64)
    X = np.asarray(data["xyz"], np.float64)
    Nrm = np.asarray(data["nrm"], np.float64)
    T, V, _ = fw["xhat"].shape
    gx = chamfer_backward(fw["xhat"], P, data["frame_off"], ls["a"], ls["b"], ls["w"])
    if cfg.get("w_iso", 0.0) > 0:
        gx = gx + cfg["w_iso"] * iso_backward(fw["xhat"], np.asarray(data["edges"]), ls["t_key"], iso_sign)
    go = transform_backward(gx.reshape(T * V, 3), fw["o"], fw["Xt"], fw["R"], fw["dh"], cfg["alpha_t"],
                            cfg.get("rot_head", "expmap"))
    gmlp, gY = mlp_backward(params["mlp"], go, fw["pres"], fw["ins"], cfg["act"], cfg["leaky_slope"],
                            cfg.get("precision", "fp32") == "bf16")
    Fz = cfg["feat_n"] + cfg["feat_p"]
    gz = gY[:, :Fz].reshape(T, V, Fz).sum(0)
    gp, gn = encode_backward(gz, X, Nrm, cfg["levels"], cfg["res_n"], cfg["feat_p"], cfg["feat_n"])
    return dict(grid_p=gp, grid_n=gn, mlp=gmlp), dict(gxhat=gx, go=go, gz=gz)


# --------------------------------------------------------------------------
# Sec. 3.5 "Preconditioning": g~ = (I + lambda L)^-2 g per grid level and per
# feature channel, with L the combinatorial Laplacian (degree minus adjacency)
# of the 6-neighbour node lattice with free boundary.
# --------------------------------------------------------------------------
def laplacian_apply(p, R):
    """(L p) for p of shape [R^3, F], as sums of differences along lattice edges."""
    F = p.shape[1]
    q = p.reshape(R, R, R, F)          # [iz, iy, ix, f]
    out = np.zeros_like(q)
    for ax in range(3):
        d = np.diff(q, axis=ax)         # p[n+1] - p[n] along this axis
        sl_lo = [slice(None)] * 4
        sl_hi = [slice(None)] * 4
        sl_lo[ax] = slice(0, R - 1)
        sl_hi[ax] = slice(1, R)
        out[tuple(sl_lo)] -= d
        out[tuple(sl_hi)] += d
    return out.reshape(R ** 3, F)


def precond_dct(g, R, lam):
    """Exact (I + lam L)^-2 g. The free-boundary path-graph Laplacian has the
    DCT-II vectors as eigenvectors with eigenvalues 2 - 2 cos(pi k / R); the
    lattice Laplacian is their Kronecker sum, so the orthonormal 3-D DCT-II
    diagonalises the operator."""
    F = g.shape[1]
    q = g.reshape(R, R, R, F)
    k = np.arange(R)
    mu1 = 2.0 - 2.0 * np.cos(np.pi * k / R)
    mu = mu1[:, None, None] + mu1[None, :, None] + mu1[None, None, :]
    s = 1.0 / (1.0 + lam * mu) ** 2
    c = scipy.fft.dctn(q, type=2, norm="ortho", axes=(0, 1, 2), workers=-1)
    c *= s[..., None]
    return scipy.fft.idctn(c, type=2, norm="ortho", axes=(0, 1, 2), workers=-1).reshape(R ** 3, F)


def precond_cg(g, R, lam, rtol=1e-13, maxit=10000):
    """Second path: two conjugate-gradient solves with (I + lam L), per channel,
    from a zero start. Returns (result, iterations of each solve)."""
    def solve(b):
        x = np.zeros_like(b)
        r = b.copy()
        p = r.copy()
        rr = (r * r).sum(0)
        bb = np.sqrt(rr)
        it = 0
        while it < maxit:
            active = np.sqrt(rr) > rtol * bb
            if not active.any():
                break
            q = p + lam * laplacian_apply(p, R)
            pq = (p * q).sum(0)
            alpha = np.where(active, rr / np.where(active, pq, 1.0), 0.0)
            x += alpha * p
            r -= alpha * q
            rr_new = (r * r).sum(0)
            beta = np.where(active, rr_new / np.where(active, rr, 1.0), 0.0)
            p = r + beta * p
            rr = rr_new
            it += 1
        return x, it

    y, i1 = solve(g)
    x, i2 = solve(y)
    return x, (i1, i2)


def precondition(grads, cfg, method="dct"):
    """Apply the preconditioner to every grid block (levels and normal grid);
    the MLP gradient is left unchanged."""
    f = precond_dct if method == "dct" else (lambda g, R, lam: precond_cg(g, R, lam)[0])
    gp = [f(g, R, lam) for g, R, lam in zip(grads["grid_p"], cfg["levels"], cfg["lam"])]
    gn = f(grads["grid_n"], cfg["res_n"], cfg["lam_n"])
    return dict(grid_p=gp, grid_n=gn, mlp=grads["mlp"])


# --------------------------------------------------------------------------
# Sec. 3.5 "Implementation Details": Adam with default parameters, bias
# corrected, step count k 1-based.
# --------------------------------------------------------------------------
def adam(theta, g, m, v, k, lr, b1, b2, eps):
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** k)
    vh = v / (1.0 - b2 ** k)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def _lr_blocks(cfg):
    return dict(grid_p=list(cfg["lr_grid"]), grid_n=cfg["lr_n"], mlp=cfg["lr_mlp"])


def step(params, m, v, k, data, cfg, epoch, n_epochs, precond="dct", iso_sign=None):
    """One full optimization step (forward, loss, backward, preconditioning,
    Adam). k is the 1-based Adam step count of this update; iso_sign as in
    iso_backward. Returns (params, m, v, diagnostics)."""
    fw = forward(params, data, cfg)
    ls = losses(fw, data, cfg, epoch, n_epochs)
    grads, aux = backward(params, data, cfg, fw, ls, iso_sign)
    pg = precondition(grads, cfg, precond)
    b1, b2, eps = cfg["beta1"], cfg["beta2"], cfg["eps"]
    lrs = _lr_blocks(cfg)
    np_, nm, nv = {}, {}, {}
    res = [adam(th, g, mm, vv, k, lr, b1, b2, eps)
           for th, g, mm, vv, lr in zip(params["grid_p"], pg["grid_p"], m["grid_p"], v["grid_p"], lrs["grid_p"])]
    np_["grid_p"] = [r[0] for r in res]
    nm["grid_p"] = [r[1] for r in res]
    nv["grid_p"] = [r[2] for r in res]
    np_["grid_n"], nm["grid_n"], nv["grid_n"] = adam(params["grid_n"], pg["grid_n"], m["grid_n"],
                                                     v["grid_n"], k, lrs["grid_n"], b1, b2, eps)
    np_["mlp"], nm["mlp"], nv["mlp"] = [], [], []
    for (W, b), (gW, gb), (mW, mb), (vW, vb) in zip(params["mlp"], pg["mlp"], m["mlp"], v["mlp"]):
        W2, mW2, vW2 = adam(W, gW, mW, vW, k, lrs["mlp"], b1, b2, eps)
        b2_, mb2, vb2 = adam(b, gb, mb, vb, k, lrs["mlp"], b1, b2, eps)
        np_["mlp"].append((W2, b2_))
        nm["mlp"].append((mW2, mb2))
        nv["mlp"].append((vW2, vb2))
    diag = dict(fw=fw, ls=ls, grads=grads, pgrads=pg, aux=aux)
    return np_, nm, nv, diag


# --------------------------------------------------------------------------
# Sec. 4 "Evaluation Metrics" on ground truth (readings; the paper gives the
# names only). Predicted normals are the reference normals turned by each
# vertex's predicted rotation. Per frame t, with nearest neighbours a (from
# the prediction into the truth) and b (from the truth into the prediction):
#   CD   = mean_i |x^_i - g_a_i|^2 + mean_j |g_j - x^_b_j|^2
#   NC   = (mean_i |n^_i . m_a_i| + mean_j |m_j . n^_b_j|) / 2
#   F    = 2 P R / (P + R), P = share of i with |x^_i - g_a_i| < tau,
#          R = share of j with |g_j - x^_b_j| < tau (0 when P + R = 0)
#   Corr = mean_i |x^_i - g_i| (each vertex against its own true position)
# --------------------------------------------------------------------------
def deformed_normals(fw, Nrm):
    """R_i,t n_i for every frame and vertex [T, V, 3] from a forward pass."""
    T, V, _ = fw["xhat"].shape
    n = np.einsum("sab,sb->sa", fw["R"], np.tile(np.asarray(Nrm, np.float64), (T, 1)))
    return n.reshape(T, V, 3)


def metrics(xhat, nhat, gt, gt_n, tau):
    """Per-frame (CD, NC, F, Corr) [T, 4] of predicted vertices/normals
    against true vertices/normals [T, V, 3] (same vertex order)."""
    out = []
    for t in range(len(xhat)):
        a, b, da, db, cd = chamfer(xhat[t], gt[t])
        nc = 0.5 * (np.abs((nhat[t] * gt_n[t][a]).sum(1)).mean() + np.abs((gt_n[t] * nhat[t][b]).sum(1)).mean())
        prec = (da < tau * tau).mean()
        rec = (db < tau * tau).mean()
        f = 2 * prec * rec / (prec + rec) if prec + rec > 0 else 0.0
        corr = np.linalg.norm(xhat[t] - gt[t], axis=1).mean()
        out.append((cd, nc, f, corr))
    return np.array(out)
