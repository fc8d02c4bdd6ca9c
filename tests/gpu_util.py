"""Helpers shared by the GPU parity tests (not collected by pytest)."""
import numpy as np

U32 = 2.0 ** -24  # float32 unit roundoff


def rel(a, b):
    """Norm-wise relative difference ||a - b|| / ||b|| (||b|| = 0: absolute)."""
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    nb = np.linalg.norm(b)
    d = np.linalg.norm(a - b)
    return d / nb if nb > 0 else d


def to_np(t):
    return t.detach().cpu().numpy()


def nn_check(X, P, a_gpu, b_gpu, block=4096):
    """Near-tie protocol for nearest-neighbour indices computed on the GPU.

    X, P are the float32 inputs the GPU used (promoted to float64 here); the
    float64 brute force gives the lowest-index argmins a_o, b_o. A GPU index
    may differ only when its float64 distance exceeds the best one by at most
    8 u d (u = 2^-24), the float32 rounding of the direct form. Returns
    (number of documented ties in rows, in columns); raises on any other
    difference."""
    X = np.asarray(X, np.float64)
    P = np.asarray(P, np.float64)
    V, N = len(X), len(P)
    a_gpu = np.asarray(a_gpu)
    b_gpu = np.asarray(b_gpu)
    assert a_gpu.min() >= 0 and a_gpu.max() < N and b_gpu.min() >= 0 and b_gpu.max() < V
    ties_a = ties_b = 0
    colbest = np.full(N, np.inf)
    colarg = np.zeros(N, np.int64)
    colgpu = np.zeros(N)
    for s in range(0, V, block):
        D = ((X[s:s + block, None, :] - P[None, :, :]) ** 2).sum(-1)
        ao = D.argmin(1)
        r = np.arange(len(D))
        dbest = D[r, ao]
        dg = D[r, a_gpu[s:s + block]]
        bad = a_gpu[s:s + block] != ao
        if bad.any():
            ok = dg[bad] - dbest[bad] <= 8 * U32 * dg[bad]
            assert ok.all(), f"row NN mismatch beyond the tie bound at vertices {np.flatnonzero(bad)[~ok][:5] + s}"
            ties_a += int(bad.sum())
        j = D.argmin(0)
        m = D[j, np.arange(N)]
        upd = m < colbest
        colbest[upd] = m[upd]
        colarg[upd] = j[upd] + s
        inblk = (b_gpu >= s) & (b_gpu < s + block)
        colgpu[inblk] = D[b_gpu[inblk] - s, np.flatnonzero(inblk)]
    bad = b_gpu != colarg
    if bad.any():
        ok = colgpu[bad] - colbest[bad] <= 8 * U32 * colgpu[bad]
        assert ok.all(), f"column NN mismatch beyond the tie bound at points {np.flatnonzero(bad)[~ok][:5]}"
        ties_b = int(bad.sum())
    return ties_a, ties_b


def gpu_plan(cfg, data):
    import paper_2602_22212_amd as npg
    return npg.plan_from_workload(cfg, data)


def flat_params(cfg, p):
    import torch

    import paper_2602_22212_amd as npg
    return torch.from_numpy(npg.pack_params(cfg, p)).cuda()


def block_rel(cfg, flat_gpu, structured_ref):
    """Per-block relative differences of a flat GPU vector vs structured ref."""
    import paper_2602_22212_amd as npg
    got = npg.unpack_params(cfg, np.asarray(flat_gpu))
    out = {}
    for l, (g, r) in enumerate(zip(got["grid_p"], structured_ref["grid_p"])):
        out[f"grid_p{l}"] = rel(g, r)
    out["grid_n"] = rel(got["grid_n"], structured_ref["grid_n"])
    for k, ((W, b), (Wr, br)) in enumerate(zip(got["mlp"], structured_ref["mlp"])):
        out[f"W{k}"] = rel(W, Wr)
        out[f"b{k}"] = rel(b, br)
    return out


def touched_nodes(cfg, data):
    """Nodes read by the grid lookup of some reference vertex (per grid:
    position levels, then the normal grid)."""
    import oracle as O
    X = data["xyz"].astype(np.float64)
    Nr = data["nrm"].astype(np.float64)
    out = []
    for R in list(cfg["levels"]) + [cfg["res_n"]]:
        Q = X if len(out) < len(cfg["levels"]) else Nr
        nodes = set()
        for node, _ in O.neupig._corners(Q, R):
            nodes.update(node.tolist())
        out.append(np.array(sorted(nodes)))
    return out


def f32_hyper(cfg):
    """The config with every hyper-parameter the C ABI carries as float32
    (learning rates, smoothness weights, Adam constants, activation slope,
    displacement scale) replaced by its float32 value, so that a float64
    oracle step runs the constants the library was given (1 - 0.999 and
    1 - float32(0.999) differ by 1.3e-5 relative)."""
    f = lambda x: float(np.float32(x))
    out = dict(cfg)
    for k in ("beta1", "beta2", "eps", "lr_mlp", "lr_n", "lam_n", "leaky_slope", "alpha_t"):
        out[k] = f(cfg[k])
    out["lr_grid"] = [f(x) for x in cfg["lr_grid"]]
    out["lam"] = [f(x) for x in cfg["lam"]]
    return out
