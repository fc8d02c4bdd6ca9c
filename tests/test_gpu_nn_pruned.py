"""The pruned nearest-neighbour search against the exhaustive one (needs a GPU).

Both searches are selected by the config's nn_search and must give the same
indices, distances and per-frame Chamfer sums bit for bit: the pruned search
skips only tiles whose every point is strictly farther than a query's
minimum, and takes the lowest original index among equal distances. Cases:
the human and quadruped workloads at the benchmark state and at the identity
start, exact ties placed across tile boundaries, and ragged sizes around the
tile (128 targets) and wave (256 queries) boundaries. The exact-tie case is
also compared with the oracle's lowest-index brute force.
"""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import flat_params, gpu_plan, to_np

pytestmark = pytest.mark.gpu


def _xhat(plan, cfg, params, T, V):
    import torch
    flat = flat_params(cfg, params)
    z = torch.empty(V * plan.Fz, dtype=torch.float32, device="cuda")
    xh = torch.empty(T * V * 4, dtype=torch.float32, device="cuda")
    plan.encode_fwd(flat, z)
    plan.decode_fwd(flat, z, xh)
    return xh


def _nn(plan, xh, T, V):
    import torch
    N = plan.Ntot
    out = dict(a=torch.empty(T * V, dtype=torch.int32, device="cuda"), da=torch.empty(T * V, device="cuda"),
               b=torch.empty(N, dtype=torch.int32, device="cuda"), db=torch.empty(N, device="cuda"),
               cd=torch.empty(T, dtype=torch.float64, device="cuda"))
    plan.chamfer_fwd(xh, out["a"], out["da"], out["b"], out["db"], out["cd"])
    torch.cuda.synchronize()
    return {k: to_np(v) for k, v in out.items()}


def _compare(cfg, data, xh_from=None, params=None, label=""):
    T, V = len(data["frame_off"]) - 1, len(data["xyz"])
    pr = gpu_plan(dict(cfg, nn_search="pruned"), data)
    ex = gpu_plan(dict(cfg, nn_search="exhaustive"), data)
    try:
        xh = xh_from if xh_from is not None else _xhat(pr, cfg, params, T, V)
        r_p = _nn(pr, xh, T, V)
        r_e = _nn(ex, xh, T, V)
        for k in ("a", "da", "b", "db", "cd"):
            np.testing.assert_array_equal(r_p[k], r_e[k], err_msg=f"{label}: {k}")
        print(f"{label}: T={T} V={V} N={pr.Ntot}: a, da, b, db, cd bitwise equal", flush=True)
        return r_p, xh
    finally:
        pr.close()
        ex.close()


@pytest.mark.parametrize("state", ["bench", "identity"])
def test_pruned_equals_exhaustive_human(state):
    cfg = synth.config_c2()
    data = synth.make_workload(cfg)
    p = synth.random_state(cfg, 9, grid_std=0.05) if state == "bench" else synth.init_params(cfg)
    _compare(cfg, data, params=p, label=f"human/{state}")


def test_pruned_equals_exhaustive_quadruped():
    cfg = synth.config_c3()
    data = synth.make_workload(cfg)
    _compare(cfg, data, params=synth.random_state(cfg, 9, grid_std=0.05), label="quadruped/bench")


def _lattice_case():
    # Points on a lattice of spacing 2^-4, vertices at cell centres and on
    # lattice nodes: every distance is exact in float32, a centre vertex has 8
    # nearest points at exactly equal distance and a node vertex coincides
    # with a point; duplicated points add equal distances at separate
    # indices. A random permutation of the points scatters equal-distance
    # points over different Morton tiles and index orders.
    rng = np.random.default_rng(7)
    h = 2.0 ** -4
    g = np.arange(-6, 7) * h
    P = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    P = np.concatenate([P, P[rng.choice(len(P), 300, replace=False)]])
    P = P[rng.permutation(len(P))].astype(np.float32)
    cells = (rng.integers(-6, 6, size=(200, 3)) + 0.5) * h
    nodes = rng.integers(-6, 7, size=(157, 3)) * h
    X = np.concatenate([cells, nodes]).astype(np.float32)
    return X, P


def test_exact_ties_across_tiles():
    X, P = _lattice_case()
    V = len(X)
    cfg = synth.config_small(mlp_width=32, V=V, T=2, N=[len(P), 129], t_key=0)
    data = synth.make_workload(cfg)
    data["xyz"] = X
    data["nrm"] = np.tile(np.array([[0, 0, 1]], np.float32), (V, 1))
    data["pts"] = np.concatenate([P, P[:129][::-1]]).astype(np.float32)
    data["frame_off"] = np.array([0, len(P), len(P) + 129])
    # identity start: x^ = x exactly in both frames
    r, xh = _compare(cfg, data, params=synth.init_params(cfg), label="lattice ties")
    xh = to_np(xh).reshape(2, V, 4)[..., :3]
    np.testing.assert_array_equal(xh[0], X)
    off = data["frame_off"]
    for t in range(2):
        Pt = data["pts"][off[t]:off[t + 1]].astype(np.float64)
        ao, bo, dao, dbo, _ = O.chamfer(X.astype(np.float64), Pt)
        np.testing.assert_array_equal(r["a"][t * V:(t + 1) * V], ao)
        np.testing.assert_array_equal(r["b"][off[t]:off[t + 1]], bo)
        np.testing.assert_array_equal(r["da"][t * V:(t + 1) * V], dao.astype(np.float32))
    D = ((X[:, None].astype(np.float64) - P[None].astype(np.float64)) ** 2).sum(-1)
    n_tied = int(((D == D.min(1, keepdims=True)).sum(1) > 1).sum())
    print("vertices with several nearest points at equal distance:", n_tied)
    assert n_tied > 100


@pytest.mark.parametrize("V,N", [(1, [1, 2]), (255, [127, 128, 129]), (256, [1, 300]), (257, [128, 257, 5]),
                                 (700, [1000, 1])])
def test_ragged_sizes(V, N):
    cfg = synth.config_small(mlp_width=32, V=V, T=len(N), N=N, t_key=0, seed=40 + V)
    data = synth.make_workload(cfg)
    _compare(cfg, data, params=synth.random_state(cfg, 3), label=f"ragged V={V} N={N}")
