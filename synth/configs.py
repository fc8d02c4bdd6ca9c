"""Hyper-parameter sets for the synthetic workloads.

Every value here is an input handed to both the oracle and the HIP library.
Level indices are 1-based when read against the paper's schedules
(Sec. 3.5, "Implementation Details": per-level learning rate 0.005*2.5^l and
smoothness 0.4*1.5^l, with Table 7 naming the base level lambda^1 = 0.4).
"""
import copy


def _geometric_res(r0, r1, levels):
    # Nodes per axis growing geometrically from r0 to r1 (grid corners on +-1).
    if levels == 1:
        return [r1]
    g = (r1 / r0) ** (1.0 / (levels - 1))
    return [int(round(r0 * g ** l)) for l in range(levels)]


def _base(**kw):
    cfg = dict(
        name="custom",
        levels=[8, 16, 32, 64],     # nodes per axis of each position-grid level
        feat_p=2,                   # features per position-grid node
        res_n=4, feat_n=2,          # normal-direction grid (Sec. 3.2: 4^3, 2-dim)
        time_freqs=0,               # 0 = scalar normalised time, else M Fourier freqs
        mlp_hidden=2, mlp_width=64, # hidden layers and their width
        act="relu", leaky_slope=0.01,
        alpha_t=0.1,                # displacement squashing tanh(alpha d)
        rot_head="expmap",          # "expmap" (6 outputs) or "quat" (7 outputs)
        w_iso=0.0,                  # isometry-loss weight (paper: 100); 0 = off
        precision="fp32",           # "fp32" or "bf16" (MLP matrix operands in bfloat16)
        lr_mlp=1e-3,
        lr_grid=None, lr_n=0.005,
        lam=None, lam_n=0.4,
        beta1=0.9, beta2=0.999, eps=1e-8,
        conf_weight=1, t_key=None,
        cg_rtol=1e-7, cg_maxit=400,
        cg_mg=1,                    # CG form: 1 = multigrid-preconditioned solves, 0 = plain CG
        n_steps=10,
        grid_init_std=0.0,
    )
    cfg.update(kw)
    L = len(cfg["levels"])
    if cfg["lr_grid"] is None:
        cfg["lr_grid"] = [0.005 * 2.5 ** l for l in range(L)]
    if cfg["lam"] is None:
        cfg["lam"] = [0.4 * 1.5 ** l for l in range(L)]
    return cfg


def config_c1():
    """Oracle-size parity workload: icosphere, 10 frames, 4 levels 8..64, F=2."""
    return _base(name="c1_icosphere", levels=[8, 16, 32, 64], feat_p=2,
                 time_freqs=0, mlp_hidden=2, mlp_width=64, act="relu",
                 t_key=4, n_steps=10, grid_init_std=1e-4,
                 seed=1, V=2562, T=10, N=2048)


def config_c2():
    """Human-scale headline workload: 30k vertices, 100 frames, 10k points."""
    return _base(name="c2_human", levels=_geometric_res(16, 256, 8), feat_p=4,
                 time_freqs=4, mlp_hidden=3, mlp_width=128, act="leaky",
                 t_key=None, n_steps=500, grid_init_std=0.0,
                 seed=2, V=30000, T=100, N=10000)


def config_c3():
    """Long quadruped sequence: 50k vertices, 1000 frames, ~7.6k points."""
    return _base(name="c3_quadruped", levels=_geometric_res(16, 256, 8), feat_p=4,
                 time_freqs=4, mlp_hidden=3, mlp_width=128, act="leaky",
                 t_key=None, n_steps=500, grid_init_std=0.0,
                 seed=3, V=50000, T=1000, N=8000, drop=0.05)


def config_c5(n_seq=16, seed=5, scale=1.0):
    """Batched sequences: n_seq independent sequences, each with its own
    headline-shaped grids and MLP in the BF16 form, human and quadruped
    alternating; V ~ U[5k, 60k], T ~ U[20, 400] and N_t ~ U[4k, 16k] drawn
    per frame (`scale` shrinks V, T and N for tests)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_seq):
        V = max(64, int(rng.integers(5000, 60001) * scale))
        T = max(2, int(rng.integers(20, 401) * scale))
        N = [max(16, int(n * scale)) for n in rng.integers(4000, 16001, size=T)]
        shape = "human" if k % 2 == 0 else "quadruped"
        out.append(_base(name=f"c5_{k:02d}_{shape}", shape=shape, levels=_geometric_res(16, 256, 8), feat_p=4,
                         time_freqs=4, mlp_hidden=3, mlp_width=128, act="leaky", t_key=None, n_steps=500,
                         grid_init_std=0.0, seed=500 + k, V=V, T=T, N=N, precision="bf16"))
    return out


def config_small(**kw):
    """Tiny sizes for finite-difference and multi-tile tests."""
    cfg = _base(name="small", levels=[3, 4, 5], feat_p=2, time_freqs=2,
                mlp_hidden=2, mlp_width=8, act="leaky", t_key=1, n_steps=3,
                grid_init_std=0.1, seed=11, V=60, T=3, N=50)
    cfg.update(kw)
    L = len(cfg["levels"])
    if len(cfg["lr_grid"]) != L:
        cfg["lr_grid"] = [0.005 * 2.5 ** l for l in range(L)]
    if len(cfg["lam"]) != L:
        cfg["lam"] = [0.4 * 1.5 ** l for l in range(L)]
    return cfg


def config_by_name(name):
    return {"c1": config_c1, "c2": config_c2, "c3": config_c3,
            "small": config_small}[name]()


def with_overrides(cfg, **kw):
    out = copy.deepcopy(cfg)
    out.update(kw)
    return out
