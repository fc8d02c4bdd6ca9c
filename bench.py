"""Benchmark: optimization steps/sec of the full Neu-PiG step on one MI355X.

One step = encode, decode (MLP + transform), bidirectional NN Chamfer and
confidence-weighted loss, backward of all of them, Sobolev preconditioning
(two CG solves per grid, each preconditioned by a multigrid V-cycle) and
Adam, on the human workload: 30,000 reference
vertices, 100 frames, 10,000 points per frame, 8-level position grid 16..256
with 4 features, normal grid 4^3 x 2, MLP 14 -> 128 x 3 -> 6 (float32).
Inputs are resident in HBM before timing starts; the state is a seeded
non-degenerate one (random grids and last layer) so every stage does its
full work from the first timed step.

Prints one JSON line (see the keys below). `roofline` is measured live for
the dominant kernel group, the preconditioner's CG iteration (k_cg_dir_ap,
k_cg_update and the V-cycle kernels), with HIP events recorded on the plan's
stream; `cpu_baseline` times the FP64 oracle on a bounded sample of the same
workload.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# MI355X published peaks (dense): MFMA fp32 157.3 and bf16 2500 TFLOP/s; fp32
# vector 157.3 TFLOP/s with packed FP32, 78.6 without (this build disables
# packed FP32 code generation, so 78.6 is the issue limit its kernels have)
MFMA_PEAK_TFS = {"f32": 157.3, "bf16": 2500.0}
VALU_F32_PEAK_TFS, VALU_F32_UNPACKED_TFS = 157.3, 78.6

# The paper's own runtime at the metric's frame count (context only: other
# hardware, data and point counts; one step here is one epoch there)
PAPER_CONTEXT = {
    "hardware": "NVIDIA RTX 4090",
    "per_sequence_runtime_s": 97.0, "frames": 100, "epochs": 1000,
    "derived_ms_per_epoch": 97.0, "derived_epochs_per_s": 10.3,
    "source": "Table 2 (AMA split into 100-frame sequences); epoch count of the method's default setting",
    "note": "context only, not like-for-like (different GPU, data, point counts); vs_baseline stays null",
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-frames", type=int, default=2, help="frames in the oracle's timed sample")
    ap.add_argument("--forms", default="cg,nn,cg_plain,dct,graph,quat,iso,metrics,bf16,batch,animal",
                    help="forms to time: cg (headline: CG preconditioned by a multigrid V-cycle), "
                         "nn (the Chamfer forward with the pruned and the exhaustive nearest-neighbour search), "
                         "cg_plain (the same solves by plain CG), dct (exact DCT preconditioner), "
                         "graph (the DCT-form step replayed as one captured HIP graph, on the human "
                         "workload and on the small icosphere one, against the eager step), "
                         "quat (quaternion rotation head, DCT preconditioner), "
                         "iso (isometry loss w_iso = 100 on a 6-NN edge graph, DCT preconditioner), "
                         "metrics (inference export + evaluation metrics on ground truth), "
                         "bf16 (BF16 MLP form: CG steps/s and time-to-target against FP32), "
                         "batch (16 independent sequences stepped together, BF16 and FP32), "
                         "animal (quadruped workload: 50000 vertices, 1000 frames, CG)")
    ap.add_argument("--no-quality", action="store_true",
                    help="skip the 100-step BF16/FP32 quality comparison (for counter runs)")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default launch shapes (no autotuner runs; for counter runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="finish with one plain 1 GiB device copy (reference dispatch for HBM counters)")
    ap.add_argument("--cg-one-stream", action="store_true",
                    help="keep every CG launch on the plan's stream (cg_one_stream = 1: the same launches, "
                         "the grid groups one after the other; for per-dispatch counter runs, whose counts "
                         "are only attributable when no two kernels run at once)")
    return ap.parse_args()


def traffic_from_profile():
    """HBM bytes per preconditioned CG iteration (CG and V-cycle kernels) from the
    committed rocprofv3 counter summary, if it was taken on the current
    kernel source (its `precond.hip sha256` line names the source)."""
    path = os.path.join(ROOT, "profiles", "cg_iteration_human_pmc.md")
    src = os.path.join(ROOT, "paper_2602_22212_amd", "csrc", "precond.hip")
    try:
        text = open(path).read()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    m_sha = re.search(r"precond\.hip sha256: ([0-9a-f]{16})", text)
    m_val = re.search(r"hbm_bytes_per_iteration: ([0-9]+)", text)
    if not m_sha or not m_val or m_sha.group(1) != sha:
        return None
    return int(m_val.group(1))


def cpu_baseline(cfg, data, P0, frames):
    """Time the FP64 oracle step on the first `frames` frames of the same
    workload; frame-proportional stages are scaled to all frames."""
    import numpy as np

    import oracle as O
    T = len(data["frame_off"]) - 1
    off = data["frame_off"][: frames + 1]
    sub = dict(data, pts=data["pts"][: off[-1]], frame_off=off)
    c = dict(cfg, t_key=min(cfg["t_key"] or 0, frames - 1))
    P = O.to64(P0)
    t = {}
    t0 = time.perf_counter()
    fw = O.forward(P, sub, c)
    t["forward"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    ls = O.losses(fw, sub, c, 0, cfg["n_steps"])
    t["chamfer"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    g, _ = O.backward(P, sub, c, fw, ls)
    t["backward"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    pg = O.precondition(g, c, "dct")
    t["precond"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    z = O.zeros_like_params(P)
    for th, gg, lr in zip(P["grid_p"], pg["grid_p"], c["lr_grid"]):
        O.adam(th, gg, np.zeros_like(th), np.zeros_like(th), 1, lr, c["beta1"], c["beta2"], c["eps"])
    O.adam(P["grid_n"], pg["grid_n"], z["grid_n"], z["grid_n"], 1, c["lr_n"], c["beta1"], c["beta2"], c["eps"])
    for (W, b), (gW, gb) in zip(P["mlp"], pg["mlp"]):
        O.adam(W, gW, 0 * W, 0 * W, 1, c["lr_mlp"], c["beta1"], c["beta2"], c["eps"])
    t["adam"] = time.perf_counter() - t0
    scale = T / frames
    # the encode inside forward is frame independent but negligible next to the decode
    per_step = (t["forward"] + t["chamfer"] + t["backward"]) * scale + t["precond"] + t["adam"]
    threads = len(os.sched_getaffinity(0))
    return dict(value=1.0 / per_step, unit="steps/s", cores=threads, kind="oracle",
                sample=(f"FP64 oracle step on frames 0..{frames - 1} of the same human workload "
                        f"({frames} of {T} frames; all 30000 vertices, 8 grid levels, exact DCT "
                        f"preconditioner); forward, Chamfer and backward times scaled x{scale:g} to "
                        f"{T} frames, preconditioner and Adam as measured; measured {sum(t.values()):.1f} s"),
                stage_seconds={k: round(v, 3) for k, v in t.items()}, seconds_per_step=per_step)


def cpu_fast(cfg, data, P0, frames):
    """The fast-CPU baseline: the same FP64 oracle step with the nearest
    neighbours from scipy's cKDTree (exact nearest-neighbour distances, all
    host threads) instead of the brute-force search, on the same frame sample
    and with the same scaling as cpu_baseline."""
    import numpy as np
    from scipy.spatial import cKDTree

    import oracle as O
    T = len(data["frame_off"]) - 1
    off = data["frame_off"][: frames + 1]
    sub = dict(data, pts=data["pts"][: off[-1]], frame_off=off)
    c = dict(cfg, t_key=min(cfg["t_key"] or 0, frames - 1))
    P = O.to64(P0)
    pts = np.asarray(sub["pts"], np.float64)
    t = {}
    t0 = time.perf_counter()
    fw = O.forward(P, sub, c)
    t["forward"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    a, b, da, db, cd = [], [], [], [], []
    for f in range(frames):
        Pt = pts[off[f]:off[f + 1]]
        dA, iA = cKDTree(Pt).query(fw["xhat"][f], workers=-1)
        dB, iB = cKDTree(fw["xhat"][f]).query(Pt, workers=-1)
        a.append(iA)
        b.append(iB)
        da.append(dA * dA)
        db.append(dB * dB)
        cd.append(da[-1].mean() + db[-1].mean())
    cd = np.array(cd)
    w = O.confidence(cd, c["t_key"], 0, cfg["n_steps"], bool(cfg["conf_weight"]))
    ls = dict(a=a, b=b, da=da, db=db, cd=cd, w=w, loss=float(np.mean(w * cd)), iso=0.0, t_key=c["t_key"])
    t["chamfer_kdtree"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    g, _ = O.backward(P, sub, c, fw, ls)
    t["backward"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.precondition(g, c, "dct")
    t["precond"] = time.perf_counter() - t0
    scale = T / frames
    per_step = (t["forward"] + t["chamfer_kdtree"] + t["backward"]) * scale + t["precond"]
    return dict(value=1.0 / per_step, unit="steps/s", cores=len(os.sched_getaffinity(0)), kind="oracle+cKDTree",
                sample=(f"the oracle step on frames 0..{frames - 1} with scipy cKDTree nearest neighbours "
                        f"(workers=-1) in place of the brute-force search; forward, Chamfer and backward scaled "
                        f"x{scale:g} to {T} frames, DCT preconditioner as measured (Adam as in cpu_baseline, "
                        f"not repeated)"),
                stage_seconds={k: round(v, 3) for k, v in t.items()})


def keeps_activations(cfg, V, T):
    """Whether the library's step keeps the decoder's hidden activations of
    layers 2..H for its backward (the rule of plan creation: FP32 form, H > 1,
    at most 8 GiB), so that the backward does not recompute them."""
    W, H = cfg["mlp_width"], cfg["mlp_hidden"]
    return cfg.get("precision", "fp32") != "bf16" and H > 1 and V * T * (H - 1) * W * 4 <= (8 << 30)


def stage_roofline(cfg, data, stage_ms, precision, prof=None):
    """Per-stage algorithmic work over the measured stage time, against the
    roofline that bounds each stage: HBM bytes for the grid encode and its
    scatter, Adam and the CG preconditioner; MFMA FLOPs for the decoder (the
    backward: back-propagation and weight gradient, twice the forward's
    FLOPs; a recomputed forward is not counted, `recomputes_forward` says
    whether the step does one); FP32 vector FLOPs (10 per vertex-point pair
    and direction pair) for the nearest-neighbour Chamfer."""
    import paper_2602_22212_amd as npg
    V, T = len(data["xyz"]), data["T"]
    Ntot = int(data["frame_off"][-1])
    L, F, Fn = len(cfg["levels"]), cfg["feat_p"], cfg["feat_n"]
    W, H = cfg["mlp_width"], cfg["mlp_hidden"]
    n_out = 7 if cfg.get("rot_head", "expmap") == "quat" else 6
    Din = Fn + F + 2 * cfg["time_freqs"]
    S = V * T
    n_par = npg.param_count(cfg)
    n_grid = sum(R ** 3 * F for R in cfg["levels"]) + cfg["res_n"] ** 3 * Fn
    fl_fwd = 2.0 * S * ((H - 1) * W * W + n_out * W) + 2.0 * (V + T) * W * Din
    work = {
        "encode": ("hbm", V * (24 + (L * 8 * F + 8 * Fn) * 4 + 4 * (F + Fn))),
        "decode": ("mfma", fl_fwd),
        "chamfer+loss": ("alu", 10.0 * V * Ntot),
        "chamfer_bwd": ("hbm", T * V * 28 + Ntot * 16),
        "decode_bwd": ("mfma", 2 * fl_fwd),
        "encode_bwd": ("hbm", V * (F + Fn) * 4 + n_grid * 4),
        "adam": ("hbm", 28 * n_par),
    }
    if prof is not None and prof.get("cg_ms", 0) > 0:
        work["precond"] = ("hbm", prof["cg_bytes"] / max(1, prof.get("steps", 1)))
    out = {}
    for k, (bound, w) in work.items():
        ms = stage_ms.get(k, 0.0)
        if ms <= 0:
            continue
        if bound == "hbm":
            a = w / 1e9 / (ms / 1e3)
            out[k] = {"bound": "hbm", "algorithmic": round(w), "unit": "GB/s", "achieved": round(a, 1),
                      "peak": HBM_PEAK_GBS, "frac": round(a / HBM_PEAK_GBS, 4)}
        elif bound == "mfma":
            a = w / 1e12 / (ms / 1e3)
            pk = MFMA_PEAK_TFS[precision]
            out[k] = {"bound": "mfma", "dtype": precision, "algorithmic": w, "unit": "TFLOP/s", "achieved": round(a, 2),
                      "peak": pk, "frac": round(a / pk, 4)}
            if k == "decode_bwd":
                out[k]["recomputes_forward"] = not keeps_activations(cfg, V, T)
        else:
            a = w / 1e12 / (ms / 1e3)
            out[k] = {"bound": "alu", "algorithmic": w, "unit": "TFLOP/s", "achieved": round(a, 2),
                      "peak": VALU_F32_PEAK_TFS, "frac": round(a / VALU_F32_PEAK_TFS, 4),
                      "frac_of_unpacked_issue_limit": round(a / VALU_F32_UNPACKED_TFS, 4),
                      "search": cfg.get("nn_search", "pruned"),
                      "note": ("algorithmic work counts every vertex-point pair (10 FLOP each); the pruned "
                               "search evaluates only the tiles it cannot rule out, so its rate can exceed "
                               "the issue limit of the pairs it evaluates (nn_search gives both searches' "
                               "times)")}
    return out


TUNE = True  # autotune the launch shapes of every benchmarked plan (bench.py --no-tune: defaults)


def run_form(cfg, data, P0, steps, warmup, profile, graph=False):
    """Time `steps` full optimization steps of one form (graph: each step
    replayed as the captured HIP graph, npg_step_graph). Every step is
    bracketed by HIP events on the plan's stream (torch's current stream) and
    by host synchronisations; value = steps / summed wall time."""
    import numpy as np
    import torch

    import paper_2602_22212_amd as npg
    plan = npg.plan_from_workload(cfg, data)
    plan.set_state(torch.from_numpy(npg.pack_params(cfg, P0)).cuda(), adam_steps=0)
    # autotuned launch shapes: nearest-neighbour work-group size, decode
    # backward frame chunks, CG tile depth
    cgf = cfg.get("precond", "cg") == "cg"
    nn_threads, nn_ms = plan.tune_nn(0 if TUNE else 128)
    mlp_chunks, mlp_cand, mlp_ms = plan.tune_mlp(0) if TUNE else (None, [], [])
    cg_zs, cg_ms = (plan.tune_cg(0) if TUNE else (64, None)) if cgf else (None, None)
    E = cfg["n_steps"]
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    step = plan.step_graph if graph else plan.step
    for e in range(warmup):
        step(e, E, loss)
    torch.cuda.synchronize()
    if profile:
        plan.profile(True)
    stage_sum = {k: 0.0 for k in npg.STAGES}
    t_total = 0.0
    statuses = []
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for k in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev[k][0].record()
        statuses.append(step(warmup + k, E, loss))
        ev[k][1].record()
        torch.cuda.synchronize()
        t_total += time.perf_counter() - t0
        if not graph:  # the graph records no per-stage events
            for name, ms in plan.stage_times().items():
                stage_sum[name] += ms
    ev_ms = np.array([a.elapsed_time(b) for a, b in ev])
    prof = plan.profile_read() if profile else None
    if prof is not None:
        prof["steps"] = steps
    relres = plan.precond_residuals() if cfg.get("precond", "cg") == "cg" else None
    plan.close()
    print(f"bench: form precond={cfg.get('precond', 'cg')} precision={cfg.get('precision', 'fp32')} "
          f"graph={graph}: {1e3 * t_total / steps:.2f} ms per step", file=sys.stderr, flush=True)
    return dict(value=steps / t_total, ms_per_step=1e3 * t_total / steps,
                event_ms={"median": round(float(np.median(ev_ms)), 4), "p90": round(float(np.percentile(ev_ms, 90)), 4),
                          "min": round(float(ev_ms.min()), 4)},
                stage_ms=None if graph else {k: round(v / steps, 3) for k, v in stage_sum.items()},
                status=sorted(set(int(s) for s in statuses)), prof=prof, loss=loss.item(),
                nn_tune={"threads": nn_threads, "ms_64_128_256": [round(m, 3) for m in nn_ms],
                         "mlp_frame_chunks": mlp_chunks,
                         "mlp_ms": {str(c): round(m, 3) for c, m in zip(mlp_cand, mlp_ms) if c},
                         "cg_tile_z": cg_zs, "cg_ms_32_64_128": None if cg_ms is None else [round(m, 3) for m in cg_ms]},
                cg_relres_max=None if relres is None else max(relres))


def run_nn_compare(cfg, data, P0, reps=5):
    """The Chamfer forward (npg_chamfer_fwd: both nearest-neighbour directions
    and the per-frame sums) with the pruned and with the exhaustive search on
    the same deformed vertices, at the benchmark state and at the identity
    start (last layer zero: x^ = x); HIP events on the plans' stream. Both
    searches give bitwise the same indices and distances."""
    import numpy as np
    import torch

    import paper_2602_22212_amd as npg
    import synth
    T, V = data["T"], len(data["xyz"])
    plans = {m: npg.plan_from_workload(dict(cfg, nn_search=m), data) for m in ("pruned", "exhaustive")}
    out = {}
    for state, P in (("benchmark", P0), ("identity", synth.init_params(cfg))):
        flat = torch.from_numpy(npg.pack_params(cfg, P)).cuda()
        z = torch.empty(V * plans["pruned"].Fz, device="cuda")
        xh = torch.empty(T * V * 4, device="cuda")
        plans["pruned"].encode_fwd(flat, z)
        plans["pruned"].decode_fwd(flat, z, xh)
        res = {}
        for m, plan in plans.items():
            plan.set_state(flat, adam_steps=0)
            plan.tune_nn(0 if TUNE else 128)
            a = torch.empty(T * V, dtype=torch.int32, device="cuda")
            da = torch.empty(T * V, device="cuda")
            b = torch.empty(plan.Ntot, dtype=torch.int32, device="cuda")
            db = torch.empty(plan.Ntot, device="cuda")
            cd = torch.empty(T, dtype=torch.float64, device="cuda")
            plan.chamfer_fwd(xh, a, da, b, db, cd)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(reps):
                plan.chamfer_fwd(xh, a, da, b, db, cd)
            e1.record()
            torch.cuda.synchronize()
            res[m] = (e0.elapsed_time(e1) / reps, [x.cpu().numpy() for x in (a, da, b, db, cd)])
        same = all(np.array_equal(u, v) for u, v in zip(res["pruned"][1], res["exhaustive"][1]))
        out[state] = {"pruned_ms": round(res["pruned"][0], 3), "exhaustive_ms": round(res["exhaustive"][0], 3),
                      "speedup": round(res["exhaustive"][0] / res["pruned"][0], 2), "bitwise_equal": bool(same)}
    for plan in plans.values():
        plan.close()
    print("bench: nearest-neighbour searches compared", file=sys.stderr, flush=True)
    out["note"] = ("npg_chamfer_fwd on the human workload with nn_search = pruned (the step's search) and "
                   "exhaustive; stage_roofline's chamfer entry counts every vertex-point pair as algorithmic work")
    return out


def run_metrics(cfg, P0, reps=3):
    """Inference export (npg_predict) and the Sec. 4 metrics against the
    generator's ground truth, timed with HIP events (inputs resident)."""
    import numpy as np
    import torch

    import paper_2602_22212_amd as npg
    import synth
    data = synth.make_workload(cfg, truth=True)
    T, V = data["T"], len(data["xyz"])
    plan = npg.plan_from_workload(cfg, data)
    plan.set_state(torch.from_numpy(npg.pack_params(cfg, P0)).cuda(), adam_steps=0)
    gt = torch.from_numpy(np.concatenate([data["truth"], np.zeros((T, V, 1))], -1).astype(np.float32).ravel()).cuda()
    gn = torch.from_numpy(np.concatenate([data["truth_nrm"], np.zeros((T, V, 1))], -1).astype(np.float32).ravel()).cuda()
    tau = 0.005 * float(np.linalg.norm(data["xyz"].max(0) - data["xyz"].min(0)))
    xh = torch.empty(T * V * 4, device="cuda")
    nh = torch.empty(T * V * 4, device="cuda")
    out = torch.empty(T * 4, dtype=torch.float64, device="cuda")
    plan.predict(xh, nh)
    plan.metrics(xh, nh, gt, gn, tau, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.predict(xh, nh)
    torch.cuda.synchronize()
    t_pred = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.metrics(xh, nh, gt, gn, tau, out)
    t_met = (time.perf_counter() - t0) / reps
    m = out.cpu().numpy().reshape(T, 4).mean(0)
    plan.close()
    return {"predict_ms": round(1e3 * t_pred, 3), "metrics_ms": round(1e3 * t_met, 3), "tau": round(tau, 6),
            "mean_over_frames": {"CD": float(m[0]), "NC": float(m[1]), "F": float(m[2]), "Corr": float(m[3])},
            "note": ("npg_predict (vertices + normals of all frames) and npg_metrics (CD, NC, F-score at tau = "
                     "0.5% of the reference bounding-box diagonal, correspondence error; Sec. 4, readings) against "
                     "the generator's ground truth, at the seeded benchmark state; metrics_ms includes its "
                     "workspace allocation and final synchronisation")}


def run_quality(cfg, steps=300):
    """BF16 against FP32 on the headline workload: `steps` steps of each form
    from the paper's identity start (CG preconditioner, graph-replayed steps),
    the mean per-frame Chamfer distance of every step's forward pass (the
    step's own float64 sums), and, for targets set by the FP32 curve at a
    quarter, half and three quarters of the run, the steps and time each form
    needs to first reach them (the FP32 curve passes each target before its
    last step by construction). The final state of each form is evaluated
    once more on the host: float64 nearest-neighbour distances (scipy cKDTree,
    exact) on the deformed vertices of every frame."""
    import numpy as np
    import torch
    from scipy.spatial import cKDTree

    import paper_2602_22212_amd as npg
    import synth
    data = synth.make_workload(cfg)
    T, V = data["T"], len(data["xyz"])
    off = data["frame_off"]
    pts = data["pts"].astype(np.float64)
    out = {}
    for prec in ("fp32", "bf16"):
        print(f"bench: quality run {prec} ({steps} steps)", file=sys.stderr, flush=True)
        c = dict(cfg, precond="cg", precision=prec)
        plan = npg.plan_from_workload(c, data)
        plan.set_state(torch.from_numpy(npg.pack_params(c, synth.init_params(c))).cuda(), adam_steps=0)
        plan.tune_nn(0)
        cd = torch.empty(T, dtype=torch.float64, device="cuda")
        curve, t_total = [], 0.0
        for e in range(steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan.step_graph(e, steps, None, cd)
            torch.cuda.synchronize()
            t_total += time.perf_counter() - t0
            curve.append(float(cd.mean().item()))
        xh = torch.empty(T * V * 3, device="cuda")
        plan.deform(xh)
        torch.cuda.synchronize()
        xh = xh.cpu().numpy().reshape(T, V, 3).astype(np.float64)
        plan.close()
        fin = []
        for t in range(T):
            Pt = pts[off[t]:off[t + 1]]
            fin.append((cKDTree(Pt).query(xh[t], workers=-1)[0] ** 2).mean()
                       + (cKDTree(xh[t]).query(Pt, workers=-1)[0] ** 2).mean())
        out[prec] = dict(curve=curve, ms_per_step=1e3 * t_total / steps, final_cd=float(np.mean(fin)))
    marks = [steps // 4, steps // 2, (3 * steps) // 4]
    res = {"steps": steps, "start": "identity (the paper's init)", "preconditioner": "cg (V-cycle), graph-replayed",
           "note": ("mean per-frame Chamfer distance of each step's forward pass; targets = the FP32 curve at the "
                    "given step; steps_to_target = first step whose value is <= the target; time = that count x the "
                    "form's ms/step; final_cd = after the last update, float64 k-d tree distances on the host")}
    for prec, r in out.items():
        res[prec] = {"final_cd": r["final_cd"], "cd_at_last_step": r["curve"][-1],
                     "ms_per_step": round(r["ms_per_step"], 3)}
    res["targets"] = []
    for k in marks:
        tgt = out["fp32"]["curve"][k - 1]
        row = {"fp32_step": k, "target_cd": tgt}
        for prec, r in out.items():
            hit = next((j + 1 for j, v in enumerate(r["curve"]) if v <= tgt), None)
            row[prec] = {"steps_to_target": hit,
                         "time_to_target_s": None if hit is None else round(hit * r["ms_per_step"] / 1e3, 3)}
        res["targets"].append(row)
    mid = res["targets"][1]
    if mid["bf16"]["time_to_target_s"]:
        res["fp32_over_bf16_time_to_target"] = round(mid["fp32"]["time_to_target_s"] / mid["bf16"]["time_to_target_s"],
                                                      4)
    res["final_cd_ratio_bf16_over_fp32"] = round(out["bf16"]["final_cd"] / out["fp32"]["final_cd"], 5)
    return res


def _batch_time(cfgs, datas, steps, warmup, state, modes=("eager",)):
    """One batch of the sequences (autotuned once); for every timing mode
    ("eager": npg_batch_step; "graph": npg_batch_step_graph with each
    recording on its sequence's stream; "one_graph": one batch graph) the
    state is reset, `warmup` steps run, then `steps` are timed. Returns
    {mode: seconds per batch step}, the final mean Chamfer distances of the
    last mode, the tuned launch shapes and the step statuses."""
    import torch

    import paper_2602_22212_amd as npg
    import synth
    batch = npg.Batch(cfgs, datas)
    tuned, states = [], []
    for k, (c, p) in enumerate(zip(cfgs, batch.plans)):
        P = synth.random_state(c, 900 + k, grid_std=0.05) if state == "random" else synth.init_params(c)
        states.append(torch.from_numpy(npg.pack_params(c, P)).cuda())
        p.set_state(states[-1], adam_steps=0)
        cgf = c.get("precond", "cg") == "cg"
        tuned.append((p.tune_nn(0 if TUNE else 128)[0], p.tune_mlp(0)[0] if TUNE else None,
                      (p.tune_cg(0)[0] if TUNE else 64) if cgf else None))
    E = max(steps + warmup, 500)
    out, statuses = {}, set()
    for mode in modes:
        for p, st in zip(batch.plans, states):
            p.set_state(st, adam_steps=0)
        if mode != "eager":
            batch.graph_mode(mode == "graph")
        step = batch.step if mode == "eager" else batch.step_graph
        for e in range(warmup):
            step(e, E)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for e in range(steps):
            statuses.add(int(step(warmup + e, E)))
        torch.cuda.synchronize()
        out[mode] = (time.perf_counter() - t0) / steps
        print(f"bench: batch {mode} {1e3 * out[mode]:.1f} ms per batch step", file=sys.stderr, flush=True)
    final = [plan_cd(p) for p in batch.plans]
    batch.close()
    return out, final, tuned, sorted(statuses)


def plan_cd(plan):
    """Mean per-frame Chamfer distance at the plan's current parameters
    (the library's forward stages and float64 frame sums)."""
    import torch
    f = dict(device="cuda")
    params = plan.get_state()[0]
    z = torch.empty(plan.V * plan.Fz, **f)
    xh = torch.empty(plan.T * plan.V * 4, **f)
    plan.encode_fwd(params, z)
    plan.decode_fwd(params, z, xh)
    a = torch.empty(plan.T * plan.V, dtype=torch.int32, **f)
    da = torch.empty(plan.T * plan.V, **f)
    b = torch.empty(plan.Ntot, dtype=torch.int32, **f)
    db = torch.empty(plan.Ntot, **f)
    cd = torch.empty(plan.T, dtype=torch.float64, **f)
    plan.chamfer_fwd(xh, a, da, b, db, cd)
    torch.cuda.synchronize()  # the plan's stream may differ from torch's
    return float(cd.mean().item())


def run_batch(steps=3, warmup=2, quality_steps=20):
    """Batched sequences (16 independent sequences, survey config 5): one
    npg_batch_step advances every sequence by one step, concurrently; the
    BF16 form (default of the batch configs) and the FP32 form on the same
    sequences, and both forms from the identity start for quality_steps
    steps (DCT preconditioner) to compare their final Chamfer distances."""
    import numpy as np

    import synth
    cfgs = synth.config_c5()
    t0 = time.perf_counter()
    datas = []
    for c in cfgs:
        datas.append(synth.make_workload(c))
        print(f"bench: batch workload {len(datas)} of {len(cfgs)} generated", file=sys.stderr, flush=True)
    t_gen = time.perf_counter() - t0
    res = {}
    for prec in ("bf16", "fp32"):
        cs = [dict(c, precision=prec) for c in cfgs]
        t, _, tuned, st = _batch_time(cs, datas, steps, warmup, "random", modes=("eager", "graph", "one_graph"))
        tq, final, _, _ = _batch_time([dict(c, precond="dct") for c in cs], datas, quality_steps, 0, "init",
                                      modes=("eager",))
        res[prec] = dict(dt=t["graph"], d1=t["one_graph"], de=t["eager"], dq=tq["eager"], final=final, tuned=tuned,
                         status=st)
    pairs = sum(len(d["xyz"]) * int(d["frame_off"][-1]) for d in datas)
    samples = sum(len(d["xyz"]) * d["T"] for d in datas)
    b, f = res["bf16"], res["fp32"]
    ratio = float(np.mean(np.array(b["final"]) / np.array(f["final"])))
    return {"value": round(1.0 / b["de"], 4), "unit": "batch steps/s", "ms_per_step": round(1e3 * b["de"], 2),
            "timing": ("value: npg_batch_step (eager steps, one host thread and stream per sequence); "
                       "graph_per_stream: npg_batch_step_graph with each sequence's recorded step graph replayed on "
                       "its own stream (NPG_BATCH_GRAPH_PER_STREAM); one_graph: the same recordings as branches of "
                       "one batch graph (NPG_BATCH_ONE_GRAPH); all three bitwise equal"),
            "graph_per_stream": {"value": round(1.0 / b["dt"], 4), "ms_per_step": round(1e3 * b["dt"], 2)},
            "one_graph": {"value": round(1.0 / b["d1"], 4), "ms_per_step": round(1e3 * b["d1"], 2)},
            "fp32": {"value": round(1.0 / f["de"], 4), "ms_per_step": round(1e3 * f["de"], 2),
                     "graph_per_stream_value": round(1.0 / f["dt"], 4), "one_graph_value": round(1.0 / f["d1"], 4)},
            "bf16_over_fp32_steps_per_s": round(f["de"] / b["de"], 4),
            "quality": {"steps": quality_steps, "preconditioner": "dct", "start": "identity (the paper's init)",
                        "bf16_ms_per_step": round(1e3 * b["dq"], 2), "fp32_ms_per_step": round(1e3 * f["dq"], 2),
                        "bf16_final_cd_mean": float(np.mean(b["final"])), "fp32_final_cd_mean": float(np.mean(f["final"])),
                        "mean_ratio_bf16_over_fp32_final_cd": round(ratio, 5),
                        "note": "mean per-frame Chamfer distance of each sequence after the last step, averaged"},
            "autotuned_nn_threads_mlp_chunks_cg_tile_z": res["bf16"]["tuned"],
            "step_status": {"bf16": res["bf16"]["status"], "fp32": res["fp32"]["status"]},
            "sequences": len(cfgs), "steps": steps, "warmup": warmup,
            "samples_per_step": samples, "chamfer_pairs_per_direction": pairs,
            "sequence_shapes": [(len(d["xyz"]), d["T"], int(d["frame_off"][-1])) for d in datas],
            "note": ("16 sequences (V ~ U[5k,60k], T ~ U[20,400], N_t ~ U[4k,16k] per frame; human and quadruped "
                     "alternating), each with its own 8-level grids and 14->128x3->6 MLP; value: the BF16 form, "
                     "CG preconditioner, seeded non-degenerate state; one batch step = one step of every "
                     "sequence; inputs generated in "
                     f"{t_gen:.0f} s and resident before timing")}


def run_animal(steps=2, warmup=1):
    """The quadruped (animal-shaped) workload: 50 000 vertices, 1000 frames,
    ~7600 points per frame (5 % dropped), CG preconditioner, FP32."""
    import synth
    cfg = dict(synth.config_c3(), precond="cg")
    print("bench: generating the quadruped workload", file=sys.stderr, flush=True)
    data = synth.make_workload(cfg)
    r = run_form(cfg, data, synth.random_state(cfg, 9, grid_std=0.05), steps, warmup, profile=False)
    return {"value": round(r["value"], 4), "unit": "steps/s", "ms_per_step": round(r["ms_per_step"], 2),
            "steps": steps, "warmup": warmup, "stage_ms": r["stage_ms"],
            "step_status": r["status"], "cg_final_relres_max": r["cg_relres_max"],
            "stage_roofline": stage_roofline(cfg, data, r["stage_ms"], "f32"),
            "workload": f"quadruped_v{len(data['xyz'])}_t{data['T']}_n{int(data['frame_off'][-1])}",
            "note": "13-capsule quadruped, 8-level grids 16..256 x 4, 14->128x3->6 MLP, float32, CG with the V-cycle"}


def main():
    args = parse()
    global TUNE
    TUNE = not args.no_tune
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the method is single-GPU; sharding is described, "
              f"not built): --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)
    import synth

    cfg = dict(synth.config_c2(), cg_one_stream=int(args.cg_one_stream))
    data = synth.make_workload(cfg)
    T, V = data["T"], len(data["xyz"])
    P0 = synth.random_state(cfg, 9, grid_std=0.05)
    forms = set(args.forms.split(","))
    if "cg" not in forms:
        print("the headline form is cg: --forms must include it", file=sys.stderr)
        sys.exit(2)
    # headline: the CG-form step launched eagerly (npg_step, per-stage times);
    # the same step replayed as one captured HIP graph beside it (on this
    # runtime the graph's parallel branches of CG work overlap less than the
    # eager launches on two streams do), and the eager step with CG iteration
    # profiling (the groups of grids in step, each batch of iterations
    # bracketed by events): the roofline's measurement
    cgg = run_form(dict(cfg, precond="cg"), data, P0, args.steps, args.warmup, profile=False, graph=True)
    cg = run_form(dict(cfg, precond="cg"), data, P0, args.steps, args.warmup, profile=False)
    cgp = run_form(dict(cfg, precond="cg"), data, P0, args.steps, args.warmup, profile=True)
    plain = (run_form(dict(cfg, precond="cg", cg_mg=0), data, P0, args.steps, args.warmup, profile=True)
             if "cg_plain" in forms else None)
    dct = run_form(dict(cfg, precond="dct"), data, P0, args.steps, args.warmup, profile=False) if "dct" in forms else None
    graph = None
    if "graph" in forms:
        gh = run_form(dict(cfg, precond="dct"), data, P0, args.steps, args.warmup, profile=False, graph=True)
        cs = dict(synth.config_c1(), precond="dct", n_steps=100)
        ds = synth.make_workload(cs)
        Ps = synth.random_state(cs, 5, grid_std=0.05)
        small = {m: run_form(cs, ds, Ps, 50, 5, profile=False, graph=(m == "graph")) for m in ("eager", "graph")}
        graph = {"value": round(gh["value"], 4), "unit": "steps/s", "ms_per_step": round(gh["ms_per_step"], 3),
                 "status": gh["status"],
                 "eager_value": None if dct is None else round(dct["value"], 4),
                 "small": {"workload": f"icosphere_v{len(ds['xyz'])}_t{ds['T']}_n{int(ds['frame_off'][-1])}",
                           "steps": 50,
                           "eager": {"value": round(small["eager"]["value"], 2),
                                     "ms_per_step": round(small["eager"]["ms_per_step"], 4)},
                           "graph": {"value": round(small["graph"]["value"], 2),
                                     "ms_per_step": round(small["graph"]["ms_per_step"], 4)}},
                 "note": "npg_step_graph: the DCT-form step recorded once as a HIP graph and replayed (results "
                         "bitwise those of npg_step); value on the human workload, eager_value = precond_dct; "
                         "small = the 2562-vertex, 10-frame icosphere workload, where launches dominate"}
    quat = None
    if "quat" in forms:
        cq = dict(cfg, precond="dct", rot_head="quat")
        quat = run_form(cq, data, synth.random_state(cq, 9, grid_std=0.05), args.steps, args.warmup, profile=False)
    iso = None
    if "iso" in forms:
        iso = run_form(dict(cfg, precond="dct", w_iso=100.0), data, P0, args.steps, args.warmup, profile=False)
    prof = cgp["prof"]
    n_it = max(prof["cg_iters"], 1)
    cg_iter_ms = prof["cg_ms"] / n_it
    achieved = (prof["cg_bytes"] / 1e9) / (prof["cg_ms"] / 1e3) if prof["cg_ms"] > 0 else 0.0
    achieved_mg = (prof["cg_bytes_mg"] / 1e9) / (prof["cg_ms"] / 1e3) if prof["cg_ms"] > 0 else 0.0
    traffic = traffic_from_profile()
    # algorithmic bytes of one iteration with every grid active (the unit the
    # counter summary measures): 6 passes over the grid unknowns, and for the
    # V-cycle form 8 passes plus 4 over every coarse level's unknowns (levels
    # halve per axis, at most 3, down to 8 nodes per axis)
    systems = [(R, cfg["feat_p"]) for R in cfg["levels"]] + [(cfg["res_n"], cfg["feat_n"])]
    n_fine = sum(R ** 3 * F for R, F in systems)
    n_coarse = 0
    for R, F in systems:
        n, lev = R, 0
        while True:
            n, lev = (n + 1) // 2, lev + 1
            n_coarse += n ** 3 * F
            if n <= 8 or lev >= 3:
                break
    # the large grids (R >= 100, 4 features: z-column tiles) store no z: the
    # V-cycle's finest prolongation forms their next direction itself
    n_split = sum(R ** 3 * F for R, F in systems if R >= 100 and F == 4)
    full6, full_mg = 24.0 * n_fine, 32.0 * n_fine - 8.0 * n_split + 16.0 * n_coarse
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4),
                    traffic=traffic,
                    traffic_unit=("HBM bytes per preconditioned CG iteration with every grid active (rocprofv3 "
                                  "FETCH_SIZE + WRITE_SIZE, copy-calibrated)"),
                    traffic_over_algorithmic=(None if traffic is None else round(traffic / full6, 4)),
                    alg_bytes_full_iteration=full6,
                    kernel=("preconditioned CG iteration (k_cg_dir_ap, k_cg_reduce, k_cg_update, the V-cycle: "
                            "k_mg_down0, k_mg_down, k_mg_coarse, k_mg_up, k_mg_up0, and k_cg_reduce)"),
                    alg_bytes_definition=("per iteration a grid takes: 6 float32 passes over its R^3 F unknowns "
                                          "(x, r, p each read and written; A p formed in-kernel)"),
                    avg_ms_per_iteration=round(cg_iter_ms, 4),
                    alg_bytes_per_iteration=round(prof["cg_bytes"] / n_it),
                    iterations_timed=prof["cg_iters"],
                    vcycle_form_bytes={
                        "alg_bytes_per_iteration": round(prof["cg_bytes_mg"] / n_it),
                        "achieved": round(achieved_mg, 1), "frac": round(achieved_mg / HBM_PEAK_GBS, 4),
                        "alg_bytes_full_iteration": full_mg,
                        "traffic_over_these_bytes": (None if traffic is None else round(traffic / full_mg, 4)),
                        "definition": ("the same iterations counting also the preconditioned residual z (written "
                                       "and read) where it is stored (grids below 100 nodes per axis; the larger "
                                       "ones get their next direction from the V-cycle's finest prolongation) and "
                                       "every coarse V-cycle level's right-hand side and correction (written and "
                                       "read)")})
    out = {
        "metric": "optimization steps/sec (fwd+bwd+precond) at 100 frames; fraction of FP32/MFMA peak",
        "value": round(cg["value"], 4),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(cg["ms_per_step"], 3),
        "step_ms_events": cg["event_ms"],
        "timing": ("npg_step: every step launched eagerly (each group of CG grids on its own stream, its "
                   "iterations in batches between host checks of its flags); per-step HIP events on the plan's "
                   "stream give median / p90"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"human_v{V}_t{T}_n{cfg['N']}", "levels": cfg["levels"], "feat_p": cfg["feat_p"],
                   "mlp": f"{cfg['feat_n'] + cfg['feat_p'] + 2 * cfg['time_freqs']}->{cfg['mlp_width']}x"
                          f"{cfg['mlp_hidden']}->6", "precond": "cg", "cg_mg": 1, "cg_rtol": cfg["cg_rtol"],
                   "parallelism": "single-gpu"},
        "cg_profiled": {"value": round(cgp["value"], 4), "ms_per_step": round(cgp["ms_per_step"], 3),
                        "stage_ms": cgp["stage_ms"], "step_status": cgp["status"],
                        "note": ("the same eager step with CG iteration profiling (the groups of grids in step, "
                                 "HIP events around each batch of iterations): the run roofline is measured on")},
        "graph_replay": {"value": round(cgg["value"], 4), "ms_per_step": round(cgg["ms_per_step"], 3),
                         "step_ms_events": cgg["event_ms"], "step_status": cgg["status"],
                         "note": ("the same step replayed as one captured HIP graph (npg_step_graph; results "
                                  "bitwise those of npg_step)")},
        "stage_ms": cg["stage_ms"],
        "nn_autotune": cg["nn_tune"],
        "stage_roofline": stage_roofline(cfg, data, cg["stage_ms"], "f32", prof),
        "paper_context": PAPER_CONTEXT,
        "cg_iterations_per_step": round(prof["cg_iters"] / args.steps, 1),
        "cg_final_relres_max": cg["cg_relres_max"],
        "step_status": cg["status"],
        "roofline": roofline,
        "precond_cg_plain": None if plain is None else {
            "value": round(plain["value"], 4), "unit": "steps/s", "ms_per_step": round(plain["ms_per_step"], 3),
            "stage_ms": plain["stage_ms"],
            "cg_iterations_per_step": round(plain["prof"]["cg_iters"] / args.steps, 1),
            "cg_final_relres_max": plain["cg_relres_max"],
            "note": "same step with the solves by plain CG (no V-cycle, cg_mg = 0)"},
        "precond_dct": None if dct is None else {
            "value": round(dct["value"], 4), "unit": "steps/s", "ms_per_step": round(dct["ms_per_step"], 3),
            "stage_ms": dct["stage_ms"], "note": "same step with the exact DCT form of (I + lambda L)^-2"},
        "step_graph": graph,
        "rot_quat": None if quat is None else {
            "value": round(quat["value"], 4), "unit": "steps/s", "ms_per_step": round(quat["ms_per_step"], 3),
            "stage_ms": quat["stage_ms"],
            "note": "quaternion rotation head (7 outputs, Sec. 3.4) with the DCT preconditioner; compare precond_dct"},
        "isometry": None if iso is None else {
            "value": round(iso["value"], 4), "unit": "steps/s", "ms_per_step": round(iso["ms_per_step"], 3),
            "stage_ms": iso["stage_ms"], "edges": int(len(data["edges"])),
            "note": "objective L_def + 100 L_iso (Sec. 3.5) with the DCT preconditioner; compare precond_dct"},
        "evaluation": run_metrics(cfg, P0) if "metrics" in forms else None,
        "nn_search": run_nn_compare(cfg, data, P0) if "nn" in forms else None,
        "bf16": None,
        "batch": None,
        "cpu_baseline": None,
    }
    if "bf16" in forms:
        b16 = run_form(dict(cfg, precond="cg", precision="bf16"), data, P0, args.steps, args.warmup, profile=False)
        out["bf16"] = {"value": round(b16["value"], 4), "unit": "steps/s", "ms_per_step": round(b16["ms_per_step"], 3),
                       "stage_ms": b16["stage_ms"],
                       "stage_roofline": stage_roofline(cfg, data, b16["stage_ms"], "bf16"),
                       "step_status": b16["status"],
                       "note": "headline step with the MLP's matrix operands in bfloat16 (float32 accumulation)",
                       "quality": None if args.no_quality else run_quality(cfg)}
    if "batch" in forms:
        out["batch"] = run_batch()
    if "animal" in forms:
        out["animal"] = run_animal()
    if not args.no_cpu_baseline:
        print("bench: CPU baselines (oracle, then oracle with k-d tree nearest neighbours)", file=sys.stderr,
              flush=True)
        cb = cpu_baseline(cfg, data, P0, args.cpu_frames)
        out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
        out["cpu_baseline"]["stage_seconds"] = cb["stage_seconds"]
        cf = cpu_fast(cfg, data, P0, args.cpu_frames)
        # Adam of the full parameter vector as measured in the oracle leg
        cf["value"] = 1.0 / (1.0 / cf["value"] + cb["stage_seconds"]["adam"])
        out["cpu_fast_baseline"] = cf
    print(json.dumps(out), flush=True)
    if args.copy_calibration:
        import torch
        a = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device="cuda")  # 1 GiB
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()


if __name__ == "__main__":
    main()
