"""Python binding of libneupig.so (the MI355X Neu-PiG optimization-step library).

Argument marshalling only: every computation runs in the library's HIP
kernels. Tensors must be contiguous torch tensors on the plan's GPU; their
device pointers and the current HIP stream are passed through the C ABI
declared in include/neupig.h. If the library is missing this module fails
loudly: there is no CPU fallback.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libneupig.so")

NPG_MAX_LEVELS = 16
NPG_OK, NPG_EINVAL, NPG_ENOMEM, NPG_EHIP, NPG_ENOTCONV, NPG_ENONFINITE = range(6)
NPG_ACT_RELU, NPG_ACT_LEAKY = 0, 1
NPG_PRECOND_CG, NPG_PRECOND_DCT = 0, 1
NPG_ROT_EXPMAP, NPG_ROT_QUAT = 0, 1
NPG_PREC_FP32, NPG_PREC_BF16 = 0, 1
NPG_NN_PRUNED, NPG_NN_EXHAUSTIVE = 0, 1
STAGES = ("encode", "decode", "chamfer+loss", "chamfer_bwd", "iso", "decode_bwd", "encode_bwd", "precond", "adam")


class NpgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"neupig status {status}: {msg}")
        self.status = status


class npg_config(ctypes.Structure):
    _fields_ = [
        ("n_levels", ctypes.c_int32), ("res", ctypes.c_int32 * NPG_MAX_LEVELS),
        ("feat_p", ctypes.c_int32), ("res_n", ctypes.c_int32), ("feat_n", ctypes.c_int32),
        ("time_freqs", ctypes.c_int32), ("mlp_hidden", ctypes.c_int32), ("mlp_width", ctypes.c_int32),
        ("act", ctypes.c_int32), ("leaky_slope", ctypes.c_float), ("alpha_t", ctypes.c_float),
        ("lr_mlp", ctypes.c_float), ("lr_grid", ctypes.c_float * NPG_MAX_LEVELS), ("lr_n", ctypes.c_float),
        ("lam", ctypes.c_float * NPG_MAX_LEVELS), ("lam_n", ctypes.c_float),
        ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
        ("conf_weight", ctypes.c_int32), ("t_key", ctypes.c_int32),
        ("cg_rtol", ctypes.c_double), ("cg_maxit", ctypes.c_int32), ("precond", ctypes.c_int32),
        ("rot_head", ctypes.c_int32), ("w_iso", ctypes.c_float), ("precision", ctypes.c_int32),
        ("cg_mg", ctypes.c_int32), ("nn_search", ctypes.c_int32), ("cg_one_stream", ctypes.c_int32),
    ]


_lib = None
_P = ctypes.c_void_p
_I32, _I64, _D = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
_SIGS = {
    "npg_last_error": ([], ctypes.c_char_p),
    "npg_param_count": ([ctypes.POINTER(npg_config), ctypes.POINTER(_I64)], ctypes.c_int),
    "npg_plan_create": ([ctypes.POINTER(npg_config), _I64, _P, _P, _I32, _P, ctypes.POINTER(_I64), _P,
                         ctypes.POINTER(_P)], ctypes.c_int),
    "npg_plan_destroy": ([_P], ctypes.c_int),
    "npg_set_state": ([_P, _P, _P, _P, _I64], ctypes.c_int),
    "npg_get_state": ([_P, _P, _P, _P, ctypes.POINTER(_I64)], ctypes.c_int),
    "npg_step": ([_P, _I32, _I32, _P, _P], ctypes.c_int),
    "npg_step_graph": ([_P, _I32, _I32, _P, _P], ctypes.c_int),
    "npg_deform": ([_P, _P], ctypes.c_int),
    "npg_encode_fwd": ([_P, _P, _P], ctypes.c_int),
    "npg_decode_fwd": ([_P, _P, _P, _P], ctypes.c_int),
    "npg_chamfer_fwd": ([_P, _P, _P, _P, _P, _P, _P], ctypes.c_int),
    "npg_loss": ([_P, _P, _I32, _I32, _P, _P], ctypes.c_int),
    "npg_chamfer_bwd": ([_P, _P, _P, _P, _P, _P], ctypes.c_int),
    "npg_decode_bwd": ([_P, _P, _P, _P, _P, _P], ctypes.c_int),
    "npg_encode_bwd": ([_P, _P, _P], ctypes.c_int),
    "npg_precond": ([_P, _P, ctypes.POINTER(_I32)], ctypes.c_int),
    "npg_adam": ([_P, _P, _P, _P, _P, _I64], ctypes.c_int),
    "npg_stage_times": ([_P, ctypes.POINTER(ctypes.c_float)], ctypes.c_int),
    "npg_plan_set_edges": ([_P, _I64, ctypes.POINTER(_I32)], ctypes.c_int),
    "npg_iso": ([_P, _P, _P, _P, _P], ctypes.c_int),
    "npg_predict": ([_P, _P, _P], ctypes.c_int),
    "npg_plan_create_batched": ([ctypes.POINTER(npg_config), _I32, ctypes.POINTER(_I64), ctypes.POINTER(_P),
                                 ctypes.POINTER(_P), ctypes.POINTER(_I32), ctypes.POINTER(_P),
                                 ctypes.POINTER(ctypes.POINTER(_I64)), ctypes.POINTER(_P)], ctypes.c_int),
    "npg_batch_plan": ([_P, _I32, ctypes.POINTER(_P)], ctypes.c_int),
    "npg_batch_step": ([_P, _I32, _I32, ctypes.POINTER(_P)], ctypes.c_int),
    "npg_batch_step_graph": ([_P, _I32, _I32, ctypes.POINTER(_P)], ctypes.c_int),
    "npg_batch_graph_mode": ([_P, _I32], ctypes.c_int),
    "npg_batch_destroy": ([_P], ctypes.c_int),
    "npg_metrics": ([_P, _P, _P, _P, _P, ctypes.c_float, _P], ctypes.c_int),
    "npg_metrics_noalloc": ([_P, _P, _P, _P, _P, ctypes.c_float, _P], ctypes.c_int),
    "npg_objective_fwd": ([_P, _P, _I32, _I32, _P, _P, _P, _P, _P, _P, _P, _P], ctypes.c_int),
    "npg_objective_bwd": ([_P, _P, _P, _P, _P, _P, _P], ctypes.c_int),
    "npg_scale": ([_P, _P, _D, _P, _I32, _I64], ctypes.c_int),
    "npg_tune_nn": ([_P, _I32, ctypes.POINTER(_I32), ctypes.POINTER(ctypes.c_float)], ctypes.c_int),
    "npg_tune_mlp": ([_P, _I32, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(ctypes.c_float)],
                     ctypes.c_int),
    "npg_tune_cg": ([_P, _I32, ctypes.POINTER(_I32), ctypes.POINTER(ctypes.c_float)], ctypes.c_int),
    "npg_precond_residuals": ([_P, ctypes.POINTER(_D)], ctypes.c_int),
    "npg_params_import": ([_P, ctypes.POINTER(_P)], ctypes.c_int),
    "npg_params_export": ([_P, ctypes.POINTER(_P)], ctypes.c_int),
    "npg_state_import": ([_P, _P, _P, _P, _I64], ctypes.c_int),
    "npg_state_export": ([_P, _P, _P, _P, ctypes.POINTER(_I64)], ctypes.c_int),
    "npg_profile": ([_P, _I32], ctypes.c_int),
    "npg_profile_read": ([_P, ctypes.POINTER(_D), ctypes.POINTER(_I64), ctypes.POINTER(_D), ctypes.POINTER(_D)],
                         ctypes.c_int),
}


def lib():
    """Load libneupig.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2602_22212_amd.build.build() "
                               "(there is no fallback path)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(status):
    if status != NPG_OK:
        raise NpgError(status, lib().npg_last_error().decode())
    return status


def make_config(cfg):
    """Marshal a hyper-parameter dict (see synth.configs) into npg_config."""
    c = npg_config()
    levels = list(cfg["levels"])
    c.n_levels = len(levels)
    for l, r in enumerate(levels):
        c.res[l] = int(r)
        c.lr_grid[l] = float(cfg["lr_grid"][l])
        c.lam[l] = float(cfg["lam"][l])
    c.feat_p, c.res_n, c.feat_n = int(cfg["feat_p"]), int(cfg["res_n"]), int(cfg["feat_n"])
    c.time_freqs = int(cfg["time_freqs"])
    c.mlp_hidden, c.mlp_width = int(cfg["mlp_hidden"]), int(cfg["mlp_width"])
    c.act = NPG_ACT_RELU if cfg["act"] == "relu" else NPG_ACT_LEAKY
    c.leaky_slope, c.alpha_t = float(cfg["leaky_slope"]), float(cfg["alpha_t"])
    c.lr_mlp, c.lr_n, c.lam_n = float(cfg["lr_mlp"]), float(cfg["lr_n"]), float(cfg["lam_n"])
    c.beta1, c.beta2, c.eps = float(cfg["beta1"]), float(cfg["beta2"]), float(cfg["eps"])
    c.conf_weight = int(cfg["conf_weight"])
    c.t_key = -1 if cfg.get("t_key") is None else int(cfg["t_key"])
    c.cg_rtol, c.cg_maxit = float(cfg["cg_rtol"]), int(cfg["cg_maxit"])
    c.precond = NPG_PRECOND_DCT if cfg.get("precond", "cg") == "dct" else NPG_PRECOND_CG
    c.cg_mg = int(cfg.get("cg_mg", 1))
    c.cg_one_stream = int(cfg.get("cg_one_stream", 0))
    nn = cfg.get("nn_search", "pruned")
    if nn not in ("pruned", "exhaustive"):
        raise ValueError(f"nn_search must be 'pruned' or 'exhaustive', not {nn!r}")
    c.nn_search = NPG_NN_EXHAUSTIVE if nn == "exhaustive" else NPG_NN_PRUNED
    head = cfg.get("rot_head", "expmap")
    if head not in ("expmap", "quat"):
        raise ValueError(f"rot_head must be 'expmap' or 'quat', not {head!r}")
    c.rot_head = NPG_ROT_QUAT if head == "quat" else NPG_ROT_EXPMAP
    c.w_iso = float(cfg.get("w_iso", 0.0))
    prec = cfg.get("precision", "fp32")
    if prec not in ("fp32", "bf16"):
        raise ValueError(f"precision must be 'fp32' or 'bf16', not {prec!r}")
    c.precision = NPG_PREC_BF16 if prec == "bf16" else NPG_PREC_FP32
    return c


def param_count(cfg):
    n = _I64()
    _check(lib().npg_param_count(ctypes.byref(make_config(cfg)), ctypes.byref(n)))
    return n.value


def param_layout(cfg):
    """(name, offset, shape) of every block of the flat parameter vector
    (layout stated in include/neupig.h)."""
    out, off = [], 0
    F, Fn, Rn = cfg["feat_p"], cfg["feat_n"], cfg["res_n"]
    for l, R in enumerate(cfg["levels"]):
        out.append((f"grid_p{l}", off, (R ** 3, F)))
        off += R ** 3 * F
    out.append(("grid_n", off, (Rn ** 3, Fn)))
    off += Rn ** 3 * Fn
    M = cfg["time_freqs"]
    n_out = 7 if cfg.get("rot_head", "expmap") == "quat" else 6
    dims = [Fn + F + (2 * M if M > 0 else 1)] + [cfg["mlp_width"]] * cfg["mlp_hidden"] + [n_out]
    for k in range(len(dims) - 1):
        out.append((f"W{k}", off, (dims[k + 1], dims[k])))
        off += dims[k + 1] * dims[k]
        out.append((f"b{k}", off, (dims[k + 1],)))
        off += dims[k + 1]
    return out, off


def pack_params(cfg, p):
    """Structured parameters (grid_p list, grid_n, mlp [(W, b)]) -> flat float32."""
    parts = [np.asarray(g, np.float32).ravel() for g in p["grid_p"]]
    parts.append(np.asarray(p["grid_n"], np.float32).ravel())
    for W, b in p["mlp"]:
        parts += [np.asarray(W, np.float32).ravel(), np.asarray(b, np.float32).ravel()]
    return np.concatenate(parts)


def unpack_params(cfg, flat):
    flat = np.asarray(flat)
    lay, _ = param_layout(cfg)
    d = {name: flat[o:o + int(np.prod(s))].reshape(s) for name, o, s in lay}
    L = len(cfg["levels"])
    H = cfg["mlp_hidden"]
    return dict(grid_p=[d[f"grid_p{l}"] for l in range(L)], grid_n=d["grid_n"],
                mlp=[(d[f"W{k}"], d[f"b{k}"]) for k in range(H + 1)])


def _ptr(t, dtype=None, n=None, name="tensor"):
    import torch
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} must have {n} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """One sequence's plan (npg_plan): static tables, optimizer state and
    workspace live on the GPU; methods mirror the C entry points."""

    def __init__(self, cfg, xyz, nrm, pts, frame_off, stream=None):
        import torch
        self.cfg = dict(cfg)
        self._c = make_config(cfg)
        self.V = int(xyz.shape[0])
        self.T = int(len(frame_off) - 1)
        off = np.ascontiguousarray(np.asarray(frame_off, dtype=np.int64))
        self.frame_off = off
        self.Ntot = int(off[-1])
        self.n_params = param_count(cfg)
        f32 = torch.float32
        px = _ptr(xyz, f32, 3 * self.V, "xyz")
        pn = _ptr(nrm, f32, 3 * self.V, "nrm")
        pp = _ptr(pts, f32, 3 * self.Ntot, "pts")
        self.device = xyz.device
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = _P()
        _check(lib().npg_plan_create(ctypes.byref(self._c), self.V, px, pn, self.T, pp,
                                     off.ctypes.data_as(ctypes.POINTER(_I64)),
                                     ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self.Fz = cfg["feat_n"] + cfg["feat_p"]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value and getattr(self, "_owned", True):
            lib().npg_plan_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- state --------------------------------------------------------------
    def set_state(self, params, m=None, v=None, adam_steps=0):
        import torch
        f = torch.float32
        _check(lib().npg_set_state(self._h, _ptr(params, f, self.n_params, "params"),
                                   _ptr(m, f, self.n_params, "m"), _ptr(v, f, self.n_params, "v"),
                                   int(adam_steps)))

    def get_state(self):
        import torch
        p = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        m, v = torch.empty_like(p), torch.empty_like(p)
        k = _I64()
        _check(lib().npg_get_state(self._h, _ptr(p), _ptr(m), _ptr(v), ctypes.byref(k)))
        return p, m, v, k.value

    def step(self, epoch, n_epochs, loss=None, cd=None):
        import torch
        st = lib().npg_step(self._h, int(epoch), int(n_epochs), _ptr(loss, torch.float64, 1, "loss"),
                            _ptr(cd, torch.float64, self.T, "cd"))
        if st == NPG_ENOTCONV:
            return st
        return _check(st)

    def step_graph(self, epoch, n_epochs, loss=None, cd=None):
        """npg_step replayed as one captured HIP graph (both preconditioners)."""
        import torch
        st = lib().npg_step_graph(self._h, int(epoch), int(n_epochs), _ptr(loss, torch.float64, 1, "loss"),
                                  _ptr(cd, torch.float64, self.T, "cd"))
        if st == NPG_ENOTCONV:
            return st
        return _check(st)

    def set_edges(self, edges):
        """Mesh edges [E, 2] (host array) for the isometry loss."""
        e = np.ascontiguousarray(edges, np.int32)
        if e.ndim != 2 or e.shape[1] != 2:
            raise ValueError("edges must have shape [E, 2]")
        _check(lib().npg_plan_set_edges(self._h, len(e), e.ctypes.data_as(ctypes.POINTER(_I32))))
        self.n_edges = len(e)

    def iso(self, xhat, iso, gxhat=None, sign=None):
        import torch
        TV = self.T * self.V
        _check(lib().npg_iso(self._h, _ptr(xhat, torch.float32, 4 * TV, "xhat"),
                             _ptr(gxhat, torch.float32, 4 * TV, "gxhat"), _ptr(iso, torch.float64, 1, "iso"),
                             _ptr(sign, torch.int8, self.T * getattr(self, "n_edges", 0), "sign")))

    def predict(self, xhat, nhat=None):
        """Deformed vertices (and normals) [T][V][4] with the plan's parameters."""
        import torch
        TV = self.T * self.V
        _check(lib().npg_predict(self._h, _ptr(xhat, torch.float32, 4 * TV, "xhat"),
                                 _ptr(nhat, torch.float32, 4 * TV, "nhat")))

    def metrics(self, xhat, nhat, gt, gtn, tau, out):
        """Per-frame (CD, NC, F, Corr) [T][4] float64 against true vertices/normals [T][V][4]."""
        import torch
        TV = self.T * self.V
        _check(lib().npg_metrics(self._h, _ptr(xhat, torch.float32, 4 * TV, "xhat"),
                                 _ptr(nhat, torch.float32, 4 * TV, "nhat"), _ptr(gt, torch.float32, 4 * TV, "gt"),
                                 _ptr(gtn, torch.float32, 4 * TV, "gtn"), float(tau),
                                 _ptr(out, torch.float64, 4 * self.T, "out")))

    def metrics_noalloc(self, xhat, nhat, gt, gtn, tau, out):
        """npg_metrics with the library's fixed scratch array (no device
        allocation, no synchronisation)."""
        import torch
        TV = self.T * self.V
        _check(lib().npg_metrics_noalloc(self._h, _ptr(xhat, torch.float32, 4 * TV, "xhat"),
                                         _ptr(nhat, torch.float32, 4 * TV, "nhat"), _ptr(gt, torch.float32, 4 * TV, "gt"),
                                         _ptr(gtn, torch.float32, 4 * TV, "gtn"), float(tau),
                                         _ptr(out, torch.float64, 4 * self.T, "out")))

    def deform(self, out):
        import torch
        _check(lib().npg_deform(self._h, _ptr(out, torch.float32, 3 * self.T * self.V, "out")))

    def stage_times(self):
        buf = (ctypes.c_float * len(STAGES))()
        _check(lib().npg_stage_times(self._h, buf))
        return dict(zip(STAGES, list(buf)))

    def profile(self, enable=True):
        _check(lib().npg_profile(self._h, int(bool(enable))))

    def profile_read(self):
        ms, it, by, bm = _D(), _I64(), _D(), _D()
        _check(lib().npg_profile_read(self._h, ctypes.byref(ms), ctypes.byref(it), ctypes.byref(by),
                                      ctypes.byref(bm)))
        return dict(cg_ms=ms.value, cg_iters=it.value, cg_bytes=by.value, cg_bytes_mg=bm.value)

    # -- stages ---------------------------------------------------------------
    def encode_fwd(self, params, z):
        import torch
        f = torch.float32
        _check(lib().npg_encode_fwd(self._h, _ptr(params, f, self.n_params, "params"),
                                    _ptr(z, f, self.V * self.Fz, "z")))

    def decode_fwd(self, params, z, xhat):
        import torch
        f = torch.float32
        _check(lib().npg_decode_fwd(self._h, _ptr(params, f, self.n_params, "params"),
                                    _ptr(z, f, self.V * self.Fz, "z"), _ptr(xhat, f, 4 * self.T * self.V, "xhat")))

    def chamfer_fwd(self, xhat, a, da, b, db, cd):
        import torch
        TV = self.T * self.V
        _check(lib().npg_chamfer_fwd(self._h, _ptr(xhat, torch.float32, 4 * TV, "xhat"),
                                     _ptr(a, torch.int32, TV, "a"), _ptr(da, torch.float32, TV, "da"),
                                     _ptr(b, torch.int32, self.Ntot, "b"), _ptr(db, torch.float32, self.Ntot, "db"),
                                     _ptr(cd, torch.float64, self.T, "cd")))

    def loss(self, cd, epoch, n_epochs, w, loss):
        import torch
        d = torch.float64
        _check(lib().npg_loss(self._h, _ptr(cd, d, self.T, "cd"), int(epoch), int(n_epochs),
                              _ptr(w, d, self.T, "w"), _ptr(loss, d, 1, "loss")))

    def objective_fwd(self, xhat, epoch, n_epochs, a, da, b, db, cd, w, loss, iso=None):
        """L_def + w_iso L_iso (Sec. 3.5) with the Chamfer outputs and weights."""
        import torch
        TV = self.T * self.V
        _check(lib().npg_objective_fwd(self._h, _ptr(xhat, torch.float32, 4 * TV, "xhat"), int(epoch), int(n_epochs),
                                       _ptr(a, torch.int32, TV, "a"), _ptr(da, torch.float32, TV, "da"),
                                       _ptr(b, torch.int32, self.Ntot, "b"), _ptr(db, torch.float32, self.Ntot, "db"),
                                       _ptr(cd, torch.float64, self.T, "cd"), _ptr(w, torch.float64, self.T, "w"),
                                       _ptr(iso, torch.float64, 1, "iso"), _ptr(loss, torch.float64, 1, "loss")))

    def objective_bwd(self, xhat, a, b, w, g, gxhat):
        """g (dL_def/dx^ + w_iso dL_iso/dx^); g a one-element float64 device tensor or None (1)."""
        import torch
        TV = self.T * self.V
        _check(lib().npg_objective_bwd(self._h, _ptr(xhat, torch.float32, 4 * TV, "xhat"),
                                       _ptr(a, torch.int32, TV, "a"), _ptr(b, torch.int32, self.Ntot, "b"),
                                       _ptr(w, torch.float64, self.T, "w"), _ptr(g, torch.float64, 1, "g"),
                                       _ptr(gxhat, torch.float32, 4 * TV, "gxhat")))

    def chamfer_bwd(self, xhat, a, b, w, gxhat):
        import torch
        TV = self.T * self.V
        _check(lib().npg_chamfer_bwd(self._h, _ptr(xhat, torch.float32, 4 * TV, "xhat"),
                                     _ptr(a, torch.int32, TV, "a"), _ptr(b, torch.int32, self.Ntot, "b"),
                                     _ptr(w, torch.float64, self.T, "w"), _ptr(gxhat, torch.float32, 4 * TV, "gxhat")))

    def decode_bwd(self, params, z, gxhat, grad, gz):
        import torch
        f = torch.float32
        _check(lib().npg_decode_bwd(self._h, _ptr(params, f, self.n_params, "params"),
                                    _ptr(z, f, self.V * self.Fz, "z"),
                                    _ptr(gxhat, f, 4 * self.T * self.V, "gxhat"),
                                    _ptr(grad, f, self.n_params, "grad"), _ptr(gz, f, self.V * self.Fz, "gz")))

    def encode_bwd(self, gz, grad):
        import torch
        f = torch.float32
        _check(lib().npg_encode_bwd(self._h, _ptr(gz, f, self.V * self.Fz, "gz"),
                                    _ptr(grad, f, self.n_params, "grad")))

    def precond(self, grad):
        import torch
        it = (_I32 * (2 * (len(self.cfg["levels"]) + 1)))()
        st = lib().npg_precond(self._h, _ptr(grad, torch.float32, self.n_params, "grad"), it)
        if st not in (NPG_OK, NPG_ENOTCONV):
            _check(st)
        return list(it), st

    def precond_residuals(self):
        """Final relative residuals of the last preconditioning (CG form),
        [first solve per grid..., second solve per grid...]."""
        out = (_D * (2 * (len(self.cfg["levels"]) + 1)))()
        _check(lib().npg_precond_residuals(self._h, out))
        return list(out)

    def adam(self, params, grad, m, v, adam_step):
        import torch
        f = torch.float32
        n = self.n_params
        _check(lib().npg_adam(self._h, _ptr(params, f, n, "params"), _ptr(grad, f, n, "grad"),
                              _ptr(m, f, n, "m"), _ptr(v, f, n, "v"), int(adam_step)))


    def params_import(self, blocks):
        """Replace the parameters from per-block device tensors (order and
        shapes of param_layout)."""
        import torch
        lay, _ = param_layout(self.cfg)
        if len(blocks) != len(lay):
            raise ValueError(f"need {len(lay)} blocks, got {len(blocks)}")
        ptrs = (_P * len(lay))(*[_ptr(b, torch.float32, int(np.prod(s)), n).value for b, (n, _, s) in zip(blocks, lay)])
        _check(lib().npg_params_import(self._h, ptrs))

    def params_export(self):
        """The parameters as per-block device tensors (param_layout order)."""
        import torch
        lay, _ = param_layout(self.cfg)
        out = [torch.empty(s, dtype=torch.float32, device=self.device) for _, _, s in lay]
        ptrs = (_P * len(lay))(*[t.data_ptr() for t in out])
        _check(lib().npg_params_export(self._h, ptrs))
        return out

    def tune_nn(self, threads=0):
        """Work-group size of the nearest-neighbour pass: 0 = time 64/128/256
        on the current state and keep the fastest. Returns (chosen, ms [3])."""
        ch = _I32()
        ms = (ctypes.c_float * 3)()
        _check(lib().npg_tune_nn(self._h, int(threads), ctypes.byref(ch), ms))
        return ch.value, list(ms)

    def tune_mlp(self, nch=0):
        """Frame chunks of the decode backward: 0 = time the candidates and
        keep the fastest. Returns (chosen, candidates [4], ms [4])."""
        ch = _I32()
        cand = (_I32 * 4)()
        ms = (ctypes.c_float * 4)()
        _check(lib().npg_tune_mlp(self._h, int(nch), ctypes.byref(ch), cand, ms))
        return ch.value, list(cand), list(ms)

    def tune_cg(self, zs=0):
        """z planes per CG tile (32/64/128): 0 = time them and keep the
        fastest. Returns (chosen, ms [3])."""
        ch = _I32()
        ms = (ctypes.c_float * 3)()
        _check(lib().npg_tune_cg(self._h, int(zs), ctypes.byref(ch), ms))
        return ch.value, list(ms)

    def scale(self, s, x, c=1.0):
        """x *= c * s[0] on the device (s: one float64; x: float32 or float64)."""
        import torch
        if x.dtype not in (torch.float32, torch.float64):
            raise TypeError("scale: x must be float32 or float64")
        _check(lib().npg_scale(self._h, _ptr(s, torch.float64, 1, "s"), float(c), _ptr(x, x.dtype, x.numel(), "x"),
                               int(x.dtype == torch.float64), x.numel()))


class Batch:
    """Many independent sequences (npg_batch): one plan and stream per
    sequence, stepped concurrently by npg_batch_step."""

    def __init__(self, cfgs, datas, device="cuda:0"):
        import torch
        n = len(cfgs)
        if n < 1 or len(datas) != n:
            raise ValueError("need one workload per config and at least one sequence")
        self.cfgs = [dict(c) for c in cfgs]
        self._keep = []
        confs = (npg_config * n)(*[make_config(c) for c in cfgs])
        V = (_I64 * n)()
        T = (_I32 * n)()
        xyz, nrm, pts = (_P * n)(), (_P * n)(), (_P * n)()
        offs = (ctypes.POINTER(_I64) * n)()
        for k, d in enumerate(datas):
            tx = torch.from_numpy(np.ascontiguousarray(d["xyz"], np.float32)).to(device)
            tn = torch.from_numpy(np.ascontiguousarray(d["nrm"], np.float32)).to(device)
            tp = torch.from_numpy(np.ascontiguousarray(d["pts"], np.float32)).to(device)
            off = np.ascontiguousarray(np.asarray(d["frame_off"], np.int64))
            self._keep += [tx, tn, tp, off]
            V[k], T[k] = len(d["xyz"]), len(off) - 1
            xyz[k], nrm[k], pts[k] = tx.data_ptr(), tn.data_ptr(), tp.data_ptr()
            offs[k] = off.ctypes.data_as(ctypes.POINTER(_I64))
        h = _P()
        _check(lib().npg_plan_create_batched(confs, n, V, xyz, nrm, T, pts, offs, ctypes.byref(h)))
        self._h = h
        self.plans = []
        for k, (c, d) in enumerate(zip(cfgs, datas)):
            ph = _P()
            _check(lib().npg_batch_plan(self._h, k, ctypes.byref(ph)))
            v = Plan.__new__(Plan)
            v.cfg, v._c, v._owned, v._h = dict(c), make_config(c), False, ph
            v.V, v.T = int(V[k]), int(T[k])
            v.frame_off = self._keep[4 * k + 3]
            v.Ntot = int(v.frame_off[-1])
            v.n_params = param_count(c)
            v.device, v.stream = torch.device(device), None
            v.Fz = c["feat_n"] + c["feat_p"]
            if c.get("w_iso", 0.0) > 0:
                v.set_edges(d["edges"])
            self.plans.append(v)

    def step(self, epoch, n_epochs, losses=None):
        import torch
        arr = None
        if losses is not None:
            arr = (_P * len(self.plans))(*[None if l is None else _ptr(l, torch.float64, 1, "loss").value
                                          for l in losses])
        st = lib().npg_batch_step(self._h, int(epoch), int(n_epochs), arr)
        if st == NPG_ENOTCONV:
            return st
        return _check(st)

    def graph_mode(self, per_stream):
        """npg_batch_graph_mode: False = one batch graph, True = each
        sequence's recording on its own stream."""
        _check(lib().npg_batch_graph_mode(self._h, 1 if per_stream else 0))

    def step_graph(self, epoch, n_epochs, losses=None):
        """The batch step replayed from recorded HIP graphs (npg_batch_step_graph)."""
        import torch
        arr = None
        if losses is not None:
            arr = (_P * len(self.plans))(*[None if l is None else _ptr(l, torch.float64, 1, "loss").value
                                          for l in losses])
        st = lib().npg_batch_step_graph(self._h, int(epoch), int(n_epochs), arr)
        if st == NPG_ENOTCONV:
            return st
        return _check(st)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            for v in self.plans:
                v._h = None
            lib().npg_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan_from_workload(cfg, data, device="cuda:0"):
    """Upload a synth workload dict and create a Plan."""
    import torch
    xyz = torch.from_numpy(np.ascontiguousarray(data["xyz"], np.float32)).to(device)
    nrm = torch.from_numpy(np.ascontiguousarray(data["nrm"], np.float32)).to(device)
    pts = torch.from_numpy(np.ascontiguousarray(data["pts"], np.float32)).to(device)
    plan = Plan(cfg, xyz, nrm, pts, data["frame_off"])
    if cfg.get("w_iso", 0.0) > 0:
        plan.set_edges(data["edges"])
    return plan
