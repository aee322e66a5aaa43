"""Python binding of libddpinn (ctypes): argument marshalling only.

Every step of the training step runs in the HIP kernels of libddpinn.so;
torch supplies device memory and the stream.  There is no fallback: if the
library is missing, loading raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

from . import workloads as W

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libddpinn.so")

DDP_OK, DDP_EINVAL, DDP_ENOMEM, DDP_EHIP, DDP_ESTATE, DDP_ENONFINITE = 0, -1, -2, -3, -4, -5
DDP_CPINN, DDP_XPINN = 0, 1
DDP_POISSON2D, DDP_BURGERS1D, DDP_NS2D_STEADY, DDP_DIFFUSION2D_INV = 0, 1, 2, 3
DDP_RESIDUAL, DDP_DATA, DDP_DATA_AUX = 0, 1, 2
(DDP_OPT_CHUNK_POINTS, DDP_OPT_BLOCKS_PER_CU, DDP_OPT_ITEMS_PER_SLOT, DDP_OPT_RECOMPUTE, DDP_OPT_CONCURRENT,
 DDP_OPT_TAIL) = 0, 1, 2, 3, 4, 5
DDP_ACT_TANH, DDP_ACT_SIN, DDP_ACT_COS = 0, 1, 2
_ACT = {"tanh": DDP_ACT_TANH, "sin": DDP_ACT_SIN, "cos": DDP_ACT_COS}

EXPORTED = [
    "ddp_create", "ddp_add_subdomain", "ddp_set_points", "ddp_add_interface", "ddp_set_interface_method",
    "ddp_set_activation",
    "ddp_set_option",
    "ddp_finalize", "ddp_param_count", "ddp_set_params", "ddp_get_params", "ddp_loss_and_grad",
    "ddp_step", "ddp_get_state", "ddp_set_state", "ddp_eval", "ddp_sync", "ddp_time_kernels",
    "ddp_plan_dump", "ddp_plan", "ddp_last_error", "ddp_destroy", "ddp_autotune", "ddp_mfma_probe",
    "ddp_time_phases", "ddp_loss_and_grad_static",
]

_METHOD = {W.METHOD_CPINN: DDP_CPINN, W.METHOD_XPINN: DDP_XPINN}
_PDE = {W.PDE_POISSON2D: DDP_POISSON2D, W.PDE_BURGERS1D: DDP_BURGERS1D, W.PDE_NS2D: DDP_NS2D_STEADY,
        W.PDE_DIFFUSION2D_INV: DDP_DIFFUSION2D_INV}

_lib = None


class DDPError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libddpinn error {code}: {msg}")
        self.code = code


def load_library(path=LIB_PATH):
    """Load libddpinn.so and declare the C signatures.  Raises if missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run paper_2104_10013_amd.build.build()")
    L = ctypes.CDLL(path)
    P, I, I64, F, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_float, ctypes.c_double
    pI, pF, pI64 = ctypes.POINTER(I), ctypes.POINTER(F), ctypes.POINTER(I64)
    sig = {
        "ddp_create": ([ctypes.POINTER(P), I, I, ctypes.POINTER(D), I], I),
        "ddp_add_subdomain": ([P, I, pI, pI, pF, F, pI], I),
        "ddp_set_points": ([P, I, I, I, P, P, I], I),
        "ddp_add_interface": ([P, I, I, I, P, pF, I, pI], I),
        "ddp_set_interface_method": ([P, I, I], I),
        "ddp_set_activation": ([P, I, I, I, F], I),
        "ddp_set_option": ([P, I, I64], I),
        "ddp_finalize": ([P, P, I], I),
        "ddp_param_count": ([P, I, pI64], I),
        "ddp_set_params": ([P, I, P, I], I),
        "ddp_get_params": ([P, I, P, I], I),
        "ddp_loss_and_grad": ([P, P, P], I),
        "ddp_step": ([P, I, P], I),
        "ddp_get_state": ([P, P, P, pI64], I),
        "ddp_set_state": ([P, P, P, I64], I),
        "ddp_eval": ([P, I, P, P, P], I),
        "ddp_sync": ([P], I),
        "ddp_time_kernels": ([P, I, pF], I),
        "ddp_plan_dump": ([P, ctypes.c_char_p], I),
        "ddp_plan": ([P], I),
        "ddp_last_error": ([], ctypes.c_char_p),
        "ddp_destroy": ([P], I),
        "ddp_autotune": ([P, I, ctypes.c_char_p, pI64], I),
        "ddp_mfma_probe": ([I, ctypes.POINTER(D)], I),
        "ddp_time_phases": ([P, I, pF], I),
        "ddp_loss_and_grad_static": ([P, P, P], I),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def mfma_probe(iters=2000):
    """FP32 MFMA rate (TFLOP/s) the current device sustains on a pure MFMA
    loop (the attainable matrix-core peak)."""
    L = load_library()
    t = ctypes.c_double()
    _check(L.ddp_mfma_probe(int(iters), ctypes.byref(t)))
    return t.value


def _check(rc):
    if rc != DDP_OK:
        raise DDPError(rc, _lib.ddp_last_error().decode())


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, torch.Tensor):
        return ctypes.c_void_p(a.data_ptr())
    return a.ctypes.data_as(ctypes.c_void_p)


def _host_f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


class Problem:
    """One domain-decomposed PINN problem on one GPU (libddpinn handle).

    fused=True: all subdomains in one persistent launch, step captured as a
    HIP graph.  fused=False: the same kernels launched per subdomain."""

    def __init__(self, prob: W.Problem, fused=True, device="cuda", stream=None, chunk_points=None,
                 blocks_per_cu=None, items_per_slot=None, recompute=None, concurrent=None, tail=None,
                 plan_only=False):
        L = load_library()
        self.prob = prob
        self.fused = bool(fused)
        self.n_sd = prob.n_sd
        self.d_out = prob.d_out
        # columns of eval(): the inverse problem stitches (u, K)
        self.n_eval_cols = prob.d_out + (1 if prob.pde == W.PDE_DIFFUSION2D_INV else 0)
        self._h = ctypes.c_void_p()
        coef = (ctypes.c_double * 4)(*([float(c) for c in prob.coef] + [0.0] * (4 - len(prob.coef))))
        _check(L.ddp_create(ctypes.byref(self._h), _METHOD[prob.method], _PDE[prob.pde], coef, len(prob.coef)))
        try:
            for s in prob.subdomains:
                nets = [s.widths] + ([s.aux_widths] if s.aux_widths is not None else [])
                allw = [w for n in nets for w in n]
                wd = (ctypes.c_int * len(allw))(*allw)
                nl = (ctypes.c_int * len(nets))(*[len(n) for n in nets])
                lw = (ctypes.c_float * 4)(*s.loss_w)
                sid = ctypes.c_int()
                _check(L.ddp_add_subdomain(self._h, len(nets), nl, wd, lw, float(s.lr), ctypes.byref(sid)))
                rx, rf = _host_f32(s.res_xy), _host_f32(s.res_f)
                _check(L.ddp_set_points(self._h, sid.value, DDP_RESIDUAL, rx.shape[0], _ptr(rx), _ptr(rf), 0))
                bx, bg = _host_f32(s.bnd_xy), _host_f32(s.bnd_g)
                _check(L.ddp_set_points(self._h, sid.value, DDP_DATA, bx.shape[0], _ptr(bx), _ptr(bg), 0))
                if s.aux_widths is not None:
                    ax, ag = _host_f32(s.aux_xy), _host_f32(s.aux_g)
                    _check(L.ddp_set_points(self._h, sid.value, DDP_DATA_AUX, ax.shape[0], _ptr(ax), _ptr(ag), 0))
                act, adaptive = getattr(s, "act", "tanh"), bool(getattr(s, "adaptive", False))
                if act != "tanh" or adaptive:
                    _check(L.ddp_set_activation(self._h, sid.value, _ACT[act], int(adaptive),
                                                float(getattr(s, "slope_n", 10.0))))
            for e in prob.interfaces:
                xy = _host_f32(e.xy)
                nrm = (ctypes.c_float * 2)(*[float(v) for v in e.normal])
                eid = ctypes.c_int()
                _check(L.ddp_add_interface(self._h, e.a, e.b, xy.shape[0], _ptr(xy), nrm, 0, ctypes.byref(eid)))
                if getattr(e, "method", None) is not None:
                    _check(L.ddp_set_interface_method(self._h, eid.value, _METHOD[e.method]))
            if chunk_points is not None:
                _check(L.ddp_set_option(self._h, DDP_OPT_CHUNK_POINTS, int(chunk_points)))
            if blocks_per_cu is not None:
                _check(L.ddp_set_option(self._h, DDP_OPT_BLOCKS_PER_CU, int(blocks_per_cu)))
            if items_per_slot is not None:
                _check(L.ddp_set_option(self._h, DDP_OPT_ITEMS_PER_SLOT, int(items_per_slot)))
            if recompute is not None:
                _check(L.ddp_set_option(self._h, DDP_OPT_RECOMPUTE, int(recompute)))
            if concurrent is not None:
                _check(L.ddp_set_option(self._h, DDP_OPT_CONCURRENT, int(concurrent)))
            if tail is not None:
                _check(L.ddp_set_option(self._h, DDP_OPT_TAIL, int(tail)))
            self.n_params = []
            for q in range(self.n_sd):
                n = ctypes.c_int64()
                _check(L.ddp_param_count(self._h, q, ctypes.byref(n)))
                self.n_params.append(n.value)
            self.offsets = np.concatenate([[0], np.cumsum(self.n_params)]).astype(np.int64)
            if plan_only:
                _check(L.ddp_plan(self._h))
                self.device = None
                return
            self.device = torch.device(device)
            if stream is None:
                stream = torch.cuda.current_stream(self.device)
            self.stream = stream
            _check(L.ddp_finalize(self._h, ctypes.c_void_p(stream.cuda_stream), 1 if fused else 0))
            self.set_params([s.params for s in prob.subdomains])
            self._loss = torch.zeros(self.n_sd, 5, dtype=torch.float32, device=self.device)
        except Exception:
            L.ddp_destroy(self._h)
            self._h = None
            raise

    # -- parameters -------------------------------------------------------
    def set_params(self, params):
        for q, p in enumerate(params):
            if isinstance(p, torch.Tensor) and p.is_cuda:
                t = p.detach().to(torch.float32).contiguous()
                _check(_lib.ddp_set_params(self._h, q, _ptr(t), 1))
            else:
                a = _host_f32(p)
                assert a.size == self.n_params[q]
                _check(_lib.ddp_set_params(self._h, q, _ptr(a), 0))

    def set_params_flat(self, flat):
        t = flat.detach().to(torch.float32).contiguous()
        for q in range(self.n_sd):
            _check(_lib.ddp_set_params(self._h, q, ctypes.c_void_p(t[self.offsets[q]:].data_ptr()), 1))

    def get_params(self):
        out = []
        for q in range(self.n_sd):
            a = np.empty(self.n_params[q], np.float32)
            _check(_lib.ddp_get_params(self._h, q, _ptr(a), 0))
            out.append(a)
        return out

    def split(self, flat):
        return [flat[self.offsets[q]:self.offsets[q + 1]] for q in range(self.n_sd)]

    # -- the training step ---------------------------------------------------
    def loss_and_grad(self):
        """(loss_terms (n_sd, 5), gradient (sum P_q,)) as device tensors."""
        lt = torch.empty(self.n_sd, 5, dtype=torch.float32, device=self.device)
        g = torch.empty(int(self.offsets[-1]), dtype=torch.float32, device=self.device)
        _check(_lib.ddp_loss_and_grad(self._h, _ptr(lt), _ptr(g)))
        return lt, g

    def loss_and_grad_static(self):
        """loss_and_grad through the allocation-free entry point (counters and
        activation stash in the library's static device scratch); the output
        tensors are allocated here, by the caller, as for loss_and_grad."""
        lt = torch.empty(self.n_sd, 5, dtype=torch.float32, device=self.device)
        g = torch.empty(int(self.offsets[-1]), dtype=torch.float32, device=self.device)
        _check(_lib.ddp_loss_and_grad_static(self._h, _ptr(lt), _ptr(g)))
        return lt, g

    def step(self, n=1):
        """n Adam steps; returns the loss terms of the last one (device tensor)."""
        _check(_lib.ddp_step(self._h, int(n), _ptr(self._loss)))
        return self._loss

    def get_state(self):
        n = int(self.offsets[-1])
        m = np.empty(n, np.float32)
        v = np.empty(n, np.float32)
        t = ctypes.c_int64()
        _check(_lib.ddp_get_state(self._h, _ptr(m), _ptr(v), ctypes.byref(t)))
        return {"params": self.get_params(), "m": m, "v": v, "t": t.value}

    def set_state(self, state):
        self.set_params(state["params"])
        m, v = _host_f32(state["m"]), _host_f32(state["v"])
        _check(_lib.ddp_set_state(self._h, _ptr(m), _ptr(v), int(state["t"])))

    def eval(self, xy, owner):
        xy = torch.as_tensor(np.asarray(xy, np.float32), device=self.device).contiguous()
        ow = torch.as_tensor(np.asarray(owner, np.int32), device=self.device).contiguous()
        out = torch.empty(xy.shape[0], self.n_eval_cols, dtype=torch.float32, device=self.device)
        _check(_lib.ddp_eval(self._h, xy.shape[0], _ptr(xy), _ptr(ow), _ptr(out)))
        return out

    def sync(self):
        _check(_lib.ddp_sync(self._h))

    def time_kernels(self, iters=10):
        ms = (ctypes.c_float * 2)()
        _check(_lib.ddp_time_kernels(self._h, int(iters), ms))
        return {"train_ms": ms[0], "reduce_ms": ms[1]}

    def time_phases(self, iters=10):
        """Mean ms of the fused step's train launches per phase: residual,
        data and interface items, and all items."""
        ms = (ctypes.c_float * 4)()
        _check(_lib.ddp_time_phases(self._h, int(iters), ms))
        return {"residual_ms": ms[0], "data_ms": ms[1], "interface_ms": ms[2], "all_ms": ms[3]}

    def autotune(self, iters=5, cache_path=None):
        """Pick the fastest work plan (see ddp_autotune); returns the choice."""
        ch = (ctypes.c_int64 * 6)()
        path = None if cache_path is None else str(cache_path).encode()
        _check(_lib.ddp_autotune(self._h, int(iters), path, ch))
        return {"chunk_points": ch[0], "items_per_slot": ch[1], "blocks_per_cu": ch[2], "recompute": ch[3],
                "concurrent": ch[4], "tail": ch[5]}

    def plan_dump(self, path):
        _check(_lib.ddp_plan_dump(self._h, str(path).encode()))

    def close(self):
        if self._h:
            _lib.ddp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DDPLoss(torch.autograd.Function):
    """J_q of every subdomain as a differentiable function of the flat
    parameters; backward returns gJ[q] * dJ_q/dTheta_q per subdomain (each
    subdomain's loss depends on its own parameters, neighbours held fixed)."""

    @staticmethod
    def forward(ctx, params_flat, problem):
        problem.set_params_flat(params_flat)
        lt, g = problem.loss_and_grad()
        ctx.problem = problem
        ctx.save_for_backward(g)
        return lt[:, 0].clone()

    @staticmethod
    def backward(ctx, gJ):
        g, = ctx.saved_tensors
        pb = ctx.problem
        counts = torch.as_tensor(pb.n_params, device=g.device)
        scale = torch.repeat_interleave(gJ.to(g.dtype), counts)
        return g * scale, None
