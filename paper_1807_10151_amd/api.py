"""Thin PyTorch binding over libsuppcg (same names as the C ABI).

PyTorch provides device memory and the stream; every step runs in the HIP
library.  Tensors must be float32, contiguous and on the context's GPU;
outputs are allocated here when not given.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib as L


class SupPCGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{L.STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


@dataclass(frozen=True)
class Geometry:
    """Parallel-beam geometry; dtheta = None means pi / n_angles."""
    rows: int
    cols: int
    n_angles: int
    n_bins: int
    pixel: float = 1.0
    theta0: float = 0.0
    dtheta: float | None = None
    bin_spacing: float = 1.0
    bin_offset: float = 0.0

    @property
    def n(self):
        return self.rows * self.cols

    @property
    def m(self):
        return self.n_angles * self.n_bins

    def c(self):
        return L.sp_geometry(self.rows, self.cols, self.pixel, self.n_angles, self.theta0,
                             -1.0 if self.dtheta is None else self.dtheta, self.n_bins,
                             self.bin_spacing, self.bin_offset)


class Context:
    """Owns one sp_ctx on a GPU; calls enqueue on torch's current stream."""

    def __init__(self, device: int = 0):
        self.lib = L.load()
        self.device = device
        h = ctypes.c_void_p()
        with torch.cuda.device(device):
            stream = torch.cuda.current_stream(device).cuda_stream
            rc = self.lib.sp_ctx_create(device, ctypes.c_void_p(stream), ctypes.byref(h))
        if rc != L.SP_OK:
            raise SupPCGError(rc, "sp_ctx_create failed")
        self.h = h

    def close(self):
        if self.h:
            self.lib.sp_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        self.lib.sp_ctx_set_stream(self.h, ctypes.c_void_p(s))

    def profile_enable(self, on: bool = True):
        """Time every projector/backprojector/preconditioner/S_TV launch with HIP
        events (the solver then runs its loop eagerly)."""
        self._stream()
        self._check(self.lib.sp_profile_enable(self.h, 1 if on else 0))

    def profile_read(self, kind: int):
        """(total_ms, launches) of one SP_PROF_* kind since profile_enable."""
        self._stream()
        ms = ctypes.c_double()
        n = ctypes.c_int32()
        self._check(self.lib.sp_profile_read(self.h, kind, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def _check(self, rc, ok=(L.SP_OK,)):
        if rc not in ok:
            raise SupPCGError(rc, self.lib.sp_last_error(self.h).decode())
        return rc


_CTX: dict = {}


def context(device: int = 0) -> Context:
    if device not in _CTX:
        _CTX[device] = Context(device)
    return _CTX[device]


def _dev(t: torch.Tensor, n: int, name: str, device: int):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or not t.is_cuda:
        raise TypeError(f"{name} must be a float32 CUDA tensor")
    if t.device.index != device:
        raise ValueError(f"{name} is on cuda:{t.device.index}, context is on cuda:{device}")
    if not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name} must be contiguous with {n} elements (got {tuple(t.shape)})")
    return ctypes.c_void_p(t.data_ptr())


def _out(t, shape, device):
    if t is None:
        return torch.empty(shape, dtype=torch.float32, device=f"cuda:{device}")
    return t


def sp_project(g: Geometry, x: torch.Tensor, y: torch.Tensor | None = None, ctx: Context | None = None):
    """y = R x: [rows, cols] -> [n_angles, n_bins]."""
    ctx = ctx or context(x.device.index or 0)
    y = _out(y, (g.n_angles, g.n_bins), ctx.device)
    ctx._stream()
    gc = g.c()
    ctx._check(ctx.lib.sp_project(ctx.h, ctypes.byref(gc), _dev(x, g.n, "x", ctx.device),
                                  _dev(y, g.m, "y", ctx.device)))
    return y


def sp_backproject(g: Geometry, y: torch.Tensor, x: torch.Tensor | None = None, ctx: Context | None = None):
    """x = R^T y: [n_angles, n_bins] -> [rows, cols]."""
    ctx = ctx or context(y.device.index or 0)
    x = _out(x, (g.rows, g.cols), ctx.device)
    ctx._stream()
    gc = g.c()
    ctx._check(ctx.lib.sp_backproject(ctx.h, ctypes.byref(gc), _dev(y, g.m, "y", ctx.device),
                                      _dev(x, g.n, "x", ctx.device)))
    return x


def sp_residual(g: Geometry, x: torch.Tensor, b: torch.Tensor, ctx: Context | None = None):
    """(r, f): r = R x - b and f = ||r||^2 (float64, 0-d CUDA tensor)."""
    ctx = ctx or context(x.device.index or 0)
    r = _out(None, (g.n_angles, g.n_bins), ctx.device)
    f = torch.empty((), dtype=torch.float64, device=f"cuda:{ctx.device}")
    ctx._stream()
    gc = g.c()
    ctx._check(ctx.lib.sp_residual(ctx.h, ctypes.byref(gc), _dev(x, g.n, "x", ctx.device),
                                   _dev(b, g.m, "b", ctx.device), _dev(r, g.m, "r", ctx.device),
                                   ctypes.c_void_p(f.data_ptr())))
    return r, f


def sp_gradient(g: Geometry, x: torch.Tensor, b: torch.Tensor, grad: torch.Tensor | None = None,
                ctx: Context | None = None):
    """(grad, f): grad = R^T (R x - b) with the residual kept in float64, and
    f = ||R x - b||^2 (float64, 0-d CUDA tensor)."""
    ctx = ctx or context(x.device.index or 0)
    grad = _out(grad, (g.rows, g.cols), ctx.device)
    f = torch.empty((), dtype=torch.float64, device=f"cuda:{ctx.device}")
    ctx._stream()
    gc = g.c()
    ctx._check(ctx.lib.sp_gradient(ctx.h, ctypes.byref(gc), _dev(x, g.n, "x", ctx.device),
                                   _dev(b, g.m, "b", ctx.device), _dev(grad, g.n, "grad", ctx.device),
                                   ctypes.c_void_p(f.data_ptr())))
    return grad, f


def sp_suppcg_solve_batched(geoms, bs, x0s=None, *, K: int = 1, a: float = 0.5, gamma: float = 0.5,
                            max_trials: int = 100, precond="ramp", mu: float = 1e-5,
                            rho: float = 0.8, max_iter: int = 20, eps: float = 0.0,
                            graph: bool = True, autotune: bool = False, trace: bool = True,
                            x_half=None, x_last=None, ctx: Context | None = None):
    """Algorithm 3 on a batch of slices in lockstep (one launch per stage for
    all slices).  geoms, bs (and optional x0s, x_half, x_last): per-slice lists.
    Returns one SolveResult per slice (trace: f_half, tv_half, ell)."""
    n = len(geoms)
    if n < 1 or len(bs) != n:
        raise ValueError("need one data tensor per geometry")
    ctx = ctx or context(bs[0].device.index or 0)
    dev = ctx.device
    x_half = list(x_half) if x_half is not None else [None] * n
    x_last = list(x_last) if x_last is not None else [None] * n
    for i, g in enumerate(geoms):
        x_half[i] = _out(x_half[i], (g.rows, g.cols), dev)
        x_last[i] = _out(x_last[i], (g.rows, g.cols), dev)
    garr = (L.sp_geometry * n)(*[g.c() for g in geoms])
    ptrs = lambda ts, size, name: (ctypes.c_void_p * n)(
        *[_dev(t, sz, name, dev).value if t is not None else None for t, sz in zip(ts, size)])
    b_arr = ptrs(bs, [g.m for g in geoms], "b")
    x0_arr = ptrs(x0s, [g.n for g in geoms], "x0") if x0s is not None else None
    xh_arr = ptrs(x_half, [g.n for g in geoms], "x_half")
    xl_arr = ptrs(x_last, [g.n for g in geoms], "x_last")
    tvp = L.sp_tv_params(K, a, gamma, max_trials)
    pc = _precond(precond, mu, rho, None)
    flags = (L.SP_FLAG_GRAPH if graph else 0) | (L.SP_FLAG_AUTOTUNE if autotune else 0)
    sp = L.sp_solve_params(eps, max_iter, flags, None)
    cap = max(max_iter, 1)
    k_out = (ctypes.c_int32 * n)()
    status = np.zeros(n, dtype=np.int32)
    f_half = np.zeros((n, cap))
    tv_half = np.zeros((n, cap))
    ell = np.zeros((n, cap), dtype=np.int32)
    dp = lambda a_: a_.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    ip = lambda a_: a_.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    tr = L.sp_batch_trace(dp(f_half), dp(tv_half), ip(ell), cap, ip(status))
    ctx._stream()
    rc = ctx.lib.sp_suppcg_solve_batched(
        ctx.h, n, garr, b_arr, x0_arr, ctypes.byref(tvp), ctypes.byref(pc), ctypes.byref(sp), xh_arr,
        xl_arr, k_out, ctypes.byref(tr))
    ctx._check(rc)
    out = []
    for i in range(n):
        done = min(max(k_out[i] - 1, 0), cap)
        tr_i = {"f_half": f_half[i, :done], "tv_half": tv_half[i, :done], "ell": ell[i, :done]} if trace else {}
        out.append(SolveResult(int(k_out[i]), x_half[i], x_last[i], int(status[i]), tr_i))
    return out


def sp_suppcg_solve_async(g: Geometry, b: torch.Tensor, x0: torch.Tensor | None = None, *,
                          K: int = 1, a: float = 0.5, gamma: float = 0.5, max_trials: int = 100,
                          precond="ramp", mu: float = 1e-5, rho: float = 0.8, max_iter: int = 20,
                          eps: float = 0.0, graph: bool = True, resume: bool = False,
                          x_half: torch.Tensor | None = None, x_last: torch.Tensor | None = None,
                          net: "LearnedPrecond | None" = None, ctx: Context | None = None):
    """SP_FLAG_ASYNC solve: enqueues the run and returns at once.  Returns
    (k, x_half, x_last) with k an int32 CUDA tensor written when the run
    completes; sp_solve_status() gives the status afterwards."""
    ctx = ctx or context(b.device.index or 0)
    dev = ctx.device
    x_half = _out(x_half, (g.rows, g.cols), dev)
    x_last = _out(x_last, (g.rows, g.cols), dev)
    k = torch.zeros((), dtype=torch.int32, device=f"cuda:{dev}")
    gc = g.c()
    tvp = L.sp_tv_params(K, a, gamma, max_trials)
    pc = _precond(precond, mu, rho, net)
    flags = L.SP_FLAG_ASYNC | (L.SP_FLAG_GRAPH if graph else 0) | (L.SP_FLAG_RESUME if resume else 0)
    sp = L.sp_solve_params(eps, max_iter, flags, None)
    ctx._stream()
    rc = ctx.lib.sp_suppcg_solve(ctx.h, ctypes.byref(gc), _dev(b, g.m, "b", dev),
                                 _dev(x0, g.n, "x0", dev) if x0 is not None else None,
                                 ctypes.byref(tvp), ctypes.byref(pc), ctypes.byref(sp),
                                 _dev(x_half, g.n, "x_half", dev), _dev(x_last, g.n, "x_last", dev),
                                 ctypes.cast(ctypes.c_void_p(k.data_ptr()), ctypes.POINTER(ctypes.c_int32)),
                                 None)
    ctx._check(rc)
    return k, x_half, x_last


def sp_solve_status(count: int = 1, ctx: Context | None = None):
    """(k list, status list) of the slices of the last solve (waits for it)."""
    ctx = ctx or context(0)
    k = (ctypes.c_int32 * count)()
    st = (ctypes.c_int32 * count)()
    ctx._stream()
    ctx._check(ctx.lib.sp_solve_status(ctx.h, count, k, st))
    return list(k), list(st)


def sp_state_save(ctx: Context | None = None) -> bytes:
    """Algorithm 3's carried state of the context's last single-slice solve."""
    ctx = ctx or context(0)
    ctx._stream()
    size = ctypes.c_int64(0)
    ctx._check(ctx.lib.sp_state_save(ctx.h, None, ctypes.byref(size)))
    buf = ctypes.create_string_buffer(size.value)
    ctx._check(ctx.lib.sp_state_save(ctx.h, buf, ctypes.byref(size)))
    return buf.raw[:size.value]


def sp_state_load(blob: bytes, ctx: Context | None = None):
    """Puts a saved state into the context (the next solve may resume from it)."""
    ctx = ctx or context(0)
    ctx._stream()
    buf = ctypes.create_string_buffer(bytes(blob), len(blob))
    ctx._check(ctx.lib.sp_state_load(ctx.h, buf, len(blob)))


def batch_tuning(ctx: Context | None = None) -> dict:
    """Launch shapes the batched solver uses, per stage: (order, workgroups per CU)."""
    ctx = ctx or context(0)
    arr = (ctypes.c_int32 * 16)()
    ctx._check(ctx.lib.sp_batch_tuning(ctx.h, arr, 16))
    names = ["prep", "project", "backproject", "fft_rows", "fft_cols", "tv", "vector", "per_slice"]
    return {nm: ("xcd" if arr[2 * i] else "slice", int(arr[2 * i + 1])) for i, nm in enumerate(names)}


def tune_shapes(g: Geometry, ctx: Context | None = None) -> dict:
    """Times R's ray parts (1, 2, 4, 8) and R^T's pixels per lane (2, 4) for g on
    the GPU and stores the fastest in the process-wide shape table."""
    ctx = ctx or context(0)
    parts, px = ctypes.c_int32(0), ctypes.c_int32(0)
    ms = (ctypes.c_double * 6)()
    gc = g.c()
    ctx._stream()
    ctx._check(ctx.lib.sp_tune_shapes(ctx.h, ctypes.byref(gc), ctypes.byref(parts), ctypes.byref(px), ms))
    return {"parts": parts.value, "px": px.value,
            "R_ms": {p_: ms[i] for i, p_ in enumerate((1, 2, 4, 8))},
            "RT_ms": {2: ms[4], 4: ms[5]}}


def tuning_set(g: Geometry, parts: int, px: int):
    """Stores launch shapes for g (parts = px = 0 erases the entry)."""
    gc = g.c()
    rc = L.load().sp_tuning_set(ctypes.byref(gc), parts, px)
    if rc != L.SP_OK:
        raise SupPCGError(rc, f"sp_tuning_set rejected parts={parts} px={px}")


def tuning_list():
    """[(Geometry, parts, px)] of the shape table."""
    lib = L.load()
    cnt = ctypes.c_int32(0)
    lib.sp_tuning_list(None, None, None, 0, ctypes.byref(cnt))
    n = cnt.value
    gs = (L.sp_geometry * max(n, 1))()
    parts = (ctypes.c_int32 * max(n, 1))()
    px = (ctypes.c_int32 * max(n, 1))()
    lib.sp_tuning_list(gs, parts, px, n, ctypes.byref(cnt))
    out = []
    for i in range(min(n, cnt.value)):
        c = gs[i]
        out.append((Geometry(c.rows, c.cols, c.n_angles, c.n_bins, c.pixel, c.theta0,
                             None if c.dtheta <= 0 else c.dtheta, c.bin_spacing, c.bin_offset),
                    parts[i], px[i]))
    return out


def tuning_clear():
    L.load().sp_tuning_clear()


def tuning_save(path: str):
    """Writes the shape table as JSON (one record per geometry)."""
    import json
    recs = [{"rows": g.rows, "cols": g.cols, "n_angles": g.n_angles, "n_bins": g.n_bins, "pixel": g.pixel,
             "theta0": g.theta0, "dtheta": g.dtheta, "bin_spacing": g.bin_spacing, "bin_offset": g.bin_offset,
             "parts": p_, "px": x_} for g, p_, x_ in tuning_list()]
    with open(path, "w") as f:
        json.dump({"shapes": recs}, f, indent=1)


def tuning_load(path: str):
    """Adds the records of a JSON file written by tuning_save to the shape table."""
    import json
    with open(path) as f:
        recs = json.load(f)["shapes"]
    for r in recs:
        g = Geometry(r["rows"], r["cols"], r["n_angles"], r["n_bins"], r["pixel"], r["theta0"], r["dtheta"],
                     r["bin_spacing"], r["bin_offset"])
        tuning_set(g, int(r["parts"]), int(r["px"]))


class StoredMatrix:
    """R and R^T of geometry g as stored CSR matrices on the GPU (sp_matrix_*)."""

    def __init__(self, g: Geometry, ctx: Context | None = None):
        self.ctx = ctx or context(0)
        self.g = g
        h = ctypes.c_void_p()
        gc = g.c()
        self.ctx._stream()
        self.ctx._check(self.ctx.lib.sp_matrix_build(self.ctx.h, ctypes.byref(gc), ctypes.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            self.ctx.lib.sp_matrix_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        """(nonzeros of R, device bytes of both sides)."""
        nnz, nbytes = ctypes.c_int64(0), ctypes.c_int64(0)
        self.ctx._check(self.ctx.lib.sp_matrix_info(self.h, ctypes.byref(nnz), ctypes.byref(nbytes)))
        return nnz.value, nbytes.value

    def project(self, x: torch.Tensor, y: torch.Tensor | None = None):
        """y = R x."""
        g = self.g
        y = _out(y, (g.n_angles, g.n_bins), self.ctx.device)
        self.ctx._stream()
        self.ctx._check(self.ctx.lib.sp_matrix_project(self.ctx.h, self.h, _dev(x, g.n, "x", self.ctx.device),
                                                       _dev(y, g.m, "y", self.ctx.device)))
        return y

    def backproject(self, y: torch.Tensor, x: torch.Tensor | None = None):
        """x = R^T y."""
        g = self.g
        x = _out(x, (g.rows, g.cols), self.ctx.device)
        self.ctx._stream()
        self.ctx._check(self.ctx.lib.sp_matrix_backproject(self.ctx.h, self.h, _dev(y, g.m, "y", self.ctx.device),
                                                           _dev(x, g.n, "x", self.ctx.device)))
        return x

    def export(self, side: int):
        """(row_ptr int64, col int32, val float32) of R (side 0) or R^T (side 1), on the host."""
        nnz, _ = self.info()
        rows = self.g.m if side == 0 else self.g.n
        rp = np.zeros(rows + 1, dtype=np.int64)
        col = np.zeros(nnz, dtype=np.int32)
        val = np.zeros(nnz, dtype=np.float32)
        self.ctx._stream()
        self.ctx._check(self.ctx.lib.sp_matrix_export(self.ctx.h, self.h, side, rp.ctypes.data_as(ctypes.c_void_p),
                                                      col.ctypes.data_as(ctypes.c_void_p),
                                                      val.ctypes.data_as(ctypes.c_void_p)))
        return rp, col, val


class LearnedPrecond:
    """M = C^T diag(softplus(d)) C (sp_lp_* calls); parameters live on the GPU."""

    def __init__(self, layers: int = 4, channels: int = 16, ctx: Context | None = None):
        self.ctx = ctx or context(0)
        h = ctypes.c_void_p()
        self.ctx._check(self.ctx.lib.sp_lp_create(self.ctx.h, layers, channels, ctypes.byref(h)))
        self.h = h
        self.layers = layers
        self.channels = channels

    def close(self):
        if self.h:
            self.ctx.lib.sp_lp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def num_params(self) -> int:
        return int(self.ctx.lib.sp_lp_num_params(self.h))

    def set_params(self, theta):
        a = np.ascontiguousarray(np.asarray(theta, dtype=np.float32).ravel())
        self.ctx._stream()
        self.ctx._check(self.ctx.lib.sp_lp_set_params(
            self.ctx.h, self.h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), a.size))

    def get_params(self) -> np.ndarray:
        a = np.zeros(self.num_params, dtype=np.float32)
        self.ctx._stream()
        self.ctx._check(self.ctx.lib.sp_lp_get_params(
            self.ctx.h, self.h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), a.size))
        return a

    def apply(self, u: torch.Tensor, z: torch.Tensor | None = None):
        """z = M u for u of shape [B, H, W] or [H, W]."""
        shape = tuple(u.shape)
        B, H, W = (1,) + shape if len(shape) == 2 else shape
        z = _out(z, shape, self.ctx.device)
        self.ctx._stream()
        n = B * H * W
        self.ctx._check(self.ctx.lib.sp_lp_apply(self.ctx.h, self.h, B, H, W,
                                                 _dev(u, n, "u", self.ctx.device),
                                                 _dev(z, n, "z", self.ctx.device)))
        return z

    def loss_grad(self, Av: torch.Tensor, v: torch.Tensor, idx: torch.Tensor,
                  grad: torch.Tensor | None = None, margin: int = 0):
        """(loss [float64 0-d], grad [num_params]) on the minibatch idx of (Av, v),
        the loss taken over pixels at least `margin` from every edge."""
        N, H, W = Av.shape
        if idx.dtype != torch.int32 or not idx.is_cuda or not idx.is_contiguous():
            raise TypeError("idx must be a contiguous int32 CUDA tensor")
        dev = f"cuda:{self.ctx.device}"
        loss = torch.empty((), dtype=torch.float64, device=dev)
        grad = _out(grad, (self.num_params,), self.ctx.device)
        self.ctx._stream()
        self.ctx._check(self.ctx.lib.sp_lp_loss_grad(
            self.ctx.h, self.h, H, W, _dev(Av, N * H * W, "Av", self.ctx.device),
            _dev(v, N * H * W, "v", self.ctx.device), N, ctypes.c_void_p(idx.data_ptr()),
            idx.numel(), int(margin), ctypes.c_void_p(loss.data_ptr()),
            _dev(grad, self.num_params, "grad", self.ctx.device)))
        return loss, grad

    def adam_step(self, grad: torch.Tensor, lr: float, step: int, beta1=0.9, beta2=0.999, eps=1e-8):
        self.ctx._stream()
        self.ctx._check(self.ctx.lib.sp_lp_adam_step(
            self.ctx.h, self.h, _dev(grad, self.num_params, "grad", self.ctx.device), lr, beta1,
            beta2, eps, step))


def _precond(kind, mu, rho, net=None):
    k = {"ramp": L.SP_PRECOND_RAMP, "none": L.SP_PRECOND_NONE,
         "learned": L.SP_PRECOND_LEARNED}[kind] if isinstance(kind, str) else kind
    return L.sp_precond(k, mu, rho, net.h if net is not None else None)


def sp_precond_apply(g: Geometry, gin: torch.Tensor, mu: float = 1e-5, rho: float = 0.8,
                     kind="ramp", z: torch.Tensor | None = None, net=None,
                     ctx: Context | None = None):
    """z = M g with the ramp-Hamming Fourier preconditioner (or M = I)."""
    ctx = ctx or context(gin.device.index or 0)
    z = _out(z, (g.rows, g.cols), ctx.device)
    ctx._stream()
    gc = g.c()
    pc = _precond(kind, mu, rho, net)
    ctx._check(ctx.lib.sp_precond_apply(ctx.h, ctypes.byref(gc), ctypes.byref(pc),
                                        _dev(gin, g.n, "g", ctx.device), _dev(z, g.n, "z", ctx.device)))
    return z


def sp_tv(g: Geometry, x: torch.Tensor, ctx: Context | None = None):
    """TV(x) as a float64 0-d CUDA tensor."""
    ctx = ctx or context(x.device.index or 0)
    out = torch.empty((), dtype=torch.float64, device=f"cuda:{ctx.device}")
    ctx._stream()
    gc = g.c()
    ctx._check(ctx.lib.sp_tv(ctx.h, ctypes.byref(gc), _dev(x, g.n, "x", ctx.device),
                             ctypes.c_void_p(out.data_ptr())))
    return out


@dataclass
class ARTResult:
    x: torch.Tensor
    status: int
    trace: dict = field(default_factory=dict)


def _art_call(g, b, x0, K, a, gamma, max_trials, r, lam, max_iter, graph, se_ref, se_axes, se_c, timing, x_out,
              ctx, blob):
    ctx = ctx or context(b.device.index or 0)
    dev = ctx.device
    x_out = _out(x_out, (g.rows, g.cols), dev)
    gc = g.c()
    tvp = L.sp_tv_params(K, a, gamma, max_trials)
    sp = L.sp_solve_params(0.0, max_iter, L.SP_FLAG_GRAPH if graph else 0, None)
    cap = max(max_iter, 1)
    dp = lambda a_: a_.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    ip = lambda a_: a_.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    arrs = {"tv_half": np.zeros(cap), "ell": np.zeros(cap, dtype=np.int32),
            "trials": np.zeros(cap * max(K, 1), dtype=np.int32)}
    tr = L.sp_trace(None, dp(arrs["tv_half"]), None, None, None, ip(arrs["ell"]), ip(arrs["trials"]), cap,
                    0.0, 0.0, 0, None, 0, 0)
    if se_ref is not None:
        _dev(se_ref, g.n, "se_ref", dev)
        axes = paper_se_axes(g) if se_axes is None else tuple(float(v) for v in se_axes)
        arrs["se"] = np.full(cap, np.nan)
        tr.se_ref = ctypes.c_void_p(se_ref.data_ptr())
        tr.se_axes[0], tr.se_axes[1] = axes
        tr.se_c = se_c
        tr.se = dp(arrs["se"])
    if timing:
        arrs["t_ms"] = np.zeros(cap)
        tr.t_ms = dp(arrs["t_ms"])
    ctx._stream()
    if blob:
        rc = ctx.lib.sp_blobart_solve(ctx.h, ctypes.byref(gc), _dev(b, g.m, "b", dev), r, lam, ctypes.byref(sp),
                                      _dev(x_out, g.n, "x_out", dev), ctypes.byref(tr))
    else:
        rc = ctx.lib.sp_supart_solve(ctx.h, ctypes.byref(gc), _dev(b, g.m, "b", dev),
                                     _dev(x0, g.n, "x0", dev) if x0 is not None else None, ctypes.byref(tvp),
                                     r, lam, ctypes.byref(sp), _dev(x_out, g.n, "x_out", dev), ctypes.byref(tr))
    ctx._check(rc, ok=(L.SP_MAXITER, L.SP_TRIALS_EXHAUSTED))
    done = min(tr.bodies, cap)
    out = {}
    if K > 0:
        out["tv_half"] = arrs["tv_half"][:done]
        out["ell"] = arrs["ell"][:done]
        out["trials"] = arrs["trials"][:done * K].reshape(done, K)
    if se_ref is not None:
        out["se"] = np.concatenate([[tr.se0], arrs["se"][:done]])
    if timing:
        out["t_ms"] = np.concatenate([[0.0], arrs["t_ms"][:done]])
    return ARTResult(x_out, rc, out)


def sp_supart_solve(g: Geometry, b: torch.Tensor, x0: torch.Tensor | None = None, *, K: int = 0,
                    a: float = 1 - 1e-5, gamma: float = 1e-2, max_trials: int = 100, r: float = 5.0,
                    lam: float = 0.05, max_iter: int = 10, graph: bool = True, se_ref: torch.Tensor | None = None,
                    se_axes=None, se_c: float = 0.0, timing: bool = False, x_out: torch.Tensor | None = None,
                    ctx: Context | None = None) -> ARTResult:
    """ART for the Bayesian criterion (K = 0) or SupART (K > 0), max_iter cycles
    through the rays (sp_supart_solve).  The trace holds ell, tv_half and
    trials (SupART), "se" = [SE(x_0), SE(x_1), ...] with se_ref, and
    "t_ms" = [0, t(x_1), ...] with timing."""
    return _art_call(g, b, x0, K, a, gamma, max_trials, r, lam, max_iter, graph, se_ref, se_axes, se_c, timing,
                     x_out, ctx, False)


def sp_blobart_solve(g: Geometry, b: torch.Tensor, *, r: float = 5.0, lam: float = 1e-2, max_iter: int = 10,
                     graph: bool = True, se_ref: torch.Tensor | None = None, se_axes=None, se_c: float = 0.0,
                     timing: bool = False, x_out: torch.Tensor | None = None,
                     ctx: Context | None = None) -> ARTResult:
    """BlobART (sp_blobart_solve): ART on Kaiser-Bessel blob coefficients; x is
    the blob image at the pixel centres; trace as for sp_supart_solve."""
    return _art_call(g, b, None, 0, 0.5, 0.0, 100, r, lam, max_iter, graph, se_ref, se_axes, se_c, timing, x_out,
                     ctx, True)


# The paper's ellipse for the selective error: semi-axes 5 cm (horizontal) and
# 7 cm (vertical) on a phantom 243 pixels of 0.0752 cm wide (Section 4.2);
# other images keep the same share of their width.
_SE_WIDTH = 243 * 0.0752
_SE_AXES = (5.0, 7.0)


def paper_se_axes(g: Geometry):
    """(horizontal, vertical) semi-axes of the selective-error ellipse for g."""
    w = g.cols * g.pixel
    return (_SE_AXES[0] / _SE_WIDTH * w, _SE_AXES[1] / _SE_WIDTH * w)


def sp_selective_error(g: Geometry, x: torch.Tensor, ref: torch.Tensor, axes=None, C: float = 0.0,
                       ctx: Context | None = None):
    """SE(x) of eq. (4.1) as a float64 0-d CUDA tensor (axes default: paper_se_axes)."""
    ctx = ctx or context(x.device.index or 0)
    out = torch.empty((), dtype=torch.float64, device=f"cuda:{ctx.device}")
    ax = paper_se_axes(g) if axes is None else tuple(float(v) for v in axes)
    axc = (ctypes.c_double * 2)(*ax)
    ctx._stream()
    gc = g.c()
    ctx._check(ctx.lib.sp_selective_error(ctx.h, ctypes.byref(gc), _dev(x, g.n, "x", ctx.device),
                                          _dev(ref, g.n, "ref", ctx.device), axc, C,
                                          ctypes.c_void_p(out.data_ptr())))
    return out


def sp_tv_grad(g: Geometry, x: torch.Tensor, ctx: Context | None = None):
    """(t_bar, ||t_bar||^2)."""
    ctx = ctx or context(x.device.index or 0)
    tb = _out(None, (g.rows, g.cols), ctx.device)
    n2 = torch.empty((), dtype=torch.float64, device=f"cuda:{ctx.device}")
    ctx._stream()
    gc = g.c()
    ctx._check(ctx.lib.sp_tv_grad(ctx.h, ctypes.byref(gc), _dev(x, g.n, "x", ctx.device),
                                  _dev(tb, g.n, "tbar", ctx.device), ctypes.c_void_p(n2.data_ptr())))
    return tb, n2


def sp_tv_perturb(g: Geometry, x: torch.Tensor, ell: int, K: int, a: float, gamma: float,
                  max_trials: int = 100, ctx: Context | None = None):
    """Algorithm 1.  Returns (x_half, ell, TV(x_half), trials per inner step)."""
    ctx = ctx or context(x.device.index or 0)
    dev = f"cuda:{ctx.device}"
    xh = torch.empty((g.rows, g.cols), dtype=torch.float32, device=dev)
    ell_t = torch.tensor([ell], dtype=torch.int32, device=dev)
    tvh = torch.empty((), dtype=torch.float64, device=dev)
    trials = torch.zeros(max(K, 1), dtype=torch.int32, device=dev)
    ctx._stream()
    gc = g.c()
    p = L.sp_tv_params(K, a, gamma, max_trials)
    ctx._check(ctx.lib.sp_tv_perturb(ctx.h, ctypes.byref(gc), ctypes.byref(p),
                                     _dev(x, g.n, "x", ctx.device), ctypes.c_void_p(ell_t.data_ptr()),
                                     _dev(xh, g.n, "x_half", ctx.device),
                                     ctypes.c_void_p(tvh.data_ptr()),
                                     ctypes.c_void_p(trials.data_ptr())))
    return xh, int(ell_t.item()), float(tvh.item()), trials[:K].cpu().tolist()


@dataclass
class SolveResult:
    k: int
    x_half: torch.Tensor
    x_last: torch.Tensor
    status: int
    trace: dict = field(default_factory=dict)

    @property
    def status_name(self):
        return L.STATUS_NAMES.get(self.status, str(self.status))


def sp_suppcg_solve(g: Geometry, b: torch.Tensor, x0: torch.Tensor | None = None, *,
                    K: int = 1, a: float = 0.5, gamma: float = 0.5, max_trials: int = 100,
                    precond="ramp", mu: float = 1e-5, rho: float = 0.8, max_iter: int = 20,
                    eps: float = 0.0, graph: bool = False, replay=None, trace: bool = True,
                    x_half: torch.Tensor | None = None, x_last: torch.Tensor | None = None,
                    net: "LearnedPrecond | None" = None, g_snap: torch.Tensor | None = None,
                    resume: bool = False, se_ref: torch.Tensor | None = None, se_axes=None,
                    se_c: float = 0.0, timing: bool = False,
                    ctx: Context | None = None) -> SolveResult:
    """Algorithm 3 (SupPCG); K = 0 gives plain PCG, precond="none" gives CG.

    g_snap (optional, float32 device tensor [count, rows, cols]): receives the
    gradient g_{k+1/2} that loop body k hands to the preconditioner.
    resume: continue for max_iter more loop bodies from the state the context
    holds (the previous solve, or state_load); x0 is ignored.
    se_ref (optional phantom, float32 device tensor [rows, cols]): the trace
    gets "se" = [SE(x_0), SE(x_1), SE(x_2), ...], the selective error of eq.
    (4.1) of every iterate, over the ellipse se_axes (default: paper_se_axes)
    with constant se_c (<= 0: relative to the phantom inside the ellipse).
    timing: the trace gets "t_ms" = [0, t(x_1), t(x_2), ...], milliseconds
    from the call's first launch to the moment each iterate is formed."""
    ctx = ctx or context(b.device.index or 0)
    dev = ctx.device
    snap_count = 0
    if g_snap is not None:
        if g_snap.dim() != 3 or tuple(g_snap.shape[1:]) != (g.rows, g.cols):
            raise ValueError("g_snap must have shape [count, rows, cols]")
        snap_count = int(g_snap.shape[0])
        _dev(g_snap, snap_count * g.n, "g_snap", dev)
    x_half = _out(x_half, (g.rows, g.cols), dev)
    x_last = _out(x_last, (g.rows, g.cols), dev)
    gc = g.c()
    tvp = L.sp_tv_params(K, a, gamma, max_trials)
    pc = _precond(precond, mu, rho, net)
    flags = (L.SP_FLAG_GRAPH if graph else 0) | (L.SP_FLAG_RESUME if resume else 0)
    rep_arr = None
    if replay is not None:
        flags |= L.SP_FLAG_REPLAY
        rep = np.ascontiguousarray(np.asarray(replay, dtype=np.int32).reshape(-1))
        if rep.size < max_iter * max(K, 1):
            raise ValueError("replay needs max_iter * K entries")
        rep_arr = (ctypes.c_int32 * rep.size)(*rep.tolist())
    sp = L.sp_solve_params(eps, max_iter, flags,
                           ctypes.cast(rep_arr, ctypes.POINTER(ctypes.c_int32)) if rep_arr is not None else None)
    cap = max(max_iter, 1)
    tr = None
    arrs = {}
    if se_ref is not None:
        _dev(se_ref, g.n, "se_ref", dev)
        se_axes = paper_se_axes(g) if se_axes is None else tuple(float(v) for v in se_axes)
    if trace or g_snap is not None or se_ref is not None or timing:
        arrs = {"f_half": np.zeros(cap), "tv_half": np.zeros(cap), "alpha": np.zeros(cap),
                "beta": np.zeros(cap), "s_norm": np.zeros(cap),
                "ell": np.zeros(cap, dtype=np.int32), "trials": np.zeros(cap * max(K, 1), dtype=np.int32)}
        dp = lambda a_: a_.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        ip = lambda a_: a_.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        tr = L.sp_trace(dp(arrs["f_half"]), dp(arrs["tv_half"]), dp(arrs["alpha"]), dp(arrs["beta"]),
                        dp(arrs["s_norm"]), ip(arrs["ell"]), ip(arrs["trials"]), cap, 0.0, 0.0, 0,
                        ctypes.c_void_p(g_snap.data_ptr()) if g_snap is not None else None,
                        snap_count, 0)
        if se_ref is not None:
            arrs_se = np.full(cap, np.nan)
            tr.se_ref = ctypes.c_void_p(se_ref.data_ptr())
            tr.se_axes[0], tr.se_axes[1] = se_axes
            tr.se_c = se_c
            tr.se = dp(arrs_se)
        if timing:
            arrs_t = np.zeros(cap)
            tr.t_ms = dp(arrs_t)
    k_out = ctypes.c_int32(0)
    ctx._stream()
    rc = ctx.lib.sp_suppcg_solve(ctx.h, ctypes.byref(gc), _dev(b, g.m, "b", dev),
                                 _dev(x0, g.n, "x0", dev) if x0 is not None else None,
                                 ctypes.byref(tvp), ctypes.byref(pc), ctypes.byref(sp),
                                 _dev(x_half, g.n, "x_half", dev), _dev(x_last, g.n, "x_last", dev),
                                 ctypes.byref(k_out), ctypes.byref(tr) if tr is not None else None)
    ctx._check(rc, ok=(L.SP_MAXITER, L.SP_CONVERGED, L.SP_BREAKDOWN_CONVERGED, L.SP_TRIALS_EXHAUSTED))
    out = {}
    if tr is not None:
        done = min(tr.bodies, cap)
        out = {key: v[:done] if key != "trials" else v[:done * max(K, 1)].reshape(done, max(K, 1))
               for key, v in arrs.items()}
        out["f0"] = tr.f0
        out["alpha0"] = tr.alpha0
        out["fallbacks"] = tr.fallbacks
        if se_ref is not None:
            out["se"] = np.concatenate([[tr.se0, tr.se1], arrs_se[:done]])
        if timing:
            out["t_ms"] = np.concatenate([[0.0, tr.t1_ms], arrs_t[:done]])
    return SolveResult(k_out.value, x_half, x_last, rc, out)
