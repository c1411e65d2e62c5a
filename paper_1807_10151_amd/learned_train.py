"""Training and evaluation of the learned preconditioner M = C^T diag(softplus(d)) C.

Everything that touches an image runs in libsuppcg's kernels: probe data
A v = R^T R v through the projector and backprojector, the network's forward
and backward passes and Adam through the sp_lp_* calls, the Krylov probes
through the solver's gradient snapshots.  This module only orchestrates.

The paper defines the Fourier preconditioner of Section 3.2 (eq. 3.2) and no
learned one; the recipe below is this library's own:
  * probes: Gaussian vectors plus Krylov vectors, the normalised gradients
    g_{k+1/2} (Algorithm 2, step 1) that the plain solver (the Fourier M)
    hands to its preconditioner in loop bodies 1..64 on a set of phantoms;
  * loss: mean over a minibatch of ||M A v - v||^2 / ||v||^2 with A = R^T R;
  * Adam (lr 1e-3, betas 0.9/0.999), minibatch 256, He-normal C, and d
    started at one common value per channel, the one that minimises the loss
    of the initial network over a global scale of M (the loss is not scale
    invariant while PCG is, so a badly scaled start wastes the Adam steps);
  * evaluation (time to target): the plain solver's f(x_{100+1/2}) and
    TV(x_{100+1/2}) are the targets; the learned run reports the first loop
    body that reaches each, and both forms are timed to their targets.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import api

__all__ = ["TrainConfig", "CropConfig", "phantom_data", "gaussian_probes", "krylov_probes",
           "normal_op", "crop_probes", "init_theta", "scale_init", "train", "train_crops",
           "time_to_target"]


@dataclass
class TrainConfig:
    layers: int = 4
    channels: int = 16
    steps: int = 2000
    batch: int = 256
    lr: float = 1e-3
    n_gauss: int = 2048
    krylov_seeds: tuple = tuple(range(10, 42))
    krylov_per_seed: int = 64
    seed: int = 0
    # SupPCG settings of the plain runs that produce the Krylov probes
    K: int = 1
    a: float = 0.5
    gamma: float = 0.5
    mu: float = 1e-5
    rho: float = 0.8
    n_ellipses: int = 5
    noise: float = 0.01
    # choose d at the start so that the loss is minimal over a common scale
    # of M (A v is O(1e3) |v| here, so softplus(d) = 1 starts ~1e10 off)
    scale_init: bool = True
    scale_sample: int = 256


def phantom_data(g: api.Geometry, seed: int, n_ellipses: int, noise: float,
                 ctx: api.Context | None = None):
    """(phantom, b) on the GPU: b = R x + sigma * N(0, 1), sigma = noise * max(R x).

    The phantom and the noise come from the shared seeded generators; R x is
    this library's projector."""
    from synth import noisy_data, random_ellipses, unit_noise
    ctx = ctx or api.context(0)
    img, rng = random_ellipses(g.rows, g.cols, n_ellipses, seed)
    x = torch.from_numpy(img.astype(np.float32)).to(f"cuda:{ctx.device}")
    bx = api.sp_project(g, x, ctx=ctx)
    b_exact = bx.double().cpu().numpy().ravel()
    b = noisy_data(b_exact, unit_noise(rng, g.m), noise).astype(np.float32)
    return x, torch.from_numpy(b.reshape(g.n_angles, g.n_bins)).to(x.device)


def gaussian_probes(count: int, rows: int, cols: int, seed: int, device) -> torch.Tensor:
    """count unit-norm Gaussian images [count, rows, cols] from default_rng(seed)."""
    v = np.random.default_rng(seed).standard_normal((count, rows * cols))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return torch.from_numpy(v.astype(np.float32).reshape(count, rows, cols)).to(device)


def krylov_probes(g: api.Geometry, cfg: TrainConfig, ctx: api.Context | None = None) -> torch.Tensor:
    """Normalised g_{k+1/2}, k = 1..per_seed, of plain SupPCG runs, one per seed."""
    ctx = ctx or api.context(0)
    dev = f"cuda:{ctx.device}"
    per = cfg.krylov_per_seed
    out = torch.empty((len(cfg.krylov_seeds) * per, g.rows, g.cols), dtype=torch.float32, device=dev)
    for i, seed in enumerate(cfg.krylov_seeds):
        _, b = phantom_data(g, seed, cfg.n_ellipses, cfg.noise, ctx)
        snap = out[i * per:(i + 1) * per]
        api.sp_suppcg_solve(g, b, None, K=cfg.K, a=cfg.a, gamma=cfg.gamma, precond="ramp",
                            mu=cfg.mu, rho=cfg.rho, max_iter=per, graph=True, trace=False,
                            g_snap=snap, ctx=ctx)
    norms = out.flatten(1).double().norm(dim=1)
    if not bool(torch.all(norms > 0)):
        raise RuntimeError("a Krylov probe is zero (the solver stopped early)")
    return (out.double() / norms[:, None, None]).float().contiguous()


def normal_op(g: api.Geometry, V: torch.Tensor, ctx: api.Context | None = None) -> torch.Tensor:
    """A v = R^T R v for each probe v of V [N, rows, cols]."""
    ctx = ctx or api.context(0)
    AV = torch.empty_like(V)
    y = torch.empty((g.n_angles, g.n_bins), dtype=torch.float32, device=V.device)
    for j in range(V.shape[0]):
        api.sp_project(g, V[j], y, ctx=ctx)
        api.sp_backproject(g, y, AV[j], ctx=ctx)
    return AV


def init_theta(layers: int, channels: int, seed: int) -> np.ndarray:
    """He-normal conv weights (fan-in = in-channels x 9) and d = softplus^-1(1).

    Flat layout: W_1 [channels][1][3][3], W_2..W_L [channels][channels][3][3],
    then d [channels]."""
    rng = np.random.default_rng(seed)
    parts = [rng.standard_normal(channels * 9) * math.sqrt(2.0 / 9.0)]
    for _ in range(layers - 1):
        parts.append(rng.standard_normal(channels * channels * 9) * math.sqrt(2.0 / (channels * 9)))
    parts.append(np.full(channels, math.log(math.e - 1.0)))
    return np.concatenate(parts).astype(np.float32)


def scale_init(net: api.LearnedPrecond, theta: np.ndarray, V: torch.Tensor, AV: torch.Tensor,
               channels: int, sample: int = 256) -> np.ndarray:
    """Rescale M by the s minimising sum ||s M A v - v||^2 over `sample`
    probes spread evenly over the set, s = sum <M A v, v> / sum ||M A v||^2,
    by moving every d_c to softplus^-1(s softplus(d_c)).  Returns the new
    parameters."""
    k = min(sample, V.shape[0])
    pick = torch.from_numpy(np.linspace(0, V.shape[0] - 1, k).round().astype(np.int64)).to(V.device)
    MAV = net.apply(AV[pick].contiguous())
    mav = MAV.double().cpu().numpy().reshape(k, -1)
    v = V[pick].double().cpu().numpy().reshape(k, -1)
    den = float(np.sum(mav * mav))
    num = float(np.sum(mav * v))
    if not (den > 0.0 and num > 0.0 and math.isfinite(num / den)):
        return theta
    sc = num / den
    d = theta[-channels:].astype(np.float64)
    sp = np.logaddexp(0.0, d) * sc
    theta = theta.copy()
    theta[-channels:] = (sp + np.log(-np.expm1(-sp))).astype(np.float32)   # softplus^-1
    net.set_params(theta)
    return theta


@dataclass
class TrainResult:
    net: api.LearnedPrecond
    losses: list                     # (step, minibatch loss) every log_every steps
    seconds: float                   # wall time of the optimisation loop
    probe_seconds: float             # wall time to build the probes and A v
    n_probes: int
    extra: dict = field(default_factory=dict)


def train(g: api.Geometry, cfg: TrainConfig = TrainConfig(), ctx: api.Context | None = None,
          log_every: int = 100, probes=None, margin: int = 0) -> TrainResult:
    """Build the probes, then run cfg.steps Adam steps on the GPU."""
    ctx = ctx or api.context(0)
    dev = f"cuda:{ctx.device}"
    t0 = time.perf_counter()
    if probes is None:
        parts = []
        if cfg.n_gauss:
            parts.append(gaussian_probes(cfg.n_gauss, g.rows, g.cols, cfg.seed + 1, dev))
        if cfg.krylov_seeds and cfg.krylov_per_seed:
            parts.append(krylov_probes(g, cfg, ctx))
        V = torch.cat(parts).contiguous()
        AV = normal_op(g, V, ctx)
    else:
        V, AV = probes
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    net = api.LearnedPrecond(cfg.layers, cfg.channels, ctx)
    theta = init_theta(cfg.layers, cfg.channels, cfg.seed)
    net.set_params(theta)
    if cfg.scale_init:
        theta = scale_init(net, theta, V, AV, cfg.channels, cfg.scale_sample)
    n = V.shape[0]
    rng = np.random.default_rng(cfg.seed + 2)
    idx = torch.from_numpy(
        np.stack([rng.choice(n, cfg.batch, replace=False) for _ in range(cfg.steps)]).astype(np.int32)
    ).to(dev)
    grad = torch.empty(net.num_params, dtype=torch.float32, device=dev)
    losses = []
    pending = []
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for step in range(1, cfg.steps + 1):
        loss, _ = net.loss_grad(AV, V, idx[step - 1], grad, margin=margin)
        net.adam_step(grad, cfg.lr, step)
        if step % log_every == 0 or step == 1 or step == cfg.steps:
            pending.append((step, loss))
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    losses = [(s, float(l.item())) for s, l in pending]
    if not all(math.isfinite(l) for _, l in losses):
        raise RuntimeError("training diverged (non-finite loss)")
    return TrainResult(net, losses, t3 - t2, t1 - t0, n, {"V": V, "AV": AV})


@dataclass
class CropConfig:
    """Training on crops of large images: M reaches 2 * layers pixels, so the
    loss on crop interiors with that margin is the full-size loss there."""
    crop: int = 96
    margin: int = 8
    crops_per_image: int = 64
    n_gauss_images: int = 32
    krylov_seeds: tuple = (5100, 5101)
    krylov_per_seed: int = 16
    n_ellipses: int = 50
    noise: float = 0.005
    seed: int = 0


def _crops(img: torch.Tensor, other: torch.Tensor, rng, cc: CropConfig):
    """Random crops (same positions) of two [H, W] device images, scaled so the
    first crop's interior has unit norm."""
    H, W = img.shape
    c, m = cc.crop, cc.margin
    ys = rng.integers(0, H - c + 1, cc.crops_per_image)
    xs = rng.integers(0, W - c + 1, cc.crops_per_image)
    a = torch.stack([img[y:y + c, x:x + c] for y, x in zip(ys, xs)])
    b = torch.stack([other[y:y + c, x:x + c] for y, x in zip(ys, xs)])
    nrm = a[:, m:c - m, m:c - m].double().flatten(1).norm(dim=1).clamp_min(1e-30)
    return (a.double() / nrm[:, None, None]).float(), (b.double() / nrm[:, None, None]).float()


def crop_probes(g: api.Geometry, cfg: TrainConfig, cc: CropConfig, ctx: api.Context | None = None):
    """(V, AV) crops [N, crop, crop] from full-size Gaussian images and from the
    gradients g_{k+1/2} of plain runs, with A v = R^T R v computed at full size."""
    ctx = ctx or api.context(0)
    dev = f"cuda:{ctx.device}"
    rng = np.random.default_rng(cc.seed + 7)
    y = torch.empty((g.n_angles, g.n_bins), dtype=torch.float32, device=dev)
    av = torch.empty((g.rows, g.cols), dtype=torch.float32, device=dev)
    Vs, AVs = [], []
    for i in range(cc.n_gauss_images):
        v = torch.from_numpy(np.random.default_rng(cc.seed + 1000 + i).standard_normal(
            (g.rows, g.cols)).astype(np.float32)).to(dev)
        api.sp_project(g, v, y, ctx=ctx)
        api.sp_backproject(g, y, av, ctx=ctx)
        a, b = _crops(v, av, rng, cc)
        Vs.append(a)
        AVs.append(b)
    for seed in cc.krylov_seeds:
        _, bdat = phantom_data(g, seed, cc.n_ellipses, cc.noise, ctx)
        snap = torch.empty((cc.krylov_per_seed, g.rows, g.cols), dtype=torch.float32, device=dev)
        api.sp_suppcg_solve(g, bdat, None, K=cfg.K, a=cfg.a, gamma=cfg.gamma, precond="ramp",
                            mu=cfg.mu, rho=cfg.rho, max_iter=cc.krylov_per_seed, graph=True,
                            trace=False, g_snap=snap, ctx=ctx)
        for j in range(cc.krylov_per_seed):
            api.sp_project(g, snap[j], y, ctx=ctx)
            api.sp_backproject(g, y, av, ctx=ctx)
            a, b = _crops(snap[j], av, rng, cc)
            Vs.append(a)
            AVs.append(b)
        del snap
    return torch.cat(Vs).contiguous(), torch.cat(AVs).contiguous()


def train_crops(g: api.Geometry, cfg: TrainConfig = TrainConfig(), cc: CropConfig = CropConfig(),
                ctx: api.Context | None = None, log_every: int = 100) -> TrainResult:
    """train() on crop probes of a large geometry, loss over the crop interiors."""
    ctx = ctx or api.context(0)
    t0 = time.perf_counter()
    V, AV = crop_probes(g, cfg, cc, ctx)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    res = train(g, cfg, ctx, log_every, probes=(V, AV), margin=cc.margin)
    res.probe_seconds = t1 - t0
    return res


def _first(arr, target):
    hit = np.nonzero(np.asarray(arr) <= target)[0]
    return int(hit[0]) + 1 if hit.size else None


def _timed_solve(g, b, reps, **kw):
    api.sp_suppcg_solve(g, b, None, **kw)        # warm: geometry, plans, graph
    torch.cuda.synchronize()
    t = []
    for _ in range(reps):
        t0 = time.perf_counter()
        api.sp_suppcg_solve(g, b, None, **kw)
        torch.cuda.synchronize()
        t.append(time.perf_counter() - t0)
    return float(np.median(t))


def time_to_target(g: api.Geometry, net: api.LearnedPrecond, seeds, cfg: TrainConfig = TrainConfig(),
                   plain_iters: int = 100, max_iters: int = 400, reps: int = 3,
                   ctx: api.Context | None = None):
    """Per seed: targets from the plain (Fourier M) run at loop body plain_iters;
    the learned run's first loop body reaching f, TV and both; wall time of
    each form to its target (median of reps graph-mode solves)."""
    ctx = ctx or api.context(0)
    common = dict(K=cfg.K, a=cfg.a, gamma=cfg.gamma, mu=cfg.mu, rho=cfg.rho, graph=True, ctx=ctx)
    rows = []
    for seed in seeds:
        _, b = phantom_data(g, seed, cfg.n_ellipses, cfg.noise, ctx)
        plain = api.sp_suppcg_solve(g, b, None, precond="ramp", max_iter=plain_iters, **common)
        f_star = float(plain.trace["f_half"][plain_iters - 1])
        tv_star = float(plain.trace["tv_half"][plain_iters - 1])
        lrn = api.sp_suppcg_solve(g, b, None, precond="learned", net=net, max_iter=max_iters, **common)
        f_tr, tv_tr = lrn.trace["f_half"], lrn.trace["tv_half"]
        k_f, k_tv = _first(f_tr, f_star), _first(tv_tr, tv_star)
        both = np.nonzero((f_tr <= f_star) & (tv_tr <= tv_star))[0]
        k_both = int(both[0]) + 1 if both.size else None
        row = {"seed": seed, "f_star": f_star, "tv_star": tv_star, "k_f": k_f, "k_tv": k_tv,
               "k_both": k_both, "fallbacks": lrn.trace["fallbacks"],
               "learned_f_at_plain_iters": float(f_tr[min(plain_iters, len(f_tr)) - 1])}
        if reps:
            row["plain_s"] = _timed_solve(g, b, reps, precond="ramp", max_iter=plain_iters, **common)
            row["learned_s"] = (_timed_solve(g, b, reps, precond="learned", net=net, max_iter=k_both,
                                             **common) if k_both else None)
        rows.append(row)
    return rows
