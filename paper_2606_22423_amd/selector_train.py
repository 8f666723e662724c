"""Training harness of the learned strategy selector.

1. Draws fresh synthetic columns with the mixed-column workload's shape
   (lengths 2^10..2^24, widths 1..24, frame-of-reference / delta /
   dictionary, log-uniform selectivity, zone maps on every column), from a
   seed of its own so that they never coincide with evaluation columns.
2. Times each of the eight row-major strategies on each column: one scan
   launch between two HIP events on the context stream, after a cache-evicting
   overwrite of a 512 MiB buffer, median of `reps`.
3. Computes each column's selector features on the device (zone maps only).
4. Fits the 6 -> 64 -> 64 -> 8 network to log-time per strategy (masked mean
   squared error, Adam, mini-batches) with the library's device kernels.

Everything numeric runs in libscan; this module only orchestrates.
"""
from __future__ import annotations

import math
import time

import numpy as np

import synth
from . import api
from ._lib import ENC_DELTA, ENC_DICT, ENC_FOR, strategy

K = 8
TRAIN_SEED = synth.SEED_BASE + 50


def class_strategy(c: int) -> int:
    """Selector class c -> strategy id: decoder c&1, SV (c>>1)&1, zone maps (c>>2)&1."""
    return strategy(c & 1, (c >> 1) & 1, (c >> 2) & 1)


STRATEGIES = [class_strategy(c) for c in range(K)]


def make_column(spec, device="cuda"):
    """(Column, lo, hi) of one workload column, encoded by the library."""
    v, lo, hi, dct = synth.config4_values(spec)
    if spec.enc == ENC_FOR:
        col = api.encode_for(v, spec.b, device=device)
    elif spec.enc == ENC_DELTA:
        col = api.encode_delta(v, spec.b, device=device)
    else:
        col = api.encode_dict(v, spec.b, dct, device=device)
    return col, lo, hi


class Timer:
    """Cold single-launch timings of one scan on the context stream."""

    def __init__(self, ctx: api.Context, evict_bytes: int = 512 << 20):
        import torch
        self.torch = torch
        self.ctx = ctx
        self.evict = torch.empty(evict_bytes // 4, dtype=torch.int32, device="cuda")
        self.evict_bytes = evict_bytes
        self.out = torch.zeros(64, dtype=torch.uint8, device="cuda")

    def time_strategies(self, col, lo, hi, strategies, reps: int):
        """times[s][r] in seconds for every strategy s and repetition r."""
        torch = self.torch
        ev = []
        for _ in range(reps):
            for s in strategies:
                self.ctx.cache_flush(self.evict, self.evict_bytes)
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(self.ctx.stream)
                self.ctx.run_async(col, lo, hi, s, self.out)
                b.record(self.ctx.stream)
                ev.append((s, a, b))
        self.ctx.sync()
        times = {s: [] for s in strategies}
        for s, a, b in ev:
            times[s].append(a.elapsed_time(b) * 1e-3)
        return times


def collect(ctx: api.Context, n_cols: int = 2560, reps: int = 5, seed: int = TRAIN_SEED, log=print,
            log2_max: float = 24.0):
    """Time all eight strategies on n_cols fresh columns.

    Returns (X [n, 6] float32 features, T [n, 8] float64 median seconds)."""
    import torch
    specs = synth.config4_specs(n_cols, seed=seed, log2_max=log2_max)
    timer = Timer(ctx)
    X = torch.zeros(n_cols, 6, dtype=torch.float32, device="cuda")
    T = np.zeros((n_cols, K))
    t0 = time.time()
    for i, spec in enumerate(specs):
        col, lo, hi = make_column(spec)
        ctx.features([col.item(lo, hi, -1)], X[i:i + 1])
        times = timer.time_strategies(col, lo, hi, STRATEGIES, reps)
        T[i] = [float(np.median(times[s])) for s in STRATEGIES]
        del col
        if log and (i + 1) % 256 == 0:
            log("selector timings: %d/%d columns, %.0f s" % (i + 1, n_cols, time.time() - t0))
    return X.cpu().numpy(), T


def targets(T: np.ndarray) -> np.ndarray:
    """Regression target: natural log of the time in microseconds."""
    return np.log(np.maximum(T, 1e-9) * 1e6).astype(np.float32)


def train(ctx: api.Context, X: np.ndarray, Y: np.ndarray, M: np.ndarray | None = None, epochs: int = 400,
          batch: int = 256, lr: float = 1e-3, seed: int = 1, log=print):
    """Adam on the masked squared error with the library's device kernels.

    Returns the parameter vector (float32 numpy) and the final full-data loss."""
    import torch
    rng = np.random.default_rng(seed)
    n = X.shape[0]
    P = api.Context.mlp_param_count()
    # He-style initialisation for the ReLU layers, small output layer
    shapes = [(64, 6), (64,), (64, 64), (64,), (K, 64), (K,)]
    parts = []
    for shp in shapes:
        if len(shp) == 2:
            parts.append(rng.standard_normal(shp) * math.sqrt(2.0 / shp[1]) * (0.5 if shp[0] == K else 1.0))
        else:
            parts.append(np.zeros(shp))
    theta0 = np.concatenate([p.ravel() for p in parts]).astype(np.float32)
    # output bias starts at the mean target of each strategy
    ymean = (Y * (M if M is not None else 1)).sum(axis=0) / np.maximum(
        (M if M is not None else np.ones_like(Y)).sum(axis=0), 1)
    theta0[P - K:] = ymean.astype(np.float32)
    M = np.ones_like(Y) if M is None else M
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()  # noqa: E731
    Xd, Yd, Md = dev(X), dev(Y), dev(M)
    theta, m, v = dev(theta0), torch.zeros(P, device="cuda"), torch.zeros(P, device="cuda")
    grad = torch.empty(P, device="cuda")
    loss = torch.empty(1, device="cuda")
    step = 0
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).cuda()
        for s0 in range(0, n, batch):
            idx = perm[s0:s0 + batch]
            xb, yb, mb = Xd[idx].contiguous(), Yd[idx].contiguous(), Md[idx].contiguous()
            denom = mb.sum().item()
            if denom <= 0:
                continue
            ctx.mlp_loss_grad(theta, xb, yb, mb, 1.0 / denom, grad, loss)
            step += 1
            ctx.adam_step(theta, grad, m, v, step, lr=lr)
        if log and (ep + 1) % 100 == 0:
            ctx.mlp_loss_grad(theta, Xd, Yd, Md, 1.0 / float(M.sum()), grad, loss)
            log("selector training: epoch %d, loss %.4f" % (ep + 1, float(loss.item())))
    ctx.mlp_loss_grad(theta, Xd, Yd, Md, 1.0 / float(M.sum()), grad, loss)
    return theta.cpu().numpy(), float(loss.item())


def predict(ctx: api.Context, theta: np.ndarray, X: np.ndarray) -> np.ndarray:
    import torch
    out = torch.empty(X.shape[0], K, dtype=torch.float32, device="cuda")
    ctx.mlp_forward(torch.from_numpy(np.ascontiguousarray(theta)).cuda(),
                    torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda(), out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def regret(T: np.ndarray, choice: np.ndarray) -> dict:
    """Total-time regret sum t(chosen)/sum t(best) - 1 and the per-column mean."""
    rows = np.arange(T.shape[0])
    chosen = T[rows, choice]
    best = T.min(axis=1)
    return {"total": float(chosen.sum() / best.sum() - 1.0), "mean": float(np.mean(chosen / best - 1.0))}
