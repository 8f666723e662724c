"""Training harness of the learned strategy selector.

1. Draws fresh synthetic columns with the mixed-column workload's shape
   (lengths 2^10..2^24, widths 1..24, frame-of-reference / delta /
   dictionary, log-uniform selectivity, zone maps on every column), from a
   seed of its own so that they never coincide with evaluation columns.
2. Times each of the eight row-major strategies on each column: one scan
   launch between two HIP events on the context stream, after a cache-evicting
   read of a 512 MiB scratch buffer (the shipped parameters were trained when
   the eviction overwrote it), median of `reps`.
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


def _host_column(spec):
    """Raw values -> host-encoded arrays (library encoder) of one column."""
    v, lo, hi, dct = synth.config4_values(spec)
    if spec.enc == ENC_FOR:
        payload, refs, zmin, zmax = api.host_encode_for(v, spec.b)
        extra = None
    elif spec.enc == ENC_DELTA:
        payload, extra, zmin, zmax = api.host_encode_delta(v, spec.b)
    else:
        payload, zmin, zmax = api.host_encode_dict(v, spec.b, len(dct))
        extra = np.ascontiguousarray(dct, dtype=np.int64)
    return spec, payload, extra, zmin, zmax, lo, hi


def _upload(host, device):
    import torch
    spec, payload, extra, zmin, zmax, lo, hi = host
    dev = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(device)  # noqa: E731
    kw = {}
    if spec.enc == ENC_DELTA:
        kw["bases"] = dev(extra)
    elif spec.enc == ENC_DICT:
        kw["dct"] = dev(extra)
    col = api.Column(spec.enc, spec.b, spec.n, 0, dev(payload), zmin=dev(zmin), zmax=dev(zmax), **kw)
    return col, lo, hi


def make_column(spec, device="cuda"):
    """(Column, lo, hi) of one workload column, encoded by the library."""
    return _upload(_host_column(spec), device)


def build_columns(specs, device="cuda", threads: int = 8, window: int = 32):
    """Generate, encode and upload many columns; host work runs on `threads`
    threads, at most `window` columns ahead of the upload."""
    from concurrent.futures import ThreadPoolExecutor
    out = []
    with ThreadPoolExecutor(threads) as ex:
        pending = []
        it = iter(specs)
        for spec in it:
            pending.append(ex.submit(_host_column, spec))
            if len(pending) >= window:
                out.append(_upload(pending.pop(0).result(), device))
        for f in pending:
            out.append(_upload(f.result(), device))
    return out


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
            log2_max: float = 24.0, threads: int = 8):
    """Time all eight strategies on n_cols fresh columns.

    Returns (X [n, 6] float32 features, T [n, 8] float64 median seconds)."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    specs = synth.config4_specs(n_cols, seed=seed, log2_max=log2_max)
    timer = Timer(ctx)
    X = torch.zeros(n_cols, 6, dtype=torch.float32, device="cuda")
    T = np.zeros((n_cols, K))
    t0 = time.time()
    with ThreadPoolExecutor(threads) as ex:
        futs = [ex.submit(_host_column, sp) for sp in specs[:2 * threads]]
        for i in range(n_cols):
            host = futs[i].result()
            futs[i] = None
            if i + 2 * threads < n_cols:
                futs.append(ex.submit(_host_column, specs[i + 2 * threads]))
            col, lo, hi = _upload(host, "cuda")
            del host
            ctx.features([col.item(lo, hi, -1)], X[i:i + 1])
            times = timer.time_strategies(col, lo, hi, STRATEGIES, reps)
            T[i] = [float(np.median(times[s])) for s in STRATEGIES]
            del col
            if log and (i + 1) % 512 == 0:
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


def evaluate(ctx: api.Context, theta: np.ndarray, X: np.ndarray, T: np.ndarray) -> dict:
    """Regret of the learned choice and of the fixed alternatives on timed columns."""
    pred = predict(ctx, theta, X)
    learned = np.argmin(pred, axis=1)  # ties to the lowest class, as on the device
    default = np.full(len(T), 5)       # row-major direct decoder, branch-free, zone maps on
    best_fixed = int(np.argmin(T.sum(axis=0)))
    return {
        "columns": int(len(T)),
        "learned": regret(T, learned),
        "fixed_default": regret(T, default),
        "best_fixed_in_hindsight": {"class": best_fixed, **regret(T, np.full(len(T), best_fixed))},
        "time_s": {"learned": float(T[np.arange(len(T)), learned].sum()), "best": float(T.min(axis=1).sum()),
                   "fixed_default": float(T[:, 5].sum())},
        "learned_class_counts": np.bincount(learned, minlength=K).tolist(),
        "best_class_counts": np.bincount(np.argmin(T, axis=1), minlength=K).tolist(),
    }


def main(argv=None):
    import argparse
    import json

    ap = argparse.ArgumentParser(description="train and evaluate the strategy selector on this GPU")
    ap.add_argument("--cols", type=int, default=2560, help="training columns (x 8 strategies timings)")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--eval-cols", type=int, default=4096, help="held-out columns (the mixed workload's own)")
    ap.add_argument("--eval-reps", type=int, default=3)
    ap.add_argument("--epochs", type=int, default=400)
    ap.add_argument("--out", required=True, help="selector file to write")
    ap.add_argument("--report", default=None, help="JSON report")
    args = ap.parse_args(argv)
    say = lambda *a: print(*a, flush=True)  # noqa: E731
    ctx = api.Context(0)
    t0 = time.time()
    X, T = collect(ctx, args.cols, args.reps, log=say)
    say("training set: %d columns x %d strategies in %.0f s" % (len(T), K, time.time() - t0))
    theta, loss = train(ctx, X, targets(T), epochs=args.epochs, log=say)
    ctx.selector_set(theta)
    ctx.selector_save(args.out)
    train_eval = evaluate(ctx, theta, X, T)
    t1 = time.time()
    Xe, Te = collect(ctx, args.eval_cols, args.eval_reps, seed=synth.SEED_BASE + 3, log=say)
    say("held-out set: %d columns in %.0f s" % (len(Te), time.time() - t1))
    held = evaluate(ctx, theta, Xe, Te)
    report = {"train_columns": len(T), "timings": int(T.size), "reps": args.reps, "epochs": args.epochs,
              "final_loss": loss, "train": train_eval, "held_out": held}
    say(json.dumps(report))
    if args.report:
        with open(args.report, "w") as fh:
            json.dump(report, fh, indent=1)
    ctx.close()


if __name__ == "__main__":
    main()
