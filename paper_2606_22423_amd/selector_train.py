"""Training harness of the learned strategy selector.

1. Draws fresh synthetic columns with the mixed-column workload's shape
   (lengths 2^10..2^24, widths 1..24, frame-of-reference / delta /
   dictionary, log-uniform selectivity, zone maps on every column), from a
   seed of its own so that they never coincide with evaluation columns.
2. Times each of the eight row-major strategies on each column where the
   selector is used, inside a batch (BatchTimer: the column's share of a
   device-filling replay), or as single cold launches (Timer).
3. Computes each column's selector features on the device (zone maps only).
4. Fits the 6 -> 64 -> 64 -> 8 network to log-time per strategy (masked mean
   squared error, Adam, mini-batches) with the library's device kernels, and
   picks the fallback margin (keep the heuristic unless the predicted gain is
   larger) of least total time on the training columns.
5. Times the held-out columns (the 4096-column mixed workload itself) the
   same way and reports the regret of the learned choice, of the heuristic
   and of the best fixed strategy against the per-column best.

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


class BatchTimer:
    """Cost of one column under each strategy inside a batch, where the
    selector works: K items of the column (the same device buffers) in one
    prepared batch with that strategy, replayed between two HIP events after
    a cache-evicting read, median of `reps`; minus the replay cost of a batch
    of one single-block column with the same strategy (the launches), divided
    by K.  K = clamp(ceil(2^30 / n), 1, 4096) fills the device with work
    items the way a large batch does, so the figure is the column's share of
    a saturated replay rather than its latency alone."""

    FILL_VALUES = 1 << 30
    MAX_COPIES = 4096

    def __init__(self, ctx: api.Context, evict_bytes: int = 512 << 20):
        import torch
        self.torch = torch
        self.ctx = ctx
        self.evict = torch.empty(evict_bytes // 4, dtype=torch.int32, device="cuda")
        self.evict_bytes = evict_bytes
        self.base = {}

    def _replay_time(self, items, reps):
        torch = self.torch
        h = self.ctx.batch_prepare(items)
        try:
            self.ctx.batch_replay(h, wait=False)  # first replay: code objects, graph upload
            ev = []
            for _ in range(reps):
                self.ctx.cache_flush(self.evict, self.evict_bytes)
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(self.ctx.stream)
                self.ctx.batch_replay(h, wait=False)
                b.record(self.ctx.stream)
                ev.append((a, b))
            self.ctx.sync()
            return float(np.median([a.elapsed_time(b) * 1e-3 for a, b in ev]))
        finally:
            self.ctx.batch_release(h)

    def _base(self, col, lo, hi, s, reps):
        key = (col.enc, s)
        if key not in self.base:
            one = api.Column(col.enc, col.b, min(col.n, 1024), col.layout, col.payload, refs=col.refs,
                             bases=col.bases, dct=col.dct, zmin=col.zmin, zmax=col.zmax)
            self.base[key] = self._replay_time([one.item(lo, hi, s)], reps)
        return self.base[key]

    def time_strategies(self, col, lo, hi, strategies, reps: int):
        """{s: seconds per column} for every strategy s."""
        k = int(min(self.MAX_COPIES, max(1, -(-self.FILL_VALUES // max(1, col.n)))))
        out = {}
        for s in strategies:
            t = self._replay_time([col.item(lo, hi, s)] * k, reps)
            out[s] = max(t - self._base(col, lo, hi, s, reps), 1e-9) / k
        return out


def collect(ctx: api.Context, n_cols: int = 2560, reps: int = 5, seed: int = TRAIN_SEED, log=print,
            log2_max: float = 24.0, threads: int = 8, context: str = "batch"):
    """Time all eight strategies on n_cols fresh columns, in a batch
    (context "batch", BatchTimer) or as single cold launches ("single", Timer).

    Returns (X [n, 6] float32 features, T [n, 8] float64 seconds)."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    specs = synth.config4_specs(n_cols, seed=seed, log2_max=log2_max)
    timer = BatchTimer(ctx) if context == "batch" else Timer(ctx)
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
            if log and (i + 1) % 128 == 0:
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


HEURISTIC_CLASS = 5  # row-major direct decoder, branch-free, zone maps (every workload column has them)


def choose(pred: np.ndarray, margin: float) -> np.ndarray:
    """The library's rule on host predictions: the heuristic's class unless its
    predicted log-time exceeds the argmin's by at least `margin` (every class
    is valid for a column with zone maps; ties to the lowest class)."""
    best = np.argmin(pred, axis=1)
    rows = np.arange(pred.shape[0])
    keep = pred[rows, HEURISTIC_CLASS] - pred[rows, best] < margin
    return np.where(keep, HEURISTIC_CLASS, best)


def pick_margin(pred: np.ndarray, T: np.ndarray, grid=(0.0, 0.02, 0.05, 0.1, 0.15, 0.2, 0.3, 0.5)) -> float:
    """The margin of smallest total time on the training columns (the
    smallest such margin on ties)."""
    rows = np.arange(len(T))
    tot = [(float(T[rows, choose(pred, m)].sum()), m) for m in grid]
    return min(tot)[1]


def evaluate(ctx: api.Context, theta: np.ndarray, X: np.ndarray, T: np.ndarray, margin: float = 0.0) -> dict:
    """Regret of the learned choice and of the fixed alternatives on timed columns."""
    pred = predict(ctx, theta, X)
    rows = np.arange(len(T))
    learned = choose(pred, margin)
    argmin = np.argmin(pred, axis=1)   # ties to the lowest class, as on the device
    default = np.full(len(T), HEURISTIC_CLASS)
    best_fixed = int(np.argmin(T.sum(axis=0)))
    return {
        "columns": int(len(T)),
        "margin": margin,
        "learned": regret(T, learned),
        "learned_plain_argmin": regret(T, argmin),
        "fixed_default": regret(T, default),
        "best_fixed_in_hindsight": {"class": best_fixed, **regret(T, np.full(len(T), best_fixed))},
        "time_s": {"learned": float(T[rows, learned].sum()), "best": float(T.min(axis=1).sum()),
                   "fixed_default": float(T[:, HEURISTIC_CLASS].sum())},
        "gain_over_heuristic": float(T[:, HEURISTIC_CLASS].sum() / T[rows, learned].sum() - 1.0),
        "learned_class_counts": np.bincount(learned, minlength=K).tolist(),
        "best_class_counts": np.bincount(np.argmin(T, axis=1), minlength=K).tolist(),
    }


def save_table(path: str, X: np.ndarray, T: np.ndarray, note: str):
    """Timing table as text: a comment line, then per column the six features
    and the eight per-strategy times in microseconds."""
    with open(path, "w") as fh:
        fh.write("# %s\n" % note)
        fh.write("# f0 f1 f2 f3 f4 f5 | t_us class 0..7 (class c: decoder c&1, sv (c>>1)&1, zone maps (c>>2)&1)\n")
        for x, t in zip(X, T):
            fh.write(" ".join("%.7g" % v for v in x) + " " + " ".join("%.5g" % (v * 1e6) for v in t) + "\n")


def load_table(path: str):
    """(X float32 [n, 6], T float64 seconds [n, 8]) of a save_table file."""
    a = np.loadtxt(path, comments="#", dtype=np.float64, ndmin=2)
    return a[:, :6].astype(np.float32), a[:, 6:] * 1e-6


def main(argv=None):
    import argparse
    import json

    ap = argparse.ArgumentParser(description="train and evaluate the strategy selector on this GPU")
    ap.add_argument("--cols", type=int, default=2560, help="training columns (x 8 strategies timings)")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--eval-cols", type=int, default=4096, help="held-out columns (the mixed workload's own)")
    ap.add_argument("--eval-reps", type=int, default=3)
    ap.add_argument("--epochs", type=int, default=400)
    ap.add_argument("--context", choices=("batch", "single"), default="batch",
                    help="time strategies inside a batch (the selector's use) or as single launches")
    ap.add_argument("--train-table", default=None, help="training timings: read if it exists, else write")
    ap.add_argument("--eval-table", default=None, help="held-out timings: read if it exists, else write")
    ap.add_argument("--no-eval", action="store_true", help="collect training timings only")
    ap.add_argument("--out", default=None, help="selector file to write")
    ap.add_argument("--report", default=None, help="JSON report")
    args = ap.parse_args(argv)
    import os
    say = lambda *a: print(*a, flush=True)  # noqa: E731
    ctx = api.Context(0)
    t0 = time.time()
    if args.train_table and os.path.exists(args.train_table):
        X, T = load_table(args.train_table)
    else:
        X, T = collect(ctx, args.cols, args.reps, log=say, context=args.context)
        if args.train_table:
            save_table(args.train_table, X, T, "selector training timings, %s context, %d columns, seed %d, "
                       "median of %d" % (args.context, len(T), TRAIN_SEED, args.reps))
    say("training set: %d columns x %d strategies in %.0f s" % (len(T), K, time.time() - t0))
    if args.no_eval:
        ctx.close()
        return
    theta, loss = train(ctx, X, targets(T), epochs=args.epochs, log=say)
    margin = pick_margin(predict(ctx, theta, X), T)
    ctx.selector_set(theta)
    ctx.selector_set_margin(margin)
    if args.out:
        ctx.selector_save(args.out)
    train_eval = evaluate(ctx, theta, X, T, margin)
    t1 = time.time()
    if args.eval_table and os.path.exists(args.eval_table):
        Xe, Te = load_table(args.eval_table)
    else:
        Xe, Te = collect(ctx, args.eval_cols, args.eval_reps, seed=synth.SEED_BASE + 3, log=say,
                         context=args.context)
        if args.eval_table:
            save_table(args.eval_table, Xe, Te, "selector held-out timings (the 4096-column mixed workload), %s "
                       "context, seed %d, median of %d" % (args.context, synth.SEED_BASE + 3, args.eval_reps))
    say("held-out set: %d columns in %.0f s" % (len(Te), time.time() - t1))
    held = evaluate(ctx, theta, Xe, Te, margin)
    report = {"context": args.context, "train_columns": len(T), "timings": int(T.size), "reps": args.reps,
              "epochs": args.epochs, "final_loss": loss, "margin": margin, "train": train_eval, "held_out": held}
    say(json.dumps(report))
    if args.report:
        with open(args.report, "w") as fh:
            json.dump(report, fh, indent=1)
    ctx.close()


if __name__ == "__main__":
    main()
