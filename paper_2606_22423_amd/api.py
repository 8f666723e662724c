"""Python face of the C ABI: device-resident columns and a scan context.

Thin wrappers only: arguments are marshalled to the C library, which does all
encoding, decoding, filtering and aggregation.  PyTorch provides device memory
(tensors) and the HIP stream.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import numpy as np

from . import _lib
from ._lib import (ENC_DELTA, ENC_DICT, ENC_FOR, LAYOUT_LI, LAYOUT_RM, STRAT_AUTO, ScanColumn, ScanError,
                   ScanItem, ScanPredicate, ScanResult, ScanTune)

L = 1024


def nblocks(n: int) -> int:
    return (n + L - 1) // L


def _ptr(a) -> int | None:
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


def _check(rc: int, what: str):
    if rc != 0:
        raise ScanError(rc, what)


# --------------------------------------------------------------- host encoders
def host_encode_for(values, b: int, layout: int = LAYOUT_RM, ref_policy: int = 0):
    """(payload, refs or None, zmin, zmax) as numpy arrays, by the library's host encoder."""
    lib = _lib.load()
    v = np.ascontiguousarray(values, dtype=np.uint32)
    n = len(v)
    payload = np.empty(int(lib.scan_payload_words(n, b)), dtype=np.uint32)
    refs = np.empty(nblocks(n), dtype=np.uint32) if ref_policy == 1 else None
    zmin = np.empty(nblocks(n), dtype=np.uint32)
    zmax = np.empty(nblocks(n), dtype=np.uint32)
    rc = lib.scan_encode_for(_ptr(v), n, b, layout, ref_policy, _ptr(payload), _ptr(refs), _ptr(zmin), _ptr(zmax))
    _check(rc, "scan_encode_for rejected the values (width %d, policy %d)" % (b, ref_policy))
    return payload, refs, zmin, zmax


def host_encode_delta(values, b: int):
    lib = _lib.load()
    v = np.ascontiguousarray(values, dtype=np.int64)
    n = len(v)
    payload = np.empty(int(lib.scan_payload_words(n, b)), dtype=np.uint32)
    bases = np.empty(nblocks(n), dtype=np.int64)
    zmin = np.empty(nblocks(n), dtype=np.int64)
    zmax = np.empty(nblocks(n), dtype=np.int64)
    rc = lib.scan_encode_delta(_ptr(v), n, b, _ptr(payload), _ptr(bases), _ptr(zmin), _ptr(zmax))
    _check(rc, "scan_encode_delta rejected the values (width %d)" % b)
    return payload, bases, zmin, zmax


def host_encode_dict(codes, b: int, dict_len: int):
    lib = _lib.load()
    c = np.ascontiguousarray(codes, dtype=np.uint32)
    n = len(c)
    payload = np.empty(int(lib.scan_payload_words(n, b)), dtype=np.uint32)
    zmin = np.empty(nblocks(n), dtype=np.uint32)
    zmax = np.empty(nblocks(n), dtype=np.uint32)
    rc = lib.scan_encode_dict(_ptr(c), n, b, dict_len, _ptr(payload), _ptr(zmin), _ptr(zmax))
    _check(rc, "scan_encode_dict rejected the codes (width %d, %d entries)" % (b, dict_len))
    return payload, zmin, zmax


# --------------------------------------------------------------- device columns
@dataclass
class Column:
    """A column resident in device memory.  Tensors own the memory."""
    enc: int
    b: int
    n: int
    layout: int
    payload: object
    refs: object = None
    bases: object = None
    dct: object = None
    zmin: object = None
    zmax: object = None
    bsum: object = None      # per-block sums of decoded values (all-match shortcut)
    _keep: list = field(default_factory=list)

    def struct(self, zone_maps: bool = True) -> ScanColumn:
        c = ScanColumn()
        c.payload = _ptr(self.payload)
        c.block_ref = _ptr(self.refs)
        c.block_base = _ptr(self.bases)
        c.dict = _ptr(self.dct)
        c.dict_len = 0 if self.dct is None else int(self.dct.numel())
        c.layout = self.layout
        c.zone_min = _ptr(self.zmin) if zone_maps else None
        c.zone_max = _ptr(self.zmax) if zone_maps else None
        c.n = self.n
        c.block_sum = _ptr(self.bsum) if zone_maps else None
        return c

    @property
    def payload_bytes(self) -> int:
        return int(self.payload.numel()) * 4

    def item(self, lo: int, hi: int, strategy: int = STRAT_AUTO, zone_maps: bool = True) -> ScanItem:
        it = ScanItem()
        it.col = self.struct(zone_maps)
        it.enc = self.enc
        it.b = self.b
        it.pred = ScanPredicate(int(lo), int(hi))
        it.agg = 3
        it.strategy = strategy
        return it


def host_block_sums(enc: int, values, dct=None):
    """Per-block sums of decoded values mod 2^64 (uint64 numpy), by the library's host code."""
    lib = _lib.load()
    if enc == ENC_DELTA:
        v = np.ascontiguousarray(values, dtype=np.int64)
    else:
        v = np.ascontiguousarray(values, dtype=np.uint32)
    d = None if dct is None else np.ascontiguousarray(dct, dtype=np.int64)
    out = np.zeros(max(1, nblocks(len(v))), dtype=np.uint64)
    _check(lib.scan_block_sums(enc, v.ctypes.data, len(v), None if d is None else d.ctypes.data,
                               0 if d is None else len(d), out.ctypes.data), "scan_block_sums")
    return out[:nblocks(len(v))]


def _to_dev(a, device):
    import torch
    if a is None:
        return None
    return torch.from_numpy(np.ascontiguousarray(a)).to(device)


def encode_for(values, b: int, layout: int = LAYOUT_RM, ref_policy: int = 0, device="cuda",
               block_sums: bool = True) -> Column:
    payload, refs, zmin, zmax = host_encode_for(values, b, layout, ref_policy)
    bs = host_block_sums(ENC_FOR, values) if block_sums else None
    return Column(ENC_FOR, b, len(values), layout, _to_dev(payload, device), refs=_to_dev(refs, device),
                  zmin=_to_dev(zmin, device), zmax=_to_dev(zmax, device), bsum=_to_dev(bs, device))


def encode_delta(values, b: int, device="cuda", block_sums: bool = True) -> Column:
    payload, bases, zmin, zmax = host_encode_delta(values, b)
    bs = host_block_sums(ENC_DELTA, values) if block_sums else None
    return Column(ENC_DELTA, b, len(values), LAYOUT_RM, _to_dev(payload, device), bases=_to_dev(bases, device),
                  zmin=_to_dev(zmin, device), zmax=_to_dev(zmax, device), bsum=_to_dev(bs, device))


def encode_dict(codes, b: int, dct, device="cuda", block_sums: bool = True) -> Column:
    dct = np.ascontiguousarray(dct, dtype=np.int64)
    payload, zmin, zmax = host_encode_dict(codes, b, len(dct))
    bs = host_block_sums(ENC_DICT, codes, dct) if block_sums else None
    return Column(ENC_DICT, b, len(codes), LAYOUT_RM, _to_dev(payload, device), dct=_to_dev(dct, device),
                  zmin=_to_dev(zmin, device), zmax=_to_dev(zmax, device), bsum=_to_dev(bs, device))


@dataclass
class RleColumn:
    """A run-length encoded u32 column in device memory."""
    n: int
    run_value: object
    run_len: object
    block_run: object
    zmin: object = None
    zmax: object = None

    @property
    def runs(self) -> int:
        return int(self.run_value.numel())

    def struct(self, zone_maps: bool = True) -> "_lib.ScanRleColumn":
        c = _lib.ScanRleColumn()
        c.run_value = _ptr(self.run_value)
        c.run_len = _ptr(self.run_len)
        c.block_run = _ptr(self.block_run)
        c.zone_min = _ptr(self.zmin) if zone_maps else None
        c.zone_max = _ptr(self.zmax) if zone_maps else None
        c.n = self.n
        return c


def host_encode_rle(values):
    """(run values, run lengths, block run starts, zmin, zmax) by the library's host encoder."""
    lib = _lib.load()
    v = np.ascontiguousarray(values, dtype=np.uint32)
    n = len(v)
    rv = np.empty(max(n, 1), dtype=np.uint32)
    rl = np.empty(max(n, 1), dtype=np.uint16)
    br = np.empty(nblocks(n) + 1, dtype=np.uint64)
    zmin = np.empty(max(nblocks(n), 1), dtype=np.uint32)
    zmax = np.empty(max(nblocks(n), 1), dtype=np.uint32)
    runs = ctypes.c_uint64()
    _check(lib.scan_rle_encode(_ptr(v), n, _ptr(rv), _ptr(rl), _ptr(br), _ptr(zmin), _ptr(zmax), ctypes.byref(runs)),
           "scan_rle_encode")
    r = runs.value
    return rv[:r], rl[:r], br, zmin[:nblocks(n)], zmax[:nblocks(n)]


def encode_rle(values, device="cuda") -> RleColumn:
    rv, rl, br, zmin, zmax = host_encode_rle(values)
    return RleColumn(len(values), _to_dev(rv.view(np.int32), device), _to_dev(rl.view(np.int16), device),
                     _to_dev(br.view(np.int64), device), _to_dev(zmin, device), _to_dev(zmax, device))


def run_static(col: Column, lo: int, hi: int, strategy: int, out_dev, stream=None, zone_maps: bool = True):
    """scan_run_static: enqueue one scan with no context and no allocation on
    `stream` (a torch stream; default torch's current stream) of the current
    device; the 40-byte result lands in out_dev (a device tensor of >= 40 bytes)."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    it = col.item(lo, hi, strategy, zone_maps)
    rc = _lib.load().scan_run_static(ctypes.byref(it), ctypes.c_void_p(s.cuda_stream), ctypes.c_void_p(_ptr(out_dev)))
    _check(rc, "scan_run_static")


# --------------------------------------------------------------- context
class Context:
    """One scan_ctx bound to a device and to torch's current stream on it."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.lib = _lib.load()
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = ctypes.c_void_p()
        rc = self.lib.scan_create(ctypes.byref(h), device, ctypes.c_void_p(self.stream.cuda_stream))
        _check(rc, "scan_create(device=%d)" % device)
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.scan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def error(self) -> str:
        return self.lib.scan_last_error(self.h).decode()

    def check(self, rc: int, what: str):
        if rc != 0:
            raise ScanError(rc, "%s: %s" % (what, self.error()))

    @property
    def cus(self) -> int:
        return int(self.lib.scan_device_cus(self.h))

    def run(self, col: Column, lo: int, hi: int, strategy: int = STRAT_AUTO, zone_maps: bool = True) -> dict:
        c = col.struct(zone_maps)
        r = ScanResult()
        pred = ScanPredicate(int(lo), int(hi))
        rc = self.lib.scan_run(self.h, ctypes.byref(c), col.enc, col.b, ctypes.byref(pred), 3, strategy,
                               ctypes.byref(r))
        self.check(rc, "scan_run")
        return r.as_dict()

    def run_async(self, col: Column, lo: int, hi: int, strategy: int, out_dev, zone_maps: bool = True):
        """Enqueue; the 40-byte result lands in out_dev (a device tensor of >= 40 bytes)."""
        it = col.item(lo, hi, strategy, zone_maps)
        rc = self.lib.scan_run_async(self.h, ctypes.byref(it), ctypes.c_void_p(_ptr(out_dev)))
        self.check(rc, "scan_run_async")

    def sync(self):
        self.check(self.lib.scan_sync(self.h), "scan_sync")

    def set_tune(self, enc: int, b: int, strategy: int, wg_size=0, wgs_per_cu=0, window_blocks=0, depth=0):
        t = ScanTune(wg_size, wgs_per_cu, window_blocks, depth)
        self.check(self.lib.scan_set_tune(self.h, enc, b, strategy, ctypes.byref(t)), "scan_set_tune")

    def get_tune(self, enc: int, b: int, strategy: int) -> tuple:
        """(wg_size, wgs_per_cu, window_blocks, depth) as the scan will use it."""
        t = ScanTune()
        self.check(self.lib.scan_get_tune(self.h, enc, b, strategy, ctypes.byref(t)), "scan_get_tune")
        return (t.wg_size, t.wgs_per_cu, t.window_blocks, t.depth)

    def autotune(self, col: Column, lo: int, hi: int, strategy: int, reps: int = 3, zone_maps: bool = True):
        """Exhaustive launch-configuration search; returns ((wg, per_cu, window, depth), best ms)."""
        c = col.struct(zone_maps)
        t = ScanTune()
        ms = ctypes.c_float()
        pred = ScanPredicate(int(lo), int(hi))
        self.check(self.lib.scan_autotune(self.h, ctypes.byref(c), col.enc, col.b, ctypes.byref(pred), strategy,
                                          reps, ctypes.byref(t), ctypes.byref(ms)), "scan_autotune")
        return (t.wg_size, t.wgs_per_cu, t.window_blocks, t.depth), float(ms.value)

    def tune_save(self, path: str):
        self.check(self.lib.scan_tune_save(self.h, path.encode()), "scan_tune_save")

    def tune_load(self, path: str):
        self.check(self.lib.scan_tune_load(self.h, path.encode()), "scan_tune_load")

    def run_rle(self, col: RleColumn, lo: int, hi: int, zone_maps: bool = True, all_match: bool = True) -> dict:
        c = col.struct(zone_maps)
        flags = (1 if zone_maps and col.zmin is not None else 0)
        flags |= 2 if flags and all_match else 0
        r = ScanResult()
        pred = ScanPredicate(int(lo), int(hi))
        self.check(self.lib.scan_run_rle(self.h, ctypes.byref(c), ctypes.byref(pred), flags, ctypes.byref(r)),
                   "scan_run_rle")
        return r.as_dict()

    def run_rle_async(self, col: RleColumn, lo: int, hi: int, out_dev, zone_maps: bool = True,
                      all_match: bool = True):
        """Enqueue; the 40-byte result lands in out_dev (a device tensor of >= 40 bytes)."""
        c = col.struct(zone_maps)
        flags = (1 if zone_maps and col.zmin is not None else 0)
        flags |= 2 if flags and all_match else 0
        pred = ScanPredicate(int(lo), int(hi))
        self.check(self.lib.scan_run_rle_async(self.h, ctypes.byref(c), ctypes.byref(pred), flags,
                                               ctypes.c_void_p(_ptr(out_dev))), "scan_run_rle_async")

    # ------------------------------------------------ materializing select
    def select(self, col: Column, lo: int, hi: int, zone_maps: bool = True, all_match: bool = True,
               out=None):
        """Ascending positions (device uint32 tensor) of the rows with lo <= v < hi.

        With `out` (a device int32 tensor of at least col.n entries, reused
        across calls) the count and the writes run in one call with a single
        wait; without it the matches are counted first and a buffer of that
        size is allocated."""
        import torch
        c = col.struct(zone_maps)
        pred = ScanPredicate(int(lo), int(hi))
        flags = (1 if zone_maps and col.zmin is not None else 0)
        flags |= 2 if flags and all_match and col.bsum is not None else 0
        cnt = ctypes.c_uint64()
        if out is not None:
            if out.dtype != torch.int32 or not out.is_cuda or out.numel() < col.n:
                raise ValueError("out must be a device int32 tensor of at least %d entries" % col.n)
            self.check(self.lib.scan_select(self.h, ctypes.byref(c), col.enc, col.b, ctypes.byref(pred), flags,
                                            _ptr(out), out.numel(), ctypes.byref(cnt)), "scan_select")
            return out[:cnt.value]
        rc = self.lib.scan_select(self.h, ctypes.byref(c), col.enc, col.b, ctypes.byref(pred), flags, None, 0,
                                  ctypes.byref(cnt))
        if rc not in (0, _lib.SCAN_ENOMEM):
            self.check(rc, "scan_select")
        out = torch.empty(max(1, cnt.value), dtype=torch.int32, device="cuda")
        if cnt.value:
            self.check(self.lib.scan_select(self.h, ctypes.byref(c), col.enc, col.b, ctypes.byref(pred), flags,
                                            _ptr(out), cnt.value, ctypes.byref(cnt)), "scan_select")
        return out[:cnt.value]

    def refine(self, col: Column, lo: int, hi: int, positions):
        import torch
        c = col.struct(False)
        pred = ScanPredicate(int(lo), int(hi))
        out = torch.empty(max(1, positions.numel()), dtype=torch.int32, device="cuda")
        cnt = ctypes.c_uint64()
        self.check(self.lib.scan_refine(self.h, ctypes.byref(c), col.enc, col.b, ctypes.byref(pred), _ptr(positions),
                                        positions.numel(), _ptr(out), ctypes.byref(cnt)), "scan_refine")
        return out[:cnt.value]

    def gather(self, col: Column, positions):
        import torch
        c = col.struct(False)
        out = torch.empty(max(1, positions.numel()), dtype=torch.int64, device="cuda")
        self.check(self.lib.scan_gather(self.h, ctypes.byref(c), col.enc, col.b, _ptr(positions), positions.numel(),
                                        _ptr(out)), "scan_gather")
        return out[:positions.numel()]

    # ------------------------------------------------------------ batches
    @staticmethod
    def _items(items):
        arr = (ScanItem * max(1, len(items)))()
        for i, it in enumerate(items):
            arr[i] = it
        return arr

    def batch_prepare(self, items) -> int:
        """Plan a batch of ScanItem (see Column.item) once; returns its handle."""
        arr = self._items(items)
        h = ctypes.c_uint64()
        self.check(self.lib.scan_batch_prepare(self.h, arr, len(items), ctypes.byref(h)), "scan_batch_prepare")
        return int(h.value)

    def batch_replay(self, handle: int, n_items: int | None = None, wait: bool = True):
        """Replay; with wait, returns the list of per-item result dicts."""
        if not wait:
            self.check(self.lib.scan_batch_replay(self.h, handle, None), "scan_batch_replay")
            return None
        out = (ScanResult * max(1, n_items or 0))()
        self.check(self.lib.scan_batch_replay(self.h, handle, out), "scan_batch_replay")
        return [out[i].as_dict() for i in range(n_items or 0)]

    def batch_release(self, handle: int):
        self.check(self.lib.scan_batch_release(self.h, handle), "scan_batch_release")

    def batch_run(self, items) -> list:
        arr = self._items(items)
        out = (ScanResult * max(1, len(items)))()
        self.check(self.lib.scan_batch_run(self.h, arr, len(items), out), "scan_batch_run")
        return [out[i].as_dict() for i in range(len(items))]

    def batch_set_graph(self, mode: int):
        """Replay form of later prepared batches: 0 direct launches, 1 one graph
        (the default), 2 one graph with the class scans forked over branches."""
        self.check(self.lib.scan_batch_set_graph(self.h, int(mode)), "scan_batch_set_graph")

    def batch_info(self, handle: int) -> dict:
        s = _lib.ScanBatchStats()
        self.check(self.lib.scan_batch_info(self.h, handle, ctypes.byref(s)), "scan_batch_info")
        return {"captured": int(s.captured), "kernels": int(s.kernels), "class_mask": int(s.class_mask),
                "work_items": int(s.work_items), "pruned": int(s.pruned)}

    def batch_set_order(self, order: int):
        self.check(self.lib.scan_batch_set_order(self.h, int(order)), "scan_batch_set_order")

    def batch_set_class_cost(self, us: float):
        self.check(self.lib.scan_batch_set_class_cost(self.h, float(us)), "scan_batch_set_class_cost")

    def batch_autotune(self, items, reps: int = 3):
        """Search list order x work-groups per CU x window for this batch;
        returns ((wgs_per_cu, window, order), best ms)."""
        arr = self._items(items)
        t = ScanTune()
        ms = ctypes.c_float()
        self.check(self.lib.scan_batch_autotune(self.h, arr, len(items), reps, ctypes.byref(t), ctypes.byref(ms)),
                   "scan_batch_autotune")
        return (t.wgs_per_cu, t.window_blocks, t.depth), float(ms.value)

    def batch_set_tune(self, wgs_per_cu=0, window_blocks=0):
        t = ScanTune(0, wgs_per_cu, window_blocks, 0)
        self.check(self.lib.scan_batch_set_tune(self.h, ctypes.byref(t)), "scan_batch_set_tune")

    # ----------------------------------------------------------- selector
    @staticmethod
    def mlp_param_count() -> int:
        return int(_lib.load().scan_mlp_param_count())

    def selector_set(self, theta):
        """Install network parameters (any array-like of param_count floats)."""
        a = np.ascontiguousarray(np.asarray(theta, dtype=np.float32).ravel())
        self.check(self.lib.scan_selector_set(self.h, a.ctypes.data, a.size), "scan_selector_set")

    def selector_set_margin(self, margin: float):
        """Keep the heuristic unless the network predicts a log-time gain of at least `margin`."""
        self.check(self.lib.scan_selector_set_margin(self.h, float(margin)), "scan_selector_set_margin")

    def selector_clear(self):
        self.check(self.lib.scan_selector_clear(self.h), "scan_selector_clear")

    @property
    def selector_loaded(self) -> bool:
        return bool(self.lib.scan_selector_loaded(self.h))

    def selector_load(self, path: str):
        self.check(self.lib.scan_selector_load(self.h, path.encode()), "scan_selector_load")

    def selector_save(self, path: str):
        self.check(self.lib.scan_selector_save(self.h, path.encode()), "scan_selector_save")

    def features(self, items, X_dev):
        """Selector features of the items into X_dev (device float32 [len(items), 6])."""
        arr = self._items(items)
        self.check(self.lib.scan_features(self.h, arr, len(items), _ptr(X_dev)), "scan_features")

    def mlp_forward(self, theta, X, out):
        self.check(self.lib.scan_mlp_forward(self.h, _ptr(theta), _ptr(X), X.shape[0], _ptr(out)),
                   "scan_mlp_forward")

    def mlp_loss_grad(self, theta, X, Y, M, inv_denom: float, grad, loss=None):
        self.check(self.lib.scan_mlp_loss_grad(self.h, _ptr(theta), _ptr(X), _ptr(Y), _ptr(M), X.shape[0],
                                               float(inv_denom), _ptr(grad), _ptr(loss)), "scan_mlp_loss_grad")

    def adam_step(self, theta, grad, m, v, step: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.check(self.lib.scan_adam_step(self.h, _ptr(theta), _ptr(grad), _ptr(m), _ptr(v), theta.numel(), step,
                                           lr, beta1, beta2, eps), "scan_adam_step")

    # ------------------------------------------------------ bandwidth probes
    def beta_read(self, buf, nbytes: int, sink, wgs=0, wg_size=0, unroll=0):
        self.check(self.lib.scan_beta_read(self.h, _ptr(buf), nbytes, wgs, wg_size, unroll, _ptr(sink)),
                   "scan_beta_read")

    def beta_triad(self, a, b, c, s: float):
        self.check(self.lib.scan_beta_triad(self.h, _ptr(a), _ptr(b), _ptr(c), s, a.numel()), "scan_beta_triad")

    def cache_flush(self, buf, nbytes: int):
        self.check(self.lib.scan_cache_flush(self.h, _ptr(buf), nbytes), "scan_cache_flush")


def result_from_tensor(t) -> dict:
    """Decode a 40-byte scan_result held in a (host) tensor/array."""
    raw = t.cpu().numpy().tobytes() if hasattr(t, "cpu") else bytes(t)
    r = ScanResult.from_buffer_copy(raw[:ctypes.sizeof(ScanResult)])
    return r.as_dict()
