"""ctypes binding of libflashgmm.so (argument marshalling only).

Torch tensors supply device memory and the current HIP stream; every step of
the coder runs in the library's HIP kernels. The binding raises if the
library is missing or a tensor is not a contiguous device tensor of the
expected dtype: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libflashgmm.so")

OK, EINVAL, ERANGE, ECORRUPT, ENOSPC, EDEVICE, ENOMEM, E2BIG = range(8)


class GmmError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_str(status)} (status {status})")


class Cfg(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("lo", ctypes.c_int32), ("hi", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("num_streams", ctypes.c_int32),
                ("cdf_kind", ctypes.c_int32), ("param_kind", ctypes.c_int32)]


# cdf_kind values (Sec. III-B and Table II of the paper)
CDF_AS, CDF_LOGISTIC, CDF_POLYA, CDF_REFERENCE = 0, 1, 2, 3
# param_kind values: planes hold (weights, means, scales) or raw outputs
# (weight logits, means, log-scales)
PARAMS_PLAIN, PARAMS_RAW = 0, 1


class DecodeStats(ctypes.Structure):
    _fields_ = [("hits", ctypes.c_uint64), ("misses", ctypes.c_uint64),
                ("wave_all_hit", ctypes.c_uint64), ("wave_steps", ctypes.c_uint64)]


class LatentIO(ctypes.Structure):
    _fields_ = [("symbols", ctypes.c_void_p), ("weights", ctypes.c_void_p),
                ("means", ctypes.c_void_p), ("scales", ctypes.c_void_p),
                ("bitstream", ctypes.c_void_p), ("words", ctypes.c_int64),
                ("offsets", ctypes.c_void_p), ("decoded", ctypes.c_void_p)]


class PlanConfig(ctypes.Structure):
    _fields_ = [("lanes_per_stream", ctypes.c_int32), ("streams_per_lane", ctypes.c_int32),
                ("schedule", ctypes.c_int32), ("waves_per_cu", ctypes.c_int32),
                ("lds_staging", ctypes.c_int32)]

    def astuple(self):
        return (self.lanes_per_stream, self.streams_per_lane, self.schedule, self.waves_per_cu,
                self.lds_staging)


class PlanInfo(ctypes.Structure):
    _fields_ = [("tuned", ctypes.c_int32), ("candidates", ctypes.c_int32),
                ("graph_captured", ctypes.c_int32), ("config", PlanConfig),
                ("best_ms", ctypes.c_double)]


_lib = None
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_CFG = ctypes.POINTER(Cfg)

_SIGS = {
    "gmm_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "gmm_version": (_I32, []),
    "gmm_encode_max_words": (_I64, [_I64, _I32]),
    "gmm_workspace_bytes": (_I64, [_CFG, _I64, _I32]),
    "gmm_cdf_table": (ctypes.c_int, [_CFG, _I64, _P, _P, _P, _P, _P]),
    "gmm_inverse_cdf": (ctypes.c_int, [_CFG, _I64, _P, _P, _P, _P, _P, _P]),
    "gmm_encode": (ctypes.c_int, [_CFG, _I64, _P, _P, _P, _P, _P, _I64, _P, _P, _I64, _P, _P]),
    "gmm_encode_noalloc": (ctypes.c_int, [_CFG, _I64, _P, _P, _P, _P, _P, _I64, _P, _P, _P]),
    "gmm_decode": (ctypes.c_int, [_CFG, _I64, _P, _I64, _P, _P, _P, _P, _P, _P, _P, _P, _I64,
                                  _P, _P]),
    "gmm_fast_recip_mismatches": (ctypes.c_int, [_P, _P]),
    "gmm_params_from_raw": (ctypes.c_int, [_I32, _I64, _P, _P, _P, _P, _P]),
    "gmm_set_decode_lanes": (ctypes.c_int, [_I32]),
    "gmm_decode_lanes": (ctypes.c_int, [_CFG]),
    "gmm_set_wave_priority": (ctypes.c_int, [_I32]),
    "gmm_plan_create": (ctypes.c_int, [_CFG, _I32, _P, _P, _I32, _I32, _P]),
    "gmm_plan_exec": (ctypes.c_int, [_P, _P, _P, _P]),
    "gmm_plan_info": (ctypes.c_int, [_P, _P]),
    "gmm_plan_set_config": (ctypes.c_int, [_P, _P]),
    "gmm_plan_candidates": (ctypes.c_int, [_P, _P, _I32]),
    "gmm_plan_destroy": (ctypes.c_int, [_P]),
    "gmm_plan_set_bracket": (ctypes.c_int, [_P, _P, _P]),
    "gmm_encode_subset": (ctypes.c_int, [_CFG, _I64, _P, _I64, _P, _P, _P, _P, _P, _I64, _P, _P,
                                         _I64, _P, _P]),
    "gmm_decode_subset": (ctypes.c_int, [_CFG, _I64, _P, _I64, _P, _I64, _P, _P, _P, _P, _P, _P,
                                         _I64, _P, _P]),
    "gmm_bracket_create": (ctypes.c_int, [_P, _P]),
    "gmm_bracket_destroy": (ctypes.c_int, [_P]),
    "gmm_bracket_predict": (ctypes.c_int, [_P, _I32, _I64, _P, _P, _P, _P, _P, _P]),
    "gmm_fma_probe": (ctypes.c_int, [_P, _I64, _I32, _P]),
    "gmm_copy_probe": (ctypes.c_int, [_P, _P, _I64, _P]),
    "gmm_mlp_num_params": (ctypes.c_int, [_I32]),
    "gmm_mlp_workspace_bytes": (_I64, [_I32, _I64]),
    "gmm_mlp_features": (ctypes.c_int, [_I32, _I64, _P, _P, _P, _P, _I32, _P, _P, _I32, _P, _P]),
    "gmm_mlp_loss_grad": (ctypes.c_int, [_I32, _I64, _P, _P, _P, ctypes.c_float, _I32, _P, _P,
                                         _I64, _P]),
    "gmm_mlp_forward": (ctypes.c_int, [_I32, _I64, _P, _P, _I32, _P, _P]),
    "gmm_mlp_adam": (ctypes.c_int, [_I32, _P, _P, _P, _P, ctypes.c_float, ctypes.c_float,
                                    ctypes.c_float, ctypes.c_float, _I32, ctypes.c_float, _P,
                                    _P]),
}


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            if hasattr(L, name):
                f = getattr(L, name)
                f.restype, f.argtypes = res, args
        _lib = L
    return _lib


def status_str(s: int) -> str:
    return lib().gmm_status_str(int(s)).decode()


def make_cfg(K, lo, hi, precision=16, streams=256, cdf_kind=0, param_kind=0) -> Cfg:
    return Cfg(int(K), int(lo), int(hi), int(precision), int(streams), int(cdf_kind),
               int(param_kind))


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t: torch.Tensor, dtype, name: str):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _opt(t, dtype, name):
    return _dev(t, dtype, name) if t is not None else ctypes.c_void_p(0)


def _params(weights, means, scales, K):
    for t, nm in ((weights, "weights"), (means, "means"), (scales, "scales")):
        if t.dim() != 2 or t.shape[0] != K:
            raise ValueError(f"{nm} must be a [K][n] plane tensor")
    return (_dev(weights, torch.float32, "weights"), _dev(means, torch.float32, "means"),
            _dev(scales, torch.float32, "scales"))


def _check(st: int, what: str):
    if st != OK:
        raise GmmError(st, what)


def max_words(n: int, streams: int) -> int:
    return int(lib().gmm_encode_max_words(n, streams))


def workspace_bytes(cfg: Cfg, n: int, op: int) -> int:
    b = int(lib().gmm_workspace_bytes(ctypes.byref(cfg), n, op))
    if b < 0:
        raise GmmError(EINVAL, "workspace_bytes")
    return b


def cdf_table(cfg: Cfg, weights, means, scales) -> torch.Tensor:
    n = weights.shape[1]
    N = cfg.hi - cfg.lo + 1
    out = torch.empty((n, N + 1), dtype=torch.int32, device=weights.device)
    w, m, s = _params(weights, means, scales, cfg.K)
    _check(lib().gmm_cdf_table(ctypes.byref(cfg), n, w, m, s, ctypes.c_void_p(out.data_ptr()),
                               _stream()), "cdf_table")
    return out


def inverse_cdf(cfg: Cfg, weights, means, scales, slot: torch.Tensor) -> torch.Tensor:
    n = weights.shape[1]
    out = torch.empty((n,), dtype=torch.int32, device=weights.device)
    w, m, s = _params(weights, means, scales, cfg.K)
    _check(lib().gmm_inverse_cdf(ctypes.byref(cfg), n, w, m, s, _dev(slot, torch.int32, "slot"),
                                 ctypes.c_void_p(out.data_ptr()), _stream()), "inverse_cdf")
    return out


def encode_into(cfg: Cfg, symbols, weights, means, scales, bitstream, offsets, ws=None,
                status=None, stream=None) -> int:
    """Low-level encode into caller buffers. With ``status`` (int32 device
    tensor) the call is asynchronous; otherwise it returns the status."""
    n = symbols.numel()
    w, m, s = _params(weights, means, scales, cfg.K)
    if offsets.numel() != cfg.num_streams + 1:
        raise ValueError("offsets must hold num_streams + 1 entries")
    return lib().gmm_encode(ctypes.byref(cfg), n, _dev(symbols, torch.int32, "symbols"), w, m, s,
                            _dev(bitstream, torch.int16, "bitstream"), bitstream.numel(),
                            _dev(offsets, torch.int64, "offsets"), _opt(ws, torch.uint8, "ws"),
                            ws.numel() if ws is not None else 0,
                            _opt(status, torch.int32, "status"), _stream(stream))


def encode_noalloc_into(cfg: Cfg, symbols, weights, means, scales, bitstream, offsets,
                       status=None, stream=None) -> int:
    """gmm_encode_noalloc into caller buffers: the library allocates nothing
    (its workspace is a static device array). With ``status`` asynchronous;
    otherwise it returns the status."""
    n = symbols.numel()
    w, m, s = _params(weights, means, scales, cfg.K)
    if offsets.numel() != cfg.num_streams + 1:
        raise ValueError("offsets must hold num_streams + 1 entries")
    return lib().gmm_encode_noalloc(ctypes.byref(cfg), n, _dev(symbols, torch.int32, "symbols"),
                                    w, m, s, _dev(bitstream, torch.int16, "bitstream"),
                                    bitstream.numel(), _dev(offsets, torch.int64, "offsets"),
                                    _opt(status, torch.int32, "status"), _stream(stream))


def decode_into(cfg: Cfg, bitstream, offsets, weights, means, scales, symbols, total_words=None,
                bracket=None, stats=None, ws=None, status=None, stream=None) -> int:
    n = symbols.numel()
    w, m, s = _params(weights, means, scales, cfg.K)
    if offsets.numel() != cfg.num_streams + 1:
        raise ValueError("offsets must hold num_streams + 1 entries")
    tw = bitstream.numel() if total_words is None else int(total_words)
    if tw > bitstream.numel():
        raise ValueError("total_words exceeds the bitstream tensor")
    bh = ctypes.c_void_p(bracket.handle) if bracket is not None else ctypes.c_void_p(0)
    return lib().gmm_decode(ctypes.byref(cfg), n, _dev(bitstream, torch.int16, "bitstream"), tw,
                            _dev(offsets, torch.int64, "offsets"), w, m, s,
                            _dev(symbols, torch.int32, "symbols"), bh,
                            _opt(stats, torch.int64, "stats"), _opt(ws, torch.uint8, "ws"),
                            ws.numel() if ws is not None else 0,
                            _opt(status, torch.int32, "status"), _stream(stream))


def encode(symbols, weights, means, scales, lo, hi, precision=16, streams=256, cdf_kind=0,
           param_kind=0):
    """Encode int32 symbols [n] with [K][n] float32 parameter planes.
    Returns (bitstream int16 tensor of the exact encoded size, offsets int64
    tensor [streams+1]); bitstream words are uint16 values stored as int16."""
    K = weights.shape[0]
    cfg = make_cfg(K, lo, hi, precision, streams, cdf_kind, param_kind)
    n = symbols.numel()
    cap = max_words(n, streams)
    bs = torch.empty((max(cap, 1),), dtype=torch.int16, device=symbols.device)
    off = torch.empty((streams + 1,), dtype=torch.int64, device=symbols.device)
    _check(encode_into(cfg, symbols, weights, means, scales, bs, off), "encode")
    total = int(off[-1].item())
    return bs[:total], off


def decode(bitstream, offsets, weights, means, scales, lo, hi, precision=16, streams=256,
           cdf_kind=0, bracket=None, stats=None, param_kind=0):
    K = weights.shape[0]
    cfg = make_cfg(K, lo, hi, precision, streams, cdf_kind, param_kind)
    n = weights.shape[1]
    sym = torch.empty((n,), dtype=torch.int32, device=weights.device)
    bs = bitstream if bitstream.numel() else torch.zeros(1, dtype=torch.int16,
                                                         device=weights.device)
    _check(decode_into(cfg, bs, offsets, weights, means, scales, sym,
                       total_words=bitstream.numel(), bracket=bracket, stats=stats), "decode")
    return sym


def params_from_raw(logits, log_scales, stream=None):
    """Raw network outputs [K][n] (weight logits, log-scales; float32 on the
    device) to (weights, scales) [K][n], by the library's kernel."""
    assert logits.shape == log_scales.shape and logits.dim() == 2
    w = torch.empty_like(logits)
    sg = torch.empty_like(log_scales)
    _check(lib().gmm_params_from_raw(int(logits.shape[0]), int(logits.shape[1]),
                                     _dev(logits, torch.float32, "logits"),
                                     _dev(log_scales, torch.float32, "log_scales"),
                                     _dev(w, torch.float32, "weights"),
                                     _dev(sg, torch.float32, "scales"), _stream(stream)),
           "params_from_raw")
    return w, sg


def set_decode_lanes(lanes: int) -> None:
    """Lanes per stream of later decodes (0 = automatic); output unchanged."""
    _check(lib().gmm_set_decode_lanes(int(lanes)), "set_decode_lanes")


def decode_lanes(cfg: Cfg) -> int:
    """Lanes per stream a plain decode of cfg uses now (the
    set_decode_lanes choice, or the automatic one)."""
    L = lib().gmm_decode_lanes(ctypes.byref(cfg))
    if L < 0:
        _check(-L, "decode_lanes")
    return L


def set_wave_priority(priority: int) -> None:
    """Wavefront issue priority (0..3) of this thread's later encode and
    decode calls; output unchanged."""
    _check(lib().gmm_set_wave_priority(int(priority)), "set_wave_priority")


def fast_recip_mismatches() -> int:
    c = ctypes.c_uint64(0)
    _check(lib().gmm_fast_recip_mismatches(ctypes.byref(c), _stream()), "fast_recip_check")
    return int(c.value)


PLAN_AUTOTUNE = 1
SCHEDULES = ("flat", "dynamic", "static")


class Plan:
    """Batched encode (op=0) or decode (op=1) of B latents with fixed shapes
    (n_b elements, S_b streams each), run as one captured hipGraph."""

    def __init__(self, K, lo, hi, precision, ns, streams, op, autotune=True, cdf_kind=0,
                 param_kind=0):
        self.cfg = make_cfg(K, lo, hi, precision, 1, cdf_kind, param_kind)
        self.ns = [int(v) for v in ns]
        self.streams = [int(v) for v in streams]
        self.B, self.op = len(self.ns), int(op)
        n_arr = (ctypes.c_int64 * self.B)(*self.ns)
        s_arr = (ctypes.c_int32 * self.B)(*self.streams)
        h = ctypes.c_void_p(0)
        _check(lib().gmm_plan_create(ctypes.byref(self.cfg), self.B, n_arr, s_arr, self.op,
                                     PLAN_AUTOTUNE if autotune else 0, ctypes.byref(h)),
               "plan_create")
        self.handle = h
        self._io = (LatentIO * self.B)()

    def _fill(self, latents):
        if len(latents) != self.B:
            raise ValueError("one io dict per latent")
        for b, d in enumerate(latents):
            x = self._io[b]
            K = self.cfg.K
            if self.ns[b] != d["weights"].shape[1]:
                raise ValueError(f"latent {b}: n differs from the plan")
            w, m, s = _params(d["weights"], d["means"], d["scales"], K)
            x.weights, x.means, x.scales = w.value, m.value, s.value
            if d["offsets"].numel() != self.streams[b] + 1:
                raise ValueError(f"latent {b}: offsets must hold S+1 entries")
            x.offsets = _dev(d["offsets"], torch.int64, "offsets").value
            bs = d["bitstream"]
            x.bitstream = _dev(bs, torch.int16, "bitstream").value
            x.words = int(d.get("words", bs.numel()))
            if x.words > bs.numel():
                raise ValueError("words exceeds the bitstream tensor")
            if self.op == 0:
                x.symbols = _dev(d["symbols"], torch.int32, "symbols").value
                x.decoded = None
            else:
                x.decoded = _dev(d["decoded"], torch.int32, "decoded").value
                x.symbols = None

    def run(self, latents, status=None, stream=None) -> int:
        """latents: list of dicts of tensors (weights, means, scales,
        bitstream, offsets, words?, symbols | decoded). With ``status`` (int32
        device tensor [B]) asynchronous; otherwise returns the worst status."""
        self._fill(latents)
        return lib().gmm_plan_exec(self.handle, self._io, _opt(status, torch.int32, "status"),
                                   _stream(stream))

    def info(self) -> dict:
        inf = PlanInfo()
        _check(lib().gmm_plan_info(self.handle, ctypes.byref(inf)), "plan_info")
        c = inf.config
        return {"tuned": bool(inf.tuned), "lanes_per_stream": c.lanes_per_stream,
                "streams_per_lane": c.streams_per_lane, "schedule": SCHEDULES[c.schedule],
                "waves_per_cu": c.waves_per_cu, "lds_staging": bool(c.lds_staging),
                "candidates": inf.candidates, "graph_captured": bool(inf.graph_captured),
                "best_ms": inf.best_ms}

    def set_config(self, lanes, streams_per_lane, schedule, waves_per_cu, lds_staging):
        """Forces a launch shape; the arguments are a candidate tuple."""
        c = PlanConfig(int(lanes), int(streams_per_lane), int(schedule), int(waves_per_cu),
                       int(lds_staging))
        _check(lib().gmm_plan_set_config(self.handle, ctypes.byref(c)), "plan_set_config")

    def set_bracket(self, bracket, stats=None):
        """Decode plans: use the learned bracket (None = plain search)."""
        h = ctypes.c_void_p(bracket.handle if bracket is not None else 0)
        _check(lib().gmm_plan_set_bracket(self.handle, h, _opt(stats, torch.int64, "stats")),
               "plan_set_bracket")
        self._bracket = bracket

    def candidates(self):
        """The tuner's launch shapes as tuples (lanes_per_stream,
        streams_per_lane, schedule, waves_per_cu, lds_staging)."""
        n = lib().gmm_plan_candidates(self.handle, None, 0)
        buf = (PlanConfig * max(n, 1))()
        lib().gmm_plan_candidates(self.handle, buf, n)
        return [buf[i].astuple() for i in range(n)]

    def close(self):
        if self.handle:
            lib().gmm_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BracketDesc(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("radius", ctypes.c_int32),
                ("params", ctypes.c_void_p), ("in_mean", ctypes.c_void_p),
                ("in_std", ctypes.c_void_p), ("out_mean", ctypes.c_float),
                ("out_std", ctypes.c_float)]


class Bracket:
    """A learned search-bracket model loaded into the library (handle for
    decode). ``params`` float32 [P], ``in_mean``/``in_std`` float32 [3K+1]."""

    def __init__(self, K, params, in_mean, in_std, out_mean, out_std, radius=4):
        import numpy as np
        self.K, self.radius = int(K), int(radius)
        self._keep = [np.ascontiguousarray(np.asarray(a, dtype=np.float32))
                      for a in (params, in_mean, in_std)]
        d = BracketDesc(self.K, self.radius, self._keep[0].ctypes.data,
                        self._keep[1].ctypes.data, self._keep[2].ctypes.data,
                        float(out_mean), float(out_std))
        h = ctypes.c_void_p(0)
        _check(lib().gmm_bracket_create(ctypes.byref(d), ctypes.byref(h)), "bracket_create")
        self.handle = h.value

    def predict(self, precision, weights, means, scales, slot):
        n = weights.shape[1]
        out = torch.empty(n, dtype=torch.float32, device=weights.device)
        w, m, s = _params(weights, means, scales, self.K)
        _check(lib().gmm_bracket_predict(ctypes.c_void_p(self.handle), precision, n, w, m, s,
                                         _dev(slot, torch.int32, "slot"),
                                         ctypes.c_void_p(out.data_ptr()), _stream()),
               "bracket_predict")
        return out

    def close(self):
        if self.handle:
            lib().gmm_bracket_destroy(ctypes.c_void_p(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mlp_num_params(D: int) -> int:
    return int(lib().gmm_mlp_num_params(D))


def mlp_features(K, weights, means, scales, slot, precision, mean=None, inv_std=None,
                 round_bf16=False):
    n = weights.shape[1]
    D = 3 * K + 1
    X = torch.empty((n, D), dtype=torch.float32, device=weights.device)
    w, m, s = _params(weights, means, scales, K)
    _check(lib().gmm_mlp_features(K, n, w, m, s, _dev(slot, torch.int32, "slot"), precision,
                                  _opt(mean, torch.float32, "mean"),
                                  _opt(inv_std, torch.float32, "inv_std"), int(round_bf16),
                                  ctypes.c_void_p(X.data_ptr()), _stream()), "mlp_features")
    return X


def mlp_loss_grad(X, y, params, delta, round_act=True, ws=None):
    """Returns a float32 device tensor [P + 1]: summed gradients, then loss."""
    n, D = X.shape
    P = mlp_num_params(D)
    out = torch.empty(P + 1, dtype=torch.float32, device=X.device)
    need = int(lib().gmm_mlp_workspace_bytes(D, n))
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=X.device)
    _check(lib().gmm_mlp_loss_grad(D, n, _dev(X, torch.float32, "X"),
                                   _dev(y, torch.float32, "y"),
                                   _dev(params, torch.float32, "params"), float(delta),
                                   int(round_act), ctypes.c_void_p(out.data_ptr()),
                                   ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()),
           "mlp_loss_grad")
    return out


def mlp_forward(X, params, round_act=True):
    n, D = X.shape
    out = torch.empty(n, dtype=torch.float32, device=X.device)
    _check(lib().gmm_mlp_forward(D, n, _dev(X, torch.float32, "X"),
                                 _dev(params, torch.float32, "params"), int(round_act),
                                 ctypes.c_void_p(out.data_ptr()), _stream()), "mlp_forward")
    return out


def mlp_adam(params, grad, m, v, lr, step, grad_scale, shadow=None, beta1=0.9, beta2=0.999,
             eps=1e-8):
    P = params.numel()
    _check(lib().gmm_mlp_adam(P, _dev(params, torch.float32, "params"),
                              _dev(grad, torch.float32, "grad"), _dev(m, torch.float32, "m"),
                              _dev(v, torch.float32, "v"), float(lr), float(beta1),
                              float(beta2), float(eps), int(step), float(grad_scale),
                              _opt(shadow, torch.float32, "shadow"), _stream()), "mlp_adam")


def fma_probe(out, iters, stream=None):
    """Launches the FP32 fma issue probe over out.numel() lanes (see
    gmm_fma_probe); lane-fmas = out.numel() * iters * 8."""
    _check(lib().gmm_fma_probe(_dev(out, torch.float32, "out"), out.numel(), int(iters),
                               _stream(stream)), "fma_probe")


def copy_probe(src, dst, stream=None):
    """Launches the device copy probe of src into dst (same byte size)."""
    if src.numel() * src.element_size() != dst.numel() * dst.element_size():
        raise ValueError("src and dst differ in size")
    _check(lib().gmm_copy_probe(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                src.numel() * src.element_size(), _stream(stream)),
           "copy_probe")


def checkerboard_indices(C, H, W, anchor=True, device="cuda"):
    """Element indices (int32, latent order c*H*W + h*W + w) of the anchors
    ((h + w) even) or of the non-anchors of a Checkerboard two-pass model."""
    h = torch.arange(H, device=device).view(H, 1)
    w = torch.arange(W, device=device).view(1, W)
    sel = ((h + w) % 2 == 0) if anchor else ((h + w) % 2 == 1)
    plane = torch.nonzero(sel.flatten(), as_tuple=False).flatten()
    c = torch.arange(C, device=device).view(C, 1) * (H * W)
    return (c + plane.view(1, -1)).flatten().to(torch.int32).contiguous()


def encode_subset_into(cfg, idx, symbols, weights, means, scales, bitstream, offsets, ws=None,
                       status=None, stream=None) -> int:
    """Codes elements idx of the latent (symbols [n_total], planes [K][n_total])."""
    n_total = symbols.numel()
    w, m, s = _params(weights, means, scales, cfg.K)
    if offsets.numel() != cfg.num_streams + 1:
        raise ValueError("offsets must hold num_streams + 1 entries")
    return lib().gmm_encode_subset(ctypes.byref(cfg), n_total, _dev(idx, torch.int32, "idx"),
                                   idx.numel(), _dev(symbols, torch.int32, "symbols"), w, m, s,
                                   _dev(bitstream, torch.int16, "bitstream"), bitstream.numel(),
                                   _dev(offsets, torch.int64, "offsets"),
                                   _opt(ws, torch.uint8, "ws"),
                                   ws.numel() if ws is not None else 0,
                                   _opt(status, torch.int32, "status"), _stream(stream))


def decode_subset_into(cfg, idx, bitstream, offsets, weights, means, scales, symbols,
                       total_words=None, ws=None, status=None, stream=None) -> int:
    """Decodes a subset pass into symbols[idx] (symbols is the full latent)."""
    n_total = symbols.numel()
    w, m, s = _params(weights, means, scales, cfg.K)
    if offsets.numel() != cfg.num_streams + 1:
        raise ValueError("offsets must hold num_streams + 1 entries")
    tw = bitstream.numel() if total_words is None else int(total_words)
    return lib().gmm_decode_subset(ctypes.byref(cfg), n_total, _dev(idx, torch.int32, "idx"),
                                   idx.numel(), _dev(bitstream, torch.int16, "bitstream"), tw,
                                   _dev(offsets, torch.int64, "offsets"), w, m, s,
                                   _dev(symbols, torch.int32, "symbols"),
                                   _opt(ws, torch.uint8, "ws"),
                                   ws.numel() if ws is not None else 0,
                                   _opt(status, torch.int32, "status"), _stream(stream))
