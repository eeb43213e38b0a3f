"""CPU oracle of the GMM rANS coder: TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. It wraps ``liboracle.so`` (plain C,
built from ``gmm_oracle.c`` and ``mlp_oracle.c`` by :func:`build`) with
numpy arrays. Nothing here is shared with the GPU library.

The C functions restate the classic per-element CDF table method of the
FlashGMM paper (Sec. II-C, Eqs. (4)-(6)) with the paper's rANS map (Sec. II-B,
Eq. (3)) and its Gaussian-CDF approximations (Sec. III-B).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["gmm_oracle.c", "mlp_oracle.c"]

OK, EINVAL, ERANGE, ECORRUPT, ENOSPC = 0, 1, 2, 3, 4


def build(verbose: bool = False) -> str:
    """Compile liboracle.so with gcc (no FMA contraction, no fast-math)."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES if os.path.exists(os.path.join(_HERE, s))]
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", _LIB_PATH + ".tmp"] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class Cfg(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("lo", ctypes.c_int32), ("hi", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("num_streams", ctypes.c_int32),
                ("cdf_kind", ctypes.c_int32), ("param_kind", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i64, i32 = ctypes.c_int64, ctypes.c_int32
        cfgp = ctypes.POINTER(Cfg)
        sigs = {
            "gmm_oracle_phi": (ctypes.c_float, [ctypes.c_float, i32]),
            "gmm_oracle_exp": (ctypes.c_float, [ctypes.c_float]),
            "gmm_oracle_as_tail": (ctypes.c_double, [ctypes.c_float]),
            "gmm_oracle_as_constants": (None, [P]),
            "gmm_oracle_as_half": (ctypes.c_float, [ctypes.c_float, ctypes.c_float]),
            "gmm_oracle_phi_batch": (None, [P, P, i64, i32]),
            "gmm_oracle_exp_batch": (None, [P, P, i64]),
            "gmm_oracle_F_table": (ctypes.c_int, [cfgp, i64, P, P, P, P]),
            "gmm_oracle_cdf_table": (ctypes.c_int, [cfgp, i64, P, P, P, P]),
            "gmm_oracle_encode": (ctypes.c_int, [cfgp, i64, P, P, P, P, P, i64, P]),
            "gmm_oracle_decode": (ctypes.c_int, [cfgp, i64, P, i64, P, P, P, P, P]),
            "gmm_oracle_inverse": (ctypes.c_int, [cfgp, i64, P, P, P, P, P]),
            "gmm_oracle_num_threads": (i32, []),
            "gmm_oracle_set_num_threads": (None, [i32]),
            "gmm_oracle_exp_d": (ctypes.c_double, [ctypes.c_double]),
            "gmm_oracle_tail_ref": (ctypes.c_double, [ctypes.c_double]),
            "gmm_oracle_phi_ref": (ctypes.c_double, [ctypes.c_double]),
            "gmm_oracle_ref_batch": (None, [P, P, i64, i32]),
            "gmm_oracle_params_from_raw": (ctypes.c_int, [i32, i64, P, P, P, P]),
            "gmm_oracle_mlp_num_params": (i64, [i32, i32]),
            "gmm_oracle_mlp_forward": (None, [i32, i32, P, i64, P, i32, P]),
            "gmm_oracle_mlp_loss_grad": (ctypes.c_double, [i32, i32, P, i64, P, P,
                                                           ctypes.c_double, i32, P]),
        }
        for name, (res, args) in sigs.items():
            f = getattr(L, name)
            f.restype, f.argtypes = res, args
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def make_cfg(K, lo, hi, precision=16, num_streams=1, cdf_kind=0, param_kind=0) -> Cfg:
    return Cfg(K, lo, hi, precision, num_streams, cdf_kind, param_kind)


def _params(w, mu, sig):
    w = np.ascontiguousarray(w, dtype=np.float32)
    mu = np.ascontiguousarray(mu, dtype=np.float32)
    sig = np.ascontiguousarray(sig, dtype=np.float32)
    assert w.shape == mu.shape == sig.shape and w.ndim == 2, "params are [K][n] planes"
    return w, mu, sig


def phi(z, kind=0) -> np.ndarray:
    z = np.ascontiguousarray(z, dtype=np.float32).ravel()
    out = np.empty_like(z)
    lib().gmm_oracle_phi_batch(_p(z), _p(out), z.size, kind)
    return out


def as_tail(a) -> np.ndarray:
    """Kind 0's tail at a = |z|/9, the exact (binary64) product of its two
    binary32 factors (one call per value)."""
    a = np.asarray(a, dtype=np.float32).ravel()
    f = lib().gmm_oracle_as_tail
    return np.array([f(float(v)) for v in a], dtype=np.float64)


def as_constants() -> np.ndarray:
    """Kind 0's constants: 9p, 1/9, 81 log2(e)/2, density coefficients 0..5."""
    out = np.zeros(9, dtype=np.float32)
    lib().gmm_oracle_as_constants(_p(out))
    return out


def as_half(d, rn) -> np.ndarray:
    """Kind 0's signed half Phi~ - 1/2 of one component from d = b - mu and
    rn = r/9 (one call per pair)."""
    d = np.asarray(d, dtype=np.float32).ravel()
    rn = np.broadcast_to(np.asarray(rn, dtype=np.float32), d.shape)
    f = lib().gmm_oracle_as_half
    return np.array([f(float(x), float(y)) for x, y in zip(d, rn)], dtype=np.float32)


def ref_batch(x, which: str) -> np.ndarray:
    """binary64 reference functions over an array: 'exp' (exp of g in
    [-686, 0]), 'tail' (Q(a) = erfc(a/sqrt 2)/2, a in [0, 37]) or 'phi'."""
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    out = np.empty_like(x)
    lib().gmm_oracle_ref_batch(_p(x), _p(out), x.size, {"exp": 0, "tail": 1, "phi": 2}[which])
    return out


def params_from_raw(logits, log_scales):
    """Raw outputs [K][n] (weight logits, log-scales) -> (weights, scales)."""
    l = np.ascontiguousarray(logits, dtype=np.float32)
    t = np.ascontiguousarray(log_scales, dtype=np.float32)
    assert l.shape == t.shape and l.ndim == 2
    w, sg = np.empty_like(l), np.empty_like(t)
    st = lib().gmm_oracle_params_from_raw(l.shape[0], l.shape[1], _p(l), _p(t), _p(w), _p(sg))
    assert st == OK, st
    return w, sg


def exp(g) -> np.ndarray:
    g = np.ascontiguousarray(g, dtype=np.float32).ravel()
    out = np.empty_like(g)
    lib().gmm_oracle_exp_batch(_p(g), _p(out), g.size)
    return out


def F_table(cfg: Cfg, w, mu, sig) -> np.ndarray:
    w, mu, sig = _params(w, mu, sig)
    n = w.shape[1]
    N = cfg.hi - cfg.lo + 1
    out = np.empty((n, N + 1), dtype=np.float32)
    st = lib().gmm_oracle_F_table(ctypes.byref(cfg), n, _p(w), _p(mu), _p(sig), _p(out))
    if st:
        raise ValueError(f"oracle F_table status {st}")
    return out


def cdf_table(cfg: Cfg, w, mu, sig) -> np.ndarray:
    w, mu, sig = _params(w, mu, sig)
    n = w.shape[1]
    N = cfg.hi - cfg.lo + 1
    out = np.empty((n, N + 1), dtype=np.uint32)
    st = lib().gmm_oracle_cdf_table(ctypes.byref(cfg), n, _p(w), _p(mu), _p(sig), _p(out))
    if st:
        raise ValueError(f"oracle cdf_table status {st}")
    return out


def inverse(cfg: Cfg, w, mu, sig, slot) -> np.ndarray:
    w, mu, sig = _params(w, mu, sig)
    slot = np.ascontiguousarray(slot, dtype=np.uint32)
    out = np.empty(slot.shape, dtype=np.int32)
    st = lib().gmm_oracle_inverse(ctypes.byref(cfg), w.shape[1], _p(w), _p(mu), _p(sig),
                                  _p(slot), _p(out))
    if st:
        raise ValueError(f"oracle inverse status {st}")
    return out


def encode(cfg: Cfg, sym, w, mu, sig, capacity=None):
    """Returns (status, bitstream[uint16], offsets[int64, S+1])."""
    w, mu, sig = _params(w, mu, sig)
    sym = np.ascontiguousarray(sym, dtype=np.int32)
    n = sym.size
    S = cfg.num_streams
    cap = n + 2 * S if capacity is None else capacity
    bs = np.zeros(max(cap, 1), dtype=np.uint16)
    off = np.zeros(S + 1, dtype=np.int64)
    st = lib().gmm_oracle_encode(ctypes.byref(cfg), n, _p(sym), _p(w), _p(mu), _p(sig),
                                 _p(bs), cap, _p(off))
    if st == OK:
        bs = bs[: off[S]].copy()
    return st, bs, off


def decode(cfg: Cfg, bitstream, offsets, w, mu, sig, n=None):
    """Returns (status, symbols[int32])."""
    w, mu, sig = _params(w, mu, sig)
    n = w.shape[1] if n is None else n
    bs = np.ascontiguousarray(bitstream, dtype=np.uint16)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    assert off.size == cfg.num_streams + 1
    sym = np.zeros(n, dtype=np.int32)
    bs_arg = bs if bs.size else np.zeros(1, dtype=np.uint16)
    st = lib().gmm_oracle_decode(ctypes.byref(cfg), n, _p(bs_arg), bs.size, _p(off),
                                 _p(w), _p(mu), _p(sig), _p(sym))
    return st, sym


def num_threads() -> int:
    return int(lib().gmm_oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's later parallel loops."""
    lib().gmm_oracle_set_num_threads(int(n))


def mlp_num_params(D: int, H: int = 64) -> int:
    return int(lib().gmm_oracle_mlp_num_params(D, H))


def mlp_forward(params, X, H: int = 64, round_act: bool = False) -> np.ndarray:
    """FP64 forward of the bracket MLP (parameter layout W1, b1, W2, b2, w3, b3);
    with round_act the first layer's activations are rounded to bfloat16."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    p = np.ascontiguousarray(params, dtype=np.float64)
    n, D = X.shape
    assert p.size == mlp_num_params(D, H)
    out = np.empty(n, dtype=np.float64)
    lib().gmm_oracle_mlp_forward(D, H, _p(p), n, _p(X), int(bool(round_act)), _p(out))
    return out


def mlp_loss_grad(params, X, y, delta=1.0, H: int = 64, round_act: bool = False):
    """Sum of Huber losses and its FP64 gradient (same layout as params);
    with round_act the first layer's activations are rounded to bfloat16
    and the gradient passes straight through the rounding."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    p = np.ascontiguousarray(params, dtype=np.float64)
    n, D = X.shape
    g = np.empty_like(p)
    loss = lib().gmm_oracle_mlp_loss_grad(D, H, _p(p), n, _p(X), _p(y), float(delta),
                                          int(bool(round_act)), _p(g))
    return float(loss), g
