"""Pins of the oracle's Gaussian-CDF variants of the paper's Table II ablation
and of the raw-output parameter mapping (no GPU).

- Polya's approximation (FlashGMM Sec. III-B, first candidate; read as
  (1 + sign(x) sqrt(1 - exp(-2 x^2 / pi))) / 2): against that closed form in
  binary64, its known maximum error against the Gaussian CDF, and a
  monotonicity lemma for its float evaluation (exhaustive scans).
- the binary64 reference CDF standing in for the unapproximated erfc of
  Table II: against libm's erfc and numpy's exp, symmetry, and the step
  monotonicity that follows from its error bound.
- the raw-output mapping (softmax of weight logits, exponential of
  log-scales with the 0.11 scale bound of Sec. II-B): against binary64.
- coder plumbing: raw-output encode equals plain encode of mapped params;
  round trips and table invariants for every CDF kind.
"""
import ctypes
import math
import os
import struct
import subprocess

import numpy as np
import pytest
from scipy.special import ndtr

from conftest import ROOT
from paper_2509_18815_amd import synth

POLYA_C = float(np.float32(2.0 / math.pi))


def _fbits(f):
    return struct.unpack("<I", struct.pack("<f", f))[0]


def _scan_lib():
    so = os.path.join("/tmp", f"lemma_scan_abl_{os.getpid()}.so")
    subprocess.run(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-o", so,
                    os.path.join(ROOT, "tests", "lemma_scan.c"),
                    os.path.join(ROOT, "oracle", "liboracle.so"), "-lm"], check=True)
    return ctypes.CDLL(so)


def polya64(z):
    z = np.asarray(z, np.float64)
    return 0.5 * (1.0 + np.sign(z) * np.sqrt(-np.expm1(-POLYA_C * z * z)))


# ----------------------------------------------------------------- exp~

def test_exp_tilde_extended_range(orc):
    """exp~ on the whole range the contract uses: [-51.6, 0] (Polya's
    exponent at |z| <= 9) and [0, 7] (log-scales): within 2^-23 relative."""
    rng = np.random.default_rng(5)
    g = np.concatenate([np.linspace(-51.6, 7.0, 1_000_001),
                        rng.uniform(-51.6, 7.0, 500_000)]).astype(np.float32)
    e = orc.exp(g).astype(np.float64)
    ref = np.exp(g.astype(np.float64))
    assert (np.abs(e - ref) / ref).max() <= 2.0 ** -23


# ----------------------------------------------------------------- Polya

def test_polya_matches_closed_form(orc):
    z = np.concatenate([np.linspace(-9, 9, 400_001),
                        np.random.default_rng(6).uniform(-9, 9, 200_000)]).astype(np.float32)
    ph = orc.phi(z, 2).astype(np.float64)
    ref = polya64(z.astype(np.float64))
    assert np.abs(ph - ref).max() <= 2.0 ** -23
    # the tail itself, in relative terms (u = c a^2 is rounded: |du| <= 81 c 2^-23)
    a = np.linspace(0.0, 9.0, 200_001).astype(np.float32)
    t = orc.phi(-a, 2).astype(np.float64)
    ref_t = 1.0 - polya64(a.astype(np.float64))
    a64 = a.astype(np.float64)
    ref_t = 0.5 * np.exp(-POLYA_C * a64 * a64) / (1 + np.sqrt(-np.expm1(-POLYA_C * a64 * a64)))
    assert (np.abs(t - ref_t) / ref_t).max() <= 1e-5
    assert orc.phi(np.float32([0.0]), 2)[0] == 0.5
    assert 0.0 < orc.phi(np.float32([-9.0]), 2)[0] < 1e-22


def test_polya_error_against_gaussian(orc):
    """The formula with 2/pi is within about 3.2e-3 of Phi (its known
    accuracy); the variant printed without 2/pi would be off by > 0.05."""
    z = np.linspace(-9, 9, 200_001).astype(np.float32)
    err = np.abs(orc.phi(z, 2).astype(np.float64) - ndtr(z.astype(np.float64)))
    assert 2.5e-3 < err.max() < 3.3e-3, err.max()
    zz = z.astype(np.float64)
    printed = 0.5 * (1 + np.sign(zz) * np.sqrt(1 - np.exp(-zz * zz)))
    assert np.abs(printed - ndtr(zz)).max() > 0.05


def test_polya_monotonicity_lemma(orc):
    """The float Polya tail is T = RN(RN(e/2) / RN(1 + sqrt(E))) with
    e = exp~(-u), E = 1 - exp(-u) (Taylor series below u = 1/4, else
    RN(1 - e)) and u = RN(RN(a a) c): T does not increase when e does not
    increase and E does not decrease, each step being a correctly rounded
    monotone map. Boundary steps in a are at least d = 2^-11 (z steps by
    r >= 2^-10 less two roundings), and for a1 >= a0 + d,
    u1 - u0 >= D(a0) = c (2 a0 d + d^2) - c (a0^2 + a1^2) th, th = 2.0001 2^-24.
      e-part, a0 >= aB: exp~'s exhaustive relative error eps and
        exp(-D)(1+eps)/(1-eps) < 1 give exp~(-u1) < exp~(-u0);
      e-part, a0 < aB: u0 <= c aB^2 (1+th) and u1 >= c d^2 (1-th), and the
        largest exp~ on the second range is at most the smallest on the
        first (exhaustive);
      E-part, u0 < 1/4: E's exhaustive relative error eta on [0, 1] and
        (1 - e^-(u0+D)) / (1 - e^-u0) > (1+eta)/(1-eta);
      E-part, u0 >= 1/4: E = RN(1 - e) follows the e-part.
    The tail never exceeds 1/2 (the branches meet in order at z = 0) and
    its smallest value over [0, 9] is the one at the clamp a = 9."""
    L = _scan_lib()
    L.polya_E_scan.restype = ctypes.c_double
    d, th, aB = 2.0 ** -11, 2.0001 * 2.0 ** -24, 4e-4
    ua, ub = POLYA_C * aB * aB * (1 + th), POLYA_C * d * d * (1 - th)
    out = (ctypes.c_double * 3)()
    L.polya_exp_scan(ctypes.c_uint32(_fbits(51.6)), ctypes.c_double(ua), ctypes.c_double(ub), out)
    eps, min_a, max_b = out[0], out[1], out[2]
    assert eps <= 2.0 ** -23
    assert max_b <= min_a
    a0 = np.linspace(aB, 9.0, 200_001)
    a1 = a0 + d
    D = POLYA_C * (2 * a0 * d + d * d) - POLYA_C * (a0 * a0 + a1 * a1) * th
    assert np.all(np.exp(-D) * (1 + eps) / (1 - eps) < 1.0)
    eta = L.polya_E_scan(ctypes.c_uint32(_fbits(1.0)))
    assert eta <= 2.0 ** -22
    a0 = np.linspace(1e-6, 1.05 * math.sqrt(0.25 / POLYA_C), 200_001)
    a1 = a0 + d
    u0 = POLYA_C * a0 * a0 * (1 + th)
    D = POLYA_C * (2 * a0 * d + d * d) - POLYA_C * (a0 * a0 + a1 * a1) * th
    assert np.all(-np.expm1(-(u0 + D)) / -np.expm1(-u0) > (1 + eta) / (1 - eta))
    rng = (ctypes.c_double * 2)()
    L.tail_range_scan(ctypes.c_uint32(_fbits(9.0)), ctypes.c_int(2), rng)
    assert rng[0] <= 0.5
    assert rng[1] == float(orc.phi(np.float32([-9.0]), 2)[0]) > 0.0


# ------------------------------------------------------- binary64 reference

def test_reference_tail_against_libm_erfc(orc):
    rng = np.random.default_rng(7)
    a = np.concatenate([np.linspace(0.0, 37.0, 400_001), rng.uniform(0, 37, 100_000),
                        rng.uniform(2.8, 2.86, 50_000)])  # around the series / CF switch
    q = orc.ref_batch(a, "tail")
    ref = np.array([0.5 * math.erfc(x / math.sqrt(2.0)) for x in a])
    assert (np.abs(q - ref) / ref).max() <= 1e-12


def test_reference_exp_against_numpy(orc):
    g = np.concatenate([np.linspace(-686.0, 0.0, 500_001),
                        np.random.default_rng(8).uniform(-686, 0, 100_000)])
    e = orc.ref_batch(g, "exp")
    ref = np.exp(g)
    assert (np.abs(e - ref) / ref).max() <= 2.0 ** -52


def test_reference_phi_symmetry_and_center(orc):
    z = np.random.default_rng(9).uniform(-37, 37, 100_000)
    p, m = orc.ref_batch(z, "phi"), orc.ref_batch(-z, "phi")
    assert np.abs(p + m - 1.0).max() <= 2.0 ** -52
    assert orc.ref_batch(np.array([0.0, -0.0]), "phi").tolist() == [0.5, 0.5]


def test_reference_step_monotonicity():
    """Phi's tail has hazard phi(a)/Q(a) >= sqrt(2/pi) on a >= 0 (the Mills
    ratio bound, equality at 0), so across a z step of at least
    d = 2^-10 (1 - 2^-50) the true tail drops by a factor <= exp(-0.797 d);
    a relative error below 1e-12 cannot undo that, and 1 - Q, fma with
    w >= 0, min and floor are monotone. The reference coder therefore keeps
    every frequency >= 1."""
    h, d, E = math.sqrt(2.0 / math.pi), 2.0 ** -10 * (1 - 2.0 ** -50), 1e-12
    a = np.linspace(0.0, 37.0, 100_001)
    mills = np.exp(-a * a / 2) / math.sqrt(2 * math.pi) / (0.5 * np.array(
        [math.erfc(x / math.sqrt(2)) for x in a]))
    assert mills.min() >= h * (1 - 1e-9)
    assert math.exp(-h * d) * (1 + E) / (1 - E) < 1.0


def test_k1_reference_equals_textbook_bins(orc):
    """K = 1 with the reference CDF: the column is exactly
    j + floor(Phi((b_j - mu)/sigma) (M - N)) (Phi from libm's erfc) wherever
    Phi (M - N) is not within 1e-9 of a positive integer."""
    rng = np.random.default_rng(32)
    n, lo, hi, P = 2000, -100, 100, 16
    w, mu, sig = synth.random_params(rng, n, 1)
    w[:] = 1.0
    c = orc.cdf_table(orc.make_cfg(1, lo, hi, P, 1, 3), w, mu, sig).astype(np.int64)
    N, M = hi - lo + 1, 1 << P
    j = np.arange(1, N)
    b = (lo + j - 0.5)[None, :]
    s = np.clip(sig[0].astype(np.float64), 2.0 ** -10, 2.0 ** 10)[:, None]
    z = (b - mu[0].astype(np.float64)[:, None]) / s
    F = 0.5 * np.vectorize(math.erfc)(-z / math.sqrt(2.0))
    x = F * (M - N)
    ref = j[None, :] + np.floor(x)
    # the floor is decided unless x is within 1e-9 of a positive integer
    safe = (np.abs(x - np.round(x)) > 1e-9) | (x < 0.5)
    assert np.all((c[:, 1:-1] == ref)[safe])
    assert safe.mean() > 0.6          # the rest is mostly the saturated upper tail
    assert np.abs(c[:, 1:-1] - ref).max() <= 1


@pytest.mark.parametrize("kind", [2, 3])
def test_table_invariants_new_kinds(orc, kind):
    rng = np.random.default_rng(23 + kind)
    for K, lo, hi, P in [(3, -128, 127, 16), (5, -511, 511, 16), (2, -3, 4, 5), (8, -20, 20, 12)]:
        w, mu, sig = synth.random_params(rng, 600, K)
        wa, mua, siga = synth.adversarial_params(rng, 600, K)
        w, mu, sig = (np.ascontiguousarray(np.concatenate(x, axis=1))
                      for x in ((w, wa), (mu, mua), (sig, siga)))
        c = orc.cdf_table(orc.make_cfg(K, lo, hi, P, 1, kind), w, mu, sig).astype(np.int64)
        assert np.all(c[:, 0] == 0) and np.all(c[:, -1] == (1 << P))
        f = np.diff(c, axis=1)
        assert f.min() >= 1
        assert np.all(f.sum(axis=1) == (1 << P))


@pytest.mark.parametrize("kind", [2, 3])
def test_round_trip_new_kinds(orc, kind):
    cfgd = synth.CONFIGS["c1"]
    lat = synth.make_latents(cfgd)[0]
    n = 6000
    sym = np.ascontiguousarray(lat.symbols[:n])
    w, mu, sg = (np.ascontiguousarray(x[:, :n]) for x in (lat.weights, lat.means, lat.scales))
    cfg = orc.make_cfg(cfgd.K, cfgd.lo, cfgd.hi, 16, 64, kind)
    st, bs, off = orc.encode(cfg, sym, w, mu, sg)
    assert st == orc.OK
    st, out = orc.decode(cfg, bs, off, w, mu, sg)
    assert st == orc.OK and np.array_equal(out, sym)


# ------------------------------------------------------ raw-output mapping

def _raw_params(rng, n, K):
    logits = rng.normal(0.0, 3.0, size=(K, n)).astype(np.float32)
    logits[:, :50] = rng.uniform(-120, 120, size=(K, 50)).astype(np.float32)  # wide spreads
    log_s = rng.normal(0.5, 2.0, size=(K, n)).astype(np.float32)
    log_s[:, :20] = rng.uniform(-100, 100, size=(K, 20)).astype(np.float32)   # clamp region
    return logits, log_s


@pytest.mark.parametrize("K", [1, 2, 3, 5, 8])
def test_params_from_raw_against_binary64(orc, K):
    rng = np.random.default_rng(60 + K)
    logits, log_s = _raw_params(rng, 20_000, K)
    w, sg = orc.params_from_raw(logits, log_s)
    # the difference to the largest logit is taken in binary32, as specified
    d = np.maximum((logits - logits.max(axis=0)).astype(np.float64), -40.5)
    e = np.exp(d)
    w64 = e / e.sum(axis=0)
    assert (np.abs(w - w64) / w64).max() <= 2.0 ** -21
    assert np.abs(w.astype(np.float64).sum(axis=0) - 1.0).max() <= K * 2.0 ** -22
    s64 = np.maximum(np.exp(np.clip(log_s.astype(np.float64), -7, 7)), float(np.float32(0.11)))
    assert (np.abs(sg - s64) / s64).max() <= 2.0 ** -23
    assert sg.min() >= np.float32(0.11)
    if K == 1:
        assert np.all(w == 1.0)


def test_params_from_raw_edge_values(orc):
    l = np.array([[0.0, 0.0, 50.0], [-100.0, 0.0, -50.0]], np.float32)
    t = np.array([[-100.0, 0.0, 100.0], [7.0, -7.0, 1e30]], np.float32)
    w, sg = orc.params_from_raw(l, t)
    assert w[0, 1] == 0.5 and w[1, 1] == 0.5
    assert 0.0 < w[1, 0] < 1e-17 and w[1, 2] > 0.0    # difference clamped at -40.5
    assert sg[0, 0] == np.float32(0.11) and sg[1, 1] == np.float32(0.11)
    assert sg[0, 2] == sg[1, 0] == sg[1, 2] == orc.exp(np.float32([7.0]))[0]
    assert sg[0, 1] == 1.0


@pytest.mark.parametrize("kind", [0, 1, 2, 3])
def test_raw_encode_equals_plain_encode_of_mapped(orc, kind):
    rng = np.random.default_rng(70 + kind)
    K, lo, hi, n, S = 3, -40, 40, 4000, 32
    logits, log_s = _raw_params(rng, n, K)
    mu = rng.normal(0, 6, size=(K, n)).astype(np.float32)
    sym = np.clip(np.rint(rng.normal(0, 8, n)), lo, hi).astype(np.int32)
    w, sg = orc.params_from_raw(logits, log_s)
    plain = orc.make_cfg(K, lo, hi, 16, S, kind, 0)
    raw = orc.make_cfg(K, lo, hi, 16, S, kind, 1)
    st_p, bs_p, off_p = orc.encode(plain, sym, w, mu, sg)
    st_r, bs_r, off_r = orc.encode(raw, sym, logits, mu, log_s)
    assert st_p == st_r == orc.OK
    assert np.array_equal(off_p, off_r) and np.array_equal(bs_p, bs_r)
    st, out = orc.decode(raw, bs_r, off_r, logits, mu, log_s)
    assert st == orc.OK and np.array_equal(out, sym)
