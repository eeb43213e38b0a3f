"""The decoder's candidate search uses two handbook approximations (not part
of the coding contract: a wrong constant would only make candidates fail
more often, never change a decoded symbol). This pins the constants as
typed in the kernel source against the normal distribution itself:

- A&S 26.2.16, Q(x) = Z(x)(a1 t + a2 t^2 + a3 t^3), t = 1/(1 + p x):
  the handbook bounds the error by 1e-5; its printed constants, evaluated
  in binary64, reach 1.15e-5, so the check here is against 1.2e-5;
- A&S 26.2.23, the upper quantile x_p = t - (c0 + c1 t + c2 t^2) /
  (1 + d1 t + d2 t^2 + d3 t^3), t = sqrt(-2 ln p): |error| < 4.5e-4 for
  0 < p <= 1/2;
- kappa = sqrt(log2(e)/2), so that exp(-z^2/2) = exp2(-(kappa z)^2).
"""
import math
import os
import re

import numpy as np
from scipy.special import ndtr, ndtri

SRC = os.path.join(os.path.dirname(__file__), "..", "paper_2509_18815_amd", "csrc",
                   "gmm_stream.h")


def _consts():
    text = open(SRC).read()
    out = {}
    for name, val in re.findall(r"\b(k(?:A16|Q23)\w+|kKappa)\s*=\s*(-?[0-9.]+(?:e-?\d+)?)f", text):
        out[name] = float(val)
    return out


def test_constants_present():
    c = _consts()
    for k in ("kA16P", "kA16A1", "kA16A2", "kA16A3", "kQ23C0", "kQ23C1", "kQ23C2", "kQ23D1",
              "kQ23D2", "kQ23D3", "kKappa"):
        assert k in c, k


def test_as_26_2_16_tail_within_bound():
    c = _consts()
    x = np.linspace(0.0, 12.0, 200001)
    t = 1.0 / (1.0 + c["kA16P"] * x)
    z = np.exp(-x * x / 2) / math.sqrt(2 * math.pi)
    q = z * t * (c["kA16A1"] + t * (c["kA16A2"] + t * c["kA16A3"]))
    err = np.max(np.abs(q - ndtr(-x)))
    assert err < 1.2e-5, err


def test_as_26_2_23_quantile_within_bound():
    c = _consts()
    p = np.concatenate([np.logspace(-30, -1, 20001), np.linspace(0.1, 0.5, 20001)])
    t = np.sqrt(-2.0 * np.log(p))
    num = c["kQ23C0"] + t * (c["kQ23C1"] + t * c["kQ23C2"])
    den = 1.0 + t * (c["kQ23D1"] + t * (c["kQ23D2"] + t * c["kQ23D3"]))
    xp = t - num / den
    err = np.max(np.abs(xp + ndtri(p)))
    assert err < 4.5e-4, err


def test_kappa_scaling():
    c = _consts()
    assert abs(c["kKappa"] - math.sqrt(math.log2(math.e) / 2)) < 1e-12
    z = np.linspace(-10, 10, 1001)
    assert np.allclose(np.exp2(-(c["kKappa"] * z) ** 2), np.exp(-z * z / 2), rtol=1e-12,
                       atol=0)
