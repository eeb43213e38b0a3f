"""Host-side pieces of bench.py (no GPU): the one-core CPU baseline's
stream sample codes exactly the sampled streams of the latent (the oracle's
segments of those streams are unchanged), and the algorithmic flop counts
follow the per-evaluation cost."""
import numpy as np

import bench
from paper_2509_18815_amd import synth


def test_stream_sample_keeps_the_streams(orc):
    rng = np.random.default_rng(3)
    n, S, k, K, lo, hi = 6001, 64, 8, 3, -60, 60
    w, mu, sig = synth.random_params(rng, n, K)
    sym = np.clip(np.rint(rng.normal(0, 6, size=n)), lo, hi).astype(np.int32)
    st, bs, off = orc.encode(orc.make_cfg(K, lo, hi, 16, S), sym, w, mu, sig)
    assert st == orc.OK
    sub = bench._stream_sample(sym, w, mu, sig, S, k)
    assert sub[0].size == sum(len(range(s, n, S)) for s in range(k))
    st2, bs2, off2 = orc.encode(orc.make_cfg(K, lo, hi, 16, k), *sub)
    assert st2 == orc.OK
    for s in range(k):
        assert np.array_equal(bs2[off2[s]:off2[s + 1]], bs[off[s]:off[s + 1]]), s


def test_flop_counts():
    assert bench.flops_per_eval(3) == 118
    # 9 rounds for N = 511 plus the per-element set-up
    assert bench.decode_flops_per_symbol(3, 511) == 9 * 118 + 18 == 1080
    assert bench.encode_flops_per_symbol(3) == 2 * 118 + 18
