"""GPU parity of the Gaussian-CDF kinds of the paper's Table II comparison
(Polya, binary64 reference) and of raw network outputs as parameters
(param_kind 1, the fused mapping), bit-exact against the oracle.

Tables, inverse CDF, bitstreams, offsets and decoded symbols must equal the
oracle's on the same seeded inputs (ragged sizes, several workgroups, both
decode shapes the comparison kinds are built for); the mapping kernel must
equal the oracle's mapping; a raw-output encode must equal the plain encode
of the mapped parameters, also inside a batched plan.
"""
import numpy as np
import pytest

from paper_2509_18815_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    from paper_2509_18815_amd import api as a
    a.lib()
    assert torch.cuda.is_available()
    return a


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def u16(t):
    return t.cpu().numpy().view(np.uint16)


def mixed_params(rng, n, K):
    w, mu, sig = synth.random_params(rng, n, K)
    wa, ma, sa = synth.adversarial_params(rng, n, K)
    return tuple(np.ascontiguousarray(np.concatenate(x, axis=1))
                 for x in ((w, wa), (mu, ma), (sig, sa)))


@pytest.mark.parametrize("kind", [2, 3])
@pytest.mark.parametrize("K,lo,hi,P", [(1, -8, 7, 8), (3, -128, 127, 16), (5, -511, 511, 16),
                                       (8, -30, 33, 12), (2, 0, 1, 2)])
def test_cdf_table_bit_exact(api, orc, K, lo, hi, P, kind):
    rng = np.random.default_rng(11 * K + hi + kind)
    w, mu, sig = mixed_params(rng, 400, K)
    ref = orc.cdf_table(orc.make_cfg(K, lo, hi, P, 1, kind), w, mu, sig)
    got = api.cdf_table(api.make_cfg(K, lo, hi, P, 1, kind), dev(w), dev(mu), dev(sig))
    assert np.array_equal(got.cpu().numpy().view(np.uint32), ref)


@pytest.mark.parametrize("kind", [2, 3])
def test_inverse_cdf_bit_exact(api, orc, kind):
    rng = np.random.default_rng(88 + kind)
    for K, lo, hi, P in [(3, -255, 255, 16), (5, -511, 511, 16), (1, -3, 3, 5)]:
        n = 3000
        w, mu, sig = synth.random_params(rng, n, K)
        slot = rng.integers(0, 1 << P, size=n).astype(np.uint32)
        ref = orc.inverse(orc.make_cfg(K, lo, hi, P, 1, kind), w, mu, sig, slot)
        got = api.inverse_cdf(api.make_cfg(K, lo, hi, P, 1, kind), dev(w), dev(mu), dev(sig),
                              dev(slot.view(np.int32)))
        assert np.array_equal(got.cpu().numpy(), ref)


CASES = [  # (n, S, K, lo, hi, P)
    (0, 1, 3, -128, 127, 16),
    (1, 1, 1, -4, 3, 8),
    (1000, 7, 3, -128, 127, 16),
    (4099, 256, 3, -255, 255, 16),
    (20000, 257, 8, -64, 63, 14),
    (12345, 1000, 5, -511, 511, 16),
]


@pytest.mark.parametrize("kind", [2, 3])
@pytest.mark.parametrize("n,S,K,lo,hi,P", CASES)
def test_encode_decode_bit_exact(api, orc, n, S, K, lo, hi, P, kind):
    rng = np.random.default_rng(n + S + K + 100 * kind)
    w, mu, sig = synth.random_params(rng, n, K)
    sym = np.clip(np.rint(rng.normal(0, 8, size=n)), lo, hi).astype(np.int32)
    if n > 10:
        sym[:3] = [lo, hi, 0]
    st, obs, ooff = orc.encode(orc.make_cfg(K, lo, hi, P, S, kind), sym, w, mu, sig)
    assert st == orc.OK
    dsym, dw, dm, ds = dev(sym), dev(w), dev(mu), dev(sig)
    bs, off = api.encode(dsym, dw, dm, ds, lo, hi, P, S, kind)
    assert np.array_equal(off.cpu().numpy(), ooff)
    assert np.array_equal(u16(bs), obs)
    cfg = api.make_cfg(K, lo, hi, P, S, kind)
    try:
        for lanes in (1, 16, 0):      # both built decode shapes, then automatic
            api.set_decode_lanes(lanes)
            dec = torch.full((max(n, 1),), 7777, dtype=torch.int32, device="cuda")[:n]
            bsd = bs if bs.numel() else torch.zeros(1, dtype=torch.int16, device="cuda")
            assert api.decode_into(cfg, bsd, off, dw, dm, ds, dec,
                                   total_words=bs.numel()) == api.OK
            assert np.array_equal(dec.cpu().numpy(), sym), lanes
    finally:
        api.set_decode_lanes(0)


def test_comparison_kinds_rejected_where_not_built(api):
    n, S = 100, 4
    dw = torch.ones((1, n), device="cuda")
    dsym = torch.zeros(n, dtype=torch.int32, device="cuda")
    with pytest.raises(api.GmmError) as e:
        api.Plan(1, -4, 3, 8, [n], [S], op=0, autotune=False, cdf_kind=2)
    assert e.value.status == api.EINVAL
    idx = torch.arange(n, dtype=torch.int32, device="cuda")
    bs = torch.zeros(n + 2 * S, dtype=torch.int16, device="cuda")
    off = torch.zeros(S + 1, dtype=torch.int64, device="cuda")
    st = api.encode_subset_into(api.make_cfg(1, -4, 3, 8, S, 3), idx, dsym, dw, dw, dw, bs, off)
    assert st == api.EINVAL


# ------------------------------------------------------------ raw outputs

@pytest.mark.parametrize("K", [1, 2, 3, 5, 8])
def test_params_from_raw_kernel_bit_exact(api, orc, K):
    rng = np.random.default_rng(500 + K)
    logits, _, log_s = synth.raw_params(rng, 70_001, K)
    rw, rs = orc.params_from_raw(logits, log_s)
    gw, gs = api.params_from_raw(dev(logits), dev(log_s))
    assert np.array_equal(gw.cpu().numpy().view(np.uint32), rw.view(np.uint32))
    assert np.array_equal(gs.cpu().numpy().view(np.uint32), rs.view(np.uint32))


@pytest.mark.parametrize("kind", [0, 1, 2, 3])
def test_raw_outputs_encode_decode_bit_exact(api, orc, kind):
    rng = np.random.default_rng(600 + kind)
    K, lo, hi, P, n, S = 3, -255, 255, 16, 30_011, 256
    logits, mu, log_s = synth.raw_params(rng, n, K)
    sym = np.clip(np.rint(rng.normal(0, 6, size=n)), lo, hi).astype(np.int32)
    st, obs, ooff = orc.encode(orc.make_cfg(K, lo, hi, P, S, kind, 1), sym, logits, mu, log_s)
    assert st == orc.OK
    dl, dm, dt, dsym = dev(logits), dev(mu), dev(log_s), dev(sym)
    bs, off = api.encode(dsym, dl, dm, dt, lo, hi, P, S, kind, param_kind=1)
    assert np.array_equal(off.cpu().numpy(), ooff)
    assert np.array_equal(u16(bs), obs)
    # the fused mapping equals the separate mapping pass followed by a plain encode
    gw, gs = api.params_from_raw(dl, dt)
    bs2, off2 = api.encode(dsym, gw, dm, gs, lo, hi, P, S, kind)
    assert torch.equal(off2, off) and torch.equal(bs2, bs)
    dec = api.decode(bs, off, dl, dm, dt, lo, hi, P, S, kind, param_kind=1)
    assert np.array_equal(dec.cpu().numpy(), sym)


def test_raw_outputs_in_batched_plan(api):
    K, lo, hi, P = 3, -128, 127, 16
    rng = np.random.default_rng(700)
    shapes = [(0, 1), (37, 8), (5000, 64), (40000, 512), (123, 300)]
    lats = []
    for n, S in shapes:
        logits, mu, log_s = synth.raw_params(rng, n, K)
        sym = np.clip(np.rint(rng.normal(0, 7, size=n)), lo, hi).astype(np.int32)
        lats.append((n, S, dev(sym), dev(logits), dev(mu), dev(log_s), sym))
    ref = [api.encode(d_sym, d_l, d_m, d_t, lo, hi, P, S, 0, param_kind=1)
           for n, S, d_sym, d_l, d_m, d_t, _ in lats]
    ns, Ss = [L[0] for L in lats], [L[1] for L in lats]
    pe = api.Plan(K, lo, hi, P, ns, Ss, op=0, autotune=False, param_kind=1)
    io = []
    for n, S, d_sym, d_l, d_m, d_t, _ in lats:
        cap = n + 2 * S
        io.append({"symbols": d_sym, "weights": d_l, "means": d_m, "scales": d_t,
                   "bitstream": torch.zeros(max(cap, 1), dtype=torch.int16, device="cuda"),
                   "words": cap, "offsets": torch.zeros(S + 1, dtype=torch.int64,
                                                        device="cuda")})
    assert pe.run(io) == api.OK
    for e, (rbs, roff) in zip(io, ref):
        assert torch.equal(e["offsets"], roff)
        total = int(roff[-1].item())
        assert torch.equal(e["bitstream"][:total], rbs)
    pd = api.Plan(K, lo, hi, P, ns, Ss, op=1, autotune=False, param_kind=1)
    dio = []
    for (n, S, d_sym, d_l, d_m, d_t, _), e in zip(lats, io):
        dio.append({"weights": d_l, "means": d_m, "scales": d_t, "bitstream": e["bitstream"],
                    "words": int(e["offsets"][-1].item()), "offsets": e["offsets"],
                    "decoded": torch.full((max(n, 1),), 9999, dtype=torch.int32,
                                          device="cuda")[:n]})
    assert pd.run(dio) == api.OK
    for d, L in zip(dio, lats):
        assert np.array_equal(d["decoded"].cpu().numpy(), L[6])
    pe.close()
    pd.close()


def test_raw_outputs_with_bracket_rejected(api):
    from paper_2509_18815_amd import train
    K, lo, hi, P, n, S = 3, -255, 255, 16, 1000, 64
    D = 3 * K + 1
    br = api.Bracket(K, train.init_params(D, 1), np.zeros(D), np.ones(D), 0.0, 1.0)
    dw = torch.ones((K, n), device="cuda")
    bs = torch.zeros(2 * S, dtype=torch.int16, device="cuda")
    off = torch.arange(0, 2 * S + 1, 2, dtype=torch.int64, device="cuda")
    sym = torch.empty(n, dtype=torch.int32, device="cuda")
    st = api.decode_into(api.make_cfg(K, lo, hi, P, S, 0, 1), bs, off, dw, dw, dw, sym,
                         bracket=br)
    assert st == api.EINVAL
    br.close()
