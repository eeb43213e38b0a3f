"""GPU parity of batched plans in the coder setting of the 256-latent batch:
K = 5 mixture components, support [-511, 511] (N = 1023), P = 16.

- Small uneven latents (empty, one element, fewer elements than streams,
  ragged tails): for every tuner candidate, each latent's offsets and
  bitstream equal the oracle's word for word, and the plain and the
  learned-bracket decode plans (a briefly trained network, so that many
  symbols miss and take the fallback search) return the symbols.
- Full-size latents of that batch (320 x H x W, several million symbols
  each, the stream-count rule of the batch): autotuned plans, round trip
  through the plain and the bracket decode, and sampled streams of every
  latent re-encoded and decoded by the oracle one by one.
- Edge-of-range parameters with uniform symbols (K = 3, N = 256 and K = 5,
  N = 1023): every decode candidate returns the oracle-encoded symbols.
"""
import numpy as np
import pytest

from paper_2509_18815_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CFG = synth.CONFIGS["c5"]
K, LO, HI, P = CFG.K, CFG.lo, CFG.hi, CFG.precision
SHAPES = [(0, 1), (1, 1), (3, 64), (1023, 7), (4097, 64), (20000, 128), (33333, 256)]


@pytest.fixture(scope="module")
def api():
    from paper_2509_18815_amd import api as a
    a.lib()
    return a


@pytest.fixture(scope="module")
def brief_model(api):
    """A K = 5 bracket network trained for one short epoch: it hits often
    enough to exercise the bracket path and misses often enough to exercise
    the fallback search."""
    from paper_2509_18815_amd import train
    return train.train_bracket(K, LO, HI, P, n_train=131072, n_eval=16384, epochs=1,
                               batch=4096, s_logit=CFG.s_logit, s_mu=CFG.s_mu,
                               sigma_max=CFG.sigma_max, seed=31)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def small_batch(seed):
    rng = np.random.default_rng(seed)
    lats = []
    for n, S in SHAPES:
        w, mu, sig = synth.random_params(rng, n, K, CFG.s_logit, CFG.s_mu, CFG.sigma_max)
        sym = np.clip(np.rint(rng.normal(0, 12, size=n)), LO, HI).astype(np.int32)
        if n > 4:
            sym[:2] = [LO, HI]
        lats.append({"n": n, "S": S, "sym": sym, "w": w, "mu": mu, "sig": sig,
                     "d": [dev(x) for x in (sym, w, mu, sig)]})
    return lats


def enc_io(lats):
    io = []
    for L in lats:
        cap = L["n"] + 2 * L["S"]
        io.append({"symbols": L["d"][0], "weights": L["d"][1], "means": L["d"][2],
                   "scales": L["d"][3],
                   "bitstream": torch.zeros(max(cap, 1), dtype=torch.int16, device="cuda"),
                   "words": cap,
                   "offsets": torch.zeros(L["S"] + 1, dtype=torch.int64, device="cuda")})
    return io


def dec_io(lats, io):
    out = []
    for L, e in zip(lats, io):
        out.append({"weights": L["d"][1], "means": L["d"][2], "scales": L["d"][3],
                    "bitstream": e["bitstream"], "words": int(e["offsets"][-1].item()),
                    "offsets": e["offsets"],
                    "decoded": torch.full((max(L["n"], 1),), 99999, dtype=torch.int32,
                                          device="cuda")[: L["n"]]})
    return out


def test_k5_plans_every_candidate_equal_oracle(api, orc, brief_model):
    lats = small_batch(51)
    ref = []
    for L in lats:
        st, obs, ooff = orc.encode(orc.make_cfg(K, LO, HI, P, L["S"]), L["sym"], L["w"],
                                   L["mu"], L["sig"])
        assert st == orc.OK
        ref.append((obs, ooff))
    ns, Ss = [L["n"] for L in lats], [L["S"] for L in lats]
    pe = api.Plan(K, LO, HI, P, ns, Ss, op=0, autotune=False)
    io = enc_io(lats)
    cands = pe.candidates()
    assert len(cands) > 1
    for cand in cands:
        pe.set_config(*cand)
        for e in io:
            e["bitstream"].zero_()
            e["offsets"].fill_(-1)
        assert pe.run(io) == api.OK, cand
        for b, (e, (obs, ooff)) in enumerate(zip(io, ref)):
            off = e["offsets"].cpu().numpy()
            assert np.array_equal(off, ooff), (cand, b)
            got = e["bitstream"].cpu().numpy().view(np.uint16)[: off[-1]]
            assert np.array_equal(got, obs), (cand, b)
    dio = dec_io(lats, io)
    pd = api.Plan(K, LO, HI, P, ns, Ss, op=1, autotune=False)
    for cand in pd.candidates():
        pd.set_config(*cand)
        for d in dio:
            d["decoded"].fill_(12345)
        assert pd.run(dio) == api.OK, cand
        for b, (d, L) in enumerate(zip(dio, lats)):
            assert np.array_equal(d["decoded"].cpu().numpy(), L["sym"]), (cand, b)
    br = brief_model.load()
    stats = torch.zeros(4, dtype=torch.int64, device="cuda")
    pb = api.Plan(K, LO, HI, P, ns, Ss, op=1, autotune=False)
    pb.set_bracket(br, stats)
    for cand in pb.candidates():
        pb.set_config(*cand)
        for d in dio:
            d["decoded"].fill_(-777)
        assert pb.run(dio) == api.OK, cand
        for b, (d, L) in enumerate(zip(dio, lats)):
            assert np.array_equal(d["decoded"].cpu().numpy(), L["sym"]), (cand, b)
    torch.cuda.synchronize()
    hits, misses, _, _ = stats.cpu().tolist()
    print(f"K=5 plans: {len(cands)} encode candidates, brief bracket hit rate "
          f"{hits / max(hits + misses, 1):.3f}")
    assert misses > 0 and hits > 0
    for p in (pe, pd, pb):
        p.close()
    br.close()


def test_k5_full_size_latents_sampled_streams(api, orc, brief_model):
    """The first three latents of the 256-latent batch at their real sizes
    (320x129x91, 320x98x123, 320x85x109: 10.6 M symbols), in autotuned
    plans: round trip through the plain and the bracket decode plans, and
    12 sampled streams per latent (the first, the last and ten random ones)
    equal to the oracle's encoding of that stream."""
    lats = synth.make_latents(CFG, backend="torch", device="cuda", limit=3)
    ns, Ss = [L.n for L in lats], [L.streams for L in lats]
    assert ns == [3756480, 3857280, 2964800]
    pe = api.Plan(K, LO, HI, P, ns, Ss, op=0, autotune=True)
    io = []
    for L in lats:
        cap = L.n + 2 * L.streams
        io.append({"symbols": L.symbols, "weights": L.weights, "means": L.means,
                   "scales": L.scales,
                   "bitstream": torch.empty(cap, dtype=torch.int16, device="cuda"),
                   "words": cap,
                   "offsets": torch.empty(L.streams + 1, dtype=torch.int64, device="cuda")})
    assert pe.run(io) == api.OK
    dio = []
    for L, e in zip(lats, io):
        dio.append({"weights": L.weights, "means": L.means, "scales": L.scales,
                    "bitstream": e["bitstream"], "words": int(e["offsets"][-1].item()),
                    "offsets": e["offsets"],
                    "decoded": torch.empty(L.n, dtype=torch.int32, device="cuda")})
    pd = api.Plan(K, LO, HI, P, ns, Ss, op=1, autotune=True)
    assert pd.run(dio) == api.OK
    for L, d in zip(lats, dio):
        assert torch.equal(d["decoded"], L.symbols)
    br = brief_model.load()
    pb = api.Plan(K, LO, HI, P, ns, Ss, op=1, autotune=True)
    pb.set_bracket(br, None)
    for d in dio:
        d["decoded"].fill_(-1)
    assert pb.run(dio) == api.OK
    for L, d in zip(lats, dio):
        assert torch.equal(d["decoded"], L.symbols)
    ocfg1 = orc.make_cfg(K, LO, HI, P, 1)
    rng = np.random.default_rng(57)
    for b, L in enumerate(lats):
        hs = [x.cpu().numpy() for x in (L.symbols, L.weights, L.means, L.scales)]
        off = io[b]["offsets"].cpu().numpy()
        bsh = io[b]["bitstream"].cpu().numpy().view(np.uint16)
        S = L.streams
        for s in np.concatenate([[0, S - 1], rng.choice(S, 10, replace=False)]):
            idx = np.arange(s, L.n, S)
            sub = [np.ascontiguousarray(x[..., idx]) for x in hs]
            st, obs, _ = orc.encode(ocfg1, *sub)
            seg = bsh[off[s]:off[s + 1]]
            assert st == orc.OK and np.array_equal(obs, seg), (b, int(s))
            st, odec = orc.decode(ocfg1, seg, np.array([0, seg.size], np.int64), *sub[1:])
            assert st == orc.OK and np.array_equal(odec, sub[0]), (b, int(s))
    for p in (pe, pd, pb):
        p.close()
    br.close()


@pytest.mark.parametrize("k,lo,hi", [(3, -128, 127), (5, -511, 511)])
def test_plans_adversarial_params_every_candidate(api, orc, k, lo, hi):
    """Batched decode plans on edge-of-range parameters (tiny and huge
    scales, zero and denormal weights, far means, means on boundaries) with
    symbols spread uniformly over the support, so that one-lane candidates
    from the bracketed search fail often and take the exact fallback: every
    decode candidate returns the oracle-encoded symbols."""
    rng = np.random.default_rng(hi - lo + k)
    lats = []
    for n, S in [(1, 1), (777, 64), (5003, 128), (12000, 256)]:
        w, mu, sig = synth.adversarial_params(rng, n, k)
        sym = rng.integers(lo, hi + 1, size=n).astype(np.int32)
        st, obs, ooff = orc.encode(orc.make_cfg(k, lo, hi, P, S), sym, w, mu, sig)
        assert st == orc.OK
        lats.append({"n": n, "S": S, "sym": sym, "d": [dev(x) for x in (w, mu, sig)],
                     "bs": dev(obs.view(np.int16)), "off": dev(ooff)})
    dio = [{"weights": L["d"][0], "means": L["d"][1], "scales": L["d"][2],
            "bitstream": L["bs"], "words": int(L["off"][-1].item()), "offsets": L["off"],
            "decoded": torch.empty(L["n"], dtype=torch.int32, device="cuda")} for L in lats]
    pd = api.Plan(k, lo, hi, P, [L["n"] for L in lats], [L["S"] for L in lats], op=1,
                  autotune=False)
    try:
        for cand in pd.candidates():
            pd.set_config(*cand)
            for d in dio:
                d["decoded"].fill_(-1)
            assert pd.run(dio) == api.OK, cand
            for b, (d, L) in enumerate(zip(dio, lats)):
                assert np.array_equal(d["decoded"].cpu().numpy(), L["sym"]), (cand, b)
    finally:
        pd.close()
