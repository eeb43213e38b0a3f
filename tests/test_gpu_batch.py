"""GPU parity of batched plans (persistent kernels + hipGraph + autotuner).

Each latent's bitstream, offsets and decoded symbols from a plan must equal
the single-latent entry points' (which are themselves bit-exact with the
oracle) and, for small latents, the oracle's directly — for the tuned shape
and for every candidate launch shape, across graph replays interleaved with
eager work.
"""
import numpy as np
import pytest

from paper_2509_18815_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

K, LO, HI, P = 3, -128, 127, 16
SHAPES = [(0, 1), (1, 1), (37, 8), (255, 64), (256, 256), (257, 300), (5000, 64), (40000, 512),
          (123457, 1000), (70000, 64)]


@pytest.fixture(scope="module")
def api():
    from paper_2509_18815_amd import api as a
    a.lib()
    return a


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def make_batch(seed, shapes):
    rng = np.random.default_rng(seed)
    lats = []
    for n, S in shapes:
        w, mu, sig = synth.random_params(rng, n, K)
        sym = np.clip(np.rint(rng.normal(0, 7, size=n)), LO, HI).astype(np.int32)
        lats.append({"n": n, "S": S, "sym": sym, "w": w, "mu": mu, "sig": sig,
                     "d_sym": dev(sym), "d_w": dev(w), "d_mu": dev(mu), "d_sig": dev(sig)})
    return lats


def enc_io(lats):
    io = []
    for L in lats:
        cap = L["n"] + 2 * L["S"]
        io.append({"symbols": L["d_sym"], "weights": L["d_w"], "means": L["d_mu"],
                   "scales": L["d_sig"],
                   "bitstream": torch.zeros(max(cap, 1), dtype=torch.int16, device="cuda"),
                   "words": cap,
                   "offsets": torch.zeros(L["S"] + 1, dtype=torch.int64, device="cuda")})
    return io


def dec_io(lats, enc):
    io = []
    for L, e in zip(lats, enc):
        total = int(e["offsets"][-1].item())
        io.append({"weights": L["d_w"], "means": L["d_mu"], "scales": L["d_sig"],
                   "bitstream": e["bitstream"], "words": total, "offsets": e["offsets"],
                   "decoded": torch.full((max(L["n"], 1),), 99999, dtype=torch.int32,
                                         device="cuda")[: L["n"]]})
    return io


def reference(api, lats):
    ref = []
    for L in lats:
        bs, off = api.encode(L["d_sym"], L["d_w"], L["d_mu"], L["d_sig"], LO, HI, P, L["S"])
        ref.append((bs.cpu().numpy().view(np.uint16).copy(), off.cpu().numpy()))
    return ref


def check_enc(io, ref):
    for b, (e, (rbs, roff)) in enumerate(zip(io, ref)):
        off = e["offsets"].cpu().numpy()
        assert np.array_equal(off, roff), b
        got = e["bitstream"].cpu().numpy().view(np.uint16)[: off[-1]]
        assert np.array_equal(got, rbs), b


def check_dec(io, lats):
    for b, (d, L) in enumerate(zip(io, lats)):
        assert np.array_equal(d["decoded"].cpu().numpy(), L["sym"]), b


def test_plan_matches_single_calls_and_oracle(api, orc):
    lats = make_batch(1, SHAPES)
    ref = reference(api, lats)
    for L, (rbs, roff) in zip(lats, ref):
        if L["n"] <= 5000:
            st, obs, ooff = orc.encode(orc.make_cfg(K, LO, HI, P, L["S"]), L["sym"], L["w"],
                                       L["mu"], L["sig"])
            assert st == 0 and np.array_equal(obs, rbs) and np.array_equal(ooff, roff)
    ns, Ss = [L["n"] for L in lats], [L["S"] for L in lats]
    pe = api.Plan(K, LO, HI, P, ns, Ss, op=0, autotune=True)
    io = enc_io(lats)
    assert pe.run(io) == api.OK
    check_enc(io, ref)
    info = pe.info()
    assert info["tuned"] and info["graph_captured"] and info["candidates"] > 1
    pd = api.Plan(K, LO, HI, P, ns, Ss, op=1, autotune=True)
    dio = dec_io(lats, io)
    assert pd.run(dio) == api.OK
    check_dec(dio, lats)
    pe.close()
    pd.close()


def test_every_candidate_and_graph_replays(api):
    lats = make_batch(2, SHAPES)
    ref = reference(api, lats)
    ns, Ss = [L["n"] for L in lats], [L["S"] for L in lats]
    pe = api.Plan(K, LO, HI, P, ns, Ss, op=0, autotune=False)
    io = enc_io(lats)
    for cand in pe.candidates():
        pe.set_config(*cand)
        for rep in range(3):
            for e in io:                      # eager work between replays
                e["bitstream"].zero_()
                e["offsets"].fill_(-1)
            torch.cuda.synchronize()
            status = torch.full((len(lats),), -7, dtype=torch.int32, device="cuda")
            assert pe.run(io, status=status) == api.OK
            torch.cuda.synchronize()
            assert status.cpu().tolist() == [0] * len(lats)
            check_enc(io, ref)
    pd = api.Plan(K, LO, HI, P, ns, Ss, op=1, autotune=False)
    dio = dec_io(lats, io)
    for cand in pd.candidates():
        pd.set_config(*cand)
        for rep in range(2):
            for d in dio:
                d["decoded"].fill_(12345)
            torch.cuda.synchronize()
            assert pd.run(dio) == api.OK, cand
            check_dec(dio, lats)
    pe.close()
    pd.close()


def test_plan_status_per_latent(api):
    lats = make_batch(3, SHAPES[2:7])
    bad = 2
    lats[bad]["sym"][5] = HI + 1
    lats[bad]["d_sym"] = dev(lats[bad]["sym"])
    ns, Ss = [L["n"] for L in lats], [L["S"] for L in lats]
    pe = api.Plan(K, LO, HI, P, ns, Ss, op=0, autotune=False)
    io = enc_io(lats)
    status = torch.zeros(len(lats), dtype=torch.int32, device="cuda")
    assert pe.run(io, status=status) == api.OK
    torch.cuda.synchronize()
    st = status.cpu().tolist()
    assert st[bad] == api.ERANGE and all(s == 0 for i, s in enumerate(st) if i != bad)
    assert pe.run(io) == api.ERANGE
    # decode with one corrupted segment in latent 1
    lats[bad]["sym"][5] = HI
    lats[bad]["d_sym"] = dev(lats[bad]["sym"])
    io = enc_io(lats)
    assert pe.run(io) == api.OK
    dio = dec_io(lats, io)
    w = dio[1]["bitstream"]
    w[int(dio[1]["offsets"][1].item()) + 2] ^= 0x0101
    pd = api.Plan(K, LO, HI, P, ns, Ss, op=1, autotune=False)
    status = torch.zeros(len(lats), dtype=torch.int32, device="cuda")
    assert pd.run(dio, status=status) == api.OK
    torch.cuda.synchronize()
    st = status.cpu().tolist()
    assert st[1] == api.ECORRUPT and all(s == 0 for i, s in enumerate(st) if i != 1)
    pe.close()
    pd.close()


def test_two_streams_per_lane_decode_corruption(api):
    """Decode with two streams per lane (every such candidate): clean
    latents decode exactly; a flipped word marks its latent corrupt and
    leaves every other stream exact; broken offsets send the lane to the
    one-stream path, which writes the smallest symbol for the broken streams
    and decodes the lane's other stream exactly. Latent 1 has 64 streams
    (lanes with one stream), latents 2 and 5 pair streams s and s + 64."""
    lats = make_batch(5, SHAPES[2:8])
    ns, Ss = [L["n"] for L in lats], [L["S"] for L in lats]
    pe = api.Plan(K, LO, HI, P, ns, Ss, op=0, autotune=False)
    io = enc_io(lats)
    assert pe.run(io) == api.OK
    pd = api.Plan(K, LO, HI, P, ns, Ss, op=1, autotune=False)
    cands = [c for c in pd.candidates() if c[1] == 2]
    assert cands, "no two-streams-per-lane decode candidate"

    def stream_elems(b, s):
        return np.arange(s, lats[b]["n"], lats[b]["S"])

    for cand in cands:
        pd.set_config(*cand)
        assert pd.info()["streams_per_lane"] == 2
        # clean
        dio = dec_io(lats, io)
        status = torch.full((len(lats),), -7, dtype=torch.int32, device="cuda")
        assert pd.run(dio, status=status) == api.OK, cand
        torch.cuda.synchronize()
        assert status.cpu().tolist() == [0] * len(lats), cand
        check_dec(dio, lats)
        # a flipped renormalisation word in latent 1 stream 1 and latent 5 stream 70
        dio = dec_io(lats, io)
        saved = []
        for b, s in ((1, 1), (5, 70)):
            bsw = dio[b]["bitstream"]
            pos = int(dio[b]["offsets"][s].item()) + 2
            saved.append((bsw, pos, bsw[pos].item()))
            bsw[pos] ^= 0x0101
        status = torch.zeros(len(lats), dtype=torch.int32, device="cuda")
        assert pd.run(dio, status=status) == api.OK, cand
        torch.cuda.synchronize()
        st = status.cpu().tolist()
        assert st[1] == api.ECORRUPT and st[5] == api.ECORRUPT, (cand, st)
        assert all(v == 0 for i, v in enumerate(st) if i not in (1, 5)), (cand, st)
        for b, d in enumerate(dio):
            got = d["decoded"].cpu().numpy()
            keep = np.ones(lats[b]["n"], dtype=bool)
            for bb, s in ((1, 1), (5, 70)):
                if bb == b:
                    keep[stream_elems(b, s)] = False
            assert np.array_equal(got[keep], lats[b]["sym"][keep]), (cand, b)
        for bsw, pos, v in saved:
            bsw[pos] = v
        # broken offsets in latent 2: streams 2 and 3 (paired with 66 and 67)
        dio = dec_io(lats, io)
        bad_off = dio[2]["offsets"].clone()
        bad_off[3] = -5
        dio[2]["offsets"] = bad_off
        status = torch.zeros(len(lats), dtype=torch.int32, device="cuda")
        assert pd.run(dio, status=status) == api.OK, cand
        torch.cuda.synchronize()
        st = status.cpu().tolist()
        assert st[2] == api.ECORRUPT and all(v == 0 for i, v in enumerate(st) if i != 2), st
        got = dio[2]["decoded"].cpu().numpy()
        broken = np.concatenate([stream_elems(2, 2), stream_elems(2, 3)])
        assert np.all(got[broken] == LO), cand
        keep = np.ones(lats[2]["n"], dtype=bool)
        keep[broken] = False
        assert np.array_equal(got[keep], lats[2]["sym"][keep]), cand
        for b in (0, 1, 3, 4, 5):
            assert np.array_equal(dio[b]["decoded"].cpu().numpy(), lats[b]["sym"]), (cand, b)
    pe.close()
    pd.close()


def test_batch_of_64_uneven_latents(api, orc):
    """The 64-latent batch (192 x H x W, H, W ~ U{8..128}), autotuned: round
    trip of every latent, three latents equal to the single-latent calls,
    and sampled streams of two latents re-encoded by the oracle."""
    cfgd = synth.CONFIGS["c3"]
    lats = synth.make_latents(cfgd, backend="torch", device="cuda")
    ns, Ss = [L.n for L in lats], [L.streams for L in lats]
    pe = api.Plan(cfgd.K, cfgd.lo, cfgd.hi, cfgd.precision, ns, Ss, op=0, autotune=True)
    pd = api.Plan(cfgd.K, cfgd.lo, cfgd.hi, cfgd.precision, ns, Ss, op=1, autotune=True)
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
    assert pd.run(dio) == api.OK
    for L, d in zip(lats, dio):
        assert torch.equal(d["decoded"], L.symbols)
    for b in (0, 17, 63):
        L = lats[b]
        bs, off = api.encode(L.symbols, L.weights, L.means, L.scales, cfgd.lo, cfgd.hi,
                             cfgd.precision, L.streams)
        assert torch.equal(off, io[b]["offsets"])
        assert torch.equal(bs, io[b]["bitstream"][: bs.numel()])
    ocfg1 = orc.make_cfg(cfgd.K, cfgd.lo, cfgd.hi, cfgd.precision, 1)
    rng = np.random.default_rng(4)
    for b in (5, 40):
        L = lats[b]
        hs = [x.cpu().numpy() for x in (L.symbols, L.weights, L.means, L.scales)]
        off = io[b]["offsets"].cpu().numpy()
        bsh = io[b]["bitstream"].cpu().numpy().view(np.uint16)
        for s in rng.choice(L.streams, 6, replace=False):
            idx = np.arange(s, L.n, L.streams)
            sub = [np.ascontiguousarray(x[..., idx]) for x in hs]
            st, obs, _ = orc.encode(ocfg1, *sub)
            assert st == 0 and np.array_equal(obs, bsh[off[s]:off[s + 1]])
    pe.close()
    pd.close()
