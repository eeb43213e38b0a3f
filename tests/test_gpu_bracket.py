"""GPU tests of the learned search bracket and its training kernels.

- MLP loss/gradients from the GPU kernels against the FP64 oracle, element
  by element (float32 activations; bfloat16 first-layer activations against
  the oracle rounding them the same way);
- forward, features and one Adam step against their definitions;
- training on exact tuples lowers the loss and reaches a useful hit rate;
- the decoder's matrix-core inference agrees with the float32 forward;
- decode with the bracket (trained or not) is bit-identical to plain decode
  and to the oracle, including corrupted streams; hit rate and the speed
  gain over plain decode are reported.
"""
import math

import numpy as np
import pytest

from paper_2509_18815_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    from paper_2509_18815_amd import api as a
    a.lib()
    return a


@pytest.fixture(scope="module")
def trained(api):
    from paper_2509_18815_amd import train
    return train.train_bracket(3, -255, 255, 16, n_train=1_048_576, n_eval=131072, epochs=4,
                               batch=4096, lr=3e-3, seed=6)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def rand_net(rng, D, orc, scale=0.3):
    return (rng.normal(0, scale, size=orc.mlp_num_params(D))).astype(np.float32)


BLOCKS = ("W1", "b1", "W2", "b2", "w3", "b3")


def _block_of(i, D, H=64):
    edges = np.cumsum([H * D, H, H * H, H, H, 1])
    b = int(np.searchsorted(edges, i, side="right"))
    return BLOCKS[b], i - (edges[b - 1] if b else 0)


def _check_elementwise(got, ref, rtol, atol_rms, D, what):
    """|got - ref| <= rtol |ref| + atol_rms rms(ref) for every element; prints
    the worst element (by its share of the allowance) and its block."""
    allow = rtol * np.abs(ref) + atol_rms * np.sqrt(np.mean(ref * ref))
    ratio = np.abs(got - ref) / allow
    i = int(np.argmax(ratio))
    blk, k = _block_of(i, D)
    print(f"{what} D={D}: worst element {i} ({blk}[{k}]): gpu {got[i]:.9g} oracle {ref[i]:.9g}, "
          f"{ratio[i]:.3f} of the allowance")
    for b, (lo, hi) in zip(BLOCKS, zip(np.r_[0, np.cumsum([64 * D, 64, 4096, 64, 64])],
                                       np.cumsum([64 * D, 64, 4096, 64, 64, 1]))):
        assert ratio[lo:hi].max() <= 1.0, (what, b, int(lo + np.argmax(ratio[lo:hi])))


@pytest.mark.parametrize("D", [10, 16])
def test_mlp_gradients_match_oracle(api, orc, D):
    """The training kernels' loss and gradients against the FP64 oracle,
    element by element: with float32 activations every gradient element is
    within 1e-4 |g| + 1e-6 rms(g) of the oracle's (binary32 accumulation of
    3,000 samples, whose residuals can cancel); with bfloat16 first-layer
    activations against the oracle that rounds them the same way, within
    2e-3 |g| + 2e-5 rms(g) (an activation whose binary32 value lies within
    a binary32 rounding of a bfloat16 tie may round the other way than the
    binary64 one: about one in 40,000 activations, each moving its sample's
    terms by 2^-8 relative)."""
    rng = np.random.default_rng(D)
    n = 3000
    p = rand_net(rng, D, orc)
    X = rng.normal(size=(n, D)).astype(np.float32)
    y = rng.normal(scale=2.0, size=n).astype(np.float32)
    P = p.size
    for round_act, rtol, atol in ((False, 1e-4, 1e-6), (True, 5e-4, 5e-6)):
        loss, g = orc.mlp_loss_grad(p.astype(np.float64), X.astype(np.float64),
                                    y.astype(np.float64), 1.0, round_act=round_act)
        out = api.mlp_loss_grad(dev(X), dev(y), dev(p), 1.0,
                                round_act=round_act).cpu().numpy().astype(np.float64)
        assert abs(out[P] - loss) <= (1e-5 if not round_act else 1e-4) * abs(loss)
        _check_elementwise(out[:P], g, rtol, atol, D,
                           "bf16 activations" if round_act else "float32")
        fwd = api.mlp_forward(dev(X), dev(p), round_act=round_act).cpu().numpy()
        ref = orc.mlp_forward(p.astype(np.float64), X.astype(np.float64), round_act=round_act)
        assert np.abs(fwd - ref).max() <= 1e-4 * max(1.0, np.abs(ref).max())


def test_mlp_gradients_bit_reproducible(api):
    rng = np.random.default_rng(3)
    X = dev(rng.normal(size=(70000, 10)).astype(np.float32))
    y = dev(rng.normal(size=70000).astype(np.float32))
    p = dev(rng.normal(0, 0.3, size=api.mlp_num_params(10)).astype(np.float32))
    a = api.mlp_loss_grad(X, y, p, 1.0)
    b = api.mlp_loss_grad(X, y, p, 1.0)
    assert torch.equal(a, b)


def test_adam_step_matches_definition(api):
    rng = np.random.default_rng(4)
    P = 5313
    p = rng.normal(size=P).astype(np.float32)
    g = rng.normal(size=P).astype(np.float32)
    m = rng.normal(scale=0.1, size=P).astype(np.float32)
    v = rng.uniform(0, 0.1, size=P).astype(np.float32)
    dp, dm, dv, dsh = dev(p), dev(m), dev(v), torch.zeros(P, device="cuda")
    api.mlp_adam(dp, dev(g), dm, dv, 1e-3, 7, 0.5, dsh)
    gs = g.astype(np.float64) * 0.5
    m1 = 0.9 * m + 0.1 * gs
    v1 = 0.999 * v + 0.001 * gs * gs
    ref = p - 1e-3 * (m1 / (1 - 0.9 ** 7)) / (np.sqrt(v1 / (1 - 0.999 ** 7)) + 1e-8)
    assert np.allclose(dp.cpu().numpy(), ref, rtol=2e-6, atol=2e-7)
    sh = dsh.cpu().numpy()
    assert np.array_equal(sh, torch.from_numpy(dp.cpu().numpy()).bfloat16().float().numpy())


def test_features_match_definition(api):
    rng = np.random.default_rng(5)
    for K in (3, 5):
        n = 4000
        w, mu, sg = synth.adversarial_params(rng, n, K)
        slot = rng.integers(0, 1 << 16, size=n).astype(np.uint32)
        X = api.mlp_features(K, dev(w), dev(mu), dev(sg), dev(slot.view(np.int32)),
                             16).cpu().numpy()
        wf = np.where(w < 2.0 ** -60, 0.0, w)
        ls = np.log(np.clip(sg.astype(np.float64), 2.0 ** -10, 2.0 ** 10))
        ref = np.concatenate([wf.T, mu.T, ls.T, (slot / 65536.0)[:, None]], axis=1)
        assert np.allclose(X, ref, rtol=1e-6, atol=1e-6)


def test_training_lowers_loss_and_hits(trained):
    h = [r for r in trained.history if "epoch" in r]
    assert h[-1]["loss_per_sample"] < h[0]["loss_per_sample"]
    assert h[-1]["hit_rate"] > 0.95
    print("bracket training:", h[-1], trained.history[-1])


def test_matrix_core_inference_matches_forward(api, trained):
    br = trained.load()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(123)
    from paper_2509_18815_amd import train
    w, mu, sg, slot, j = train.make_tuples(3, -255, 255, 16, 50000, gen, "cuda")
    pred = br.predict(16, w, mu, sg, slot)
    X = api.mlp_features(3, w, mu, sg, slot, 16, dev(trained.in_mean),
                         dev(1.0 / trained.in_std), round_bf16=True)
    shadow = torch.from_numpy(trained.params).cuda().bfloat16().float()
    ref = api.mlp_forward(X, shadow) * trained.out_std + trained.out_mean
    diff = (pred - ref).abs()
    assert float(diff.max()) <= 0.05 * trained.out_std, float(diff.max())
    same = (torch.round(pred) == torch.round(ref)).float().mean().item()
    assert same > 0.98
    br.close()


def _encode(api, n_shape, S, K, lo, hi, seed, cfgd):
    lat = synth.make_latents(cfgd, backend="torch", device="cuda", scale_hw=n_shape)[0]
    bs, off = api.encode(lat.symbols, lat.weights, lat.means, lat.scales, lo, hi, 16, S)
    return lat, bs, off


def test_bracket_decode_bit_exact_and_gain(api, orc, trained):
    cfgd = synth.CONFIGS["c4"]
    br = trained.load()
    lat, bs, off = _encode(api, (320, 48, 64), 16384, 3, cfgd.lo, cfgd.hi, 5, cfgd)
    cfg = api.make_cfg(3, cfgd.lo, cfgd.hi, 16, 16384)
    dec = torch.empty(lat.n, dtype=torch.int32, device="cuda")
    stats = torch.zeros(4, dtype=torch.int64, device="cuda")
    assert api.decode_into(cfg, bs, off, lat.weights, lat.means, lat.scales, dec, bracket=br,
                           stats=stats) == api.OK
    assert torch.equal(dec, lat.symbols)
    hits, misses, all_hit, steps = stats.cpu().tolist()
    assert hits + misses == lat.n
    # untrained (random) network: every bracket may miss, output unchanged
    rng = np.random.default_rng(9)
    bad = api.Bracket(3, rand_net(rng, 10, orc, 1.0), trained.in_mean, trained.in_std, 0.0, 50.0)
    dec2 = torch.empty_like(dec)
    assert api.decode_into(cfg, bs, off, lat.weights, lat.means, lat.scales, dec2,
                           bracket=bad) == api.OK
    assert torch.equal(dec2, lat.symbols)
    # speed against the plain search on the same bitstream
    st = torch.cuda.current_stream()

    def timed(fn, reps=5):
        fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        for _ in range(reps):
            fn()
        b.record(st)
        b.synchronize()
        return a.elapsed_time(b) / reps
    st_d = torch.zeros(1, dtype=torch.int32, device="cuda")
    t_plain = timed(lambda: api.decode_into(cfg, bs, off, lat.weights, lat.means, lat.scales,
                                            dec2, status=st_d))
    t_br = timed(lambda: api.decode_into(cfg, bs, off, lat.weights, lat.means, lat.scales,
                                         dec2, bracket=br, status=st_d))
    print(f"bracket hit rate {hits / lat.n:.4f}, all-lane wavefront steps {all_hit / steps:.3f}, "
          f"plain {t_plain:.3f} ms, bracket {t_br:.3f} ms, gain {t_plain / t_br:.3f}x")
    br.close()
    bad.close()


@pytest.fixture
def lanes(api, request):
    """Lanes per stream for the call (0: the library's choice); reset after."""
    api.set_decode_lanes(request.param)
    yield request.param
    api.set_decode_lanes(0)


@pytest.mark.parametrize("lanes", [0, 1, 8, 16], indirect=True)
def test_bracket_decode_matches_oracle_on_corruption(api, orc, trained, lanes):
    """333 streams: the group form (16 lanes per stream, partial last
    wavefront) by default and with 16 lanes, with 8 lanes per stream with
    8, the one-lane form with 1."""
    br = trained.load()
    rng = np.random.default_rng(11)
    n, K, S = 20000, 3, 333
    w, mu, sig = synth.random_params(rng, n, K)
    sym = np.clip(np.rint(rng.normal(0, 6, size=n)), -255, 255).astype(np.int32)
    ocfg = orc.make_cfg(K, -255, 255, 16, S)
    st, obs, ooff = orc.encode(ocfg, sym, w, mu, sig)
    cfg = api.make_cfg(K, -255, 255, 16, S)
    dec = torch.empty(n, dtype=torch.int32, device="cuda")
    flipped = obs.copy()
    flipped[ooff[7] + 3] ^= 0x0010
    badoff = ooff.copy()
    badoff[9] = badoff[8] + 1
    for bsx, offx in [(obs, ooff), (flipped, ooff), (obs, badoff)]:
        ost, osym = orc.decode(ocfg, bsx, offx, w, mu, sig)
        gst = api.decode_into(cfg, dev(bsx.view(np.int16)), dev(offx), dev(w), dev(mu),
                              dev(sig), dec, bracket=br)
        assert gst == ost
        assert np.array_equal(dec.cpu().numpy(), osym)
    br.close()


@pytest.mark.parametrize("lanes", [0, 8, 16], indirect=True)
def test_group_bracket_decode_kodak_latent(api, orc, trained, lanes):
    """The 320x48x32 latent at 4,096 streams with a bracket decodes by lane
    groups (8 lanes per stream by default, as the plain decode, or 16): the
    group form of the bracket (matrix-core inference for eight or four
    streams per wavefront, one window round of 8 or 16 boundaries) is
    bit-identical to the
    plain decode; a trained model hits on nearly every symbol (which also
    checks the 16x16x32 operand layout: a wrong layout predicts noise); an
    untrained one misses and takes the fallback search everywhere."""
    cfgd = synth.CONFIGS["c2a"]
    lat = synth.make_latents(cfgd, backend="torch", device="cuda")[0]
    S = lat.streams
    assert S == 4096
    bs, off = api.encode(lat.symbols, lat.weights, lat.means, lat.scales, cfgd.lo, cfgd.hi, 16, S)
    cfg = api.make_cfg(3, cfgd.lo, cfgd.hi, 16, S)
    br = trained.load()
    dec = torch.empty(lat.n, dtype=torch.int32, device="cuda")
    stats = torch.zeros(4, dtype=torch.int64, device="cuda")
    assert api.decode_into(cfg, bs, off, lat.weights, lat.means, lat.scales, dec, bracket=br,
                           stats=stats) == api.OK
    assert torch.equal(dec, lat.symbols)
    hits, misses, all_hit, steps = stats.cpu().tolist()
    assert hits + misses == lat.n
    window = lanes or api.decode_lanes(cfg)  # boundaries per window round
    assert window in (8, 16)
    assert hits / lat.n > (0.97 if window == 16 else 0.93), hits / lat.n
    rng = np.random.default_rng(19)
    bad = api.Bracket(3, rand_net(rng, 10, orc, 1.0), trained.in_mean, trained.in_std, 0.0, 50.0)
    stats.zero_()
    dec.fill_(-9)
    assert api.decode_into(cfg, bs, off, lat.weights, lat.means, lat.scales, dec, bracket=bad,
                           stats=stats) == api.OK
    assert torch.equal(dec, lat.symbols)
    h2, m2, _, _ = stats.cpu().tolist()
    assert h2 + m2 == lat.n and m2 > 0
    st = torch.cuda.current_stream()

    def timed(fn, reps=10):
        fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        for _ in range(reps):
            fn()
        b.record(st)
        b.synchronize()
        return a.elapsed_time(b) / reps
    st_d = torch.zeros(1, dtype=torch.int32, device="cuda")
    t_plain = timed(lambda: api.decode_into(cfg, bs, off, lat.weights, lat.means, lat.scales,
                                            dec, status=st_d))
    t_br = timed(lambda: api.decode_into(cfg, bs, off, lat.weights, lat.means, lat.scales,
                                         dec, bracket=br, status=st_d))
    torch.cuda.synchronize()
    assert st_d.item() == 0 and torch.equal(dec, lat.symbols)
    print(f"group bracket (320x48x32, 4096 streams, lanes {lanes}): hit rate {hits / lat.n:.4f}, all-hit "
          f"wavefront steps {all_hit / steps:.3f}, untrained hit rate {h2 / lat.n:.3f}, "
          f"plain {t_plain:.4f} ms, bracket {t_br:.4f} ms, gain {t_plain / t_br:.3f}x")
    br.close()
    bad.close()


def _plan_io(lats, S_list, api, lo, hi):
    enc, dec = [], []
    for L, S in zip(lats, S_list):
        bs, off = api.encode(L.symbols, L.weights, L.means, L.scales, lo, hi, 16, S)
        enc.append((bs, off))
        dec.append({"weights": L.weights, "means": L.means, "scales": L.scales,
                    "bitstream": bs, "words": bs.numel(), "offsets": off,
                    "decoded": torch.empty(L.n, dtype=torch.int32, device="cuda")})
    return dec


def test_batched_bracket_every_candidate(api, trained):
    cfgd = synth.CONFIGS["c4"]
    shapes = [(320, 8, 8), (320, 16, 24), (320, 3, 5), (320, 32, 32), (320, 1, 7)]
    lats = [synth.make_latents(cfgd, backend="torch", device="cuda", scale_hw=sh)[0]
            for sh in shapes]
    Ss = [synth.streams_rule(L.n) for L in lats]
    dio = _plan_io(lats, Ss, api, cfgd.lo, cfgd.hi)
    br = trained.load()
    stats = torch.zeros(4, dtype=torch.int64, device="cuda")
    pd = api.Plan(3, cfgd.lo, cfgd.hi, 16, [L.n for L in lats], Ss, op=1, autotune=True)
    pd.set_bracket(br, stats)
    assert pd.run(dio) == api.OK
    for L, d in zip(lats, dio):
        assert torch.equal(d["decoded"], L.symbols)
    for cand in pd.candidates():
        assert cand[0] == 1
        pd.set_config(*cand)
        for d in dio:
            d["decoded"].fill_(7777)
        assert pd.run(dio) == api.OK
        for L, d in zip(lats, dio):
            assert torch.equal(d["decoded"], L.symbols)
    torch.cuda.synchronize()
    hits, misses, _, _ = stats.cpu().tolist()
    assert (hits + misses) % sum(L.n for L in lats) == 0
    pd.close()
    br.close()


@pytest.mark.parametrize("lanes", [0, 1], indirect=True)
def test_k5_bracket_and_cooperative_fallback(api, orc, lanes):
    """A briefly trained K = 5 model (many misses, so the fallback searches
    run: the one-lane form's cooperative fallback with every group size, the
    group form's 17-ary search) decodes bit-exactly, and matches the oracle
    on a small latent."""
    from paper_2509_18815_amd import train
    cfgd = synth.CONFIGS["c5"]
    model = train.train_bracket(5, cfgd.lo, cfgd.hi, 16, n_train=131072, n_eval=16384,
                                epochs=1, batch=4096, s_logit=1.5, s_mu=4.0, sigma_max=40.0)
    br = model.load()
    lat = synth.make_latents(cfgd, backend="torch", device="cuda", scale_hw=(320, 20, 30))[0]
    S = synth.streams_rule(lat.n)
    bs, off = api.encode(lat.symbols, lat.weights, lat.means, lat.scales, cfgd.lo, cfgd.hi, 16, S)
    cfg = api.make_cfg(5, cfgd.lo, cfgd.hi, 16, S)
    dec = torch.empty(lat.n, dtype=torch.int32, device="cuda")
    stats = torch.zeros(4, dtype=torch.int64, device="cuda")
    assert api.decode_into(cfg, bs, off, lat.weights, lat.means, lat.scales, dec, bracket=br,
                           stats=stats) == api.OK
    assert torch.equal(dec, lat.symbols)
    hits, misses, all_hit, steps = stats.cpu().tolist()
    assert misses > 0 and hits + misses == lat.n
    print(f"K=5 short-trained bracket: hit rate {hits / lat.n:.3f}, "
          f"all-hit steps {all_hit / max(steps, 1):.3f}")
    # small latent against the oracle
    rng = np.random.default_rng(12)
    n, S2 = 3000, 64
    w, mu, sig = synth.random_params(rng, n, 5, 1.5, 4.0, 40.0)
    sym = np.clip(np.rint(rng.normal(0, 9, size=n)), cfgd.lo, cfgd.hi).astype(np.int32)
    ocfg = orc.make_cfg(5, cfgd.lo, cfgd.hi, 16, S2)
    st, obs, ooff = orc.encode(ocfg, sym, w, mu, sig)
    d2 = torch.empty(n, dtype=torch.int32, device="cuda")
    assert api.decode_into(api.make_cfg(5, cfgd.lo, cfgd.hi, 16, S2), dev(obs.view(np.int16)),
                           dev(ooff), dev(w), dev(mu), dev(sig), d2, bracket=br) == api.OK
    assert np.array_equal(d2.cpu().numpy(), sym)
    br.close()
