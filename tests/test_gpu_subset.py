"""Subset (two-pass Checkerboard) coding on the GPU: a pass over elements
idx equals the oracle's coding of the gathered sub-latent, decode fills
exactly symbols[idx], two passes reconstruct the whole latent, and invalid
indices give EINVAL without touching memory outside the buffers."""
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


@pytest.mark.parametrize("lanes", [0, 1, 16])
def test_checkerboard_two_pass_matches_oracle(api, orc, lanes):
    cfgd = synth.CONFIGS["c2a"]
    C, H, W = 24, 12, 10
    lat = synth.make_latents(cfgd, scale_hw=(C, H, W))[0]
    sym, w, mu, sg = lat.symbols, lat.weights, lat.means, lat.scales
    dsym, dw, dmu, dsg = (torch.from_numpy(x).cuda() for x in (sym, w, mu, sg))
    out = torch.full_like(dsym, -999999)
    api.set_decode_lanes(lanes)
    try:
        for anchor, S in ((True, 37), (False, 64)):
            idx = api.checkerboard_indices(C, H, W, anchor)
            ih = idx.cpu().numpy()
            cfg = api.make_cfg(cfgd.K, cfgd.lo, cfgd.hi, 16, S)
            bs = torch.empty(idx.numel() + 2 * S, dtype=torch.int16, device="cuda")
            off = torch.empty(S + 1, dtype=torch.int64, device="cuda")
            assert api.encode_subset_into(cfg, idx, dsym, dw, dmu, dsg, bs, off) == api.OK
            st, obs, ooff = orc.encode(orc.make_cfg(cfgd.K, cfgd.lo, cfgd.hi, 16, S), sym[ih],
                                       np.ascontiguousarray(w[:, ih]),
                                       np.ascontiguousarray(mu[:, ih]),
                                       np.ascontiguousarray(sg[:, ih]))
            assert st == 0 and np.array_equal(off.cpu().numpy(), ooff)
            got = bs.cpu().numpy().view(np.uint16)[: ooff[-1]]
            assert np.array_equal(got, obs)
            before = out.clone()
            assert api.decode_subset_into(cfg, idx, bs, off, dw, dmu, dsg, out,
                                          total_words=int(ooff[-1])) == api.OK
            changed = (out != before).cpu().numpy()
            mask = np.zeros(sym.size, bool)
            mask[ih] = True
            assert not changed[~mask].any()          # only the pass's elements written
            assert np.array_equal(out.cpu().numpy()[ih], sym[ih])
        assert torch.equal(out, dsym)                # both passes: the whole latent
    finally:
        api.set_decode_lanes(0)


def test_subset_invalid_index(api):
    rng = np.random.default_rng(3)
    n, K, S = 1000, 3, 16
    w, mu, sg = synth.random_params(rng, n, K)
    sym = rng.integers(-20, 20, size=n).astype(np.int32)
    d = [torch.from_numpy(x).cuda() for x in (sym, w, mu, sg)]
    idx = torch.arange(0, 500, dtype=torch.int32, device="cuda")
    idx[123] = n + 5
    cfg = api.make_cfg(K, -128, 127, 16, S)
    bs = torch.empty(500 + 2 * S, dtype=torch.int16, device="cuda")
    off = torch.empty(S + 1, dtype=torch.int64, device="cuda")
    assert api.encode_subset_into(cfg, idx, *d, bs, off) == api.EINVAL
    idx[123] = -1
    out = torch.zeros(n, dtype=torch.int32, device="cuda")
    assert api.decode_subset_into(cfg, idx, bs, off, d[1], d[2], d[3], out) == api.EINVAL
