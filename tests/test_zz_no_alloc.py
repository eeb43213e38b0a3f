"""GPU test of the allocation-free encode (gmm_encode_noalloc), called
through the C ABI: its offsets and bitstream equal gmm_encode's word for
word on two calls in a row, the second with a smaller input (the static
workspace keeps the first call's contents), in the synchronous and the
asynchronous (device status) form; an input needing more than the static
workspace gives GMM_E2BIG before any launch."""
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


def _inputs(seed, n, K, lo, hi):
    rng = np.random.default_rng(seed)
    w, mu, sig = synth.random_params(rng, n, K)
    sym = np.clip(np.rint(rng.normal(0, 7, size=n)), lo, hi).astype(np.int32)
    return [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (sym, w, mu, sig)]


def test_noalloc_equals_gmm_encode_twice_second_smaller(api):
    K, lo, hi = 3, -255, 255
    for seed, n, S in [(1, 2_000_003, 16384), (2, 50_001, 256), (3, 0, 5)]:
        sym, w, mu, sig = _inputs(seed, n, K, lo, hi)
        cfg = api.make_cfg(K, lo, hi, 16, S)
        cap = api.max_words(n, S)
        ref_bs = torch.zeros(max(cap, 1), dtype=torch.int16, device="cuda")
        ref_off = torch.zeros(S + 1, dtype=torch.int64, device="cuda")
        assert api.encode_into(cfg, sym, w, mu, sig, ref_bs, ref_off) == api.OK
        for asynchronous in (False, True):
            bs = torch.full((max(cap, 1),), -1, dtype=torch.int16, device="cuda")
            off = torch.full((S + 1,), -1, dtype=torch.int64, device="cuda")
            status = torch.full((1,), -9, dtype=torch.int32, device="cuda") if asynchronous else None
            r = api.encode_noalloc_into(cfg, sym, w, mu, sig, bs, off, status=status)
            assert r == api.OK, (n, asynchronous, r)
            torch.cuda.synchronize()
            if asynchronous:
                assert int(status.item()) == api.OK
            assert torch.equal(off, ref_off), (n, asynchronous)
            total = int(ref_off[-1].item())
            assert torch.equal(bs[:total], ref_bs[:total]), (n, asynchronous)
        print(f"gmm_encode_noalloc: n={n} S={S} {int(ref_off[-1].item())} words, equal to gmm_encode")


def test_noalloc_status_codes(api):
    K, lo, hi = 3, -128, 127
    sym, w, mu, sig = _inputs(4, 4000, K, lo, hi)
    cfg = api.make_cfg(K, lo, hi, 16, 64)
    bs = torch.zeros(api.max_words(4000, 64), dtype=torch.int16, device="cuda")
    off = torch.zeros(65, dtype=torch.int64, device="cuda")
    bad = sym.clone()
    bad[17] = hi + 1
    assert api.encode_noalloc_into(cfg, bad, w, mu, sig, bs, off) == api.ERANGE
    small = torch.zeros(10, dtype=torch.int16, device="cuda")
    assert api.encode_noalloc_into(cfg, sym, w, mu, sig, small, off) == api.ENOSPC
    assert api.encode_noalloc_into(cfg, sym, w, mu, sig, bs, off) == api.OK
    # a workspace beyond the static array: rejected on the host (a symbols
    # tensor of the claimed length is not needed: nothing is launched)
    big_n = (64 << 20) // 4
    cfg_big = api.make_cfg(K, lo, hi, 16, 1024)
    assert api.workspace_bytes(cfg_big, big_n, 0) > (64 << 20)
    lib = api.lib()
    r = lib.gmm_encode_noalloc(api.ctypes.byref(cfg_big), big_n, api._dev(sym, torch.int32, "s"),
                               api._dev(w, torch.float32, "w"), api._dev(mu, torch.float32, "m"),
                               api._dev(sig, torch.float32, "g"),
                               api._dev(bs, torch.int16, "b"), bs.numel(),
                               api._dev(off, torch.int64, "o"), None, api._stream())
    assert r == api.E2BIG
    assert "static workspace" in api.status_str(api.E2BIG)
