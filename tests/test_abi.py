"""The C-ABI library loads and exports every entry point that
include/flashgmm.h declares (no compute call: runs without a GPU)."""
import ctypes
import os
import re

from conftest import ROOT


def declared_functions():
    text = open(os.path.join(ROOT, "include", "flashgmm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gmm_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_coder_calls():
    names = declared_functions()
    for must in ("gmm_encode", "gmm_decode", "gmm_workspace_bytes", "gmm_status_str"):
        assert must in names


def test_library_exports_every_declared_symbol():
    path = os.path.join(ROOT, "paper_2509_18815_amd", "libflashgmm.so")
    assert os.path.exists(path), "build the library first (__graft_entry__.build())"
    lib = ctypes.CDLL(path)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_host_side_queries_without_gpu():
    from paper_2509_18815_amd import api
    L = api.lib()
    assert L.gmm_encode_max_words(1000, 8) == 1016
    assert api.status_str(api.ENOSPC) == "bitstream capacity too small"
    cfg = api.make_cfg(3, -128, 127, 16, 256)
    assert api.workspace_bytes(cfg, 49152, 0) > 49152 * 4
    bad = api.make_cfg(3, -128, 127, 7, 256)   # N > M/2
    assert L.gmm_workspace_bytes(ctypes.byref(bad), 10, 0) == -1
    # launch settings are host state: checked without a GPU
    assert L.gmm_set_wave_priority(4) == api.EINVAL and L.gmm_set_wave_priority(-1) == api.EINVAL
    assert L.gmm_set_wave_priority(3) == api.OK and L.gmm_set_wave_priority(0) == api.OK


def test_automatic_decode_lanes_without_gpu():
    """The automatic lanes-per-stream choice of a plain decode: enough lanes
    for 65,536 (at most 32 per stream), then halved while the (lanes+1)-ary
    search needs no more rounds; an explicit choice is returned as set."""
    from paper_2509_18815_amd import api
    cases = [((3, -255, 255, 16, 65536, 0), 1),    # 4K latent: one lane per stream
             ((3, -255, 255, 16, 4096, 0), 8),     # 9-ary and 17-ary both take 3 rounds
             ((3, -128, 127, 16, 256, 0), 16),     # 17-ary and 33-ary both take 2 rounds
             ((3, -255, 255, 16, 256, 0), 32),     # 33-ary: 2 rounds, 17-ary: 3
             ((5, -511, 511, 16, 1, 0), 32),       # 1,023 symbols: 33-ary 2 rounds, 17-ary 3
             ((3, -4, 3, 16, 64, 0), 8),           # 8 symbols: one 9-ary round
             ((3, -255, 255, 16, 4096, 1), 8),     # logistic kind: same rule
             ((3, -255, 255, 16, 4096, 2), 16),    # comparison kinds build 1 and 16 lanes
             ((3, -255, 255, 16, 65536, 3), 1)]
    for args, want in cases:
        assert api.decode_lanes(api.make_cfg(*args)) == want, (args, want)
    api.set_decode_lanes(4)
    try:
        assert api.decode_lanes(api.make_cfg(3, -255, 255, 16, 4096)) == 4
    finally:
        api.set_decode_lanes(0)
    L = api.lib()
    bad = api.make_cfg(0, -128, 127, 16, 256)
    assert L.gmm_decode_lanes(ctypes.byref(bad)) == -api.EINVAL
