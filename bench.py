"""Throughput benchmark of the GMM rANS coder on one MI355X.

A step codes the paper-scale workload once: the Kodak-size latent
(320x48x32, 4,096 streams) and the 4K latent (320x135x240, 65,536 streams),
K = 3, support [-255, 255], P = 16 — each latent encoded, then decoded. The
two latents are independent, so their chains run on two HIP streams (both
at the default priority, each running its steps back to back): the
Kodak-size latent's latency-bound kernels fill issue slots that the 4K
latent's kernels leave free. Inputs are
seeded synthetic latents resident in HBM before timing starts; every timed
step's output is the bit-exact round trip (checked after timing).

value = symbols coded per second, each symbol encoded and decoded once per
step: (n_kodak + n_4k) * steps / elapsed. It is measured first in the
process; after the other forms the same warm-up and timed steps run again
(`repeat_after_forms`), when the GPU's clocks have settled under load.

Prints one JSON line (rank 0 only; the benchmark runs on one GPU).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# HBM3E peak and FP32 vector peak of one MI355X (AMD public figures).
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3
# Non-packed FP32 VALU issue rate: 256 CU x 4 SIMD x 16 lanes x 2.4 GHz.
VALU_ISSUE_PEAK = 256 * 4 * 16 * 2.4e9


def flops_per_eval(K: int) -> int:
    """Algorithmic binary32 flops of one A&S mixture CDF evaluation (fma =
    2): per component 38 (b - mu: 1, a = min(|d| r/9, 1): 2, u: 2, 1/u: 1,
    polynomial: 9, a^2: 1, split of the exponent: 5, degree-5 polynomial of
    the density: 10, 2^n scaling: 1, density times polynomial: 1, 1/2 - T
    floored at 0: 2, sign: 1, mixture fma: 2) plus 4 per evaluation
    (boundary, clamp, scale, floor)."""
    return 38 * K + 4


def decode_flops_per_symbol(K: int, N: int) -> int:
    """ceil(log2 N) evaluations plus the per-element setup, 6 per component
    (scale clamp: 2, reciprocal: 1, weight flush: 1, r/9: 1, half-weight
    sum: 1): the binary search's work. The one-lane decode's bracketed
    search executes less (two exact evaluations after approximate rounds),
    so rates from this figure are binary-search equivalent."""
    rounds = (N - 1).bit_length()
    return rounds * flops_per_eval(K) + 6 * K


def encode_flops_per_symbol(K: int) -> int:
    return 2 * flops_per_eval(K) + 6 * K


def form_roofline(K: int, N: int, enc_sym_s: float, dec_sym_s: float, bits: float) -> dict:
    """Algorithmic rates of a form: binary32 flops (the method's, per
    symbol) and HBM bytes (3K parameter floats and one int32 symbol per
    symbol, plus the bitstream) times the measured symbol rate, as
    fractions of the MI355X FP32 vector and HBM peaks."""
    byt = 12 * K + 4 + bits / 8

    def rates(sym_s, flops):
        return {"tflops": round(flops * sym_s / 1e12, 2),
                "frac_fp32": round(flops * sym_s / 1e12 / PEAK_FP32_TFLOPS, 4),
                "hbm_GBps": round(byt * sym_s / 1e9, 1),
                "frac_hbm": round(byt * sym_s / 1e9 / PEAK_HBM_GBS, 4)}
    return {"encode": rates(enc_sym_s, encode_flops_per_symbol(K)),
            "decode": rates(dec_sym_s, decode_flops_per_symbol(K, N))}


class Latent:
    def __init__(self, api, cfgd, lat, cdf_kind=0, param_kind=0, prio=0):
        import torch
        self.api, self.cfgd, self.lat = api, cfgd, lat
        self.prio = prio  # wavefront issue priority of this latent's calls
        self.n, self.S = lat.n, lat.streams
        self.cfg = api.make_cfg(cfgd.K, cfgd.lo, cfgd.hi, cfgd.precision, self.S, cdf_kind,
                                param_kind)
        dev = lat.symbols.device
        self.bs = torch.empty(api.max_words(self.n, self.S), dtype=torch.int16, device=dev)
        self.off = torch.empty(self.S + 1, dtype=torch.int64, device=dev)
        self.dec = torch.empty(self.n, dtype=torch.int32, device=dev)
        self.ws_enc = torch.empty(api.workspace_bytes(self.cfg, self.n, 0), dtype=torch.uint8,
                                  device=dev)
        self.ws_dec = torch.empty(api.workspace_bytes(self.cfg, self.n, 1), dtype=torch.uint8,
                                  device=dev)
        self.st = torch.zeros(2, dtype=torch.int32, device=dev)

    def encode(self):
        self.api.set_wave_priority(self.prio)
        r = self.api.encode_into(self.cfg, self.lat.symbols, self.lat.weights, self.lat.means,
                                 self.lat.scales, self.bs, self.off, ws=self.ws_enc,
                                 status=self.st[0:1])
        assert r == 0, r

    def decode(self):
        self.api.set_wave_priority(self.prio)
        r = self.api.decode_into(self.cfg, self.bs, self.off, self.lat.weights, self.lat.means,
                                 self.lat.scales, self.dec, ws=self.ws_dec, status=self.st[1:2])
        assert r == 0, r

    def verify(self):
        import torch
        assert self.st.tolist() == [0, 0], self.st.tolist()
        assert torch.equal(self.dec, self.lat.symbols), "round trip failed"


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(oracle, ocfg, sym, w, mu, sg, runs=3, progress=None):
    """Median over `runs` of the oracle's encode and decode wall times on one
    latent (round trip checked); returns (enc_s, dec_s, bitstream). With
    progress, a line per run goes to stderr (long legs)."""
    import numpy as np
    te, td = [], []
    bs = None
    for r in range(runs):
        t0 = time.perf_counter()
        st, bs, off = oracle.encode(ocfg, sym, w, mu, sg)
        t1 = time.perf_counter()
        if progress:
            print(f"{progress}: run {r} encode {t1 - t0:.1f} s", file=sys.stderr, flush=True)
        st2, dec = oracle.decode(ocfg, bs, off, w, mu, sg)
        t2 = time.perf_counter()
        assert st == 0 and st2 == 0 and np.array_equal(dec, sym)
        te.append(t1 - t0)
        td.append(t2 - t1)
        if progress:
            print(f"{progress}: run {r} decode {t2 - t1:.1f} s", file=sys.stderr, flush=True)
    med = lambda v: sorted(v)[len(v) // 2]  # noqa: E731
    return med(te), med(td), bs


def _stream_sample(sym, w, mu, sg, S, streams):
    """The first `streams` of the S streams of a latent as a latent of its
    own (elements s + p S, s < streams, in the same stream layout)."""
    import numpy as np
    n = sym.size
    idx = np.concatenate([np.arange(s, n, S) for s in range(streams)])
    # element s + p S of stream s becomes element s + p streams
    order = np.lexsort((idx % S, idx // S))
    idx = idx[order]
    return (np.ascontiguousarray(sym[idx]),) + tuple(np.ascontiguousarray(x[:, idx])
                                                     for x in (w, mu, sg))


def cpu_baseline(lat_host, cfgd):
    """The oracle (whole CDF column per element, table-lookup encode,
    linear-scan decode) on the host: on all cores, the whole 320x48x32
    latent, and on one core, its first 256 of 4,096 streams (a latent of
    30,720 symbols in the same layout); each the median of 3 runs of encode
    and of decode (about 15 s of CPU work in all)."""
    import oracle
    oracle.lib()
    sym, w, mu, sg, S = lat_host["sym"], lat_host["w"], lat_host["mu"], lat_host["sg"], lat_host["S"]
    ocfg = oracle.make_cfg(cfgd.K, cfgd.lo, cfgd.hi, cfgd.precision, S)
    import numpy as np
    cores = oracle.num_threads()
    te, td, bs = _oracle_rate(oracle, ocfg, sym, w, mu, sg)
    m = sym.size
    sub = _stream_sample(sym, w, mu, sg, S, 256)
    oracle.set_num_threads(1)
    try:
        te1, td1, _ = _oracle_rate(oracle, oracle.make_cfg(cfgd.K, cfgd.lo, cfgd.hi,
                                                           cfgd.precision, 256), *sub)
    finally:
        oracle.set_num_threads(cores)
    m1 = sub[0].size
    return {"value": m / (te + td), "unit": "symbols/s", "cores": cores, "kind": "oracle",
            "sample": f"whole 320x48x32 latent, {S} streams ({m} symbols encoded and decoded), "
                      "median of 3 runs",
            "encode_sym_s": m / te, "decode_sym_s": m / td,
            "one_core": {"value": m1 / (te1 + td1), "encode_sym_s": m1 / te1,
                         "decode_sym_s": m1 / td1,
                         "sample": "first 256 of the 4,096 streams of the 320x48x32 latent "
                                   f"({m1} symbols), median of 3 runs"},
            "cpu_model": _cpu_model(),
            "bitstream_equal_to_gpu": bool(np.array_equal(bs, lat_host.get("gpu_bs", bs)))}


def cpu_baseline_legs(dev) -> dict:
    """Longer oracle legs (bench.py --cpu-baseline-legs, minutes of CPU
    work): all cores, median of 3, on the whole 320x135x240 latent; on the
    first 7 latents of the 64-latent batch (11.6% of its symbols) and on the
    first 2 latents of the 256-latent K = 5 batch (1.5% of its symbols, one
    run: the oracle's column of 1,023 entries per element makes 10% of it
    hours of CPU work), each encoded and decoded."""
    import numpy as np
    import oracle
    from paper_2509_18815_amd import synth
    oracle.lib()
    cores = oracle.num_threads()
    out = {"cores": cores, "cpu_model": _cpu_model(), "kind": "oracle", "unit": "symbols/s"}
    legs = [("c2b", None, 3), ("c3", 7, 3), ("c5", 2, 1)]
    for name, limit, runs in legs:
        cfgd = synth.CONFIGS[name]
        lats = synth.make_latents(cfgd, backend="torch", device=dev, limit=limit)
        total = sum(c * h * wd for c, h, wd in synth.batch_shapes(cfgd))
        n_all, t_e, t_d = 0, 0.0, 0.0
        for L in lats:
            h = [x.cpu().numpy() for x in (L.symbols, L.weights, L.means, L.scales)]
            ocfg = oracle.make_cfg(cfgd.K, cfgd.lo, cfgd.hi, cfgd.precision, L.streams)
            te, td, _ = _oracle_rate(oracle, ocfg, *h, runs=runs,
                                     progress=f"oracle leg {name}, latent of {L.n} symbols")
            n_all += L.n
            t_e += te
            t_d += td
        out[name] = {"latents": len(lats), "symbols": n_all, "share_of_workload": n_all / total,
                     "runs": runs, "value": n_all / (t_e + t_d), "encode_sym_s": n_all / t_e,
                     "decode_sym_s": n_all / t_d}
    return out


def peak_probes(api, dev) -> dict:
    """Measured ceilings of this GPU beside the published peaks: the issue
    rate of independent binary32 fmas in the library's (non-packed) form, and
    a 1 GiB device copy (bytes read + written per second)."""
    import torch
    stream = torch.cuda.current_stream()
    lanes = 256 * 4 * 64 * 8          # 8 wavefronts per SIMD of 256 CUs
    iters = 4096
    out = torch.empty(lanes, dtype=torch.float32, device=dev)
    t_fma = time_events(lambda: api.fma_probe(out, iters), 5, stream)
    src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    t_cp = time_events(lambda: api.copy_probe(src, dst), 5, stream)
    torch.cuda.synchronize()
    assert bool(torch.equal(src[:1024], dst[:1024]))
    del src, dst
    fma_s = lanes * iters * 8 / t_fma
    return {"fp32_fma_lane_per_s": float("%.4g" % fma_s),
            "fp32_nonpacked_TFLOPs": round(2 * fma_s / 1e12, 2),
            "hbm_copy_GBps": round(2 * (1 << 30) / t_cp / 1e9, 1)}


def _prof_tables(root: str):
    """Per (kernel, grid): kernel-trace durations (root/trace) and counter
    means (root/fetch, root/write, root/valu: FETCH_SIZE, WRITE_SIZE,
    SQ_INSTS_VALU, SQ_WAVES, ...), and the FETCH/WRITE scales that make the
    largest runtime copy (the 1 GiB calibration copy) read 1 GiB each way."""
    import collections
    import csv
    import glob

    def rows(sub, suffix):
        out = []
        for f in glob.glob(os.path.join(root, sub, f"*{suffix}")):
            out += list(csv.DictReader(open(f)))
        return out

    def short(name):
        name = name.replace("void ", "").replace("(anonymous namespace)::", "")
        return name.split("(")[0] if "(" in name else name

    dur = collections.defaultdict(list)
    for r in rows("trace", "kernel_trace.csv"):
        dur[(short(r["Kernel_Name"]), int(r.get("Grid_Size") or r["Grid_Size_X"]))].append(
            (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    ctr = collections.defaultdict(list)
    for sub in ("fetch", "write", "valu"):
        for r in rows(sub, "counter_collection.csv"):
            ctr[(short(r["Kernel_Name"]), int(r["Grid_Size"]), r["Counter_Name"])].append(
                float(r["Counter_Value"]))
    mean = lambda v: sum(v) / len(v) if v else float("nan")  # noqa: E731
    cal = [k for k in ctr if k[0].startswith("__amd_rocclr_copyBuffer") and k[2] == "WRITE_SIZE"]
    gib_kib = float(1 << 20)
    fetch_f = write_f = float("nan")
    if cal:
        kw = max(cal, key=lambda k: mean(ctr[k]))
        write_f = gib_kib / mean(ctr[kw])
        kf = (kw[0], kw[1], "FETCH_SIZE")
        if kf in ctr:
            fetch_f = gib_kib / mean(ctr[kf])
    return dur, ctr, fetch_f, write_f, mean


def kernel_records(root: str, prefixes=("k_", "kb_")) -> list:
    """One record per (kernel, grid) of this library: calls, mean and median
    duration, HBM bytes read and written per launch (scaled counters), VALU
    wavefront instructions per launch, and the rates they give at the mean
    duration: HBM GB/s against 8 TB/s and VALU lane-instructions per second
    against the non-packed issue rate of 256 CU x 4 SIMD x 16 lanes x
    2.4 GHz."""
    dur, ctr, fetch_f, write_f, mean = _prof_tables(root)
    keys = sorted({(k[0], k[1]) for k in dur} | {(k[0], k[1]) for k in ctr},
                  key=lambda k: -mean(dur.get(k, [0])) * len(dur.get(k, [0])))
    out = []
    for k in keys:
        if not k[0].startswith(prefixes):
            continue
        d = dur.get(k, [])
        t = mean(d) * 1e-6
        rd = mean(ctr.get((k[0], k[1], "FETCH_SIZE"), [])) * fetch_f * 1024
        wr = mean(ctr.get((k[0], k[1], "WRITE_SIZE"), [])) * write_f * 1024
        vi = mean(ctr.get((k[0], k[1], "SQ_INSTS_VALU"), []))
        wv = mean(ctr.get((k[0], k[1], "SQ_WAVES"), []))
        rec = {"kernel": k[0], "grid": k[1], "calls": len(d), "mean_us": round(mean(d), 2),
               "median_us": round(sorted(d)[len(d) // 2], 2) if d else None,
               "read_MB": round(rd / 1e6, 3), "write_MB": round(wr / 1e6, 3),
               "valu_wave_instructions": vi, "waves": wv}
        if d and rd == rd:
            rec["hbm_GBps"] = round((rd + wr) / t / 1e9, 1)
            rec["hbm_frac"] = round((rd + wr) / t / 1e9 / PEAK_HBM_GBS, 4)
        if d and vi == vi:
            rec["valu_issue_frac"] = round(vi * 64 / t / VALU_ISSUE_PEAK, 4)
        out.append(rec)
    return out


def most_called_shapes(records: list) -> list:
    """Per kernel, the record of its most-called launch shape (the tuned
    one: the autotuner runs every candidate shape a few times, the chosen
    one on every call; the other shapes stay in the profile summaries)."""
    best = {}
    for r in records:
        if r["calls"] > best.get(r["kernel"], {}).get("calls", 0):
            best[r["kernel"]] = r
    return [r for r in records if best.get(r["kernel"]) is r]


def summarize_prof(root: str) -> str:
    """Markdown summary of rocprofv3 CSV output under root/{trace,fetch,write,
    valu}: per (kernel, grid) mean duration, HBM bytes from FETCH_SIZE and
    WRITE_SIZE scaled so that the 1 GiB calibration copy reads 1 GiB each
    way, VALU instruction counts, and the HBM and VALU-issue fractions they
    give at the mean duration."""
    _, _, fetch_f, write_f, _ = _prof_tables(root)
    lines = ["| kernel | grid | calls | mean us | median us | HBM read MB | HBM write MB | "
             "VALU instr/wave | waves | HBM GB/s (frac of 8 TB/s) | VALU issue frac |",
             "|---|---|---|---|---|---|---|---|---|---|---|"]
    for r in kernel_records(root, ("k_", "kb_", "__amd_rocclr_copyBuffer")):
        vw = (r["valu_wave_instructions"] / r["waves"]
              if r["waves"] == r["waves"] and r["waves"] else float("nan"))
        hb = f"{r['hbm_GBps']} ({r['hbm_frac']})" if "hbm_GBps" in r else "-"
        lines.append(f"| {r['kernel']} | {r['grid']} | {r['calls']} | {r['mean_us']} | "
                     f"{r['median_us']} | {r['read_MB']} | {r['write_MB']} | {vw:.0f} | "
                     f"{r['waves']:.0f} | {hb} | {r.get('valu_issue_frac', '-')} |")
    head = [f"FETCH_SIZE scale {fetch_f:.4f}, WRITE_SIZE scale {write_f:.4f} "
            "(so that the 1 GiB calibration copy reads 1 GiB each way).", ""]
    return "\n".join(head + lines)


def library_source_hash() -> str:
    """sha256 of every HIP source of the library: per-kernel counter records
    are reported only while the sources they were taken from are unchanged."""
    import glob
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2509_18815_amd", "csrc")
    for f in sorted(glob.glob(os.path.join(csrc, "*"))):
        h.update(os.path.basename(f).encode())
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


# the sources the dominant kernel (the single-latent decode) is compiled from
DOMINANT_SOURCES = ("gmm_device.h", "gmm_stream.h", "gmm_kernels.h", "gmm_coder.hip")


def kernel_source_hash() -> str:
    """sha256 of the dominant kernel's HIP sources: counter figures recorded
    for one version of the kernel are reported only while they are
    unchanged."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2509_18815_amd", "csrc")
    for f in DOMINANT_SOURCES:
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def traffic_record(root: str, kernel: str, grid: int) -> dict:
    """HBM bytes per launch of one kernel dispatch shape from the counter
    CSVs (FETCH_SIZE and WRITE_SIZE scaled by the 1 GiB copy)."""
    import collections
    import csv
    import glob

    ctr = collections.defaultdict(list)
    for sub in ("fetch", "write", "valu"):
        for f in glob.glob(os.path.join(root, sub, "*counter_collection.csv")):
            for r in csv.DictReader(open(f)):
                ctr[(r["Kernel_Name"].replace("void ", "").split("(")[0], int(r["Grid_Size"]),
                     r["Counter_Name"])].append(float(r["Counter_Value"]))
    mean = lambda v: sum(v) / len(v)  # noqa: E731
    cal = max((k for k in ctr if k[0].startswith("__amd_rocclr_copyBuffer")
               and k[2] == "WRITE_SIZE"), key=lambda k: mean(ctr[k]))
    wf = float(1 << 20) / mean(ctr[cal])
    ff = float(1 << 20) / mean(ctr[(cal[0], cal[1], "FETCH_SIZE")])
    rd = mean(ctr[(kernel, grid, "FETCH_SIZE")]) * ff * 1024
    wr = mean(ctr[(kernel, grid, "WRITE_SIZE")]) * wf * 1024
    rec = {"kernel": kernel, "grid": grid, "read_bytes": rd, "write_bytes": wr,
           "traffic_bytes": rd + wr, "fetch_scale": ff, "write_scale": wf,
           "source_sha": kernel_source_hash()}
    vi = ctr.get((kernel, grid, "SQ_INSTS_VALU"))
    if vi:
        # wavefront VALU instructions per launch (each covers 64 lanes)
        rec["valu_wave_instructions"] = mean(vi)
    return rec


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_decode_4k_320x135x240_traffic.json")
# per-kernel counter records of the batched and bracket forms (bench.py
# --record-counters <profile dir>), tied to the library's source hash
COUNTERS_FILE = os.path.join(ROOT, "profiles", "kernel_counters.json")
# the oracle's longer CPU legs, written by a run with --cpu-baseline-legs
CPU_LEGS_FILE = os.path.join(ROOT, "profiles", "oracle_cpu_legs.json")
# the dominant kernel: plain A&S decode, K=3, one lane per stream, direct indexing
DOMINANT_KERNEL = "k_decode<3, 0, true, 1, false, true>"


def progress(msg: str) -> None:
    """A progress line on stderr (long runs, profilers)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def form_counters(name: str):
    """The committed counter records of a form's kernels (HBM and VALU-issue
    fractions per kernel from a profiled run of that form), or None once the
    library's sources have changed since they were taken."""
    if not os.path.exists(COUNTERS_FILE):
        return None
    rec = json.load(open(COUNTERS_FILE)).get(name)
    if not rec or rec.get("source_sha") != library_source_hash():
        return None
    keep = ("kernel", "grid", "calls", "mean_us", "read_MB", "write_MB", "hbm_GBps",
            "hbm_frac", "valu_issue_frac")
    prefix = {"c3": ("kb_",), "c5": ("kb_",), "c4": ("k_decode_bracket",)}.get(name, ("k",))
    recs = most_called_shapes([r for r in rec["kernels"] if r["kernel"].startswith(prefix)])
    return {"source": os.path.relpath(COUNTERS_FILE, ROOT),
            "kernels": [{k: r[k] for k in keep if k in r} for r in recs]}


class TimingEvent:
    """A HIP event for timing only, created with hipEventDisableSystemFence
    in the HIP runtime that torch loaded (the one the library's calls use).
    A default event is recorded with a system-scope release: the L2 is
    written back after the preceding kernel before the stream moves on. Two
    such events around the 4K decode were measured to add ~20 us to each
    step (0.407-0.415 against 0.383-0.395 ms without events) and ~10 us to
    the decode they bracket; these events add neither (0.391-0.394 ms)."""
    DISABLE_SYSTEM_FENCE = 0x20000000
    _hip = None

    @classmethod
    def runtime(cls):
        """The process's libamdhip64 (None if it cannot be found)."""
        if cls._hip is None:
            import ctypes
            path = None
            try:
                for line in open("/proc/self/maps"):
                    f = line.split()[-1]
                    if os.path.basename(f).startswith("libamdhip64.so"):
                        path = f
                        break
            except OSError:
                pass
            cls._hip = ctypes.CDLL(path) if path else False
        return cls._hip or None

    def __init__(self):
        import ctypes
        hip = self.runtime()
        self.ev = ctypes.c_void_p()
        if hip is None or hip.hipEventCreateWithFlags(
                ctypes.byref(self.ev), ctypes.c_uint(self.DISABLE_SYSTEM_FENCE)) != 0:
            raise RuntimeError("hipEventCreateWithFlags failed")

    def record(self, stream):
        import ctypes
        if self.runtime().hipEventRecord(self.ev, ctypes.c_void_p(stream.cuda_stream)) != 0:
            raise RuntimeError("hipEventRecord failed")

    def elapsed_time(self, end) -> float:
        """Milliseconds from this event to end (both completed)."""
        import ctypes
        ms = ctypes.c_float()
        if self.runtime().hipEventElapsedTime(ctypes.byref(ms), self.ev, end.ev) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return ms.value

    def destroy(self):
        if self.ev:
            self.runtime().hipEventDestroy(self.ev)
            self.ev = None


def timing_event_pairs(count):
    """count pairs of fence-free timing events, or of torch events where the
    HIP runtime cannot be reached; returns (pairs, kind)."""
    import torch
    try:
        return [(TimingEvent(), TimingEvent()) for _ in range(count)], \
            "hipEventDisableSystemFence"
    except (RuntimeError, OSError, AttributeError):
        return [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                for _ in range(count)], "torch.cuda.Event (system-scope release)"


def time_events(fn, reps, stream):
    import torch
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    fn()
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    b.synchronize()
    return a.elapsed_time(b) / 1e3 / reps


def batched_form(api, synth, name, dev, reps=5, bracket_model=None, loop_baseline=True):
    """One plan (hipGraph of persistent kernels, autotuned) per direction over
    a batch of uneven latents, against a loop of single-latent calls on the
    same buffers; round trip verified. With bracket_model, a second decode
    plan with the learned bracket is measured beside the plain one."""
    import torch
    cfgd = synth.CONFIGS[name]
    lats = synth.make_latents(cfgd, backend="torch", device=dev)
    ns, Ss = [L.n for L in lats], [L.streams for L in lats]
    n_tot = sum(ns)
    stream = torch.cuda.current_stream()
    pe = api.Plan(cfgd.K, cfgd.lo, cfgd.hi, cfgd.precision, ns, Ss, op=0, autotune=True)
    pd = api.Plan(cfgd.K, cfgd.lo, cfgd.hi, cfgd.precision, ns, Ss, op=1, autotune=True)
    io, dio = [], []
    for L in lats:
        cap = L.n + 2 * L.streams
        e = {"symbols": L.symbols, "weights": L.weights, "means": L.means, "scales": L.scales,
             "bitstream": torch.empty(cap, dtype=torch.int16, device=dev), "words": cap,
             "offsets": torch.empty(L.streams + 1, dtype=torch.int64, device=dev)}
        io.append(e)
    st_e = torch.zeros(len(lats), dtype=torch.int32, device=dev)
    st_d = torch.zeros(len(lats), dtype=torch.int32, device=dev)
    assert pe.run(io) == 0
    for L, e in zip(lats, io):
        dio.append({"weights": L.weights, "means": L.means, "scales": L.scales,
                    "bitstream": e["bitstream"], "words": int(e["offsets"][-1].item()),
                    "offsets": e["offsets"],
                    "decoded": torch.empty(L.n, dtype=torch.int32, device=dev)})
    assert pd.run(dio) == 0
    t_enc = time_events(lambda: pe.run(io, status=st_e), reps, stream)
    t_dec = time_events(lambda: pd.run(dio, status=st_d), reps, stream)
    torch.cuda.synchronize()
    assert st_e.abs().sum().item() == 0 and st_d.abs().sum().item() == 0
    for L, d in zip(lats, dio):
        assert torch.equal(d["decoded"], L.symbols), "batched round trip failed"
    words = sum(int(e["offsets"][-1].item()) for e in io)
    bracket_out = None
    if bracket_model is not None:
        br = bracket_model.load()
        stats = torch.zeros(4, dtype=torch.int64, device=dev)
        pb = api.Plan(cfgd.K, cfgd.lo, cfgd.hi, cfgd.precision, ns, Ss, op=1, autotune=True)
        pb.set_bracket(br, stats)
        for d in dio:
            d["decoded"].fill_(-1)
        assert pb.run(dio) == 0
        for L, d in zip(lats, dio):
            assert torch.equal(d["decoded"], L.symbols), "bracket round trip failed"
        stats.zero_()
        st_b = torch.zeros(len(lats), dtype=torch.int32, device=dev)
        t_br = time_events(lambda: pb.run(dio, status=st_b), reps, stream)
        torch.cuda.synchronize()
        assert st_b.abs().sum().item() == 0
        hits, misses, all_hit, steps = stats.cpu().tolist()
        bracket_out = {"decode_sym_s": n_tot / t_br, "gain_vs_plain_decode": t_dec / t_br,
                       "hit_rate": hits / max(hits + misses, 1),
                       "wave_all_hit": all_hit / max(steps, 1),
                       "decode_plan": pb.info(), "training": bracket_model.history[-2:]}
        pb.close()
        br.close()
    if not loop_baseline:
        out = {"latents": len(lats), "n": n_tot, "K": cfgd.K, "support": [cfgd.lo, cfgd.hi],
               "encode_sym_s": n_tot / t_enc, "decode_sym_s": n_tot / t_dec,
               "roundtrip_sym_s": n_tot / (t_enc + t_dec), "bits_per_symbol": 16.0 * words / n_tot,
               "roofline": form_roofline(cfgd.K, cfgd.hi - cfgd.lo + 1, n_tot / t_enc,
                                         n_tot / t_dec, 16.0 * words / n_tot),
               "encode_plan": pe.info(), "decode_plan": pd.info(), "bracket": bracket_out}
        pe.close()
        pd.close()
        return out
    # single-latent calls on the same buffers, for comparison
    ws = [torch.empty(api.workspace_bytes(api.make_cfg(cfgd.K, cfgd.lo, cfgd.hi, cfgd.precision,
                                                       L.streams), L.n, 0),
                      dtype=torch.uint8, device=dev) for L in lats]
    st1 = torch.zeros(1, dtype=torch.int32, device=dev)

    def loop_enc():
        for L, e, w in zip(lats, io, ws):
            api.encode_into(api.make_cfg(cfgd.K, cfgd.lo, cfgd.hi, cfgd.precision, L.streams),
                            L.symbols, L.weights, L.means, L.scales, e["bitstream"],
                            e["offsets"], ws=w, status=st1)

    def loop_dec():
        for L, d in zip(lats, dio):
            api.decode_into(api.make_cfg(cfgd.K, cfgd.lo, cfgd.hi, cfgd.precision, L.streams),
                            d["bitstream"], d["offsets"], L.weights, L.means, L.scales,
                            d["decoded"], total_words=d["words"], status=st1)
    t_enc1 = time_events(loop_enc, 2, stream)
    t_dec1 = time_events(loop_dec, 2, stream)
    out = {"latents": len(lats), "n": n_tot, "K": cfgd.K, "support": [cfgd.lo, cfgd.hi],
           "encode_sym_s": n_tot / t_enc, "decode_sym_s": n_tot / t_dec,
           "roundtrip_sym_s": n_tot / (t_enc + t_dec),
           "bits_per_symbol": 16.0 * words / n_tot,
           "roofline": form_roofline(cfgd.K, cfgd.hi - cfgd.lo + 1, n_tot / t_enc,
                                     n_tot / t_dec, 16.0 * words / n_tot),
           "encode_plan": pe.info(), "decode_plan": pd.info(),
           "single_call_loop": {"encode_sym_s": n_tot / t_enc1, "decode_sym_s": n_tot / t_dec1},
           "bracket": bracket_out}
    pe.close()
    pd.close()
    return out


def bracket_single_form(api, synth, dev, model, reps=5):
    """The 4K latent (320x135x240, 65,536 streams) decoded with the plain
    binary search and with the learned bracket, same bitstream."""
    import torch
    cfgd = synth.CONFIGS["c4"]
    lat = synth.make_latents(cfgd, backend="torch", device=dev)[0]
    L = Latent(api, cfgd, lat)
    L.encode()
    stream = torch.cuda.current_stream()
    t_plain = time_events(L.decode, reps, stream)
    br = model.load()
    stats = torch.zeros(4, dtype=torch.int64, device=dev)
    dec = torch.empty_like(L.dec)

    def run(with_stats=False):
        r = api.decode_into(L.cfg, L.bs, L.off, lat.weights, lat.means, lat.scales, dec,
                            bracket=br, stats=stats if with_stats else None, ws=L.ws_dec,
                            status=L.st[1:2])
        assert r == 0
    run(True)
    torch.cuda.synchronize()
    assert torch.equal(dec, lat.symbols), "bracket decode differs"
    hits, misses, all_hit, steps = stats.cpu().tolist()
    t_br = time_events(run, reps, stream)
    torch.cuda.synchronize()
    assert torch.equal(dec, lat.symbols) and L.st.tolist() == [0, 0]
    br.close()
    return {"n": L.n, "streams": L.S, "plain_decode_sym_s": L.n / t_plain,
            "bracket_decode_sym_s": L.n / t_br, "gain": t_plain / t_br,
            "hit_rate": hits / max(hits + misses, 1), "wave_all_hit": all_hit / max(steps, 1),
            "training": model.history[-2:]}


def bracket_few_streams_form(api, synth, dev, name, model, reps=10):
    """A latent with few streams (the 320x48x32 latent at 4,096 streams, or
    the 192x16x16 latent at 256 streams) decoded by lane groups: the plain
    (L+1)-ary search at the library's automatic L (8 and 16 lanes per stream
    here) against the group form of the learned bracket at the same L (one
    round of L boundaries around the prediction), same bitstream."""
    import torch
    cfgd = synth.CONFIGS[name]
    lat = synth.make_latents(cfgd, backend="torch", device=dev)[0]
    L = Latent(api, cfgd, lat)
    L.encode()
    stream = torch.cuda.current_stream()
    t_plain = time_events(L.decode, reps, stream)
    br = model.load()
    stats = torch.zeros(4, dtype=torch.int64, device=dev)
    dec = torch.empty_like(L.dec)

    def run(with_stats=False):
        r = api.decode_into(L.cfg, L.bs, L.off, lat.weights, lat.means, lat.scales, dec,
                            bracket=br, stats=stats if with_stats else None, ws=L.ws_dec,
                            status=L.st[1:2])
        assert r == 0
    run(True)
    torch.cuda.synchronize()
    assert torch.equal(dec, lat.symbols), "bracket decode differs"
    hits, misses, all_hit, steps = stats.cpu().tolist()
    t_br = time_events(run, reps, stream)
    torch.cuda.synchronize()
    assert torch.equal(dec, lat.symbols) and L.st.tolist() == [0, 0]
    br.close()
    return {"shape": list(lat.shape), "n": L.n, "streams": L.S,
            "plain_lanes_per_stream": api.decode_lanes(L.cfg),
            "bracket_lanes_per_stream": api.decode_lanes(L.cfg),
            "plain_decode_sym_s": L.n / t_plain, "bracket_decode_sym_s": L.n / t_br,
            "plain_decode_ms": round(t_plain * 1e3, 4), "bracket_decode_ms": round(t_br * 1e3, 4),
            "gain": t_plain / t_br, "hit_rate": hits / max(hits + misses, 1),
            "wave_all_hit": all_hit / max(steps, 1)}


def learned_step_form(api, lats, model, step, steps, warmup, plain_value, dev):
    """The timed step of the headline measurement again, with the
    Kodak-size latent decoded through the learned bracket's group form (the
    network on the matrix cores, one window round of 16 or of 8 boundaries;
    the faster is reported) while the 4K
    latent's decode runs beside it: the two decodes share the SIMDs, and the
    bracket moves most of the Kodak-latent decode off the vector ALUs that
    bound the 4K decode. Same bitstreams, outputs verified."""
    import torch
    L = lats["c2a"]
    br = model.load()
    stats = torch.zeros(4, dtype=torch.int64, device=dev)

    def kodak_decode_with(lanes):
        # lanes 16: group form of 16 lanes per stream (the automatic choice
        # with a bracket at 4,096 streams); 8: the group form of 8
        def kodak_decode():
            api.set_wave_priority(L.prio)
            api.set_decode_lanes(lanes)
            try:
                r = api.decode_into(L.cfg, L.bs, L.off, L.lat.weights, L.lat.means,
                                    L.lat.scales, L.dec, bracket=br, stats=stats, ws=L.ws_dec,
                                    status=L.st[1:2])
            finally:
                api.set_decode_lanes(0)
            assert r == 0
        return kodak_decode

    def timed(kd):
        # same procedure as the headline measurement: warm-up steps straight
        # into the synchronisation that opens the timed region
        for _ in range(warmup):
            step(kodak_decode=kd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step(kodak_decode=kd)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    # plain and learned steps (both group forms) alternately, so all see the
    # same conditions; the learned value is the faster group form's
    plain_t, learned_t, hit_rate = [], {16: [], 8: []}, {}
    for _ in range(2):
        # each timed region follows an output check (the same idle gap)
        plain_t.append(timed(None))
        for nm in lats:
            lats[nm].verify()
        for lanes in (16, 8):
            stats.zero_()
            learned_t[lanes].append(timed(kodak_decode_with(lanes)))
            for nm in lats:
                lats[nm].verify()
            hits, misses, _, _ = stats.cpu().tolist()
            hit_rate[lanes] = hits / max(hits + misses, 1)
    br.close()
    n_total = sum(lats[nm].n for nm in lats)
    best = min(learned_t, key=lambda k: sum(learned_t[k]))
    v = n_total * steps / (sum(learned_t[best]) / 2)
    vp = n_total * steps / (sum(plain_t) / 2)
    return {"value": v, "unit": "symbols/s",
            "ms_per_step": sum(learned_t[best]) / 2 / steps * 1e3,
            "kodak_group_lanes": best,
            "ms_per_step_by_group_lanes": {k: round(sum(t) / 2 / steps * 1e3, 4)
                                           for k, t in learned_t.items()},
            "plain_step_value_here": vp, "gain_vs_plain_step": v / vp,
            "kodak_latent_hit_rate": hit_rate[best],
            "kodak_latent_hit_rate_by_group_lanes": hit_rate}


# The paper's Table II (CPU, per 768x512 Kodak image; encode / decode ms),
# quoted as context for the same comparison on one MI355X.
PAPER_TABLE2_MS = {"no_approximation": (56.5, 127.0), "polya": (23.5, 34.3),
                   "as_26_2_17": (22.5, 33.7), "logistic": (22.5, 33.2)}


def table2_form(api, synth, dev, reps=5):
    """Speed of the Gaussian-CDF kinds of the paper's Table II on the
    320x48x32 latent (4,096 streams): encode and decode time per latent for
    the binary64 reference (standing in for the unapproximated erfc), Polya,
    A&S 26.2.17 and logistic, each round trip verified."""
    import torch
    cfgd = synth.CONFIGS["c2a"]
    lat = synth.make_latents(cfgd, backend="torch", device=dev)[0]
    stream = torch.cuda.current_stream()
    out = {"latent": list(lat.shape), "n": lat.n, "streams": lat.streams}
    for kind, name in ((3, "no_approximation"), (2, "polya"), (0, "as_26_2_17"),
                       (1, "logistic")):
        L = Latent(api, cfgd, lat, cdf_kind=kind)
        L.encode()
        L.decode()
        torch.cuda.synchronize()
        L.verify()
        t_e = time_events(L.encode, reps, stream)
        t_d = time_events(L.decode, reps, stream)
        torch.cuda.synchronize()
        L.verify()
        out[name] = {"encode_ms": round(t_e * 1e3, 4), "decode_ms": round(t_d * 1e3, 4),
                     "encode_sym_s": L.n / t_e, "decode_sym_s": L.n / t_d,
                     "bits_per_symbol": 16.0 * float(L.off[-1].item()) / L.n,
                     "paper_cpu_ms": PAPER_TABLE2_MS[name]}
    return out


def epilogue_form(api, synth, dev, reps=5):
    """Coding from a network's raw outputs on the 4K latent (320x135x240,
    65,536 streams): the mapping (softmax of weight logits, exp of
    log-scales) fused into the coder kernels, against a separate mapping
    pass (gmm_params_from_raw) before each plain encode and decode. The raw
    outputs are log-weights and log-scales of the plain workload, so the
    symbols and the model match the plain 4K measurement."""
    import torch
    cfgd = synth.CONFIGS["c2b"]
    lat = synth.make_latents(cfgd, backend="torch", device=dev)[0]
    logits = torch.log(lat.weights).contiguous()
    log_s = torch.log(lat.scales).contiguous()
    raw = synth.Latent(lat.symbols, logits, lat.means, log_s, lat.shape, lat.streams)
    Lr = Latent(api, cfgd, raw, param_kind=1)
    w_m = torch.empty_like(logits)
    s_m = torch.empty_like(log_s)
    mapped = synth.Latent(lat.symbols, w_m, lat.means, s_m, lat.shape, lat.streams)
    Lp = Latent(api, cfgd, mapped)
    stream = torch.cuda.current_stream()

    def mapping():
        r = api.lib().gmm_params_from_raw(cfgd.K, lat.n, api._dev(logits, torch.float32, "l"),
                                          api._dev(log_s, torch.float32, "t"),
                                          api._dev(w_m, torch.float32, "w"),
                                          api._dev(s_m, torch.float32, "s"), api._stream())
        assert r == 0

    def sep_encode():
        mapping()
        Lp.encode()

    def sep_decode():
        mapping()
        Lp.decode()

    Lr.encode()
    Lr.decode()
    sep_encode()
    sep_decode()
    torch.cuda.synchronize()
    Lr.verify()
    Lp.verify()
    assert torch.equal(Lr.off, Lp.off) and torch.equal(Lr.bs[: int(Lr.off[-1].item())],
                                                        Lp.bs[: int(Lp.off[-1].item())])
    t = {"fused_encode": time_events(Lr.encode, reps, stream),
         "fused_decode": time_events(Lr.decode, reps, stream),
         "separate_encode": time_events(sep_encode, reps, stream),
         "separate_decode": time_events(sep_decode, reps, stream),
         "mapping_pass": time_events(mapping, reps, stream)}
    torch.cuda.synchronize()
    Lr.verify()
    Lp.verify()
    out = {k + "_ms": round(v * 1e3, 4) for k, v in t.items()}
    out["n"] = lat.n
    out["fused_gain_encode"] = t["separate_encode"] / t["fused_encode"]
    out["fused_gain_decode"] = t["separate_decode"] / t["fused_decode"]
    # bytes of the separate pass: 2K planes read (logits, log-scales), 2K written
    out["mapping_pass_GBps"] = 4 * cfgd.K * 4 * lat.n / t["mapping_pass"] / 1e9
    return out


def main():
    if len(sys.argv) > 2 and sys.argv[1] == "--summarize-prof":
        print(summarize_prof(sys.argv[2]))
        return
    if len(sys.argv) > 3 and sys.argv[1] == "--record-counters":
        # bench.py --record-counters <profile dir> <form name>
        allrec = json.load(open(COUNTERS_FILE)) if os.path.exists(COUNTERS_FILE) else {}
        allrec[sys.argv[3]] = {"source_sha": library_source_hash(),
                               "kernels": most_called_shapes(kernel_records(sys.argv[2]))}
        with open(COUNTERS_FILE, "w") as fh:
            json.dump(allrec, fh, indent=1)
        print(json.dumps(allrec[sys.argv[3]])[:2000])
        return
    if len(sys.argv) > 2 and sys.argv[1] == "--record-traffic":
        rec = traffic_record(sys.argv[2], DOMINANT_KERNEL, 65536)
        with open(TRAFFIC_FILE, "w") as fh:
            json.dump(rec, fh, indent=1)
        print(json.dumps(rec))
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="c3,c4,c5,table2,epilogue",
                    help="comma list of extra forms measured after the timed steps: c3 batch "
                         "of 64 latents; c4 4K latent plain vs learned bracket; c5 batch of "
                         "256 K=5 latents, plain vs learned bracket; table2 Gaussian-CDF kinds "
                         "of the paper's Table II on the Kodak-size latent; epilogue raw "
                         "network outputs, fused vs separate mapping, 4K latent; none")
    ap.add_argument("--bracket-tuples", type=int, default=10_000_000,
                    help="training tuples of each bracket model (c4, c5)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM counters)")
    ap.add_argument("--bracket-model", default=None,
                    help="directory holding trained bracket models c1.npz, c4.npz, c5.npz "
                         "(train.BracketModel.save format): loaded instead of trained")
    ap.add_argument("--save-bracket-models", default=None,
                    help="directory to save the bracket models trained in this run")
    ap.add_argument("--cpu-baseline-legs", default=None,
                    help="also time the oracle's longer legs (whole 4K latent, subsets of the "
                         "batches; minutes of CPU work) and write them to this JSON file")
    ap.add_argument("--no-peak-probes", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only (asked for --gpus {args.gpus}); "
              "the sharded multi-GPU path is not implemented.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2509_18815_amd import api, synth
    api.lib()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    names = ("c2a", "c2b")
    stream = torch.cuda.current_stream()
    side = torch.cuda.Stream()  # default priority

    # HIP events around the 4K-latent decode (the dominant kernel) on the
    # launch stream, recorded inside the timed steps; created beforehand,
    # fence-free (TimingEvent)
    ev_pool, ev_kind = timing_event_pairs(args.steps)
    ev_pairs = []

    # Inputs are generated on the device, on the main stream; the warm-up
    # steps follow them in stream order (the side stream waits for the main
    # one below), with no host synchronisation in between: an idle device
    # before the warm-up leaves the first timed steps at lower clocks (20
    # timed steps after 5 warm-up ones: 26.7-27.0 G sym/s with a
    # synchronisation here, 27.0-27.7 without, alternated on one box).
    lats = {}
    for nm in names:
        cfgd = synth.CONFIGS[nm]
        lat = synth.make_latents(cfgd, backend="torch", device=dev)[0]
        # the 4K latent's kernels are bound by VALU issue and on the step's
        # critical path: they issue first on shared SIMDs, the Kodak-size
        # latent's latency-bound kernels fill their idle issue slots
        lats[nm] = Latent(api, cfgd, lat, prio=3 if nm == "c2b" else 0)

    def step(record=False, kodak_decode=None):
        # the Kodak-size latent's chain on the side stream, the 4K latent's
        # on the main stream. The two chains are independent and are not
        # joined step by step (a join per step was measured to leave the
        # main stream idle ~16 us per step while the cross-stream wait
        # resolved): each stream runs its steps back to back, and the timed
        # region ends when both are idle.
        with torch.cuda.stream(side):
            lats["c2a"].encode()
            (kodak_decode or lats["c2a"].decode)()
        lats["c2b"].encode()
        if record:
            a, b = ev_pool[len(ev_pairs)]
            a.record(stream)
            lats["c2b"].decode()
            b.record(stream)
            ev_pairs.append((a, b))
        else:
            lats["c2b"].decode()

    # warm-up steps run back to back into the timed region's synchronisation
    # (their outputs are checked with the timed ones: a check here would
    # leave the device idle for milliseconds, after which the first timed
    # steps were measured to run ~10% slower)
    side.wait_stream(stream)  # the inputs were written on the main stream
    for _ in range(args.warmup):
        step()

    progress(f"{args.warmup} warm-up steps done; timing {args.steps} steps")
    # timed region: K steps, bracketed by device synchronisation
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(record=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    dec_in_steps = sum(a.elapsed_time(b) for a, b in ev_pairs) / 1e3 / len(ev_pairs)
    for pair in ev_pool:
        for e in pair:
            if isinstance(e, TimingEvent):
                e.destroy()
    for nm in names:
        lats[nm].verify()
    n_total = sum(lats[nm].n for nm in names)
    value = n_total * args.steps / elapsed

    # per-call times with HIP events on the launch stream (separate pass)
    ev = {}
    reps = max(3, min(args.steps, 20))
    for nm in names:
        for op in ("encode", "decode"):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            for _ in range(reps):  # untimed calls first, back to back with the timed ones
                getattr(lats[nm], op)()
            a.record(stream)
            for _ in range(reps):
                getattr(lats[nm], op)()
            b.record(stream)
            b.synchronize()
            ev[(nm, op)] = a.elapsed_time(b) / 1e3 / reps
    api.set_wave_priority(0)
    forms = {}
    for nm in names:
        L = lats[nm]
        bps = 16.0 * float(L.off[-1].item()) / L.n
        forms[nm] = {"shape": list(L.lat.shape), "n": L.n, "streams": L.S,
                     "decode_lanes_per_stream": api.decode_lanes(L.cfg),
                     "encode_sym_s": L.n / ev[(nm, "encode")],
                     "decode_sym_s": L.n / ev[(nm, "decode")],
                     "bits_per_symbol": bps,
                     "roofline": form_roofline(L.cfgd.K, L.cfgd.hi - L.cfgd.lo + 1,
                                               L.n / ev[(nm, "encode")],
                                               L.n / ev[(nm, "decode")], bps)}
    big = lats["c2b"]
    K, N = big.cfgd.K, big.cfgd.hi - big.cfgd.lo + 1
    dec_t = dec_in_steps
    achieved = decode_flops_per_symbol(K, N) * big.n / dec_t / 1e12
    traffic = None
    counters = None
    if os.path.exists(TRAFFIC_FILE):
        rec = json.load(open(TRAFFIC_FILE))
        if rec.get("source_sha") == kernel_source_hash():
            traffic = rec["traffic_bytes"]
            # counter-derived rates at this run's in-step launch time: HBM
            # bytes against 8 TB/s, and VALU lane-instructions (64 per
            # wavefront instruction) against the issue rate of non-packed
            # FP32 instructions, 256 CU x 4 SIMD x 16 lanes x 2.4 GHz (packed
            # FP32 is disabled in the library's compile flags; the 157.3 TFLOP/s peak
            # counts packed FMA as 4 flops per lane)
            counters = {"source": os.path.relpath(TRAFFIC_FILE, ROOT),
                        "hbm_GBps": round(traffic / dec_t / 1e9, 1),
                        "hbm_frac": round(traffic / dec_t / 1e9 / PEAK_HBM_GBS, 4)}
            if "valu_wave_instructions" in rec:
                lane_ops = rec["valu_wave_instructions"] * 64 / dec_t
                counters.update({
                    "valu_instructions_per_symbol": round(
                        rec["valu_wave_instructions"] * 64 / big.n, 1),
                    "valu_lane_instr_per_s": float("%.4g" % lane_ops),
                    "valu_issue_peak_lane_instr_per_s": VALU_ISSUE_PEAK,
                    "valu_issue_frac": round(lane_ops / VALU_ISSUE_PEAK, 4)})
    roofline = {"bound": "alu", "kernel": "k_decode (4K latent, 65,536 streams)",
                "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": traffic,
                "flops_per_symbol": decode_flops_per_symbol(K, N),
                "flops_basis": "binary search: ceil(log2 N) exact evaluations + setup "
                               "(the kernel's bracketed search executes fewer; see counters)",
                "symbols_per_launch": big.n,
                "launch_ms": round(dec_t * 1e3, 4),
                "launch_timing_events": ev_kind,
                "launch_ms_isolated": round(ev[("c2b", "decode")] * 1e3, 4),
                # the same launch back to back on its own (no co-running
                # Kodak-latent kernels), for comparison
                "achieved_isolated": round(decode_flops_per_symbol(K, N) * big.n
                                           / ev[("c2b", "decode")] / 1e12, 3),
                "counters": counters}
    out = {
        "metric": "GMM rANS decode+encode symbols/s, bit-exact; plain vs batched+learned bracket",
        "value": value, "unit": "symbols/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "plain method at paper scale: 320x48x32 (4,096 streams) + "
                               "320x135x240 (65,536 streams), K=3, support [-255,255], P=16; "
                               "one HIP stream per latent",
                   "symbols_per_step": n_total},
        "roofline": roofline,
        "forms": forms,
    }
    if not args.no_peak_probes:
        roofline["peaks_measured"] = peak_probes(api, dev)
    want = [f for f in args.forms.split(",") if f and f != "none"]
    if "c3" in want:
        progress("form c3 (batch of 64 latents)")
        forms["c3_batched"] = batched_form(api, synth, "c3", dev)
        forms["c3_batched"]["counters"] = form_counters("c3")
    if "c4" in want or "c5" in want:
        from paper_2509_18815_amd import train

    def bracket_model(name, **kw):
        """A trained bracket model: loaded from --bracket-model, else
        trained here on the GPU (and saved with --save-bracket-models)."""
        if args.bracket_model:
            m = train.BracketModel.from_file(os.path.join(args.bracket_model, name + ".npz"))
            m.history.append({"loaded_from": name + ".npz"})
            return m
        cfgd = synth.CONFIGS[name]
        m = train.train_bracket(cfgd.K, cfgd.lo, cfgd.hi, cfgd.precision,
                                n_train=args.bracket_tuples, device=dev, **kw)
        if args.save_bracket_models:
            os.makedirs(args.save_bracket_models, exist_ok=True)
            m.save(os.path.join(args.save_bracket_models, name + ".npz"))
        return m
    if "c4" in want:
        progress("form c4 (learned bracket, 4K latent; Kodak and 192x16x16 latents)")
        m4 = bracket_model("c4", seed=synth.TRAIN_SEED_C4)
        forms["c4_bracket"] = bracket_single_form(api, synth, dev, m4)
        forms["c4_bracket"]["counters"] = form_counters("c4")
        # the same model (same parameter distributions and support) on the
        # Kodak-size latent, whose 4,096 streams decode by lane groups
        forms["c2a_bracket"] = bracket_few_streams_form(api, synth, dev, "c2a", m4)
        forms["step_learned_bracket"] = learned_step_form(api, lats, m4, step, args.steps,
                                                          args.warmup, value, dev)
        m1 = bracket_model("c1", seed=synth.TRAIN_SEED_C1)
        forms["c1_bracket"] = bracket_few_streams_form(api, synth, dev, "c1", m1)
    if "c5" in want:
        progress("form c5 (batch of 256 K=5 latents, plain and learned bracket)")
        c5 = synth.CONFIGS["c5"]
        # trained until the held-out hit rate stops improving (at most 24
        # epochs of the 10 M tuples)
        m5 = bracket_model("c5", seed=synth.TRAIN_SEED_C5, s_logit=c5.s_logit, s_mu=c5.s_mu,
                           sigma_max=c5.sigma_max, epochs=24, plateau=5e-4)
        forms["c5_batched_bracket"] = batched_form(api, synth, "c5", dev, reps=3,
                                                   bracket_model=m5, loop_baseline=False)
        forms["c5_batched_bracket"]["counters"] = form_counters("c5")
    if "table2" in want:
        progress("form table2 (Gaussian-CDF kinds)")
        forms["table2_cdf_kinds"] = table2_form(api, synth, dev)
    if "epilogue" in want:
        progress("form epilogue (raw network outputs)")
        forms["raw_output_mapping"] = epilogue_form(api, synth, dev)
    if want:
        # the headline procedure again (W warm-up steps, K timed steps) after
        # the forms' seconds of GPU work: the sustained rate, beside `value`,
        # which the process's first timed steps give while the GPU's clocks
        # still rise (they were measured to take ~100 ms of load to settle)
        progress("the headline steps again, after the forms")
        side.wait_stream(stream)
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        el2 = time.perf_counter() - t0
        for nm in names:
            lats[nm].verify()
        out["repeat_after_forms"] = {"value": n_total * args.steps / el2,
                                     "ms_per_step": el2 / args.steps * 1e3,
                                     "steps": args.steps, "warmup": args.warmup}
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if not args.no_cpu_baseline:
        L = lats["c2a"]
        import numpy as np
        host = {"sym": L.lat.symbols.cpu().numpy(), "w": L.lat.weights.cpu().numpy(),
                "mu": L.lat.means.cpu().numpy(), "sg": L.lat.scales.cpu().numpy(), "S": L.S,
                "gpu_bs": L.bs[: int(L.off[-1].item())].cpu().numpy().view(np.uint16)}
        out["cpu_baseline"] = cpu_baseline(host, L.cfgd)
        if os.path.exists(CPU_LEGS_FILE):
            out["cpu_baseline"]["legs"] = json.load(open(CPU_LEGS_FILE))
            out["cpu_baseline"]["legs"]["source"] = os.path.relpath(CPU_LEGS_FILE, ROOT)
    if args.cpu_baseline_legs:
        legs = cpu_baseline_legs(dev)
        with open(args.cpu_baseline_legs, "w") as fh:
            json.dump(legs, fh, indent=1)
        out.setdefault("cpu_baseline", {})["legs"] = legs
    print(json.dumps(out))


if __name__ == "__main__":
    main()
