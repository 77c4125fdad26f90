#!/usr/bin/env python3
"""Benchmark: GateKeeper-GPU filter throughput on one MI355X.

Workload (the headline configuration): a 100 Mbp seeded random reference
(41% GC), 2^24 pairs of 100 bp reads with one candidate each, e = 5; 30% true
origins with Poisson(5) edits, 70% decoys sharing an exact 12-mer with their
candidate window.  Reads are 2-bit packed and stored transposed (encoded on
the GPU before the timed region, as the paper's host-encoded kernel time).

A step is one gk_filter call over the whole batch, inputs resident in HBM.
Prints one JSON line with pairs/s, the dominant kernel's roofline fraction
(HIP events around every launch, on the launch stream) and the oracle timed
on a bounded sample on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X peaks used for the roofline.
CUS, LANES, CLOCK_GHZ = 256, 64, 2.4
VALU_PEAK_TOPS = CUS * LANES * CLOCK_GHZ / 1000.0      # int32 lane-ops, 39.32 T/s
HBM_PEAK_GBS = 8000.0


def ops_per_pair(m: int, e: int) -> int:
    """Algorithmic int32 lane-ops per pair: (2e+1) masks x W32 words x 14 ops
    (2 read-plane funnels, 2 compare, 9 amendment, 1 AND), plus 6 per word
    and 16 per pair for the window gather, count and stores."""
    w = (m + 31) // 32
    return 14 * (2 * e + 1) * w + 6 * w + 16


def bytes_per_pair(m: int) -> int:
    """Algorithmic bytes per pair for one candidate per read: packed read
    (m/4 B), window (m/4 B), read index + position (8 B), accept + est (3 B),
    read length (2 B)."""
    return m // 4 + m // 4 + 8 + 3 + 2


def kernel_source_hash(files=("gk_filter.hip", "gk_pair.h", "gk_args.h")) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2103_14978_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(kernel_hash: str, n_pairs: int,
                         name: str = "k_filter_w4_config1_e5_counters.json", kernel=None,
                         tuning=None, field: str = "hbm_bytes_per_launch"):
    """HBM bytes per launch (or another per-launch field) from the committed
    counter summary, if it was taken on this exact kernel source, batch size,
    kernel and tuning; else None."""
    path = os.path.join(ROOT, "profiles", name)
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_hash") != kernel_hash or d.get("n_pairs") != n_pairs:
        return None
    if kernel is not None and not d.get("kernel", "").startswith(kernel):
        return None
    if tuning is not None and d.get("tuning") != tuning:
        return None
    return d.get(field)


def host_encode_fixed(reads, n_reads: int, m: int, rows: int, chunk: int = 1 << 20):
    """Host-side 2-bit encoding of n_reads reads of exactly m bases (split
    layout: low code bits in bits 0-15, high in 16-31), rows words per read,
    as a mapper that keeps its reads encoded would hand them over."""
    code = np.zeros(256, np.uint32)
    for ch, c in zip(b"ACGT", range(4)):
        code[ch] = code[ch + 32] = c
    out = np.empty(n_reads * rows, np.uint32)
    k = np.arange(16, dtype=np.uint32)

    def one(r0):
        r1 = min(n_reads, r0 + chunk)
        c = np.zeros((r1 - r0, rows * 16), np.uint32)
        c[:, :m] = code[np.asarray(reads[r0 * m:r1 * m]).reshape(r1 - r0, m)]
        c = c.reshape(r1 - r0, rows, 16)
        w = ((c & 1) << k).sum(2) | ((c >> 1) << (16 + k)).sum(2)
        out[r0 * rows:r1 * rows] = w.astype(np.uint32).reshape(-1)

    import concurrent.futures as cf
    import gen
    with cf.ThreadPoolExecutor(max_workers=gen.default_threads()) as ex:
        list(ex.map(one, range(0, n_reads, chunk)))
    return out


def host_cpu_model() -> str:
    """The host's CPU model and logical CPU count, for the CPU baseline."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{model}, {os.cpu_count()} logical CPUs visible"


def plain_kernel_name(words: int, e: int, pairs_per_lane: int) -> str:
    """The plain launch's kernel for this shape: the automatic setting (0)
    takes one pair per lane."""
    if pairs_per_lane == 0:
        pairs_per_lane = 1
    return f"k_filter_single<{words}" if pairs_per_lane == 1 else f"k_filter<{words}"


# VALU instruction kinds timed by the calibration kernels of libgk_calib.so
# (kind number -> name).
CALIB_KINDS = {0: "v_bfi_b32", 1: "v_alignbit_b32", 2: "v_xor_b32", 3: "v_and_or_b32",
               4: "v_or3_b32", 5: "v_bitop3_b32", 6: "v_and_b32", 7: "v_lshlrev_b32",
               8: "v_xor_b32_e64", 9: "v_add_u32", 10: "v_perm_b32", 11: "v_bcnt_u32_b32"}

# The VALU instructions of the filter's per-mask loops (the deletion and
# insertion loops of the fast path, 96 instructions per pass of both), by the
# calibrated kind each issues like, from the gfx950 assembly of
# k_filter_single<4>: funnel shifts, three-input logic, two-input logic,
# shifts (left and right), and-or / or3, and two compares (taken at the
# and-or rate).
FILTER_LOOP_MIX = {"v_alignbit_b32": 37, "v_bitop3_b32": 26, "v_xor_b32": 9, "v_and_b32": 3,
                   "v_lshlrev_b32": 13, "v_and_or_b32": 7, "v_or3_b32": 1}


def mix_peak(rates: dict, mix: dict = FILTER_LOOP_MIX) -> float:
    """Issue ceiling (lane-ops/s) of an instruction stream holding mix[k]
    instructions of each kind k, each issuing at its measured rate."""
    return sum(mix.values()) / sum(n / rates[k] for k, n in mix.items())


def measure_peaks(log):
    """The device's measured VALU issue rate, per instruction kind (8
    independent chains per lane, all CUs), and its device copy rate, from
    the calibration kernels of libgk_calib.so.  The filter's ceiling is the
    issue rate of its own instruction mix (mix_peak); the roofline takes
    max(spec, that)."""
    import ctypes
    from paper_2103_14978_amd import build as hipbuild
    if not os.path.exists(hipbuild.CALIB_LIB):
        raise ImportError(f"{hipbuild.CALIB_LIB} is missing: build the package first")
    L = ctypes.CDLL(hipbuild.CALIB_LIB)
    d = ctypes.c_double
    L.gkc_valu_rate.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                ctypes.POINTER(d), ctypes.POINTER(d)]
    L.gkc_copy_rate.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.POINTER(d),
                                ctypes.POINTER(d)]
    valu = {}
    for k, name in CALIB_KINDS.items():
        rate, ms = d(), d()
        st = L.gkc_valu_rate(k, 8, 4096, 3, ctypes.byref(rate), ctypes.byref(ms))
        if st != 0:
            raise RuntimeError(f"gkc_valu_rate({name}) failed: {st}")
        valu[name] = round(rate.value / 1e12, 3)
    rate, ms = d(), d()
    st = L.gkc_copy_rate(2 << 30, 5, ctypes.byref(rate), ctypes.byref(ms))
    if st != 0:
        raise RuntimeError(f"gkc_copy_rate failed: {st}")
    out = {"valu_Tops": valu,
           "filter_mix_Tops": round(mix_peak(valu), 3),
           "filter_loop_mix": FILTER_LOOP_MIX,
           "copy_GBs": round(rate.value / 1e9, 1),
           "what": "8 independent chains per lane of one instruction kind, 8 workgroups of "
                   "256 lanes per CU, best of 3; filter_mix: the issue ceiling of the filter's "
                   "per-mask loops, each instruction at the measured rate of its kind; copy: "
                   "2 GiB read + 2 GiB written, best of 5"}
    log(f"calibration: VALU {valu} T lane-ops/s; filter mix {out['filter_mix_Tops']} T; "
        f"copy {out['copy_GBs']} GB/s")
    return out


def valu_peak(calib) -> float:
    """The VALU roof: max(spec, the measured ceiling of the filter's mix)."""
    return max(VALU_PEAK_TOPS, calib["filter_mix_Tops"]) if calib else VALU_PEAK_TOPS


def events_ms(fn, k: int, stream, warm: int = 2, stats: bool = False):
    """Mean milliseconds of fn() over k runs, each bracketed by HIP events on
    `stream` (the stream fn launches on), after `warm` untimed runs.  With
    stats: (mean, min, median)."""
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(k)]
    for a0, a1 in ev:
        a0.record(stream)
        fn()
        a1.record(stream)
    torch.cuda.synchronize()
    t = [a0.elapsed_time(a1) for a0, a1 in ev]
    if stats:
        return float(np.mean(t)), float(np.min(t)), float(np.median(t))
    return float(np.mean(t))


def encode_bytes_per_read(m: int, rows: int) -> int:
    """Algorithmic HBM bytes per read of gk_encode_reads: the ASCII text (m B)
    and its offset (8 B) in; rows packed words (4 B each), the length (2 B)
    and the unknown-base flag (1 B) out."""
    return m + 8 + 4 * rows + 2 + 1


# Sources of the fused encode + filter kernel (its counters are keyed on them).
FUSED_SOURCES = ("gk_fused.hip", "gk_pair.h", "gk_args.h", "gk_encode_dev.h")


def fused_bytes_per_pair(m: int) -> int:
    """Algorithmic HBM bytes per pair of gk_filter_ascii (pair i uses read i):
    the ASCII text (m B) and its offset (8 B), the window (m/4 B), the
    position (4 B) in; accept + est (3 B) out."""
    return m + 8 + m // 4 + 4 + 3


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--pairs", type=int, default=1 << 24)
    ap.add_argument("--e", type=int, default=5)
    ap.add_argument("--layout", choices=["split", "interleaved"], default="split",
                    help="2-bit read layout in HBM (both are 16 bases per 32-bit word)")
    ap.add_argument("--pairs-per-lane", type=int, default=0,
                    help="plain filter grid shape (0: automatic; 1: one pair per lane; "
                         "65536: one device residency)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--no-verify", action="store_true",
                    help="skip the verification (edit distance) measurement")
    ap.add_argument("--no-mixed", action="store_true",
                    help="plain: skip the mixed-batch section (config 3)")
    ap.add_argument("--no-served", action="store_true",
                    help="plain: skip the served section (config 4)")
    ap.add_argument("--served-pool", type=int, default=256,
                    help="plain: pool requests of the served section")
    ap.add_argument("--served-lambdas", default="3000,4000,5000,6000,7000",
                    help="plain: arrival rates of the served section")
    ap.add_argument("--served-duration", type=float, default=5.0,
                    help="plain: seconds of arrivals per rate of the served section")
    ap.add_argument("--no-calibrate", action="store_true",
                    help="skip the VALU / copy calibration kernels (the roofline then takes "
                         "the spec peak)")
    ap.add_argument("--no-device-encoded", action="store_true",
                    help="skip the device-encoded (encode + filter) measurement")
    ap.add_argument("--no-ft", action="store_true",
                    help="skip the host-to-host filter-time measurement")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 256 MiB device copy kernel first (counter calibration)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="target wall time of the CPU-baseline sample")
    ap.add_argument("--workload", choices=["plain", "mixed", "served", "sweep"],
                    default="plain",
                    help="plain: 100 bp, e=5 (the headline); mixed: 2^26 pairs of mixed "
                         "lengths and per-pair e, persistent launch vs one launch per "
                         "(length, e) group; served: Poisson request stream over a 3.1 Gbp "
                         "reference, batched server vs sequential per-request launches; "
                         "sweep: the plain launch at 100 bp for e = 0..10 and at 150 / 250 bp "
                         "for e = 2, 5, 10 %% of the length")
    ap.add_argument("--lambdas",
                    default="50,100,200,500,1000,2000,3000,3500,4000,4500,5000,6000,7000,8000",
                    help="served: arrival rates (requests/s)")
    ap.add_argument("--duration", type=float, default=20.0,
                    help="served: seconds of arrivals per rate and mode")
    ap.add_argument("--pool", type=int, default=1024,
                    help="served: distinct requests (each with the oracle's outputs)")
    ap.add_argument("--ref-len", type=int, default=3_100_000_000,
                    help="served: reference length")
    ap.add_argument("--slo-ms", type=float, default=25.0, help="served: p99 target")
    ap.add_argument("--served-modes", default="served,per_request",
                    help="served: which servers to run (served = batched, per_request)")
    ap.add_argument("--pageable", action="store_true",
                    help="served: keep requests in pageable host memory (default: pinned)")
    ap.add_argument("--tune-sample", type=int, default=1 << 26,
                    help="mixed: pairs the autotuner times each candidate on (the whole "
                         "batch by default: smaller samples have misranked close candidates)")
    ap.add_argument("--sweep-points", default=None,
                    help="sweep: 'm:e,m:e,...' instead of the default points (100 bp runs "
                         "config 1's generator, other lengths config 2's)")
    ap.add_argument("--mixed-config", default=None,
                    help="mixed: fixed tuning 'tile,ppl,sort_e,blocks_per_cu' instead of "
                         "the autotuner")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(pairs are independent: more GPUs would each filter "
                                   "their own share of the batch)"}))
        return 2

    import torch
    import gen
    from paper_2103_14978_amd import device, gk

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        return 1
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    m, e, n_pairs = 100, args.e, args.pairs

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    calib = None if args.no_calibrate else measure_peaks(log)

    if args.workload == "mixed":
        return bench_mixed(args, log, calib)
    if args.workload == "served":
        return bench_served(args, log)
    if args.workload == "sweep":
        return bench_sweep(args, log)

    t = time.time()
    ref = gen.c1_reference()
    ps = gen.c1_pairs(ref, e, n_pairs=n_pairs)
    log(f"generated reference + {ps.n_pairs} pairs in {time.time() - t:.1f}s")

    ctx = gk.gk_create(0)
    gk.gk_set_option(ctx, gk.GK_OPT_PAIRS_PER_LANE, args.pairs_per_lane)
    layout = gk.GK_READS_SPLIT if args.layout == "split" else gk.GK_READS_INTERLEAVED
    t = time.time()
    gk.gk_load_reference(ctx, ref)
    log(f"reference resident in {time.time() - t:.2f}s")
    dr = device.encode_reads(ctx, ps.reads, ps.read_off, max_len=m, layout=layout)
    # One candidate per read: pair i uses read i, which the batch states by
    # leaving pair_read NULL.
    identity = bool(np.array_equal(ps.pair_read, np.arange(n_pairs, dtype=np.uint32)))
    dp = device.upload_pairs(None if identity else ps.pair_read, ps.cand_pos, None,
                             with_bits=False)
    batch = device.batch_for(dr, dp, e_uniform=e, max_read_len=m)
    torch.cuda.synchronize()
    log("inputs resident")

    stream = torch.cuda.current_stream()
    if args.calibrate_copy:
        # An elementwise kernel reading 256 MiB and writing 256 MiB: the
        # reference point that scales the FETCH_SIZE / WRITE_SIZE counters.
        x = torch.ones(64 << 20, dtype=torch.int32, device=dev)
        y = torch.empty_like(x)
        torch.bitwise_xor(x, 0x55, out=y)
        torch.cuda.synchronize()
        del x, y
        log("copy calibration kernel: 268435456 bytes read, 268435456 bytes written")
    for _ in range(args.warmup):
        gk.gk_filter(ctx, batch, stream)
    torch.cuda.synchronize()

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        starts[i].record(stream)
        gk.gk_filter(ctx, batch, stream)
        ends[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = [s.elapsed_time(x) for s, x in zip(starts, ends)]
    k_avg_s = float(np.mean(kernel_ms)) / 1e3
    ms_per_step = wall * 1e3 / args.steps
    value = n_pairs * args.steps / wall
    log(f"{args.steps} steps in {wall:.4f}s; kernel avg {k_avg_s * 1e3:.4f} ms "
        f"(min {min(kernel_ms):.4f}, max {max(kernel_ms):.4f})")

    # Device-encoded kernel time (the paper's device-encoded rows of Table 2):
    # ASCII reads and their offsets resident in HBM, each run encodes them
    # (gk_encode_reads) and filters (gk_filter); mean of 10 runs.  The encode
    # kernel is also timed alone for its HBM roofline.
    dev_enc = None
    if not args.no_device_encoded:
        d_ascii = torch.from_numpy(np.ascontiguousarray(ps.reads)).to(dev)
        d_off = torch.from_numpy(ps.read_off.view(np.int64)).to(dev)
        rows = (m + 15) // 16
        packed2 = torch.full_like(dr.packed, -1)
        len2 = torch.full_like(dr.read_len, -1)
        hn2 = torch.full_like(dr.has_n, 0xFF)
        batch2 = gk.make_batch(n_reads=dr.n_reads, pitch=dr.pitch, max_read_len=m,
                               reads=packed2, read_len=len2, read_has_n=hn2,
                               n_pairs=n_pairs, pair_read=dp.pair_read, cand_pos=dp.cand_pos,
                               accept=dp.accept, est=dp.est, e_uniform=e, read_layout=layout)

        def enc():
            gk.gk_encode_reads(ctx, d_ascii, d_off, ps.n_reads, dr.pitch, rows, layout,
                               packed2, len2, hn2, stream)

        def enc_filter():
            enc()
            gk.gk_filter(ctx, batch2, stream)
        a_ref, s_ref = device.results(dp)
        enc_ms, enc_min, enc_med = events_ms(enc, 10, stream, warm=3, stats=True)
        ef_ms, ef_min, ef_med = events_ms(enc_filter, 10, stream, warm=3, stats=True)
        a2, s2 = device.results(dp)
        nr = ps.n_reads
        same_words = bool(torch.equal(packed2.view(rows, -1)[:, :nr],
                                      dr.packed.view(rows, -1)[:, :nr])
                          and torch.equal(len2[:nr], dr.read_len[:nr])
                          and torch.equal(hn2[:nr], dr.has_n[:nr]))
        res_mism = int(np.sum((a2 != a_ref) | (s2 != s_ref)))
        # The same work in one launch (gk_filter_ascii): the reads are encoded
        # into registers and never written to memory.
        fused = None
        if identity:
            batch3 = gk.make_batch(n_reads=0, pitch=0, max_read_len=m, reads=None,
                                   read_len=None, pair_read=None, cand_pos=dp.cand_pos,
                                   accept=dp.accept, est=dp.est, n_pairs=n_pairs, e_uniform=e)

            def fused_filter():
                gk.gk_filter_ascii(ctx, batch3, d_ascii, d_off, stream)
            dp.accept.fill_(0xEE)
            fu_ms, fu_min, fu_med = events_ms(fused_filter, 10, stream, warm=3, stats=True)
            a3, s3 = device.results(dp)
            fb = fused_bytes_per_pair(m)
            fu_gbs = fb * n_pairs / (fu_ms / 1e3) / 1e9
            fname = f"k_filter_ascii<{(rows + 1) // 2}"
            fhash = kernel_source_hash(FUSED_SOURCES)
            fprof = "k_filter_ascii_w4_config1_e5_counters.json"
            f_traffic = traffic_from_profile(fhash, n_pairs, fprof, kernel=fname)
            f_insts = traffic_from_profile(fhash, n_pairs, fprof, kernel=fname,
                                           field="valu_insts_per_launch")
            fused = {"pairs_per_s": round(n_pairs / (fu_ms / 1e3), 1),
                     "ms_per_step": round(fu_ms, 4), "ms_min": round(fu_min, 4),
                     "ms_median": round(fu_med, 4), "runs": 10,
                     "kernel": fname + ", false>",
                     "bytes_per_pair": fb, "achieved_gbs": round(fu_gbs, 1),
                     "hbm_frac": round(fu_gbs / HBM_PEAK_GBS, 4),
                     "traffic": f_traffic,
                     "traffic_GBs": (round(f_traffic / (fu_ms / 1e3) / 1e9, 1)
                                     if f_traffic else None),
                     "valu_issued_Tops": (round(f_insts * 64 / (fu_ms / 1e3) / 1e12, 3)
                                          if f_insts else None),
                     "kernel_source_hash": fhash,
                     "mismatches_vs_kernel_path": int(np.sum((a3 != a_ref) | (s3 != s_ref))),
                     "what": "gk_filter_ascii per run: ASCII reads encoded in the filter's "
                             "own launch, HIP events on the launch stream"}
            log(f"device-encoded fused: {fu_ms:.4f} ms "
                f"({n_pairs / (fu_ms / 1e3) / 1e9:.2f} G pairs/s, {fu_gbs:.0f} GB/s), "
                f"{fused['mismatches_vs_kernel_path']} result mismatches")
            del batch3
        eb = encode_bytes_per_read(m, rows) * ps.n_reads
        enc_gbs = eb / (enc_ms / 1e3) / 1e9
        dev_enc = {"pairs_per_s": round(n_pairs / (ef_ms / 1e3), 1),
                   "ms_per_step": round(ef_ms, 4), "ms_min": round(ef_min, 4),
                   "ms_median": round(ef_med, 4), "runs": 10,
                   "encode_ms": round(enc_ms, 4), "encode_ms_min": round(enc_min, 4),
                   "encode_ms_median": round(enc_med, 4),
                   "encode_roofline": {"bound": "hbm", "kernel": "k_encode_reads_staged",
                                       "achieved": round(enc_gbs, 1), "peak": HBM_PEAK_GBS,
                                       "unit": "GB/s", "frac": round(enc_gbs / HBM_PEAK_GBS, 4),
                                       "bytes_per_read": encode_bytes_per_read(m, rows)},
                   "fused": fused,
                   "words_identical_to_resident": same_words,
                   "mismatches_vs_kernel_path": res_mism,
                   "what": "ASCII reads + offsets resident in HBM: gk_encode_reads then "
                           "gk_filter per run, HIP events on the launch stream"}
        log(f"device-encoded: encode {enc_ms:.4f} ms ({enc_gbs:.0f} GB/s), encode+filter "
            f"{ef_ms:.4f} ms ({n_pairs / (ef_ms / 1e3) / 1e9:.2f} G pairs/s), words identical "
            f"{same_words}, "
            f"{res_mism} result mismatches")
        del d_ascii, d_off, packed2, len2, hn2, batch2

    # Parity on a random sample of this run's outputs (bit-exact); the CPU
    # baseline below widens it to every pair the oracle is timed on.
    parity = None
    if not args.no_parity:
        import oracle
        a_gpu, s_gpu = device.results(dp)
        rng = np.random.default_rng(12345)
        idx = np.sort(rng.choice(n_pairs, size=min(n_pairs, 1 << 15), replace=False))
        ra, rs = oracle.filter_batch(ps.reads, ps.read_off, ref, ps.pair_read[idx],
                                     ps.cand_pos[idx], e, n_threads=gen.default_threads())
        mism = int(np.sum((a_gpu[idx] != ra) | (s_gpu[idx] != rs)))
        parity = {"sampled_pairs": int(len(idx)), "mismatches": mism,
                  "accepted_frac": float(np.mean(a_gpu == 1))}
        log(f"parity sample: {mism} mismatches of {len(idx)}")

    # Verification of the accepted pairs (the step the filter exists to cut,
    # Sec. 3.5, Sec. 5.3): gk_verify after gk_filter, against gk_verify of
    # every pair with no filter.
    verify = None
    if not args.no_verify:
        dist = torch.empty(n_pairs, dtype=torch.int16, device=dev)

        def timed_ms(fn, k):
            return events_ms(fn, k, stream)
        vk = max(3, args.steps // 10)
        ms_after = timed_ms(lambda: gk.gk_verify(ctx, batch, dp.accept, dist, stream), vk)
        ms_fv = timed_ms(lambda: (gk.gk_filter(ctx, batch, stream),
                                  gk.gk_verify(ctx, batch, dp.accept, dist, stream)), vk)
        ms_all = timed_ms(lambda: gk.gk_verify(ctx, batch, None, dist, stream), vk)
        a_gpu, _ = device.results(dp)
        accepted = int(np.sum(a_gpu == gk.GK_ACCEPT))
        gk.gk_verify(ctx, batch, dp.accept, dist, stream)
        torch.cuda.synchronize()
        d_gpu = dist.cpu().numpy().view(np.uint16)
        vmism = None
        if not args.no_parity:
            import oracle
            acc_idx = np.nonzero(a_gpu == gk.GK_ACCEPT)[0]
            rng = np.random.default_rng(777)
            idx = np.sort(rng.choice(acc_idx, size=min(len(acc_idx), 1 << 14), replace=False))
            want = oracle.levenshtein_batch(ps.reads, ps.read_off, ref, ps.pair_read[idx],
                                            ps.cand_pos[idx], e, n_threads=gen.default_threads())
            vmism = int(np.sum(d_gpu[idx] != want))
        within = int(np.sum(d_gpu <= e))
        verify = {"accepted_pairs": accepted, "reduction": round(1 - accepted / n_pairs, 4),
                  "verified_within_e": within,
                  "verify_ms": round(ms_after, 4), "filter_plus_verify_ms": round(ms_fv, 4),
                  "verify_all_ms": round(ms_all, 4),
                  "filter_plus_verify_pairs_per_s": round(n_pairs / (ms_fv / 1e3), 1),
                  "speedup_vs_verify_all": round(ms_all / ms_fv, 3),
                  "sampled_mismatches": vmism,
                  "what": "banded bit-parallel edit distance (cap e+1) of the GK_ACCEPT pairs"}
        log(f"verify {ms_after:.3f} ms for {accepted} accepted pairs; filter+verify "
            f"{ms_fv:.3f} ms vs verify-all {ms_all:.3f} ms")
        del dist
        # Reads of several lengths under one e (trimmed reads, say): 2^21
        # pairs of 64/80/100/128 bp, every pair verified, beside 2^21 pairs of
        # 100 bp from the same generator.
        ml = {}
        for label, lengths in (("four_lengths", [64, 80, 100, 128]), ("one_length", [100])):
            mps = gen.pairs(ref, seed=4242, n_reads=320_000, lengths=lengths,
                            cand_kind=gen.CAND_GEOM, cand_param=1 / 8, cand_cap=64,
                            true_frac=0.5, edit_kind=gen.EDIT_RATE, edit_param=1.2, e_value=4,
                            band_cands=True).take_pairs(1 << 21)
            mdr = device.encode_reads(ctx, mps.reads, mps.read_off, max_len=128)
            mdp = device.upload_pairs(mps.pair_read, mps.cand_pos)
            mb = device.batch_for(mdr, mdp, e_uniform=4, max_read_len=128)
            mdist = torch.empty(mps.n_pairs, dtype=torch.int16, device=dev)
            torch.cuda.synchronize()
            ms_m = timed_ms(lambda: gk.gk_verify(ctx, mb, None, mdist, stream), vk)
            entry = {"pairs": int(mps.n_pairs), "verify_all_ms": round(ms_m, 4)}
            if not args.no_parity:
                import oracle
                gk.gk_verify(ctx, mb, None, mdist, stream)
                torch.cuda.synchronize()
                md = mdist.cpu().numpy().view(np.uint16)
                rng = np.random.default_rng(4243)
                idx = np.sort(rng.choice(mps.n_pairs, size=1 << 12, replace=False))
                want = oracle.levenshtein_batch(mps.reads, mps.read_off, ref,
                                                mps.pair_read[idx], mps.cand_pos[idx], 4,
                                                n_threads=gen.default_threads())
                entry["sampled_mismatches"] = int(np.sum(md[idx] != want))
            ml[label] = entry
            del mdist, mb, mdp, mdr
        verify["mixed_lengths"] = dict(ml, e=4, what="gk_verify of every pair")
        log(f"verify-all, four lengths {ml['four_lengths']['verify_all_ms']:.3f} ms, "
            f"one length {ml['one_length']['verify_all_ms']:.3f} ms (2^21 pairs)")

    # Filter time (Sec. 4.3): host ASCII reads and candidates in pinned host
    # memory -> gk_filter_host (chunked copies in, device encoding, filter,
    # copies out, overlapped on three streams) -> results in host memory.
    # PCIe-inclusive, so it is reported beside the kernel-time headline.
    ft = None
    if not args.no_ft:
        def pinned(a):
            t = torch.empty(max(a.nbytes, 1), dtype=torch.uint8, pin_memory=True)
            t.numpy()[:a.nbytes].view(a.dtype)[...] = a
            return t
        h_ascii, h_off, h_pos = pinned(ps.reads), pinned(ps.read_off), pinned(ps.cand_pos)
        h_pr = None if identity else pinned(ps.pair_read)
        h_acc = torch.empty(n_pairs, dtype=torch.uint8, pin_memory=True)
        h_est = torch.empty(2 * n_pairs, dtype=torch.uint8, pin_memory=True)

        def ft_step():
            gk.gk_filter_host(ctx, h_ascii, h_off, h_pos, h_acc, h_est, max_read_len=m,
                              e_uniform=e, n_reads=ps.n_reads, n_pairs=n_pairs,
                              pair_read=h_pr)
        ft_step()
        ft_steps = max(3, args.steps // 10)
        t = time.perf_counter()
        for _ in range(ft_steps):
            ft_step()
        ft_wall = (time.perf_counter() - t) / ft_steps
        a_dev, s_dev = device.results(dp)
        ft_mism = int(np.sum((h_acc.numpy() != a_dev) |
                             (h_est.numpy().view(np.uint16) != s_dev)))
        h2d = ps.reads.nbytes + ps.read_off.nbytes + ps.cand_pos.nbytes
        # The same batch with the reads host-encoded (the paper's host-encoded
        # mode): packed rows and lengths cross PCIe instead of ASCII.
        ft_packed = None
        fixed_len = bool(np.all(np.diff(ps.read_off) == m))
        if fixed_len:
            rows = (m + 15) // 16
            t = time.perf_counter()
            packed_np = host_encode_fixed(ps.reads, ps.n_reads, m, rows)
            enc_s = time.perf_counter() - t
            h_packed = pinned(packed_np)
            h_len = pinned(np.full(ps.n_reads, m, np.uint16))
            del packed_np

            def ftp_step():
                gk.gk_filter_host(ctx, None, None, h_pos, h_acc, h_est, max_read_len=m,
                                  e_uniform=e, n_reads=ps.n_reads, n_pairs=n_pairs,
                                  pair_read=h_pr, packed=h_packed, read_len=h_len)
            ftp_step()
            t = time.perf_counter()
            for _ in range(ft_steps):
                ftp_step()
            ftp_wall = (time.perf_counter() - t) / ft_steps
            ftp_mism = int(np.sum((h_acc.numpy() != a_dev) |
                                  (h_est.numpy().view(np.uint16) != s_dev)))
            h2d_p = ps.n_reads * rows * 4 + ps.n_reads * 2 + ps.cand_pos.nbytes
            ft_packed = {"pairs_per_s": round(n_pairs / ftp_wall, 1),
                         "ms_per_step": round(ftp_wall * 1e3, 3), "h2d_bytes": int(h2d_p),
                         "link_GBs": round((h2d_p + 3 * n_pairs) / ftp_wall / 1e9, 2),
                         "mismatches_vs_kernel_path": ftp_mism,
                         "host_encode_s_outside_timing": round(enc_s, 2)}
            log(f"filter time, host-encoded reads: {ftp_wall * 1e3:.2f} ms/batch "
                f"({n_pairs / ftp_wall / 1e6:.1f} M pairs/s), {ftp_mism} mismatches")
            del h_packed, h_len
        # The same ASCII batch with the reads encoded on host threads inside
        # gk_filter_host (GK_OPT_HOST_ENCODE_THREADS): 2-bit rows cross PCIe.
        enc_threads = gen.default_threads()
        gk.gk_set_option(ctx, gk.GK_OPT_HOST_ENCODE_THREADS, enc_threads)
        ft_step()
        t = time.perf_counter()
        for _ in range(ft_steps):
            ft_step()
        fth_wall = (time.perf_counter() - t) / ft_steps
        gk.gk_set_option(ctx, gk.GK_OPT_HOST_ENCODE_THREADS, 0)
        fth_mism = int(np.sum((h_acc.numpy() != a_dev) |
                              (h_est.numpy().view(np.uint16) != s_dev)))
        ft_host_threads = {"pairs_per_s": round(n_pairs / fth_wall, 1),
                           "ms_per_step": round(fth_wall * 1e3, 3), "threads": enc_threads,
                           "mismatches_vs_kernel_path": fth_mism}
        log(f"filter time, reads encoded on {enc_threads} host threads: "
            f"{fth_wall * 1e3:.2f} ms/batch ({n_pairs / fth_wall / 1e6:.1f} M pairs/s), "
            f"{fth_mism} mismatches")
        ft = {"pairs_per_s": round(n_pairs / ft_wall, 1), "ms_per_step": round(ft_wall * 1e3, 3),
              "steps": ft_steps, "h2d_bytes": int(h2d), "d2h_bytes": int(3 * n_pairs),
              "link_GBs": round((h2d + 3 * n_pairs) / ft_wall / 1e9, 2),
              "mismatches_vs_kernel_path": ft_mism,
              "what": "host ASCII reads + offsets + positions (pinned) to host results, "
                      "encoding on the GPU, chunks overlapped on three streams",
              "host_encoded": ft_packed, "host_encode_threads": ft_host_threads}
        log(f"filter time {ft_wall * 1e3:.2f} ms/batch ({n_pairs / ft_wall / 1e6:.1f} M pairs/s), "
            f"{ft_mism} mismatches vs the kernel path")
        del h_ascii, h_off, h_pos, h_pr, h_acc, h_est

    ops = ops_per_pair(m, e) * n_pairs
    achieved_tops = ops / k_avg_s / 1e12
    khash = kernel_source_hash()
    kname = plain_kernel_name((m + 31) // 32, e, args.pairs_per_lane)
    traffic = traffic_from_profile(khash, n_pairs, kernel=kname)
    valu_insts = traffic_from_profile(khash, n_pairs, kernel=kname,
                                      field="valu_insts_per_launch")
    peak = valu_peak(calib)
    # issued: the VALU instructions the counters saw per launch (x 64 lanes)
    # over the mean kernel time, against the same roof
    issued_tops = valu_insts * 64 / k_avg_s / 1e12 if valu_insts else None
    roofline = {"bound": "alu", "kernel": kname + ">", "achieved": round(achieved_tops, 3),
                "peak": round(peak, 3), "unit": "Tops/s",
                "frac": round(achieved_tops / peak, 4), "traffic": traffic,
                "issued": round(issued_tops, 3) if issued_tops else None,
                "issued_frac": round(issued_tops / peak, 4) if issued_tops else None,
                "peak_spec": round(VALU_PEAK_TOPS, 3),
                "peak_measured": calib["filter_mix_Tops"] if calib else None,
                "calibration": calib,
                "traffic_GBs": (round(traffic / k_avg_s / 1e9, 1) if traffic else None),
                "ops_per_pair": ops_per_pair(m, e), "kernel_ms": round(k_avg_s * 1e3, 4),
                "kernel_ms_min": round(float(np.min(kernel_ms)), 4),
                "kernel_ms_median": round(float(np.median(kernel_ms)), 4),
                "hbm_alg_GBs": round(bytes_per_pair(m) * n_pairs / k_avg_s / 1e9, 1),
                # what binds the launch in fact: the 128 B lines it fetches
                # (one per random window gather, plus the streamed reads)
                "line_rate": ({"lines_per_launch": int(traffic // 128),
                               "G_lines_per_s": round(traffic / 128 / k_avg_s / 1e9, 1),
                               "what": "counted traffic / 128 B over the mean kernel time; "
                                       "the random window gathers (one line per pair) hold "
                                       "the launch near 50 G lines/s"}
                              if traffic else None),
                "kernel_source_hash": khash}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        threads = gen.default_threads()
        cal = min(n_pairs, 1 << 15)
        t = time.perf_counter()
        oracle.filter_batch(ps.reads, ps.read_off, ref, ps.pair_read[:cal], ps.cand_pos[:cal], e,
                            n_threads=threads)
        rate = cal / max(time.perf_counter() - t, 1e-6)
        sample = int(min(n_pairs, max(cal, rate * args.cpu_seconds)))
        t = time.perf_counter()
        ra_all, rs_all = oracle.filter_batch(ps.reads, ps.read_off, ref, ps.pair_read[:sample],
                                             ps.cand_pos[:sample], e, n_threads=threads)
        dt = time.perf_counter() - t
        if parity is not None:
            a_gpu, s_gpu = device.results(dp)
            parity["all_pairs_checked"] = int(sample)
            parity["all_pairs_mismatches"] = int(np.sum((a_gpu[:sample] != ra_all) |
                                                        (s_gpu[:sample] != rs_all)))
        del ra_all, rs_all
        cpu = {"value": round(sample / dt, 1), "unit": "pairs/s", "cores": threads,
               "kind": "oracle",
               "sample": f"first {sample} pairs of the same batch, {threads} threads, "
                         f"{dt:.1f}s wall"}
        log(f"cpu baseline {sample / dt:.0f} pairs/s on {threads} threads")
        one = min(n_pairs, 1 << 18)
        t = time.perf_counter()
        oracle.filter_batch(ps.reads, ps.read_off, ref, ps.pair_read[:one], ps.cand_pos[:one], e,
                            n_threads=1)
        dt1 = time.perf_counter() - t
        cpu["one_core"] = {"value": round(one / dt1, 1), "unit": "pairs/s",
                           "sample": f"first {one} pairs, 1 thread, {dt1:.2f}s wall"}
        # Config 0 in full on one core (10,000 pairs of 100 bp, e = 2).
        ref0 = gen.c0_reference()
        ps0 = gen.c0_pairs(ref0)
        t = time.perf_counter()
        oracle.filter_batch(ps0.reads, ps0.read_off, ref0, ps0.pair_read, ps0.cand_pos, 2,
                            n_threads=1)
        dt0 = time.perf_counter() - t
        cpu["one_core_config0"] = {"value": round(ps0.n_pairs / dt0, 1), "unit": "pairs/s",
                                   "sample": f"config 0 in full ({ps0.n_pairs} pairs, e=2), "
                                             f"1 thread, {dt0 * 1e3:.1f} ms wall"}
        cpu["host_cpu"] = host_cpu_model()

    # The two added rows, measured in the same run: the mixed batch
    # (persistent launch vs one launch per (length, e) group) and the served
    # form (batched server vs per-request launches, p50/p99 latency).
    del dr, dp, batch
    torch.cuda.empty_cache()
    mixed = None
    if not args.no_mixed:
        mixed = mixed_section(args, log, calib)
        torch.cuda.empty_cache()
    served = None
    if not args.no_served:
        served = served_section(args, log, args.served_pool,
                                [float(x) for x in args.served_lambdas.split(",")],
                                args.served_duration)
    slo = served["served_at_slo"] if served else None

    out = {
        "metric": "filtered pairs/sec (100bp, e=5) on 1 MI355X, bit-exact; p99 request latency",
        "value": round(value, 1), "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"plain filter, {n_pairs} pairs of {m}bp reads, e={e}, "
                               "100 Mbp GC-41% reference, 30% true / 70% 12-mer decoys, "
                               "reads 2-bit packed transposed (16 bases per u32)",
                   "pairs_per_step": n_pairs, "read_len": m, "e": e,
                   "read_layout": args.layout, "pairs_per_lane": args.pairs_per_lane},
        "kernel_pairs_per_s": round(n_pairs / k_avg_s, 1),
        "p99_request_latency_ms": slo["p99_ms"] if slo else None,
        "p99_at": (f"served form at {slo['lambda']:.0f} requests/s, "
                   f"{slo['pairs_per_s'] / 1e6:.1f} M pairs/s (the highest rate with p99 <= "
                   f"{args.slo_ms:g} ms)") if slo else None,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "device_encoded": dev_enc,
        "filter_time": ft,
        "verification": verify,
        "parity": parity,
        "mixed": mixed,
        "served": served,
    }
    print(json.dumps(out), flush=True)
    gk.gk_destroy(ctx)
    return 0


def sweep_bytes_per_pair(m: int, cands_per_read: float) -> float:
    """Algorithmic bytes per pair when a read serves cands_per_read pairs: the
    window (m/4 B), the packed read and its length shared by its candidates,
    read index + position (8 B), accept + est (3 B)."""
    return m / 4 + (m / 4 + 2) / cands_per_read + 8 + 3


def bench_sweep(args, log) -> int:
    """The plain launch across thresholds and read lengths (the paper's Sec. 5
    sweeps of e and m): 2^24 pairs of 100 bp for each e in 0..10, and 2^25
    pairs at 150 bp (e = 3, 7, 15) and 250 bp (e = 5, 12, 25) with several
    candidates per read.  Per point: kernel time from HIP events on the launch
    stream, the VALU-roof fraction of the algorithmic op count, the
    algorithmic HBM rate, a sampled bit-exact check against the oracle, and
    the time to verify the accepted pairs (gk_verify) with sampled distances
    checked against the oracle's."""
    import torch
    import gen
    import oracle
    from paper_2103_14978_amd import device, gk

    ref = gen.c1_reference()
    ctx = gk.gk_create(0)
    gk.gk_set_option(ctx, gk.GK_OPT_PAIRS_PER_LANE, args.pairs_per_lane)
    gk.gk_load_reference(ctx, ref)
    stream = torch.cuda.current_stream()
    steps = max(3, min(args.steps, 20))
    points = [(100, e) for e in range(11)] + [(150, 3), (150, 7), (150, 15),
                                              (250, 5), (250, 12), (250, 25)]
    if args.sweep_points:
        points = [tuple(int(v) for v in pt.split(":")) for pt in args.sweep_points.split(",")]
    rows, headline = [], None
    for m, e in points:
        t = time.time()
        ps = gen.c1_pairs(ref, e) if m == 100 else gen.c2_pairs(ref, m, e)
        n = ps.n_pairs
        identity = bool(ps.n_reads == n and
                        np.array_equal(ps.pair_read, np.arange(n, dtype=np.uint32)))
        dr = device.encode_reads(ctx, ps.reads, ps.read_off, max_len=m)
        dp = device.upload_pairs(None if identity else ps.pair_read, ps.cand_pos, None)
        batch = device.batch_for(dr, dp, e_uniform=e, max_read_len=m)
        for _ in range(3):
            gk.gk_filter(ctx, batch, stream)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
        t0 = time.perf_counter()
        for a0, a1 in ev:
            a0.record(stream)
            gk.gk_filter(ctx, batch, stream)
            a1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kms = [a0.elapsed_time(a1) for a0, a1 in ev]
        k_s = float(np.mean(kms)) / 1e3
        a_gpu, s_gpu = device.results(dp)
        rng = np.random.default_rng(4321 + m + e)
        idx = np.sort(rng.choice(n, size=min(n, 1 << 13), replace=False))
        ra, rs = oracle.filter_batch(ps.reads, ps.read_off, ref, ps.pair_read[idx],
                                     ps.cand_pos[idx], e, n_threads=gen.default_threads())
        mism = int(np.sum((a_gpu[idx] != ra) | (s_gpu[idx] != rs)))
        # Verification of this point's accepted pairs (gk_verify after the
        # filter), with sampled distances against the oracle's.
        dist = torch.empty(n, dtype=torch.int16, device="cuda")
        gk.gk_verify(ctx, batch, dp.accept, dist, stream)
        torch.cuda.synchronize()
        vev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(5)]
        for a0, a1 in vev:
            a0.record(stream)
            gk.gk_verify(ctx, batch, dp.accept, dist, stream)
            a1.record(stream)
        torch.cuda.synchronize()
        v_ms = float(np.mean([a0.elapsed_time(a1) for a0, a1 in vev]))
        d_gpu = dist.cpu().numpy().view(np.uint16)
        acc_idx = np.nonzero(a_gpu == gk.GK_ACCEPT)[0]
        vidx = np.sort(rng.choice(acc_idx, size=min(len(acc_idx), 1 << 11), replace=False))
        if e <= gk.GK_VERIFY_MAX_E:
            want = oracle.levenshtein_batch(ps.reads, ps.read_off, ref, ps.pair_read[vidx],
                                            ps.cand_pos[vidx], e,
                                            n_threads=gen.default_threads())
        else:   # beyond the verification's band: GK_EST_NONE by contract
            want = np.full(len(vidx), gk.GK_EST_NONE, np.uint16)
        vmism = int(np.sum(d_gpu[vidx] != want))
        del dist
        words = (m + 31) // 32
        cpr = n / ps.n_reads
        tops = ops_per_pair(m, e) * n / k_s / 1e12
        row = {"read_len": m, "e": e, "pairs": int(n), "reads": int(ps.n_reads),
               "kernel": plain_kernel_name(words, e, args.pairs_per_lane) + ">",
               "kernel_ms": round(k_s * 1e3, 4), "kernel_ms_min": round(min(kms), 4),
               "kernel_ms_median": round(float(np.median(kms)), 4),
               "kernel_pairs_per_s": round(n / k_s, 1), "wall_pairs_per_s": round(n * steps / wall, 1),
               "ops_per_pair": ops_per_pair(m, e),
               "valu_frac": round(tops / VALU_PEAK_TOPS, 4),
               "alg_bytes_per_pair": round(sweep_bytes_per_pair(m, cpr), 2),
               "hbm_alg_GBs": round(sweep_bytes_per_pair(m, cpr) * n / k_s / 1e9, 1),
               "accepted_frac": round(float(np.mean(a_gpu == gk.GK_ACCEPT)), 4),
               "sampled_pairs": int(len(idx)), "mismatches": mism,
               "verify_ms": round(v_ms, 4), "verified_pairs": int(len(acc_idx)),
               "verify_pairs_per_s": round(len(acc_idx) / (v_ms / 1e3), 1),
               "verify_sampled": int(len(vidx)), "verify_mismatches": vmism}
        rows.append(row)
        if (m, e) == (100, 5):
            headline = (row, steps, wall)
        log(f"{m} bp e={e}: {k_s * 1e3:.4f} ms, {n / k_s / 1e9:.2f} G pairs/s, "
            f"VALU {row['valu_frac']:.3f}, {mism} mismatches of {len(idx)}; verify "
            f"{v_ms:.4f} ms for {len(acc_idx)} accepted, {vmism} mismatches "
            f"({time.time() - t:.1f}s)")
        del batch, dp, dr, ps
        torch.cuda.empty_cache()
    row, hsteps, hwall = headline if headline else (rows[0], steps, float("nan"))
    out = {
        "metric": "filtered pairs/sec (100bp, e=5) on 1 MI355X, bit-exact",
        "value": row["wall_pairs_per_s"] if headline else None, "unit": "pairs/s",
        "n_gpus": 1, "steps": hsteps,
        "warmup": 3, "ms_per_step": round(hwall * 1e3 / hsteps, 4) if headline else None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "plain filter sweep: 2^24 pairs of 100 bp for e = 0..10, "
                               "2^25 pairs at 150 bp (e = 3, 7, 15) and 250 bp (e = 5, 12, 25), "
                               "100 Mbp GC-41% reference",
                   "pairs_per_lane": args.pairs_per_lane},
        "roofline": {"bound": "alu", "kernel": row["kernel"],
                     "achieved": round(row["valu_frac"] * VALU_PEAK_TOPS, 3),
                     "peak": round(VALU_PEAK_TOPS, 3), "unit": "Tops/s",
                     "frac": row["valu_frac"], "traffic": None},
        "cpu_baseline": None,
        "sweep": rows,
    }
    print(json.dumps(out), flush=True)
    gk.gk_destroy(ctx)
    return 0


def mixed_section(args, log, calib=None, n_pairs: int = 1 << 26) -> dict:
    """Mixed batch: 2^26 pairs, read length uniform over {64, 100, 150, 200,
    250, 300}, per-pair e uniform over 0..floor(0.1 m), Zipf(1.5) candidates
    per read.  The persistent launch (gk_filter_mixed, autotuned, replayed
    from its hipGraph) against one plain launch per (length, e) group issued
    back-to-back on the same stream, the paper's compile-time design point."""
    import torch
    import gen
    from paper_2103_14978_amd import device, gk

    t = time.time()
    ref = gen.c1_reference()
    ps = gen.c3_pairs(ref, n_pairs=n_pairs)
    n_pairs = ps.n_pairs
    log(f"generated {n_pairs} mixed pairs ({ps.n_reads} reads) in {time.time() - t:.1f}s")
    m_pair = ps.read_len[ps.pair_read].astype(np.int64)
    e_pair = ps.e.astype(np.int64)

    ctx = gk.gk_create(0)
    gk.gk_load_reference(ctx, ref)
    dr = device.encode_reads(ctx, ps.reads, ps.read_off, max_len=300)
    dp = device.upload_pairs(ps.pair_read, ps.cand_pos, ps.e)
    batch = device.batch_for(dr, dp, max_read_len=300)
    stream = torch.cuda.current_stream()

    # Grouped baseline: pairs reordered by (length, e) once on the host,
    # outside the timed region; one gk_filter per group.
    key = m_pair * 256 + e_pair
    order = np.argsort(key, kind="stable")
    sk = key[order]
    bounds = np.flatnonzero(np.diff(sk)) + 1
    starts = np.concatenate([[0], bounds])
    ends = np.concatenate([bounds, [n_pairs]])
    dpg = device.upload_pairs(ps.pair_read[order], ps.cand_pos[order], None)
    groups = []
    for a0, a1 in zip(starts, ends):
        gm, ge = int(sk[a0] // 256), int(sk[a0] % 256)
        b = device.batch_for(dr, dpg, e_uniform=ge, max_read_len=gm)
        b.n_pairs = int(a1 - a0)
        b.pair_read = dpg.pair_read.data_ptr() + 4 * int(a0)
        b.cand_pos = dpg.cand_pos.data_ptr() + 4 * int(a0)
        b.accept = dpg.accept.data_ptr() + int(a0)
        b.est = dpg.est.data_ptr() + 2 * int(a0)
        groups.append(b)
    torch.cuda.synchronize()
    log(f"{len(groups)} (length, e) groups")

    if args.calibrate_copy:
        x = torch.ones(64 << 20, dtype=torch.int32, device="cuda")
        y = torch.empty_like(x)
        torch.bitwise_xor(x, 0x55, out=y)
        torch.cuda.synchronize()
        del x, y
        log("copy calibration kernel: 268435456 bytes read, 268435456 bytes written")
    t = time.time()
    if args.mixed_config:
        tile, ppl, sort_e, bpc = (int(v) for v in args.mixed_config.split(","))
        for opt, val in ((gk.GK_OPT_MIXED_TILE, tile), (gk.GK_OPT_MIXED_PAIRS_PER_LANE, ppl),
                         (gk.GK_OPT_MIXED_SORT_E, sort_e), (gk.GK_OPT_MIXED_BLOCKS_PER_CU, bpc)):
            gk.gk_set_option(ctx, opt, val)
        report = {"tile": tile, "ppl": ppl, "sort_e": sort_e, "blocks_per_cu": bpc,
                  "ms": None, "source": "fixed"}
    else:
        report = json.loads(gk.gk_tune_mixed(ctx, batch, stream, sample_pairs=args.tune_sample))
    log(f"tuning ({report.get('source')}) in {time.time() - t:.2f}s: tile {report['tile']} "
        f"ppl {report['ppl']} sort_e {report['sort_e']} blocks/CU {report['blocks_per_cu']}")

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
        t0 = time.perf_counter()
        for a, b in ev:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return wall, float(np.mean([a.elapsed_time(b) for a, b in ev])) / 1e3

    steps, warmup = max(3, args.steps // 5), max(1, args.warmup)
    wall_m, k_m = timed(lambda: gk.gk_filter_mixed(ctx, batch, stream), steps, warmup)
    wall_g, k_g = timed(lambda: [gk.gk_filter(ctx, b, stream) for b in groups], steps, warmup)
    log(f"mixed {k_m * 1e3:.3f} ms/batch, grouped {k_g * 1e3:.3f} ms/batch "
        f"({len(groups)} launches)")

    # Both forms give the same bytes on every pair, and match the oracle on a sample.
    a_m, s_m = device.results(dp)
    a_g = np.empty_like(a_m)
    s_g = np.empty_like(s_m)
    ag, sg = device.results(dpg)
    a_g[order], s_g[order] = ag, sg
    same = int(np.sum((a_m != a_g) | (s_m != s_g)))
    parity = {"mixed_vs_grouped_mismatches": same}
    if not args.no_parity:
        import oracle
        rng = np.random.default_rng(7)
        idx = np.sort(rng.choice(n_pairs, size=min(n_pairs, 1 << 15), replace=False))
        ra, rs = oracle.filter_batch(ps.reads, ps.read_off, ref, ps.pair_read[idx],
                                     ps.cand_pos[idx], ps.e[idx], n_threads=gen.default_threads())
        parity.update(sampled_pairs=int(len(idx)),
                      mismatches=int(np.sum((a_m[idx] != ra) | (s_m[idx] != rs))))
    # Verification of this batch's accepted pairs (mixed lengths, per-pair e),
    # with sampled parity against the oracle's capped edit distance.
    vmix = None
    if not args.no_verify:
        vdist = torch.empty(n_pairs, dtype=torch.int16, device="cuda")
        _, k_v = timed(lambda: gk.gk_verify(ctx, batch, dp.accept, vdist, stream), steps, 1)
        acc_idx = np.nonzero(a_m == gk.GK_ACCEPT)[0]
        vmix = {"accepted_pairs": int(len(acc_idx)), "verify_ms": round(k_v * 1e3, 4),
                "accepted_pairs_per_s": round(len(acc_idx) / k_v, 1)}
        if not args.no_parity:
            import oracle
            vd = vdist.cpu().numpy().view(np.uint16)
            rng = np.random.default_rng(8)
            idx = np.sort(rng.choice(acc_idx, size=min(len(acc_idx), 1 << 14), replace=False))
            vm = 0
            for ev in np.unique(ps.e[idx]):
                sub = idx[ps.e[idx] == ev]
                want = oracle.levenshtein_batch(ps.reads, ps.read_off, ref, ps.pair_read[sub],
                                                ps.cand_pos[sub], int(ev),
                                                n_threads=gen.default_threads())
                vm += int(np.sum(vd[sub] != want))
            vmix.update(sampled_pairs=int(len(idx)), sampled_mismatches=vm)
        log(f"verify of {len(acc_idx)} accepted pairs: {k_v * 1e3:.3f} ms")
        del vdist
    w = (m_pair + 31) // 32
    ops = int(np.sum(14 * (2 * np.minimum(e_pair, m_pair - 1) + 1) * w + 6 * w + 16))
    achieved = ops / k_m / 1e12
    mhash = kernel_source_hash(("gk_mixed.hip", "gk_pair.h", "gk_args.h"))
    tuning = [report["tile"], report["ppl"], report["sort_e"], report["blocks_per_cu"]]
    mtraffic = traffic_from_profile(mhash, n_pairs, "k_mixed_w10_config3_counters.json",
                                    tuning=tuning)
    m_insts = traffic_from_profile(mhash, n_pairs, "k_mixed_w10_config3_counters.json",
                                   tuning=tuning, field="valu_insts_per_launch")
    peak = valu_peak(calib)
    # issued: the mixed kernel's VALU instructions per launch (x 64 lanes) from
    # the committed counters, over the mean kernel time
    m_issued = m_insts * 64 / k_m / 1e12 if m_insts else None
    out = {
        "workload": f"mixed batch, {n_pairs} pairs, read length uniform over "
                    "{64,100,150,200,250,300}, e uniform 0..floor(0.1 m) per pair, "
                    "Zipf(1.5) candidates per read (<= 1024), 100 Mbp GC-41% reference",
        "pairs_per_step": n_pairs, "steps": steps, "warmup": warmup,
        "pairs_per_s": round(n_pairs * steps / wall_m, 1),
        "ms_per_step": round(wall_m * 1e3 / steps, 4),
        "mixed_kernel_pairs_per_s": round(n_pairs / k_m, 1),
        "grouped": {"launches": len(groups), "pairs_per_s": round(n_pairs * steps / wall_g, 1),
                    "kernel_pairs_per_s": round(n_pairs / k_g, 1),
                    "ms_per_step": round(wall_g * 1e3 / steps, 4)},
        "speedup_vs_grouped": round(wall_g / wall_m, 3),
        "autotune": {k: report.get(k) for k in ("source", "tile", "ppl", "sort_e",
                                                 "blocks_per_cu", "ms")},
        "roofline": {"bound": "alu", "kernel": "k_mixed<10>", "achieved": round(achieved, 3),
                     "peak": round(peak, 3), "unit": "Tops/s",
                     "frac": round(achieved / peak, 4), "traffic": mtraffic,
                     "issued": round(m_issued, 3) if m_issued else None,
                     "issued_frac": round(m_issued / peak, 4) if m_issued else None,
                     "traffic_GBs": (round(mtraffic / k_m / 1e9, 1) if mtraffic else None),
                     "ops_per_pair_mean": round(ops / n_pairs, 1),
                     "kernel_ms": round(k_m * 1e3, 4), "kernel_source_hash": mhash},
        "parity": parity,
        "verification": vmix,
    }
    gk.gk_destroy(ctx)
    return out


def bench_mixed(args, log, calib=None) -> int:
    n_pairs = args.pairs if args.pairs != (1 << 24) else (1 << 26)
    sec = mixed_section(args, log, calib, n_pairs)
    out = {"metric": "filtered pairs/sec, mixed batch (lengths 64-300, per-pair e), 1 MI355X, "
                     "bit-exact",
           "value": sec["pairs_per_s"], "unit": "pairs/s", "n_gpus": 1, "steps": sec["steps"],
           "warmup": sec["warmup"], "ms_per_step": sec["ms_per_step"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
           "config": {"workload": sec["workload"], "pairs_per_step": n_pairs}}
    out.update(sec)
    print(json.dumps(out), flush=True)
    return 0


class _PoolEntry:
    pass


def loadgen_lib():
    """libgk_loadgen.so (the native open-loop client) with its ctypes types."""
    import ctypes
    from paper_2103_14978_amd import build as hipbuild
    if not os.path.exists(hipbuild.LOADGEN_LIB):
        raise ImportError(f"{hipbuild.LOADGEN_LIB} is missing: build the package first")
    vp, u32, u64, i64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64

    class PoolEntry(ctypes.Structure):
        _fields_ = [("reads", vp), ("read_off", vp), ("n_reads", u32), ("e", u32),
                    ("pair_read", vp), ("cand_pos", vp), ("n_pairs", u64),
                    ("want_accept", vp), ("want_est", vp)]

    class RunArgs(ctypes.Structure):
        _fields_ = [("srv", vp), ("pool", ctypes.POINTER(PoolEntry)), ("n_pool", u32),
                    ("n_slots", u32), ("slot_pairs", u64), ("ring_accept", vp),
                    ("ring_est", vp), ("n_sub", u64), ("arrival_us", vp), ("which", vp),
                    ("deadline_us", i64), ("t_start_us", i64)]
    L = ctypes.CDLL(hipbuild.LOADGEN_LIB)
    L.gkl_run.argtypes = [ctypes.POINTER(RunArgs), vp]
    L.gkl_run.restype = ctypes.c_int
    return L, PoolEntry, RunArgs


# gkl_sub_result, 64 bytes
SUB_RESULT = np.dtype([("status", "<i4"), ("submit_status", "<i4"), ("t_arrival_us", "<i8"),
                       ("t_submit_us", "<i8"), ("t_admit_us", "<i8"), ("t_done_us", "<i8"),
                       ("n_pairs", "<u8"), ("mismatches", "<u8"), ("checked", "<u4"),
                       ("slot", "<u4")])


def served_section(args, log, pool_size: int, lambdas, duration: float,
                   warm_s: float = 1.5, lead: float = 0.5) -> dict:
    """Served form (config 4): a device-resident 3.1 Gbp reference; a pool of
    requests of 10^3 to 10^6 pairs (log-uniform), each with one read length
    in 100..250 and its own e; open-loop Poisson arrivals submitted by a
    native client thread (libgk_loadgen).  Latency = results in host memory
    minus the scheduled arrival, so queueing counts.  Every submission's own
    output buffer (from a bounded ring, sentinel-filled) is checked against
    the oracle's outputs for its pool request.  The batched server against
    the sequential per-request form (copy in, launch, copy out, one request
    at a time on one stream)."""
    import ctypes
    import torch
    import gen
    import oracle
    from paper_2103_14978_amd import gk

    t = time.time()
    ref = gen.c4_reference(args.ref_len)
    log(f"served: reference {len(ref)} bp generated in {time.time() - t:.1f}s")
    ctx = gk.gk_create(0)
    t = time.time()
    gk.gk_load_reference(ctx, ref)
    log(f"served: reference resident in {time.time() - t:.1f}s")
    t = time.time()
    pool = [gen.c4_request(ref, k) for k in range(pool_size)]
    pool_pairs = np.array([ps.n_pairs for ps in pool], dtype=np.float64)
    log(f"served: {len(pool)} requests generated in {time.time() - t:.1f}s, "
        f"{pool_pairs.sum():.0f} pairs, mean {pool_pairs.mean():.0f}")
    # The oracle's outputs for every pool request, computed once: every
    # submission of a request is checked against them.
    t = time.time()
    want = [oracle.filter_batch(ps.reads, ps.read_off, ref, ps.pair_read, ps.cand_pos,
                                ps.meta["e"], n_threads=gen.default_threads()) for ps in pool]
    oracle_s = time.time() - t
    log(f"served: oracle outputs of the pool in {oracle_s:.1f}s")
    del ref

    keep = []

    def pinned_view(a):
        """a copied into pinned host memory, as a numpy view of it."""
        tt = torch.empty(max(a.nbytes, 1), dtype=torch.uint8, pin_memory=not args.pageable)
        keep.append(tt)
        v = tt.numpy()[:a.nbytes].view(a.dtype)
        v[...] = a
        return v

    L, PoolEntry, RunArgs = loadgen_lib()
    entries = (PoolEntry * len(pool))()
    for k, ps in enumerate(pool):
        ps.reads, ps.read_off = pinned_view(ps.reads), pinned_view(ps.read_off)
        ps.cand_pos, ps.pair_read = pinned_view(ps.cand_pos), pinned_view(ps.pair_read)
        ra, rs = np.ascontiguousarray(want[k][0]), np.ascontiguousarray(want[k][1])
        keep.extend([ra, rs])
        en = entries[k]
        en.reads, en.read_off = ps.reads.ctypes.data, ps.read_off.ctypes.data
        en.n_reads, en.e = ps.n_reads, ps.meta["e"]
        en.pair_read, en.cand_pos = ps.pair_read.ctypes.data, ps.cand_pos.ctypes.data
        en.n_pairs = ps.n_pairs
        en.want_accept, en.want_est = ra.ctypes.data, rs.ctypes.data
    # Output ring: one buffer per submission in flight (server slots plus a
    # backlog of as many again), pinned, allocated once.
    max_slots = 128
    n_ring = 2 * max_slots
    slot_pairs = int(pool_pairs.max())
    ring_acc = pinned_view(np.zeros(n_ring * slot_pairs, np.uint8))
    ring_est = pinned_view(np.zeros(n_ring * slot_pairs, np.uint16))
    budget = 8 << 30

    def run_rate(mode, lam, dur, seed, lead=0.0):
        """lead + dur seconds of arrivals at lam on a fresh server; the first
        lead seconds warm it (their submissions are left out of the
        figures)."""
        srv = gk.gk_server_start(ctx, budget, max_slots, 256, mode)
        rng = np.random.default_rng(seed)
        n_req = max(20, int(lam * (dur + lead)))
        gaps = rng.exponential(1.0 / lam, n_req)
        which = rng.integers(0, len(pool), n_req).astype(np.uint32)
        arrivals = (np.cumsum(gaps) * 1e6).astype(np.int64)     # after the start
        deadline = int(arrivals[-1]) + 10_000_000
        res = np.zeros(n_req, SUB_RESULT)
        ra = RunArgs(srv=srv.value, pool=entries, n_pool=len(pool), n_slots=n_ring,
                     slot_pairs=slot_pairs, ring_accept=ring_acc.ctypes.data,
                     ring_est=ring_est.ctypes.data, n_sub=n_req,
                     arrival_us=arrivals.ctypes.data, which=which.ctypes.data,
                     deadline_us=deadline)
        st = L.gkl_run(ctypes.byref(ra), res.ctypes.data)
        t0 = ra.t_start_us
        ticks = gk.gk_server_tick_log(srv) if mode == gk.GK_SERVER_BATCHED else []
        n_ticks, per_tick, _ = gk.gk_server_counters(srv)
        gk.gk_server_stop(srv)       # after this no copy touches the ring
        if st != 0:
            raise RuntimeError(f"gkl_run failed: {st}")
        return res, t0, ticks, n_ticks, per_tick

    def summarise(res, t0, ticks, n_ticks, per_tick, lam, dur, lead=0.0):
        # only the submissions (and ticks) after the warm-up lead
        t0 = t0 + int(lead * 1e6)
        res = res[res["t_arrival_us"] >= t0]
        if ticks:
            ticks = [x for x in ticks if x.t_launch_us >= t0]
            n_ticks = len(ticks)
            per_tick = max((x.n_requests for x in ticks), default=0)
        ok = res["status"] == gk.GK_OK
        lat = (res["t_done_us"][ok] - res["t_arrival_us"][ok]) / 1e3
        unfinished = int(np.sum(~ok))
        lat_all = np.concatenate([lat, np.full(unfinished, np.inf)])

        def pct(v, q):
            x = float(np.percentile(v, q)) if len(v) else float("nan")
            return round(x, 3) if np.isfinite(x) else None
        done_pairs = float(np.sum(res["n_pairs"][ok]))
        end = int(res["t_done_us"][ok].max()) if ok.any() else t0
        span = max(end - t0, 1) / 1e6
        rec = {"lambda": lam, "requests": int(len(res)), "unfinished": unfinished,
               "p50_ms": pct(lat_all, 50), "p99_ms": pct(lat_all, 99),
               "p999_ms": pct(lat_all, 99.9),
               "max_ms": round(float(lat.max()), 3) if len(lat) else None,
               "pairs_per_s": round(done_pairs / span, 1),
               "checked_submissions": int(np.sum(res["checked"][ok])),
               "mismatched_submissions": int(np.sum(res["mismatches"] > 0)),
               "mismatched_pairs": int(np.sum(res["mismatches"])),
               "submit_lag_p99_ms": pct((res["t_submit_us"][ok] - res["t_arrival_us"][ok])
                                        / 1e3, 99),
               "admit_wait_p99_ms": pct((res["t_admit_us"][ok] - res["t_arrival_us"][ok])
                                        / 1e3, 99),
               "service_p99_ms": pct((res["t_done_us"][ok] - res["t_admit_us"][ok]) / 1e3, 99),
               "ticks": n_ticks, "max_requests_per_tick": per_tick}
        if ticks:
            tk = np.array([(x.t_launch_us, x.t_kernel_done_us, x.t_done_us, x.n_requests,
                            x.n_pairs) for x in ticks], dtype=np.int64)
            kern = (tk[:, 1] - tk[:, 0]) / 1e3
            gaps = np.diff(tk[:, 0]) / 1e3 if len(tk) > 1 else np.zeros(1)
            rec["tick"] = {"kernel_p50_ms": pct(kern, 50),
                           "kernel_p99_ms": pct(kern, 99),
                           "kernel_max_ms": round(float(kern.max()), 3),
                           "copy_out_p99_ms": pct((tk[:, 2] - tk[:, 1]) / 1e3, 99),
                           "copy_out_max_ms": round(float((tk[:, 2] - tk[:, 1]).max() / 1e3), 3),
                           "launch_gap_max_ms": round(float(gaps.max()), 3),
                           "pairs_p50": pct(tk[:, 4], 50), "pairs_max": int(tk[:, 4].max()),
                           "requests_p50": pct(tk[:, 3], 50),
                           # the first ticks: launch (ms after the timed
                           # start), kernel ms, pairs
                           "first": [[round((int(x[0]) - t0) / 1e3, 2),
                                      round((int(x[1]) - int(x[0])) / 1e3, 3), int(x[4])]
                                     for x in tk[:12]]}
        # The slowest submissions: where their time went, and what the
        # server's ticks did while the slowest one was in service.
        if ok.any():
            idx = np.nonzero(ok)[0]
            order = idx[np.argsort(lat)[::-1][:8]]
            rec["slowest"] = [
                {"arrival_ms": round((int(res["t_arrival_us"][i]) - t0) / 1e3, 3),
                 "latency_ms": round((int(res["t_done_us"][i]) - int(res["t_arrival_us"][i]))
                                     / 1e3, 3),
                 "admit_wait_ms": round((int(res["t_admit_us"][i]) -
                                         int(res["t_arrival_us"][i])) / 1e3, 3),
                 "n_pairs": int(res["n_pairs"][i])} for i in order]
            if ticks:
                i = order[0]
                a0, a1 = int(res["t_admit_us"][i]), int(res["t_done_us"][i])
                win = (tk[:, 0] >= a0) & (tk[:, 0] <= a1)
                if win.any():
                    w = tk[win]
                    rec["slowest_window"] = {
                        "ticks": int(win.sum()), "pairs": int(w[:, 4].sum()),
                        "parts": int(w[:, 3].sum()),
                        "kernel_max_ms": round(float((w[:, 1] - w[:, 0]).max() / 1e3), 3),
                        "copy_out_max_ms": round(float((w[:, 2] - w[:, 1]).max() / 1e3), 3)}
        return rec

    results = {"served": [], "per_request": []}
    modes = [m for m in (("served", gk.GK_SERVER_BATCHED),
                         ("per_request", gk.GK_SERVER_SEQUENTIAL))
             if m[0] in getattr(args, "served_modes", "served,per_request").split(",")]
    for mode_name, mode in modes:
        results[mode_name] = []
        saturated = False
        # An untimed first round at a moderate rate warms the server's first
        # ticks and the client, so the recorded rates measure the steady state.
        run_rate(mode, 1000.0, warm_s, 99 + mode)
        for lam in lambdas:
            if saturated:
                results[mode_name].append({"lambda": lam, "skipped": "saturated at a lower rate"})
                continue
            res, t0, ticks, n_ticks, per_tick = run_rate(mode, lam, duration,
                                                          int(lam) * 7 + mode, lead)
            rec = summarise(res, t0, ticks, n_ticks, per_tick, lam, duration, lead)
            saturated = rec["unfinished"] > 0
            results[mode_name].append(rec)
            log(f"served {mode_name} lambda={lam}: p50 {rec['p50_ms']} ms, p99 {rec['p99_ms']} "
                f"ms, {rec['pairs_per_s'] / 1e6:.1f} M pairs/s, unfinished {rec['unfinished']}, "
                f"mismatched submissions {rec['mismatched_submissions']} of "
                f"{rec['checked_submissions']} checked")

    def at_slo(rows):
        """The highest rate below the first one that misses the SLO (a later
        rate that happens to meet it again does not count)."""
        best = None
        for r in sorted(rows, key=lambda r: r["lambda"]):
            if ("p99_ms" not in r or r["p99_ms"] is None or r["p99_ms"] > args.slo_ms
                    or r["unfinished"] != 0 or r["mismatched_submissions"] != 0):
                break
            best = r
        if best is None:
            return None
        return {"lambda": best["lambda"], "pairs_per_s": best["pairs_per_s"],
                "p50_ms": best["p50_ms"], "p99_ms": best["p99_ms"]}

    served_slo, seq_slo = at_slo(results["served"]), at_slo(results["per_request"])
    all_rows = results["served"] + results["per_request"]
    out = {
        "workload": f"served: {args.ref_len} bp GC-41% reference resident, pool of "
                    f"{len(pool)} requests of 1e3..1e6 pairs (log-uniform, mean "
                    f"{pool_pairs.mean():.0f}), read length U{{100..250}}, own e "
                    "U{0..floor(0.1 m)}, open-loop Poisson arrivals from a native client "
                    f"thread, {duration:.0f} s per rate after {lead:g} s of arrivals at that "
                    "rate that warm the fresh server",
        "slo_p99_ms": args.slo_ms,
        "host_memory": "pageable" if args.pageable else "pinned",
        "served_at_slo": served_slo, "per_request_at_slo": seq_slo,
        "speedup_at_slo": (round(served_slo["pairs_per_s"] / seq_slo["pairs_per_s"], 3)
                           if served_slo and seq_slo else None),
        "by_rate": results,
        "parity": {"pool_requests_with_oracle_outputs": len(pool),
                   "checked_submissions": int(sum(r.get("checked_submissions", 0)
                                                  for r in all_rows)),
                   "mismatched_submissions": int(sum(r.get("mismatched_submissions", 0)
                                                     for r in all_rows)),
                   "oracle_s": round(oracle_s, 1)},
    }
    gk.gk_destroy(ctx)
    del keep
    return out


def bench_served(args, log) -> int:
    lambdas = [float(x) for x in args.lambdas.split(",")]
    sec = served_section(args, log, args.pool, lambdas, args.duration)
    out = {"metric": "p99 request latency and pairs/sec at p99 <= SLO, served filter, "
                     "1 MI355X, bit-exact",
           "value": sec["served_at_slo"]["pairs_per_s"] if sec["served_at_slo"] else None,
           "unit": "pairs/s", "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
           "dtype": "u32", "vs_baseline": None, "config": {"workload": sec["workload"]}}
    out.update(sec)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
