#!/usr/bin/env python3
"""Benchmark of the packed bit-matrix product path on one MI355X.

One step = the GF(2) product by the self-inverse alternative-basis Strassen
recursion (forward basis changes, expansion, batched leaves, compression,
inverse basis change) plus the Boolean product by the cubic method, both on
n x n operands (n = 2^18 by default: 8 GiB per matrix) resident in HBM.
Effective throughput = 2 n^3 bit operations per product / time.

The int8-MFMA leaf is the headline; the same step with the VALU (bitop3) leaf
is timed once beside it.  The line also carries the dominant kernel's roofline
(HIP events around the Boolean leaf launch) and the oracle's CPU rate on a
bounded sample of output rows, whose values are also compared with the GPU's.
"""
import argparse
import json
import os
import sys
import time

METRIC = "effective Pbop/s (2n^3/s), GF(2)+Boolean n=2^18: VALU vs int8-MFMA leaf"
PEAK_MFMA_I8_TOPS = 5000.0        # dense int8 MFMA, ops/s (1 MAC = 2 ops)
PEAK_MFMA_F4_TOPS = 10100.0       # dense fp4 (E2M1) MFMA
# VALU bit-operation peaks (2 bit operations, the AND and the XOR/OR, on each of 32 bit
# positions per fused v_bitop3_b32 lane-op), at 256 CUs and 2.4 GHz:
#  - single issue: 4 SIMDs x 16 lanes = 64 lane-ops/clk/CU -> 2.517e15 bop/s;
#  - gfx950 dual issue: two VALU instructions per SIMD per quad-cycle (counted by the
#    SQ_ACTIVE_INST_VALU2 counter) = 128 lane-ops/clk/CU -> 5.033e15 bop/s, the rate the
#    calibration kernel (bmm_calibrate_valu, bench --mode valu) measures.
PEAK_VALU_SINGLE_TBOPS = 2516.6
PEAK_VALU_FUSED_TBOPS = 5033.2
# Bytes that one Boolean leaf launch at n = 2^18 (sparse operands) moves between L2 and
# memory, for the int8 leaf with the tuned tile (7: 64 x 128, chunked loop, wide operand
# expansion, 16-byte C stores): reads from rocprofv3's request counts by size (128 x
# TCC_EA0_RDREQ_128B + 64 x TCC_EA0_RDREQ_64B; FETCH_SIZE counts a 128-byte read as 64
# bytes on this device, which a 4 GiB copy in the same runs shows), writes from
# WRITE_SIZE (the copy's 4 GiB read back exactly); see
# profiles/pmc_traffic_leaf_boolean_n262144.md.  Valid for that kernel only.
MEASURED_TRAFFIC = {("mfma", 7, 1 << 18): 1.76381e11 * 128 + 3.14568e7 * 64 + 1.37406e7 * 1024}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class ClockSampler:
    """The GPU's graphics clock (MHz), sampled every 20 ms on a host thread from the
    SMU metrics table (amdsmi gpu_metrics: the average graphics clock, else the mean
    of the per-XCD current clocks) while a region runs; mean_ghz() is None when the
    metrics cannot be read."""

    def __init__(self):
        self.samples, self._stop, self._t, self._h, self._smi = [], None, None, None, None
        try:
            import amdsmi
            amdsmi.amdsmi_init()
            self._smi = amdsmi
            self._h = amdsmi.amdsmi_get_processor_handles()[0]
            self._read()
        except Exception:
            self._smi = None

    def _read(self):
        m = self._smi.amdsmi_get_gpu_metrics_info(self._h)
        v = m.get("average_gfxclk_frequency")
        if not isinstance(v, (int, float)) or v <= 0 or v >= 0xFFFF:
            xs = [x for x in (m.get("current_gfxclks") or []) if isinstance(x, (int, float))
                  and 0 < x < 0xFFFF]
            v = sum(xs) / len(xs) if xs else None
        return v

    def __enter__(self):
        import threading
        self.samples = []
        if self._smi is None:
            return self
        self._stop = threading.Event()

        def run():
            while not self._stop.is_set():
                try:
                    v = self._read()
                    if v:
                        self.samples.append(float(v))
                except Exception:
                    pass
                self._stop.wait(0.02)
        self._t = threading.Thread(target=run, daemon=True)
        self._t.start()
        return self

    def __exit__(self, *exc):
        if self._t:
            self._stop.set()
            self._t.join()
            self._t = None

    def mean_ghz(self):
        return round(sum(self.samples) / len(self.samples) / 1e3, 3) if self.samples else None


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1 << 18)
    ap.add_argument("--depth", type=int, default=-1,
                    help="Strassen levels above the leaf (-1: the autotune table's choice)")
    ap.add_argument("--tune-file", default=None,
                    help="autotune table to load (default: the package's table for gfx950)")
    ap.add_argument("--depth-serial", type=int, default=-1)
    ap.add_argument("--shift", type=int, default=-1,
                    help="shifted leaf level of the GF(2) recursion: 0 off, 1 on, 2 on with "
                         "8-byte loads, -1 the autotune table's choice")
    ap.add_argument("--tile", type=int, default=0,
                    help="tile variant of the timed leaf kind (0 = the autotune table's)")
    ap.add_argument("--no-valu", action="store_true", help="skip the VALU-leaf side step")
    ap.add_argument("--cpu-rows", type=int, default=256,
                    help="rows of the GF(2) product the oracle computes for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows-1core", type=int, default=16,
                    help="rows of the GF(2) product the oracle computes on one thread")
    ap.add_argument("--freivalds", type=int, default=20,
                    help="Freivalds vectors checking the whole GF(2) product on the host")
    ap.add_argument("--leaf", choices=["mfma", "valu", "f4"], default="mfma",
                    help="leaf of the timed steps (mfma = int8 MFMA, f4 = E2M1 MFMA)")
    ap.add_argument("--no-f4", action="store_true", help="skip the fp4-leaf side step")
    ap.add_argument("--no-schemes", action="store_true",
                    help="skip timing the GF(2) recursion with the chaining and "
                         "Strassen-Winograd schemes")
    ap.add_argument("--mode", choices=["step", "leaf", "cubic", "batched", "ooc", "tune", "valu",
                                       "small"],
                    default="step",
                    help="leaf: one Boolean leaf launch plus a copy of known size (for "
                         "profiler counters); batched: 4096 uneven products in one "
                         "persistent launch; ooc: host-resident operands; valu: the VALU "
                         "issue-rate calibration and the VALU leaf on both semirings; small: "
                         "n = 2048 full products, graph-replayed, against the oracle")
    ap.add_argument("--k-panel", type=int, default=0,
                    help="leaf mode: k-panel length of the Boolean leaf in bits (0: one panel)")
    ap.add_argument("--dense", action="store_true",
                    help="leaf mode: dense Bernoulli(1/2) operands instead of the sparse ones")
    ap.add_argument("--dense-k-panel", type=int, default=16384,
                    help="step: also time the dense Boolean leaf with this k-panel length "
                         "(bits; 0 skips it)")
    ap.add_argument("--problems", type=int, default=4096, help="batched mode: problem count")
    ap.add_argument("--block", type=int, default=1 << 17, help="ooc mode: block size (bits)")
    return ap.parse_args()


def single_thread_seconds(fn):
    """Seconds fn() takes with the OpenMP runtime held to one thread (the oracle's C
    library runs its loops under OpenMP), or None if that runtime cannot be reached."""
    import ctypes
    try:
        gomp = ctypes.CDLL("libgomp.so.1")
        before = gomp.omp_get_max_threads()
    except OSError:
        return None
    gomp.omp_set_num_threads(1)
    try:
        t0 = time.perf_counter()
        fn()
        return time.perf_counter() - t0
    finally:
        gomp.omp_set_num_threads(before)


def run_small(args, torch, np, bmm, bmmgen):
    """The small plain-method workload: n = 2048, Bernoulli(1/2) bits, the GF(2) and
    the Boolean product by the cubic method with each leaf kind, each timed as the mean
    of `reps` launches replayed from one HIP graph (a single launch is microseconds) and
    checked in full against the oracle, which is timed on all threads and on one."""
    import oracle
    n = args.n if args.n <= 8192 else 2048
    reps = max(1000, args.steps)
    seed = bmmgen.config_seed(0)
    dev = torch.device("cuda:0")
    A = bmmgen.fill_cpu(n, n, seed, bmmgen.TAG_A, bmmgen.Dist.half())
    B = bmmgen.fill_cpu(n, n, seed, bmmgen.TAG_B, bmmgen.Dist.half())
    Ad = torch.from_numpy(A.view(np.int64).copy()).to(dev)
    Bd = torch.from_numpy(B.view(np.int64).copy()).to(dev)
    BTd = torch.empty_like(Bd)
    Cd = torch.empty_like(Ad)
    bmm.bmm_transpose(Bd, BTd, n, n)
    bops = 2.0 * n ** 3
    out = {"mode": "small", "n": n, "reps_per_graph": reps}
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    for sname, sr in [("gf2", bmm.GF2), ("boolean", bmm.BOOLEAN)]:
        c0 = time.perf_counter()
        want = oracle.mul(A, B, n, n, sr)
        c_all = time.perf_counter() - c0
        c_one = single_thread_seconds(lambda: oracle.mul(A, B, n, n, sr))
        out[f"{sname}_oracle"] = {"seconds_all_threads": round(c_all, 4), "threads": threads,
                                  "seconds_one_thread": round(c_one, 4) if c_one else None,
                                  "pbops_all_threads": round(bops / c_all / 1e15, 6)}
        fn = bmm.bmm_gf2 if sr == bmm.GF2 else bmm.bmm_boolean
        for lname, leaf in [("valu", bmm.LEAF_VALU), ("int8", bmm.LEAF_MFMA_I8),
                            ("fp4", bmm.LEAF_MFMA_F4)]:
            o = bmm.Options(leaf=leaf)
            s_ = torch.cuda.Stream()
            with torch.cuda.stream(s_):
                fn(Ad, BTd, Cd, n, n, n, options=o, b_transposed=True, stream=s_.cuda_stream)
                s_.synchronize()
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g, stream=s_):
                    for _ in range(reps):
                        fn(Ad, BTd, Cd, n, n, n, options=o, b_transposed=True,
                           stream=s_.cuda_stream)
            torch.cuda.synchronize()
            Cd.fill_(-1)
            g.replay()  # warm-up replay
            torch.cuda.synchronize()
            ok = bool(np.array_equal(Cd.cpu().numpy().view(np.uint64), want))
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            g.replay()
            e1.record()
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1) / 1e3 / reps
            _, tile = bmm.bmm_leaf_choice(sr, n, n, n, 1, o)
            out[f"{sname}_{lname}"] = {"tile": tile, "seconds": t,
                                       "pbops": round(bops / t / 1e15, 4),
                                       "speedup_vs_oracle_all_threads": round(c_all / t, 1),
                                       "verified_full": ok}
            log(f"[bench] small {sname} {lname}: {out[f'{sname}_{lname}']}")
            del g
    print(json.dumps(out), flush=True)


def run_batched(args, torch, np, bmm, bmmgen):
    """4096 independent products, m, k, n log-uniform in [256, 8192] (multiples of
    64); even problems GF(2) with Bernoulli(1/2) bits, odd problems Boolean with
    Bernoulli(1/sqrt(k)) bits.  One persistent launch replayed from a HIP graph
    against one launch per product."""
    import oracle
    dev = torch.device("cuda:0")
    seed = bmmgen.config_seed(3)
    shapes = bmmgen.batched_shapes(args.problems, seed)
    words = lambda x: (int(x) + 63) // 64
    na = sum(m * words(k) for _, m, k, n, _ in shapes)
    nb = sum(n * words(k) for _, m, k, n, _ in shapes)
    nc = sum(m * words(n) for _, m, k, n, _ in shapes)
    log(f"[bench] batched: {args.problems} problems, operands "
        f"{(na + nb + nc) * 8 / 2**30:.2f} GiB")
    bufA = torch.empty(na, dtype=torch.int64, device=dev)
    bufB = torch.empty(nb, dtype=torch.int64, device=dev)
    bufC = torch.empty(nc, dtype=torch.int64, device=dev)
    tmpB = torch.empty(max(k * words(n) for _, m, k, n, _ in shapes), dtype=torch.int64,
                       device=dev)
    probs, oa, ob, oc = [], 0, 0, 0
    for p, (sr, m, k, n, dist) in enumerate(shapes):
        A = bufA[oa:oa + m * words(k)].view(m, words(k))
        BT = bufB[ob:ob + n * words(k)].view(n, words(k))
        C = bufC[oc:oc + m * words(n)].view(m, words(n))
        oa, ob, oc = oa + A.numel(), ob + BT.numel(), oc + C.numel()
        bmmgen.fill_tensor(A, m, k, seed, bmmgen.batched_tag(p, "A"), dist)
        B = tmpB[:k * words(n)].view(k, words(n))
        bmmgen.fill_tensor(B, k, n, seed, bmmgen.batched_tag(p, "B"), dist)
        bmm.bmm_transpose(B, BT, k, n)
        probs.append(dict(semiring=sr, m=m, k=k, n=n, A=A, B=BT, C=C, b_transposed=True))
    torch.cuda.synchronize()
    bops = sum(2.0 * p["m"] * p["k"] * p["n"] for p in probs)
    # every (leaf, tile) candidate timed once for the record, then the autotuner's choice
    cands = {}
    for lf, lname in [(bmm.LEAF_MFMA_I8, "int8"), (bmm.LEAF_MFMA_F4, "fp4")]:
        for tl, tname in [(1, "128x64"), (2, "64x64"), (3, "64x128"), (4, "128x64lds")]:
            pl = bmm.BatchedPlan(probs, options=bmm.Options(leaf=lf, tile=tl))
            pl.launch()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            pl.launch()
            e1.record()
            torch.cuda.synchronize()
            cands[f"{lname}_{tname}"] = round(e0.elapsed_time(e1) / 1e3, 5)
            pl.destroy()
    leaf, tile, _ = bmm.bmm_autotune_batched(probs)
    # the per-size-class choices the autotuner kept (only where the mix was faster)
    import tempfile
    with tempfile.NamedTemporaryFile("r", suffix=".txt") as tf:
        bmm.bmm_autotune_save(tf.name)
        per_class = [ln.split()[3:] for ln in open(tf.name)
                     if ln.startswith(f"batched_class {args.problems} ")]
    log(f"[bench] batched candidates {cands}; autotuner: leaf {leaf} tile {tile}, "
        f"per-class choices {per_class}")
    plan = bmm.BatchedPlan(probs)  # AUTO options: the autotuner's choice
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        plan.launch(s.cuda_stream)  # warm-up outside the graph
        s.synchronize()
        with torch.cuda.graph(g, stream=s):
            plan.launch(s.cuda_stream)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.replay()
    torch.cuda.synchronize()
    t_graph = (time.perf_counter() - t0) / args.steps
    # rows of 16 problems from the graph replays, checked against the oracle below
    check = list(range(0, args.problems, max(1, args.problems // 16)))
    sample = {p: bmmgen.stratified_rows(probs[p]["m"], 8, seed + p) for p in check}
    kept = {p: probs[p]["C"][sample[p]].cpu().numpy().view(np.uint64).copy() for p in check}
    opts = bmm.Options(leaf=leaf)  # the baseline: the same leaf kind, tile chosen per product

    def one_by_one():
        for p in probs:
            fn = bmm.bmm_gf2 if p["semiring"] == bmm.GF2 else bmm.bmm_boolean
            fn(p["A"], p["B"], p["C"], p["m"], p["k"], p["n"], options=opts, b_transposed=True)
    one_by_one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one_by_one()
    torch.cuda.synchronize()
    t_loop = (time.perf_counter() - t0) / args.steps
    # both variants' rows of the 16 problems against the oracle
    ok = True
    for p in check:
        pr = probs[p]
        m, k, n = pr["m"], pr["k"], pr["n"]
        dist = bmmgen.Dist.half() if pr["semiring"] == bmm.GF2 else bmmgen.Dist.inv_sqrt(k)
        rows = sample[p]
        Ar = bmmgen.fill_rows_cpu(rows, k, seed, bmmgen.batched_tag(p, "A"), dist)
        Bh = bmmgen.fill_cpu(k, n, seed, bmmgen.batched_tag(p, "B"), dist)
        want = oracle.rows(Ar, Bh, k, n, pr["semiring"])
        got = pr["C"][rows].cpu().numpy().view(np.uint64)
        ok = ok and bool(np.array_equal(got, want)) and bool(np.array_equal(kept[p], want))
    plan.destroy()
    print(json.dumps({
        "mode": "batched", "problems": args.problems, "total_bops": bops,
        "persistent_graph_s": round(t_graph, 5), "persistent_pbops": round(bops / t_graph / 1e15, 4),
        "one_launch_per_product_s": round(t_loop, 5),
        "one_launch_per_product_pbops": round(bops / t_loop / 1e15, 4),
        "speedup": round(t_loop / t_graph, 3), "verified_16_problems": ok,
        "autotuned": {"leaf": {2: "int8", 3: "fp4"}[leaf],
                      "tile": {1: "128x64", 2: "64x64", 3: "64x128", 4: "128x64lds"}[tile],
                      "per_k_class": {f"class{c}": {"leaf": {1: "valu", 2: "int8", 3: "fp4"}[
                          int(lf)], "tile": int(t)} for c, lf, t in per_class}},
        "candidates_s": cands,
        "frac_of_peak": round(bops / t_graph / 1e12 / (PEAK_MFMA_F4_TOPS if leaf == 3
                                                        else PEAK_MFMA_I8_TOPS), 4)}), flush=True)


def run_cubic(args, torch, np, bmm, bmmgen):
    """The cubic products at one size (n = 65536 for the VALU-vs-int8 comparison):
    GF(2) on Bernoulli(1/2) bits and Boolean on Bernoulli(n^-1/2) bits (P(c = 1) ~ 0.63),
    B transposed once, then each leaf kind with its tuned or default tile; the median of
    `steps` launches after `warmup` launches, each checked on 64 stratified rows."""
    import oracle
    n = args.n
    seed = bmmgen.config_seed(1)
    dev = torch.device("cuda:0")
    bops = 2.0 * n ** 3
    peaks = {bmm.LEAF_VALU: PEAK_VALU_FUSED_TBOPS, bmm.LEAF_MFMA_I8: PEAK_MFMA_I8_TOPS,
             bmm.LEAF_MFMA_F4: PEAK_MFMA_F4_TOPS}
    names = {bmm.LEAF_VALU: "valu", bmm.LEAF_MFMA_I8: "int8", bmm.LEAF_MFMA_F4: "fp4"}
    out = {"mode": "cubic", "n": n}
    rows = bmmgen.stratified_rows(n, 64, seed)
    for sname, sr, dist in [("gf2", bmm.GF2, bmmgen.Dist.half()),
                            ("boolean", bmm.BOOLEAN,
                             bmmgen.Dist.pow2(max(1, (n.bit_length() - 1) // 2)))]:
        A = torch.empty((n, n // 64), dtype=torch.int64, device=dev)
        B = torch.empty_like(A)
        BT = torch.empty_like(A)
        C = torch.empty_like(A)
        bmmgen.fill_tensor(A, n, n, seed, 0xA if sr == bmm.GF2 else 0x1A, dist)
        bmmgen.fill_tensor(B, n, n, seed, 0xB if sr == bmm.GF2 else 0x1B, dist)
        bmm.bmm_transpose(B, BT, n, n)
        del B
        Bh = bmmgen.fill_cpu(n, n, seed, 0xB if sr == bmm.GF2 else 0x1B, dist)
        Ar = bmmgen.fill_rows_cpu(rows, n, seed, 0xA if sr == bmm.GF2 else 0x1A, dist)
        want = oracle.rows(Ar, Bh, n, n, sr)
        del Bh
        fn = bmm.bmm_gf2 if sr == bmm.GF2 else bmm.bmm_boolean
        for leaf in (bmm.LEAF_VALU, bmm.LEAF_MFMA_I8, bmm.LEAF_MFMA_F4):
            o = bmm.Options(leaf=leaf)
            _, tile = bmm.bmm_leaf_choice(sr, n, n, n, 1, o)
            for _ in range(args.warmup):
                fn(A, BT, C, n, n, n, options=o, b_transposed=True)
            times = []
            for _ in range(args.steps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                fn(A, BT, C, n, n, n, options=o, b_transposed=True)
                e1.record()
                torch.cuda.synchronize()
                times.append(e0.elapsed_time(e1) / 1e3)
            t = sorted(times)[len(times) // 2]
            got = C[rows].cpu().numpy().view(np.uint64)
            out[f"{sname}_{names[leaf]}"] = {
                "tile": tile, "seconds": round(t, 5), "pbops": round(bops / t / 1e15, 4),
                "frac_of_peak": round(bops / t / 1e12 / peaks[leaf], 4),
                "verified_rows": len(rows), "verified": bool(np.array_equal(got, want))}
            log(f"[bench] cubic {sname} {names[leaf]}: {out[f'{sname}_{names[leaf]}']}")
        del A, BT, C
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


def valu_calibration(bmm, rounds=1 << 21):
    """bmm_calibrate_valu at 1-4 waves per SIMD: measured v_bitop3_b32 lane-ops per
    core clock per CU, the waves' core clock and the aggregate bit-operation rate."""
    out = {}
    for w in (1, 2, 4, 8):
        r = bmm.bmm_calibrate_valu(w, rounds)
        out[str(w)] = {"lane_ops_per_clk_cu": round(r["lane_ops_per_clk_cu"], 2),
                       "clock_ghz": round(r["clock_ghz"], 3),
                       "seconds": round(r["seconds"], 5),
                       "tbops": round(r["aggregate_bops"] / 1e12, 1)}
        log(f"[bench] VALU calibration, {w} waves/SIMD: {out[str(w)]}")
    return out


def sustained_valu_tbops(cal):
    """The highest calibrated v_bitop3_b32 issue rate (lane-ops per clock per CU, over
    the waves-per-SIMD settings) as a bit-operation rate at 256 CUs and 2.4 GHz."""
    best = max(v["lane_ops_per_clk_cu"] for v in cal.values())
    return best * 256 * 2.4e9 * 64 / 1e12


def valu_fracs(rate_tbops, sustained_tbops):
    """A VALU leaf rate as fractions of the single-issue (64 lane-ops/clk/CU), the
    dual-issue (128) and the measured sustained bit-operation peaks."""
    return {"frac_single_issue": round(rate_tbops / PEAK_VALU_SINGLE_TBOPS, 4),
            "frac_dual_issue": round(rate_tbops / PEAK_VALU_FUSED_TBOPS, 4),
            "frac_sustained": round(rate_tbops / sustained_tbops, 4) if sustained_tbops else None}


def run_valu(args, torch, np, bmm, bmmgen):
    """The VALU roofline: the issue-rate calibration kernel, then the VALU leaf on
    the cubic products at one size (GF(2) on Bernoulli(1/2) bits, Boolean on
    Bernoulli(n^-1/2) bits), each as a fraction of the single-issue and the
    dual-issue bit-operation peaks; 64 stratified rows of each checked.  --tile 2
    runs the leaf's outer-product form (B row-major) instead of the dot-product form."""
    import oracle
    n = args.n
    outer = args.tile == 2
    cal = valu_calibration(bmm)
    sustained = sustained_valu_tbops(cal)
    out = {"mode": "valu", "n": n, "tile": 2 if outer else 1, "calibration": cal,
           "peaks_tbops": {"single_issue_64_lanes": PEAK_VALU_SINGLE_TBOPS,
                           "dual_issue_128_lanes": PEAK_VALU_FUSED_TBOPS,
                           "sustained_measured": round(sustained, 1)}}
    seed = bmmgen.config_seed(1)
    dev = torch.device("cuda:0")
    bops = 2.0 * n ** 3
    rows = bmmgen.stratified_rows(n, 64, seed)
    for sname, sr, dist in [("gf2", bmm.GF2, bmmgen.Dist.half()),
                            ("boolean", bmm.BOOLEAN,
                             bmmgen.Dist.pow2(max(1, (n.bit_length() - 1) // 2)))]:
        A = torch.empty((n, n // 64), dtype=torch.int64, device=dev)
        B = torch.empty_like(A)
        BT = None if outer else torch.empty_like(A)
        C = torch.empty_like(A)
        bmmgen.fill_tensor(A, n, n, seed, 0xA if sr == bmm.GF2 else 0x1A, dist)
        bmmgen.fill_tensor(B, n, n, seed, 0xB if sr == bmm.GF2 else 0x1B, dist)
        if outer:
            Bop = B  # the outer-product form reads B where it lies
        else:
            bmm.bmm_transpose(B, BT, n, n)
            Bop = BT
        del B
        fn = bmm.bmm_gf2 if sr == bmm.GF2 else bmm.bmm_boolean
        o = bmm.Options(leaf=bmm.LEAF_VALU, tile=2 if outer else 1)
        for _ in range(args.warmup):
            fn(A, Bop, C, n, n, n, options=o, b_transposed=not outer)
        times = []
        for _ in range(args.steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn(A, Bop, C, n, n, n, options=o, b_transposed=not outer)
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1) / 1e3)
        t = sorted(times)[len(times) // 2]
        got = C[rows].cpu().numpy().view(np.uint64)
        Bh = bmmgen.fill_cpu(n, n, seed, 0xB if sr == bmm.GF2 else 0x1B, dist)
        Ar = bmmgen.fill_rows_cpu(rows, n, seed, 0xA if sr == bmm.GF2 else 0x1A, dist)
        want = oracle.rows(Ar, Bh, n, n, sr)
        del Bh
        rate = bops / t / 1e12
        out[sname] = {"seconds": round(t, 5), "pbops": round(rate / 1e3, 4),
                      **valu_fracs(rate, sustained),
                      "verified_rows": len(rows), "verified": bool(np.array_equal(got, want))}
        log(f"[bench] VALU leaf {sname}: {out[sname]}")
        del A, BT, Bop, C
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


def run_ooc(args, torch, np, bmm, bmmgen):
    """Products with A, B, C in page-locked host memory, streamed through HBM in
    b x b blocks (copies on their own streams, overlapped with compute).  GF(2)
    (Bernoulli(1/2) bits) with the host-level recursion and with the cubic block
    order; Boolean (Bernoulli(2^-e), P(c = 1) ~ 0.63) in the block order.
    Rates include every PCIe transfer."""
    import oracle
    n, blk = args.n, min(args.block, args.n)
    nw = n // 64
    seed = bmmgen.config_seed(4)
    g = n // blk
    out = {"mode": "ooc", "n": n, "block": blk}
    log(f"[bench] ooc: {3 * n * nw * 8 / 2**30:.1f} GiB of pinned host memory")
    A = torch.empty((n, nw), dtype=torch.int64, pin_memory=True)
    B = torch.empty((n, nw), dtype=torch.int64, pin_memory=True)
    C = torch.empty((n, nw), dtype=torch.int64, pin_memory=True)
    slab = torch.empty((min(n, 1 << 15), nw), dtype=torch.int64, device="cuda")
    block_bytes = blk * blk / 8
    dh = g.bit_length() - 1 if g >= 2 and (g & (g - 1)) == 0 else 0
    runs = [("gf2_host_levels", bmm.GF2, bmmgen.Dist.half(), 0),
            ("gf2_block_order", bmm.GF2, bmmgen.Dist.half(), bmm.FLAG_OOC_BLOCK_ORDER),
            ("boolean_block_order", bmm.BOOLEAN,
             bmmgen.Dist.pow2(max(1, (n.bit_length() - 1) // 2)), 0)]
    made = None
    for name, sr, dist, flags in runs:
        if name == "gf2_host_levels" and dh == 0:
            continue
        if made != (dist.kind, dist.param):
            # generate on the GPU in row slabs and copy into the pinned buffers
            for dst, tag in [(A, bmmgen.TAG_A), (B, bmmgen.TAG_B)]:
                for r0 in range(0, n, slab.shape[0]):
                    rows = min(slab.shape[0], n - r0)
                    bmmgen.fill_tensor(slab[:rows], rows, n, seed, tag, dist, row0=r0)
                    dst[r0:r0 + rows].copy_(slab[:rows])
            torch.cuda.synchronize()
            made = (dist.kind, dist.param)
        log(f"[bench] ooc {name}")
        secs = bmm.bmm_ooc(sr, A, B, C, n, n, n, block=blk,
                           options=bmm.Options(leaf=bmm.LEAF_MFMA_I8, flags=flags))
        rows = bmmgen.stratified_rows(n, 16, seed)
        Ar = bmmgen.fill_rows_cpu(rows, n, seed, bmmgen.TAG_A, dist)
        want = oracle.rows(Ar, B.numpy().view(np.uint64), n, n, sr)
        got = C[rows].numpy().view(np.uint64)
        if name == "gf2_host_levels":  # 14 blocks of A and 14 of B per level and instance
            h2d = 2 * 14 ** dh * block_bytes
            d2h = n * n / 8
        else:
            h2d = 2 * g ** 3 * block_bytes
            d2h = n * n / 8
        hb, hs, db, dsec = bmm.bmm_ooc_last_transfers()
        out[name] = {"seconds": round(secs, 3), "pbops": round(2.0 * n ** 3 / secs / 1e15, 4),
                     "h2d_bytes": h2d, "d2h_bytes": d2h,
                     "pcie_gbs_wall": round((h2d + d2h) / secs / 1e9, 2),
                     # the copies' own durations (HIP events around each on its stream)
                     "h2d_copy_bytes": hb, "h2d_copy_s": round(hs, 4),
                     "h2d_gbs": round(hb / hs / 1e9, 2) if hs > 0 else None,
                     "d2h_copy_bytes": db, "d2h_copy_s": round(dsec, 4),
                     "d2h_gbs": round(db / dsec / 1e9, 2) if dsec > 0 else None,
                     "verified_rows": len(rows), "verified": bool(np.array_equal(got, want))}
        log(f"[bench] ooc {name}: {secs:.2f} s {out[name]}")
    del A, B, C, slab
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); this build has no "
              "multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    root = os.path.dirname(os.path.abspath(__file__))
    sys.path.insert(0, root)
    if not os.path.exists(os.path.join(root, "paper_1909_01554_amd", "libbmm.so")):
        import __graft_entry__
        __graft_entry__.build()
    import bmmgen
    import paper_1909_01554_amd as bmm

    tune_file = args.tune_file or os.path.join(root, "paper_1909_01554_amd", "tune_gfx950.txt")
    if args.mode != "tune" and os.path.exists(tune_file):
        bmm.bmm_autotune_load(tune_file)
        log(f"[bench] loaded autotune table {tune_file}")
    if args.mode == "cubic":
        return run_cubic(args, torch, np, bmm, bmmgen)
    if args.mode == "batched":
        return run_batched(args, torch, np, bmm, bmmgen)
    if args.mode == "ooc":
        return run_ooc(args, torch, np, bmm, bmmgen)
    if args.mode == "valu":
        return run_valu(args, torch, np, bmm, bmmgen)
    if args.mode == "small":
        return run_small(args, torch, np, bmm, bmmgen)

    n = args.n
    nw = n // 64
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    seed = bmmgen.config_seed(2)
    bool_dist = bmmgen.Dist.pow2(max(1, (n.bit_length() - 1) // 2))  # p = n^-1/2: P(c=1) ~ 0.63

    def mat():
        return torch.empty((n, nw), dtype=torch.int64, device=dev)

    log(f"[bench] n={n}: generating operands in HBM")
    Ag, Bg, Cg = mat(), mat(), mat()
    Ab, Bb, BTb, Cb = mat(), mat(), mat(), mat()
    bmmgen.fill_tensor(Ag, n, n, seed, bmmgen.TAG_A, bmmgen.Dist.half())
    bmmgen.fill_tensor(Bg, n, n, seed, bmmgen.TAG_B, bmmgen.Dist.half())
    bmmgen.fill_tensor(Ab, n, n, seed, 0x1A, bool_dist)
    bmmgen.fill_tensor(Bb, n, n, seed, 0x1B, bool_dist)

    stream = torch.cuda.current_stream()
    LEAF = {"mfma": bmm.LEAF_MFMA_I8, "valu": bmm.LEAF_VALU, "f4": bmm.LEAF_MFMA_F4}

    def events():
        return [torch.cuda.Event(enable_timing=True) for _ in range(4)]

    def opts(leaf):
        # --tile applies to the timed leaf kind only; side steps take their tuned tiles
        return bmm.Options(leaf=leaf, tile=args.tile if leaf == LEAF[args.leaf] else 0,
                           depth_serial=args.depth_serial,
                           depth_parallel=-1 if args.depth_serial < 0 else
                           args.depth - args.depth_serial, shift=args.shift)

    if args.mode == "leaf":
        # one Boolean leaf launch (or one per k panel) on the sparse headline operands, or
        # on the dense GF(2) ones, then a 4 GiB copy that calibrates the traffic counters
        LA, LB = (Ag, Bg) if args.dense else (Ab, Bb)
        bmm.bmm_transpose(LB, BTb, n, n)
        src = torch.empty(1 << 29, dtype=torch.int64, device=dev)  # 4 GiB
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        e = events()
        e[0].record(stream)
        bmm.bmm_boolean(LA, BTb, Cb, n, n, n, options=bmm.Options(
            leaf=LEAF[args.leaf], tile=args.tile, k_panel=args.k_panel or -1), b_transposed=True)
        e[1].record(stream)
        dst.copy_(src)
        e[2].record(stream)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "leaf", "n": n, "leaf": args.leaf,
                          "operands": "dense" if args.dense else "sparse",
                          "k_panel": args.k_panel or n,
                          "leaf_s": e[0].elapsed_time(e[1]) / 1e3,
                          "copy_bytes": 2 * src.numel() * 8,
                          "copy_s": e[1].elapsed_time(e[2]) / 1e3}), flush=True)
        return

    # the GF(2) product changes A to the alternative basis in place and restores it
    # (BMM_FLAG_INPLACE_BASIS): no 8 GiB copy of A in the workspace
    nbytes, ds, dp = bmm.bmm_gf2_strassen_workspace(n, n, n, args.depth, opts(bmm.LEAF_MFMA_I8),
                                                    inplace_basis=True)
    if args.mode == "tune":
        # room for the deeper plans the depth tuner tries
        nbytes = max(nbytes, bmm.bmm_gf2_strassen_workspace(
            n, n, n, 6, bmm.Options(depth_serial=2, depth_parallel=4))[0])
    ws = torch.empty(nbytes // 8 + 1, dtype=torch.int64, device=dev)
    if args.mode == "tune":
        out = {"mode": "tune", "n": n}
        # leaf table: the full-size cubic shapes, one timed launch per (leaf, tile) on the
        # step's own inputs for that semiring (the matrix cores' rate depends on how many
        # operand bits switch, so each semiring is timed on its own bit density), and the
        # Strassen leaf shapes of the admissible depths
        for sr, name, A_, B_ in [(bmm.BOOLEAN, "boolean", Ab, Bb), (bmm.GF2, "gf2", Ag, Bg)]:
            bmm.bmm_transpose(B_, BTb, n, n)
            BT_, C_ = BTb, Cb
            fn = bmm.bmm_boolean if sr == bmm.BOOLEAN else bmm.bmm_gf2
            best = {}
            for lf in (bmm.LEAF_VALU, bmm.LEAF_MFMA_I8, bmm.LEAF_MFMA_F4):
                for t in range(1, bmm.bmm_leaf_tiles(lf) + 1):
                    e = events()
                    e[0].record(stream)
                    fn(A_, BT_, C_, n, n, n, options=bmm.Options(leaf=lf, tile=t),
                       b_transposed=True)
                    e[1].record(stream)
                    torch.cuda.synchronize()
                    secs = e[0].elapsed_time(e[1]) / 1e3
                    log(f"[bench] cubic {name} leaf={lf} tile={t}: {secs:.3f} s")
                    if secs < best.get(lf, (1e30, 0))[0]:
                        best[lf] = (secs, t)
            order = sorted(best, key=lambda lf: -best[lf][0])  # fastest leaf set last
            for lf in order:
                bmm.bmm_autotune_set(sr, n, n, n, lf, best[lf][1])
            out[f"cubic_{name}"] = {str(lf): {"tile": best[lf][1], "s": round(best[lf][0], 4)}
                                    for lf in best}
        for d in range(4, 9):
            s_ = n >> d
            if s_ < 1024:
                break
            leaf, tile, secs = bmm.bmm_autotune_leaf(bmm.GF2, s_, s_, s_, 2401)
            out[f"strassen_leaf_{s_}"] = {"leaf": leaf, "tile": tile, "s": secs}
            log(f"[bench] tuned leaf {s_}^3 x64: leaf={leaf} tile={tile} {secs * 1e3:.2f} ms")
        # the depth tuner times the int8-MFMA leaf (the headline leaf)
        d, dsel, shift, secs = bmm.bmm_autotune_strassen(
            Ag, Bg, Cg, n, n, n, ws,
            options=bmm.Options(leaf=bmm.LEAF_MFMA_I8, flags=bmm.FLAG_INPLACE_BASIS))
        out["strassen_depth"] = {"depth": d, "depth_serial": dsel, "shift": shift,
                                 "seconds": secs}
        log(f"[bench] tuned Strassen depth {d} (serial {dsel}, shift {shift}) {secs:.3f} s")
        bmm.bmm_autotune_save(tune_file)
        out["table"] = tune_file
        print(json.dumps(out), flush=True)
        return
    log(f"[bench] Strassen depth {args.depth} (serial {ds}, parallel {dp}), workspace "
        f"{nbytes / 2**30:.1f} GiB")
    torch.cuda.synchronize()

    def step(leaf, ev=None):
        o = opts(leaf)
        if ev:
            ev[0].record(stream)
        bmm.bmm_gf2_strassen(Ag, Bg, Cg, n, n, n, ws, depth=args.depth, options=o,
                             inplace_basis=True)
        if ev:
            ev[1].record(stream)
        bmm.bmm_transpose(Bb, BTb, n, n)
        if ev:
            ev[2].record(stream)
        bmm.bmm_boolean(Ab, BTb, Cb, n, n, n, options=o, b_transposed=True)
        if ev:
            ev[3].record(stream)

    for w in range(args.warmup):
        log(f"[bench] warmup step {w}")
        step(LEAF[args.leaf])
        torch.cuda.synchronize()

    # output rows kept from every variant below, checked against the oracle at the end
    rows_sample = bmmgen.stratified_rows(n, max(2, args.cpu_rows), seed)
    idx = torch.tensor(rows_sample, device=dev)
    kept = {}

    def keep(name, with_boolean=True):
        kept[name] = (Cg.index_select(0, idx).cpu(),
                      Cb.index_select(0, idx).cpu() if with_boolean else None)

    evs = [events() for _ in range(args.steps)]
    clock = ClockSampler()
    torch.cuda.synchronize()
    with clock:
        t0 = time.perf_counter()
        for i in range(args.steps):
            step(LEAF[args.leaf], evs[i])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    step_sclk = clock.mean_ghz()
    keep(args.leaf)
    # the headline GF(2) result, for Freivalds's check of the whole matrix at the end
    C_head = (Cg.cpu().numpy().view(np.uint64)
              if args.freivalds > 0 and not args.no_cpu_baseline else None)
    step_s = (t1 - t0) / args.steps
    gf2_s = sum(e[0].elapsed_time(e[1]) for e in evs) / args.steps / 1e3
    tr_s = sum(e[1].elapsed_time(e[2]) for e in evs) / args.steps / 1e3
    leaf_s = sum(e[2].elapsed_time(e[3]) for e in evs) / args.steps / 1e3
    bops = 2.0 * n ** 3
    log(f"[bench] MFMA step {step_s:.3f} s: GF(2) Strassen {gf2_s:.3f} s, transpose {tr_s * 1e3:.2f}"
        f" ms, Boolean leaf {leaf_s:.3f} s")

    def side_step(name, peak_tbops):
        log(f"[bench] {name}-leaf step")
        e = events()
        with ClockSampler() as ck:
            step(LEAF[name], e)
            torch.cuda.synchronize()
        vg = e[0].elapsed_time(e[1]) / 1e3
        vb = e[2].elapsed_time(e[3]) / 1e3
        vt = e[0].elapsed_time(e[3]) / 1e3
        keep(name)
        log(f"[bench] {name} step {vt:.3f} s (GF(2) {vg:.3f} s, Boolean {vb:.3f} s)")
        return {"step_s": round(vt, 4), "value": round(2 * bops / vt / 1e15, 4),
                "gf2_strassen_s": round(vg, 4), "gf2_eff_pbops": round(bops / vg / 1e15, 4),
                "boolean_leaf_s": round(vb, 4), "boolean_leaf_pbops": round(bops / vb / 1e15, 4),
                "boolean_leaf_frac_of_peak": round(bops / vb / 1e12 / peak_tbops, 4),
                "sclk_ghz": ck.mean_ghz()}

    valu = None
    if not args.no_valu and args.leaf != "valu":
        valu = side_step("valu", PEAK_VALU_FUSED_TBOPS)
        # the VALU roofline three ways: 64 lane-ops/clk/CU (single issue), 128 (gfx950's
        # dual issue) and the sustained issue rate the calibration kernel measures here
        cal = valu_calibration(bmm)
        sustained = sustained_valu_tbops(cal)
        valu["boolean_leaf_fracs"] = valu_fracs(bops / valu["boolean_leaf_s"] / 1e12, sustained)
        valu["issue_calibration"] = {
            "sustained_lane_ops_per_clk_cu": max(v["lane_ops_per_clk_cu"] for v in cal.values()),
            "sustained_tbops_at_2p4ghz": round(sustained, 1),
            "by_waves_per_simd": cal}
    f4 = None
    if not args.no_f4 and args.leaf != "f4":
        f4 = side_step("f4", PEAK_MFMA_F4_TOPS)

    # the same GF(2) recursion (same depth and leaf) with the other 2 x 2 schemes
    schemes = None
    if not args.no_schemes:
        schemes = {}
        for name, sch in [("chaining", bmm.SCHEME_CHAINING),
                          ("strassen_winograd", bmm.SCHEME_WINOGRAD)]:
            o = opts(LEAF[args.leaf])
            o.scheme = sch
            e = events()
            e[0].record(stream)
            bmm.bmm_gf2_strassen(Ag, Bg, Cg, n, n, n, ws, depth=args.depth, options=o,
                             inplace_basis=True)
            e[1].record(stream)
            torch.cuda.synchronize()
            t = e[0].elapsed_time(e[1]) / 1e3
            keep(name, with_boolean=False)
            schemes[name] = {"gf2_s": round(t, 4), "gf2_eff_pbops": round(bops / t / 1e15, 4)}
            log(f"[bench] GF(2) {name} scheme {t:.3f} s")

    # The recursion's core alone (A-hat and B-hat^T in, C-hat out: no basis changes or
    # transposition, the paper's timing convention, section 4.2), on the GF(2) operands taken
    # as already changed; its output is not checked here (the tests check this mode).
    bmm.bmm_transpose(Bg, BTb, n, n)
    torch.cuda.synchronize()
    e = events()
    e[0].record(stream)
    bmm.bmm_gf2_strassen(Ag, BTb, Cb, n, n, n, ws, depth=args.depth, options=opts(LEAF[args.leaf]),
                         b_transposed=True, alt_basis_io=True)
    e[1].record(stream)
    torch.cuda.synchronize()
    core_s = e[0].elapsed_time(e[1]) / 1e3
    log(f"[bench] GF(2) core (alternative basis in and out) {core_s:.3f} s")
    # The Boolean leaf on dense operands (the GF(2) inputs, Bernoulli(1/2) bits) beside the
    # sparse headline inputs: the matrix cores draw more power, and run at a lower clock,
    # on dense bits.
    e = events()
    with ClockSampler() as ck:
        e[0].record(stream)
        bmm.bmm_boolean(Ag, BTb, Cb, n, n, n, options=opts(LEAF[args.leaf]), b_transposed=True)
        e[1].record(stream)
        torch.cuda.synchronize()
    dense_s = e[0].elapsed_time(e[1]) / 1e3
    dense = {"bits": "Bernoulli(1/2)", "leaf_s": round(dense_s, 4),
             "pbops": round(bops / dense_s / 1e15, 4), "sclk_ghz": ck.mean_ghz()}
    log(f"[bench] Boolean leaf on dense operands {dense_s:.3f} s")
    if args.dense_k_panel > 0:
        # the same product in k panels: each panel's operand rows stay in L2 while the
        # tiles that share them run, which cuts memory traffic and the power it draws
        kopt = opts(LEAF[args.leaf])
        kopt.k_panel = args.dense_k_panel
        e = events()
        with ClockSampler() as ck:
            e[0].record(stream)
            bmm.bmm_boolean(Ag, BTb, Cb, n, n, n, options=kopt, b_transposed=True)
            e[1].record(stream)
            torch.cuda.synchronize()
        kp_s = e[0].elapsed_time(e[1]) / 1e3
        dense["k_panel"] = {"bits": args.dense_k_panel, "leaf_s": round(kp_s, 4),
                            "pbops": round(bops / kp_s / 1e15, 4), "sclk_ghz": ck.mean_ghz()}
        log(f"[bench] ... in k panels of {args.dense_k_panel} bits {kp_s:.3f} s")

    # Rows of both products, checked against the oracle; the GF(2) rows time the oracle.
    cpu = None
    verified = None
    if not args.no_cpu_baseline:
        import numpy as np
        import oracle
        log(f"[bench] oracle: generating B on the host and computing {len(rows_sample)} rows")
        Bh = bmmgen.fill_cpu(n, n, seed, bmmgen.TAG_B, bmmgen.Dist.half())
        Ar = bmmgen.fill_rows_cpu(rows_sample, n, seed, bmmgen.TAG_A, bmmgen.Dist.half())
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        c0 = time.perf_counter()
        want = oracle.rows(Ar, Bh, n, n, oracle.GF2)
        c1 = time.perf_counter()
        log(f"[bench] oracle {c1 - c0:.2f} s for {len(rows_sample)} rows on {threads} threads")
        # the same oracle on one thread, on fewer rows (the first of the sample)
        r1 = max(1, min(args.cpu_rows_1core, len(rows_sample)))
        one = single_thread_seconds(lambda: oracle.rows(Ar[:r1], Bh, n, n, oracle.GF2))
        # Freivalds's check of the whole headline GF(2) product: (x^T A) B = x^T C
        freivalds = None
        if args.freivalds > 0 and C_head is not None:
            Ah = bmmgen.fill_cpu(n, n, seed, bmmgen.TAG_A, bmmgen.Dist.half())
            xs = bmmgen.freivalds_vectors(n, args.freivalds, seed)
            f0 = time.perf_counter()
            freivalds = all(oracle.freivalds(Ah, Bh, C_head, n, n, n, xs))
            log(f"[bench] {args.freivalds} Freivalds vectors in {time.perf_counter() - f0:.1f} s:"
                f" {freivalds}")
            del Ah
        del Bh
        Bbh = bmmgen.fill_cpu(n, n, seed, 0x1B, bool_dist)
        Abr = bmmgen.fill_rows_cpu(rows_sample, n, seed, 0x1A, bool_dist)
        want_b = oracle.rows(Abr, Bbh, n, n, oracle.BOOLEAN)
        del Bbh
        # every variant's kept rows: the GF(2) product and (for leaf variants) the Boolean one
        verified = {"rows": len(rows_sample)}
        if freivalds is not None:
            verified["gf2_freivalds_vectors"] = args.freivalds
            verified["gf2_freivalds"] = freivalds
        for name, (g, b) in kept.items():
            verified[name] = {"gf2": bool(np.array_equal(g.numpy().view(np.uint64), want))}
            if b is not None:
                verified[name]["boolean"] = bool(
                    np.array_equal(b.numpy().view(np.uint64), want_b))
        rate = 2.0 * len(rows_sample) * n * n / (c1 - c0)
        cpu = {"value": round(rate / 1e15, 8), "unit": "Pbop/s", "cores": threads,
               "kind": "oracle",
               "sample": f"{len(rows_sample)} stratified rows of the GF(2) product at n={n} "
                         f"(2*rows*n^2 bit ops) in {c1 - c0:.2f} s"}
        if one:
            cpu["single_core"] = {"value": round(2.0 * r1 * n * n / one / 1e15, 9), "cores": 1,
                                  "sample": f"{r1} of those rows on one thread in {one:.2f} s"}
            log(f"[bench] oracle on one thread: {r1} rows in {one:.2f} s")
        log(f"[bench] verified {verified}")

    value = 2 * bops / step_s / 1e15
    achieved = bops / leaf_s / 1e12  # TOP/s of the Boolean leaf launch
    _, leaf_tile = bmm.bmm_leaf_choice(bmm.BOOLEAN, n, n, n, 1, opts(LEAF[args.leaf]))
    traffic = MEASURED_TRAFFIC.get((args.leaf, leaf_tile, n))
    peak = {"mfma": PEAK_MFMA_I8_TOPS, "f4": PEAK_MFMA_F4_TOPS,
            "valu": PEAK_VALU_FUSED_TBOPS}[args.leaf]
    line = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "Pbop/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_s * 1e3, 2),
        "value_paper_form": round(2 * (bops - float(n) ** 2) / step_s / 1e15, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i8",
        "data": "synthetic",
        "config": {
            "workload": f"GF(2) alt-basis Strassen + Boolean cubic product, n={n} square",
            "n": n, "gf2_bits": "Bernoulli(1/2)", "boolean_bits": f"Bernoulli({bool_dist.p:g})",
            "strassen_depth": args.depth, "depth_serial": ds, "depth_parallel": dp,
            "leaf": {"mfma": "int8 MFMA", "f4": "fp4 MFMA", "valu": "VALU bitop3"}[args.leaf],
            "gf2_strassen_s": round(gf2_s, 4),
            "gf2_eff_pbops": round(bops / gf2_s / 1e15, 4),
            "gf2_core_s": round(core_s, 4),
            "gf2_core_eff_pbops": round(bops / core_s / 1e15, 4),
            "boolean_s": round(leaf_s + tr_s, 4),
            "boolean_pbops": round(bops / (leaf_s + tr_s) / 1e15, 4),
            "boolean_leaf_s": round(leaf_s, 4), "boolean_leaf_pbops": round(bops / leaf_s / 1e15, 4),
        },
        "sclk_ghz": step_sclk,
        "boolean_dense_leaf": dense,
        "valu_leaf": valu,
        "f4_leaf": f4,
        "gf2_schemes": schemes,
        "roofline": {"bound": "alu" if args.leaf == "valu" else "mfma",
                     "kernel": ("leaf_valu_kernel" if args.leaf == "valu" else "leaf_mfma_kernel")
                               + f" tile {leaf_tile} (Boolean cubic product, one launch per step)",
                     "achieved": round(achieved, 1), "peak": peak,
                     "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
                     "traffic": traffic, "sclk_ghz_step": step_sclk},
        "cpu_baseline": cpu,
        "verified": verified,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
