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
# 256 CU * 128 lane-ops/clk (the fp32 vector rate: 157.3 TFLOP/s / 2) * 2.4 GHz * 32 bits
# * 2 bit operations (AND and XOR/OR) per fused v_bitop3_b32
PEAK_VALU_FUSED_TBOPS = 5033.2


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1 << 18)
    ap.add_argument("--depth", type=int, default=6, help="Strassen levels above the leaf")
    ap.add_argument("--depth-serial", type=int, default=-1)
    ap.add_argument("--tile", type=int, default=0, help="MFMA leaf tile variant (0 = auto)")
    ap.add_argument("--no-valu", action="store_true", help="skip the VALU-leaf side step")
    ap.add_argument("--cpu-rows", type=int, default=256,
                    help="rows of the GF(2) product the oracle computes for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    return ap.parse_args()


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

    def opts(leaf):
        return bmm.Options(leaf=leaf, tile=args.tile if leaf == bmm.LEAF_MFMA_I8 else 0,
                           depth_serial=args.depth_serial,
                           depth_parallel=-1 if args.depth_serial < 0 else
                           args.depth - args.depth_serial)

    nbytes, ds, dp = bmm.bmm_gf2_strassen_workspace(n, n, n, args.depth, opts(bmm.LEAF_MFMA_I8))
    ws = torch.empty(nbytes // 8 + 1, dtype=torch.int64, device=dev)
    log(f"[bench] Strassen depth {args.depth} (serial {ds}, parallel {dp}), workspace "
        f"{nbytes / 2**30:.1f} GiB")
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()

    def step(leaf, ev=None):
        o = opts(leaf)
        if ev:
            ev[0].record(stream)
        bmm.bmm_gf2_strassen(Ag, Bg, Cg, n, n, n, ws, depth=args.depth, options=o)
        if ev:
            ev[1].record(stream)
        bmm.bmm_transpose(Bb, BTb, n, n)
        if ev:
            ev[2].record(stream)
        bmm.bmm_boolean(Ab, BTb, Cb, n, n, n, options=o, b_transposed=True)
        if ev:
            ev[3].record(stream)

    def events():
        return [torch.cuda.Event(enable_timing=True) for _ in range(4)]

    for w in range(args.warmup):
        log(f"[bench] warmup step {w}")
        step(bmm.LEAF_MFMA_I8)
        torch.cuda.synchronize()

    evs = [events() for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(bmm.LEAF_MFMA_I8, evs[i])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    step_s = (t1 - t0) / args.steps
    gf2_s = sum(e[0].elapsed_time(e[1]) for e in evs) / args.steps / 1e3
    tr_s = sum(e[1].elapsed_time(e[2]) for e in evs) / args.steps / 1e3
    leaf_s = sum(e[2].elapsed_time(e[3]) for e in evs) / args.steps / 1e3
    bops = 2.0 * n ** 3
    log(f"[bench] MFMA step {step_s:.3f} s: GF(2) Strassen {gf2_s:.3f} s, transpose {tr_s * 1e3:.2f}"
        f" ms, Boolean leaf {leaf_s:.3f} s")

    valu = None
    if not args.no_valu:
        log("[bench] VALU-leaf step")
        e = events()
        step(bmm.LEAF_VALU, e)
        torch.cuda.synchronize()
        vg = e[0].elapsed_time(e[1]) / 1e3
        vb = e[2].elapsed_time(e[3]) / 1e3
        vt = e[0].elapsed_time(e[3]) / 1e3
        valu = {"step_s": round(vt, 4), "value": round(2 * bops / vt / 1e15, 4),
                "gf2_strassen_s": round(vg, 4), "gf2_eff_pbops": round(bops / vg / 1e15, 4),
                "boolean_s": round(vb, 4), "boolean_pbops": round(bops / vb / 1e15, 4),
                "boolean_leaf_frac_of_fused_valu_peak":
                    round(bops / vb / 1e12 / PEAK_VALU_FUSED_TBOPS, 4)}
        log(f"[bench] VALU step {vt:.3f} s (GF(2) {vg:.3f} s, Boolean {vb:.3f} s)")

    # Rows of both products, checked against the oracle; the GF(2) rows time the oracle.
    cpu = None
    verified = None
    rows_sample = bmmgen.stratified_rows(n, max(2, args.cpu_rows), seed)
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
        idx = torch.tensor(rows_sample, device=dev)
        got = Cg.index_select(0, idx).cpu().numpy().view(np.uint64)
        ok_g = bool(np.array_equal(got, want))
        del Bh
        Bbh = bmmgen.fill_cpu(n, n, seed, 0x1B, bool_dist)
        Abr = bmmgen.fill_rows_cpu(rows_sample, n, seed, 0x1A, bool_dist)
        want_b = oracle.rows(Abr, Bbh, n, n, oracle.BOOLEAN)
        got_b = Cb.index_select(0, idx).cpu().numpy().view(np.uint64)
        ok_b = bool(np.array_equal(got_b, want_b))
        del Bbh
        verified = {"rows": len(rows_sample), "gf2": ok_g, "boolean": ok_b}
        rate = 2.0 * len(rows_sample) * n * n / (c1 - c0)
        cpu = {"value": round(rate / 1e15, 8), "unit": "Pbop/s", "cores": threads,
               "kind": "oracle",
               "sample": f"{len(rows_sample)} stratified rows of the GF(2) product at n={n} "
                         f"(2*rows*n^2 bit ops) in {c1 - c0:.2f} s"}
        log(f"[bench] oracle {c1 - c0:.2f} s for {len(rows_sample)} rows; verified {verified}")

    value = 2 * bops / step_s / 1e15
    achieved = bops / leaf_s / 1e12  # TOP/s of the Boolean leaf launch
    line = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "Pbop/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_s * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i8",
        "data": "synthetic",
        "config": {
            "workload": f"GF(2) alt-basis Strassen + Boolean cubic product, n={n} square",
            "n": n, "gf2_bits": "Bernoulli(1/2)", "boolean_bits": f"Bernoulli({bool_dist.p:g})",
            "strassen_depth": args.depth, "depth_serial": ds, "depth_parallel": dp,
            "leaf": "int8 MFMA", "gf2_strassen_s": round(gf2_s, 4),
            "gf2_eff_pbops": round(bops / gf2_s / 1e15, 4),
            "boolean_s": round(leaf_s + tr_s, 4), "boolean_pbops": round(bops / leaf_s / 1e15, 4),
        },
        "valu_leaf": valu,
        "roofline": {"bound": "mfma", "kernel": "leaf_mfma_kernel (Boolean, one launch)",
                     "achieved": round(achieved, 1), "peak": PEAK_MFMA_I8_TOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_MFMA_I8_TOPS, 4),
                     "traffic": None},
        "cpu_baseline": cpu,
        "verified": verified,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
