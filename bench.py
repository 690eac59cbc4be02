#!/usr/bin/env python3
"""Encrypted uint16 less-than / max / min throughput at N = 2^15 on one MI355X.

Workload (one step): 64 groups of 128 uint16 pairs, each integer split into
three base-129 digit planes (one BGV ciphertext per plane and group, p = 257,
N = 2^15, 14 x 50-bit primes, 4 x 60-bit special primes, dnum = 3); the step
evaluates the lexicographic less-than over the planes and the max and min
planes -- 98 ciphertext multiplications per group, all groups batched.
Inputs are encrypted and resident in HBM before the timed region.

Reported: uint16 comparisons per second (each comparison also yields its max
and min), the forward-NTT roofline measured with HIP events on the launch
stream during the timed steps, the plain per-operation path (one group per
call, same kernels), and the CPU oracle on a one-group sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "encrypted LT comparisons/s (slots/s) at N=2^15; NTT+keyswitch HBM GB/s"
HBM_PEAK_GBS = 8000.0
SEED = 105
BASE, NDIG = 129, 3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--groups", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-op", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--ntt-chunk-mb", type=float, default=None,
                    help="split batched transforms into launch pairs over at most this many MB")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 1 GiB device copy first (reference for hardware byte counters)")
    return ap.parse_args()


def digits(v, base, nd):
    import numpy as np

    v = np.asarray(v, dtype=np.int64)
    return [((v // base ** (nd - 1 - i)) % base).astype(np.uint32) for i in range(nd)]


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {a.gpus}). The comparison groups are "
              f"independent, so a multi-GPU run would give each GPU its own share of groups and keys; "
              f"that is not built here. Nothing was run.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2407_07308_amd as bc
    import synth

    torch.cuda.set_device(0)
    prm = dict(logN=15, p=257, nQ=14, bitsQ=50, nP=4, bitsP=60, dnum=3)
    G = a.groups
    dev = bc.Context(**prm)
    N, M = dev.N, dev.M
    rnd = synth.keygen_randomness(SEED, N, prm["nQ"], prm["nP"], prm["dnum"], 0)
    keys = dev.keygen(rnd["s"], rnd["a"], rnd["e"], ())
    tuned = dev.autotune()
    if a.ntt_chunk_mb is not None:
        dev.set_tuning(bc.BC_TUNE_NTT_CHUNK_BYTES, int(a.ntt_chunk_mb * 2**20))
        dev.set_tuning(bc.BC_TUNE_NTT_SINGLE_PASS, 0)
        tuned = {"single_pass": 0, "chunk_bytes": int(a.ntt_chunk_mb * 2**20)}
    if a.copy_calibration:
        src = torch.ones(2**27, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)  # reads and writes exactly 1 GiB
        torch.cuda.synchronize()
        del src, dst
    xs = synth.integers(SEED, (G, M), 0, 65536)
    ys = synth.integers(SEED, (G, M), 0, 65536, index=1)
    xd, yd = digits(xs, BASE, NDIG), digits(ys, BASE, NDIG)
    A, B = [], []
    for d in range(NDIG):
        ra = synth.encrypt_randomness(SEED + 10 + d, G, N)
        rb = synth.encrypt_randomness(SEED + 20 + d, G, N)
        A.append(dev.encrypt(keys, xd[d], ra["u"], ra["e"]))
        B.append(dev.encrypt(keys, yd[d], rb["u"], rb["e"]))
    outs = dev.compare_max_min(keys, A, B)  # also the first warm-up step
    for _ in range(max(0, a.warmup - 1)):
        dev.compare_max_min(keys, A, B, outs=outs)
    torch.cuda.synchronize()

    # ------------------------------------------------------------ timed
    dev.profile_enable(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    e0.record()
    for _ in range(a.steps):
        dev.compare_max_min(keys, A, B, outs=outs)
    e1.record()
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms_step = e0.elapsed_time(e1) / a.steps
    fwd_ms, fwd_n, fwd_bytes = dev.profile_read(bc.BC_PROF_NTT_FWD)
    inv_ms, inv_n, inv_bytes = dev.profile_read(bc.BC_PROF_NTT_INV)
    dev.profile_enable(False)

    # results of the last step must be the plaintext answers
    lt, mx, mn = outs
    ok = np.array_equal(dev.decrypt(keys, lt), (xs < ys).astype(np.uint32))
    val = lambda planes: sum(dev.decrypt(keys, p).astype(np.int64) * BASE ** (NDIG - 1 - i) for i, p in enumerate(planes))
    ok = ok and np.array_equal(val(mx), np.maximum(xs, ys)) and np.array_equal(val(mn), np.minimum(xs, ys))
    if not ok:
        print("bench: decrypted results are wrong", file=sys.stderr)
        sys.exit(3)

    comparisons = G * M
    value = comparisons / (ms_step / 1e3)
    achieved = fwd_bytes / (fwd_ms / 1e3) / 1e9 if fwd_ms > 0 else 0.0

    # ------------------------------------------------- per-op launch path
    # same circuit, same kernels, one ciphertext per launch
    per_op = None
    if not a.no_per_op:
        dev.set_exec_mode(bc.BC_EXEC_PER_OP)
        po = dev.compare_max_min(keys, A, B)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dev.compare_max_min(keys, A, B, outs=po)
        torch.cuda.synchronize()
        per_op = (time.perf_counter() - t0) * 1e3
        same = all(np.array_equal(dev.export(x), dev.export(y)) for x, y in [(po[0], lt)] + list(zip(po[1], mx)))
        dev.set_exec_mode(bc.BC_EXEC_BATCHED)
        if not same:
            print("bench: per-operation path differs from the batched path", file=sys.stderr)
            sys.exit(3)

    # recorded-graph replay of the batched launch sequence
    graph_ms = None
    if not a.no_graph:
        dev.set_exec_mode(bc.BC_EXEC_GRAPH)
        dev.compare_max_min(keys, A, B, outs=outs)  # records
        torch.cuda.synchronize()
        g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        g0.record()
        for _ in range(a.steps):
            dev.compare_max_min(keys, A, B, outs=outs)
        g1.record()
        torch.cuda.synchronize()
        graph_ms = g0.elapsed_time(g1) / a.steps
        dev.set_exec_mode(bc.BC_EXEC_BATCHED)

    # ------------------------------------------------------ CPU oracle
    cpu = None
    if not a.no_cpu_baseline:
        import oracle

        orc = oracle.Oracle(oracle.Params(**prm))
        orc.keygen(rnd)
        oa, ob = [], []
        for d in range(NDIG):
            ra = synth.encrypt_randomness(SEED + 10 + d, G, N)
            rb = synth.encrypt_randomness(SEED + 20 + d, G, N)
            oa.append(orc.encrypt(xd[d][0], ra["u"][0], ra["e"][0]))
            ob.append(orc.encrypt(yd[d][0], rb["u"][0], rb["e"][0]))
        ev = oracle.CtEvaluator(orc)
        t0 = time.perf_counter()
        o_lt = oracle.compare_lt(ev, oa, ob, prm["p"])
        oracle.max_min(ev, oa, ob, o_lt)
        t_cpu = time.perf_counter() - t0
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        cores = min(cores, os.cpu_count() or cores)
        cpu = {"value": M / t_cpu, "unit": "comparisons/s", "cores": cores, "kind": "oracle",
               "sample": f"1 group of {M} uint16 pairs (3 base-129 planes): LT + max + min, {ev.mults} "
                         f"multiplications at N=2^15, {t_cpu:.1f} s"}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "comparisons/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"uint16 lexicographic LT+max+min, {G} groups x {M} slots x {NDIG} base-129 planes, "
                               f"BGV N=2^15 p=257 Q=14x50b P=4x60b dnum=3, batched",
                   "groups": G, "slots": M, "planes": NDIG, "N": N},
        "slot_comparisons_per_s": value * NDIG,
        "wall_ms_per_step": t_wall * 1e3 / a.steps,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": ("forward NTT, " + ("single pass" if tuned["single_pass"] else "column pass + row pass")
                                + ", 16 N bytes per limb"),
                     "ntt_schedule": tuned,
                     "launches": fwd_n, "avg_launch_us": 1e3 * fwd_ms / max(1, fwd_n),
                     "avg_launch_MB": fwd_bytes / max(1, fwd_n) / 1e6,
                     "inverse_ntt_GBs": inv_bytes / (inv_ms / 1e3) / 1e9 if inv_ms > 0 else None},
        "graph_replay_ms_per_step": graph_ms,
        "per_op_launch": None if per_op is None else {"ms_per_step": per_op, "batched_speedup": per_op / ms_step},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
