#!/usr/bin/env python3
"""Encrypted uint16 less-than / max / min throughput at N = 2^15 on one MI355X.

Workload (one step): 64 groups of 128 uint16 pairs, each integer split into
three base-129 digit planes (one BGV ciphertext per plane and group, p = 257,
N = 2^15, 14 x 50-bit primes, 5 x 50-bit special primes, dnum = 3); the step
evaluates the lexicographic less-than over the planes and the max and min
planes -- 98 ciphertext multiplications per group, all groups batched.
Inputs are encrypted and resident in HBM before the timed region.

Reported: uint16 comparisons per second (each comparison also yields its max
and min), the forward-NTT roofline measured with HIP events on the launch
stream during the timed steps, the same step with 64-bit integer arithmetic
in place of the exact fp64 residue products (checked byte-identical), the
plain per-operation path (one group per call, same kernels), and the CPU
oracle on a one-group sample.
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
    ap.add_argument("--split", type=int, default=2,
                    help="concurrent slices of the batch, each on its own library stream (BC_TUNE_SPLIT_STREAMS)")
    ap.add_argument("--persistent", type=int, default=0,
                    help="uint16: 1 runs each step as one persistent launch (the slices as its lanes)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-op", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-int", action="store_true", help="skip the integer-arithmetic comparison run")
    ap.add_argument("--no-extra", action="store_true",
                    help="uint16 only: skip the mixed-N, serving and bivariate keys of the JSON line")
    ap.add_argument("--extra-window", type=float, default=3.0, help="serving key of the default line: seconds of arrivals")
    ap.add_argument("--biv-groups", type=int, default=4, help="bivariate: groups of 128 uint16 pairs")
    ap.add_argument("--no-mfma", action="store_true",
                    help="bivariate: the scalar combinations on the fp64 vector units instead of the matrix cores")
    ap.add_argument("--mfma-modup", type=int, default=None, choices=[0, 1],
                    help="uint16: modulus raising on the matrix cores (1) or the fp64 vector units (0); "
                         "default: the library's")
    ap.add_argument("--raw-handoff", type=int, default=None, choices=[0, 1],
                    help="uint16: limbs between key-switching kernels as reduced fp64 patterns (1) or canonical "
                         "words (0); default: what the multiplication autotuner picks (profiles pin it)")
    ap.add_argument("--packed-cts", type=int, default=64,
                    help="packed: ciphertexts per batch (32 uint16 integers each)")
    ap.add_argument("--fpd-cts", type=int, default=32,
                    help="fpd: ciphertexts per batch (128 uint16 values each, two F_p digits per F_257^256 slot)")
    ap.add_argument("--workload", choices=["uint16", "mixed", "serving", "rotate", "bivariate", "packed", "bluestein", "fpd"],
                    default="uint16",
                    help="uint16: LT+max+min at N=2^15 (default); mixed: 256 single-digit pairs over "
                         "N in {2^13,2^14,2^15} in one graph; serving: Poisson request stream; "
                         "rotate: slot rotations of 192 ciphertexts at N=2^15")
    ap.add_argument("--serve-streams", type=int, default=2, help="serving: batches in flight (streams)")
    ap.add_argument("--serve-max-groups", type=int, default=32, help="serving: groups per batch at most")
    ap.add_argument("--window", type=float, default=10.0, help="serving: seconds of arrivals")
    ap.add_argument("--rate", type=float, default=200.0, help="serving: mean requests per second")
    ap.add_argument("--pmc-summary", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "COMMAND"),
                    help="write the forward-NTT traffic summary from two rocprofv3 --pmc runs and exit")
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
    if a.pmc_summary:
        return pmc_summary(*a.pmc_summary)
    if a.workload == "mixed":
        return print(json.dumps(mixed(a)))
    if a.workload == "serving":
        return print(json.dumps(serve(a)))
    if a.workload == "bivariate":
        return print(json.dumps(bivariate(a)))
    if a.workload == "packed":
        return print(json.dumps(packed(a)))
    if a.workload == "bluestein":
        return print(json.dumps(bluestein_bench(a)))
    if a.workload == "fpd":
        return print(json.dumps(fpd_bench(a)))
    if a.workload == "rotate":
        return rotate(a)
    import numpy as np
    import torch

    import paper_2407_07308_amd as bc
    import synth

    torch.cuda.set_device(0)
    prm = dict(logN=15, p=257, nQ=14, bitsQ=50, nP=5, bitsP=50, dnum=3)
    G = a.groups
    dev = bc.Context(**prm)
    N, M = dev.N, dev.M
    rnd = synth.keygen_randomness(SEED, N, prm["nQ"], prm["nP"], prm["dnum"], 0)
    keys = dev.keygen(rnd["s"], rnd["a"], rnd["e"], ())
    dev.autotune()
    tuned = dev.autotune_mul(keys)
    # the groups run as SPLIT concurrent slices on library streams (two kept:
    # re-timed with the current kernels, 1, 2, 3 and 4 slices gave 128.0,
    # 123.0-125.7, 122.3-126.7 and 126.5-127.2 ms a step)
    dev.set_tuning(bc.BC_TUNE_SPLIT_STREAMS, a.split)
    tuned["split_streams"] = a.split
    dev.set_tuning(bc.BC_TUNE_PERSISTENT, a.persistent)
    tuned["persistent"] = a.persistent
    if a.mfma_modup is not None:
        dev.set_tuning(bc.BC_TUNE_MFMA_MODUP, a.mfma_modup)
    tuned["mfma_modup"] = dev.get_tuning(bc.BC_TUNE_MFMA_MODUP)
    if a.raw_handoff is not None:
        dev.set_tuning(bc.BC_TUNE_RAW_HANDOFF, a.raw_handoff)
        tuned["raw_handoff"] = a.raw_handoff
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
    def timed(profile: bool):
        """ms per step over a.steps steps (and the transform records when profiling)."""
        dev.profile_enable(profile)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record()
        for _ in range(a.steps):
            dev.compare_max_min(keys, A, B, outs=outs)
        e1.record()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / a.steps
        rec = None
        if profile:
            rec = {name: dev.profile_read(getattr(bc, k["prof"])) for name, k in KINDS.items()}
        dev.profile_enable(False)
        return e0.elapsed_time(e1) / a.steps, wall, rec

    if a.split > 1 or a.persistent:
        # throughput with the slices concurrent (or one persistent launch);
        # the per-launch kernel figures then come from a second pass of
        # ordinary launches with the slices one after another, where launches
        # do not overlap (an overlapped launch's duration includes the other
        # slice's kernels)
        ms_step, wall_step, _ = timed(False)
        dev.set_tuning(bc.BC_TUNE_SPLIT_STREAMS, 1)
        dev.set_tuning(bc.BC_TUNE_PERSISTENT, 0)
        dev.compare_max_min(keys, A, B, outs=outs)  # warms the unsplit workspace
        unsplit_ms, _, prof = timed(True)
        dev.set_tuning(bc.BC_TUNE_SPLIT_STREAMS, a.split)
    else:
        ms_step, wall_step, prof = timed(True)
        unsplit_ms = ms_step
    # the roofline kernel: the kernel kind of the key-switching path with the
    # most time in the step; every kind is listed with its achieved GB/s
    rk = max((k for k in KINDS if k != "mul" and prof[k][1] > 0), key=lambda k: prof[k][0])
    rk_ms, rk_n, rk_bytes = prof[rk]
    # the comparisons roofline: fused-minimum bytes of every multiplication
    # of the step at its level, at 8 TB/s, against the measured step
    mul_ms, mul_n, mul_bytes = prof["mul"]
    step_min_bytes = mul_bytes / a.steps

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
    achieved = rk_bytes / (rk_ms / 1e3) / 1e9 if rk_ms > 0 else 0.0
    traffic = measured_traffic(rk)
    step_bytes = [dev.export(x) for x in [lt] + mx + mn]  # the step's results, coefficient domain

    # ------------------------------------------------- per-op launch path
    # same circuit, same kernels, one ciphertext per launch
    per_op = None
    if not a.no_per_op:
        dev.set_exec_mode(bc.BC_EXEC_PER_OP)
        dev.set_tuning(bc.BC_TUNE_SPLIT_STREAMS, 1)  # the plain path: one stream
        po = dev.compare_max_min(keys, A, B)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dev.compare_max_min(keys, A, B, outs=po)
        torch.cuda.synchronize()
        per_op = (time.perf_counter() - t0) * 1e3
        same = all(np.array_equal(dev.export(x), dev.export(y)) for x, y in [(po[0], lt)] + list(zip(po[1], mx)))
        dev.set_exec_mode(bc.BC_EXEC_BATCHED)
        dev.set_tuning(bc.BC_TUNE_SPLIT_STREAMS, a.split)
        if not same:
            print("bench: per-operation path differs from the batched path", file=sys.stderr)
            sys.exit(3)

    # the same step with 64-bit integer arithmetic everywhere (Shoup / Barrett
    # products): must give byte-identical ciphertexts; timed for comparison
    int_path = None
    if not a.no_int and tuned.get("fp64"):
        dev.set_tuning(bc.BC_TUNE_FP64, 0)
        io = dev.compare_max_min(keys, A, B)  # warm-up, integer tables
        torch.cuda.synchronize()
        i0, i1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        i0.record()
        for _ in range(a.steps):
            dev.compare_max_min(keys, A, B, outs=io)
        i1.record()
        torch.cuda.synchronize()
        int_ms = i0.elapsed_time(i1) / a.steps
        same = all(np.array_equal(dev.export(x), dev.export(y))
                   for x, y in [(io[0], lt)] + list(zip(io[1], mx)) + list(zip(io[2], mn)))
        dev.set_tuning(bc.BC_TUNE_FP64, 1)
        if not same:
            print("bench: integer arithmetic gives different ciphertexts", file=sys.stderr)
            sys.exit(3)
        int_path = {"ms_per_step": int_ms, "value": comparisons / (int_ms / 1e3), "identical_ciphertexts": True}

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
        if not all(np.array_equal(dev.export(x), y) for x, y in zip([lt] + mx + mn, step_bytes)):
            print("bench: graph replay differs from the eager step", file=sys.stderr)
            sys.exit(3)

    # ------------------------------------------------------ CPU oracle
    cpu = None
    oracle_parity = None
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
        o_mx, o_mn = oracle.max_min(ev, oa, ob, o_lt)
        t_cpu = time.perf_counter() - t0
        # group 0 of the timed step, residue for residue
        oracle_parity = all(np.array_equal(got[0], want.data)
                            for got, want in zip(step_bytes, [o_lt] + o_mx + o_mn))
        if not oracle_parity:
            print("bench: group 0 differs from the oracle", file=sys.stderr)
            sys.exit(3)
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
                               f"BGV N=2^{prm['logN']} p={prm['p']} Q={prm['nQ']}x{prm['bitsQ']}b "
                               f"P={prm['nP']}x{prm['bitsP']}b dnum={prm['dnum']}, "
                               + (f"one persistent launch per step ({a.split} lanes)" if a.persistent else
                                  f"batched ({a.split} concurrent slices)"),
                   "groups": G, "slots": M, "planes": NDIG, "N": N},
        "slot_comparisons_per_s": value * NDIG,
        "wall_ms_per_step": wall_step,
        "unsplit_ms_per_step": unsplit_ms,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_note": "HBM bytes per launch from FETCH_SIZE/WRITE_SIZE, copy-calibrated",
                     "kernel": KINDS[rk]["desc"], "kind": rk,
                     "measured_in": ("the same step as ordinary launches with the slices one after another "
                                     "(launches do not overlap)" if a.split > 1 or a.persistent else "the timed steps"),
                     "launches": rk_n, "avg_launch_us": 1e3 * rk_ms / max(1, rk_n),
                     "avg_launch_MB": rk_bytes / max(1, rk_n) / 1e6,
                     "ntt_schedule": tuned,
                     "kernels": {k: {"GBs": b / (ms / 1e3) / 1e9, "frac": b / (ms / 1e3) / 1e9 / HBM_PEAK_GBS,
                                     "launches": n, "avg_launch_us": 1e3 * ms / n, "ms_per_step": ms / a.steps}
                                 for k, (ms, n, b) in prof.items() if n > 0 and ms > 0 and k != "mul"}},
        "comparisons_roofline": {
            "bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS,
            "min_bytes_per_step": step_min_bytes, "multiplications_per_step": mul_n / a.steps,
            "min_ms_per_step": step_min_bytes / (HBM_PEAK_GBS * 1e9) * 1e3,
            "achieved": step_min_bytes / (ms_step / 1e3) / 1e9,
            "frac": step_min_bytes / (HBM_PEAK_GBS * 1e9) / (ms_step / 1e3),
            "note": "fused-minimum bytes of every multiplication at its level (two operands, the key once per "
                    "ciphertext, the result; an addend where there is one) against ms_per_step"},
        "graph_replay_ms_per_step": graph_ms,
        "integer_arithmetic": int_path,
        "per_op_launch": None if per_op is None else {"ms_per_step": per_op, "batched_speedup": per_op / ms_step},
        "cpu_baseline": cpu,
        "oracle_parity": oracle_parity,
        "oracle_parity_sample": "group 0 of the timed step: LT, 3 max and 3 min planes, every residue" if cpu else None,
    }
    if not a.no_extra:
        # the other workloads, each checked against its plaintext answers:
        # mixed N (one persistent launch per step), a short serving window,
        # uint16 as two base-257 digits with the bivariate circuit, and uint16
        # packed four slots per integer (rotations inside the circuit)
        import gc

        # the uint16 context, its recorded graph (which holds a whole step's
        # workspace) and every buffer of this workload go first
        del outs, A, B, lt, mx, mn, step_bytes
        po = io = None  # noqa: F841 (the per-op and integer-path outputs, if any)
        del dev, keys
        gc.collect()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        sub = argparse.Namespace(**vars(a))
        sub.window = a.extra_window
        for name, fn in (("mixed", mixed), ("serving", serve), ("bivariate", bivariate), ("packed", packed),
                         ("bluestein", bluestein_bench), ("fpd", fpd_bench)):
            print(f"bench: {name}", file=sys.stderr, flush=True)
            r = fn(sub)
            for k in ("n_gpus", "higher_is_better", "scaling", "vs_baseline", "dtype", "data"):
                r.pop(k, None)
            out[name] = r
            gc.collect()
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
    print(json.dumps(out))


# Kernel kinds of the comparison step: profiler kind, the kernels' names in a
# rocprofv3 trace, the sources their code comes from, and what a launch moves.
KINDS = {
    "forward_combine": {"prof": "BC_PROF_NTT_FWD_COMBINE", "re": r"ntt_(part|full)_combine<",
                        "src": ["ntt.hip", "ntt_dev.h", "context.cpp", "bc_internal.h"],
                        "desc": "forward NTT of the relinearise+switch correction with the multiplication's last step "
                                "as its store (32 N bytes per limb: the limb, d and the accumulator read, the result "
                                "written)"},
    "forward_part": {"prof": "BC_PROF_NTT_FWD_PART", "re": r"ntt_part<\d+, [^,]+, \d+(, false(, (true|false)){0,2})?>",
                     "src": ["ntt.hip", "ntt_dev.h", "context.cpp", "bc_internal.h"],
                     "desc": "forward NTT of the raised limbs, 2^13-word part-limb blocks (16 N bytes per limb)"},
    "inverse_part": {"prof": "BC_PROF_NTT_INV_PART", "re": r"ntt_part<\d+, [^,]+, \d+, true(, (true|false)){0,2}>",
                     "src": ["ntt.hip", "ntt_dev.h", "context.cpp", "bc_internal.h"],
                     "desc": "inverse NTT of the key-switched limbs, 2^13-word part-limb blocks (16 N bytes per limb)"},
    "forward": {"prof": "BC_PROF_NTT_FWD", "re": r"ntt_(full|cols|rows)<\d+, false",
                "src": ["ntt.hip", "ntt_dev.h", "context.cpp", "bc_internal.h"], "desc": "whole-limb forward NTT (16 N bytes per limb)"},
    "inverse": {"prof": "BC_PROF_NTT_INV", "re": r"ntt_(full|cols|rows)<\d+, true",
                "src": ["ntt.hip", "ntt_dev.h", "context.cpp", "bc_internal.h"], "desc": "whole-limb inverse NTT (16 N bytes per limb)"},
    "tensor": {"prof": "BC_PROF_TENSOR", "re": r"k_tensor<", "src": ["kernels.hip", "kernels_dev.h", "bc_internal.h"],
               "desc": "tensor product / multiply-accumulate (operands read once, 3 components written)"},
    "modup": {"prof": "BC_PROF_MODUP", "re": r"k_modup<", "src": ["kernels.hip", "kernels_dev.h", "bc_internal.h"],
              "desc": "digit decomposition + basis extension (each digit's limbs read, new limbs written)"},
    "ks_inner": {"prof": "BC_PROF_KS_INNER", "re": r"k_ks_inner<", "src": ["kernels.hip", "kernels_dev.h", "bc_internal.h"],
                 "desc": "key-switch inner product (raised limbs and key read, two accumulators written)"},
    "relin_ms": {"prof": "BC_PROF_RELIN_MS", "re": r"k_relin_ms_fbc<", "src": ["kernels.hip", "kernels_dev.h", "bc_internal.h"],
                 "desc": "ModDown + modulus-switch correction (special and top limbs read, correction written)"},
    "lincomb": {"prof": "BC_PROF_LINCOMB", "re": r"k_lincomb<", "src": ["kernels.hip", "kernels_dev.h", "bc_internal.h"],
                "desc": "Paterson-Stockmeyer block combinations (babies read, blocks written)"},
    "mul": {"prof": "BC_PROF_MUL", "re": None, "src": [], "desc": "whole multiplications"},
}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "kernel_traffic_n15.json")


def source_hash(kind: str) -> str:
    import hashlib

    h = hashlib.sha256()
    for f in KINDS[kind]["src"]:
        h.update(open(os.path.join(ROOT, "paper_2407_07308_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def pmc_summary(fetch_csv: str, write_csv: str, command: str):
    """Per-launch HBM bytes of every kernel kind from two rocprofv3 --pmc runs.
    FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are scaled by what they read
    for the 1 GiB device copy the profiled run performs first; only the
    comparison's dispatches count (from the first plane subtraction on)."""
    import csv
    import re

    per = {k: {} for k in KINDS if KINDS[k]["re"]}
    scales = {}
    for path, counter in ((fetch_csv, "FETCH_SIZE"), (write_csv, "WRITE_SIZE")):
        rows = [r for r in csv.DictReader(open(path)) if r.get("Counter_Name", counter) == counter]
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
        # the calibration copy is the first copy dispatched after the 1 GiB fill
        fill = max((i for i, r in enumerate(rows) if "Fill" in r["Kernel_Name"]),
                   key=lambda i: int(rows[i]["Grid_Size"]))
        ref = next(float(r["Counter_Value"]) for r in rows[fill + 1:] if "copyBuffer" in r["Kernel_Name"])
        scales[counter] = (1 << 20) / ref  # KiB the copy should have counted / KiB counted
        first = next(i for i, r in enumerate(rows) if "k_addsub" in r["Kernel_Name"])
        for k in per:
            sel = [r for r in rows[first:] if re.search(KINDS[k]["re"], r["Kernel_Name"])]
            per[k][counter] = (sum(float(r["Counter_Value"]) for r in sel) * 1024 * scales[counter], len(sel))
    rec = {"command": command, "fetch_scale": scales["FETCH_SIZE"], "write_scale": scales["WRITE_SIZE"],
           "kinds": {}}
    for k, v in per.items():
        n = v["FETCH_SIZE"][1]
        if n:
            rec["kinds"][k] = {"source_hash": source_hash(k), "launches": n,
                               "traffic_bytes_per_launch": (v["FETCH_SIZE"][0] + v["WRITE_SIZE"][0]) / n}
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


def measured_traffic(kind: str):
    """HBM bytes per launch of `kind` from the committed counter summary, if
    its sources are unchanged since the counters were taken."""
    try:
        rec = json.load(open(TRAFFIC_FILE))["kinds"][kind]
    except (OSError, ValueError, KeyError):
        return None
    return rec["traffic_bytes_per_launch"] if rec.get("source_hash") == source_hash(kind) else None


CHAINS = {13: dict(logN=13, p=257, nQ=8, bitsQ=50, nP=4, bitsP=50, dnum=2),
          14: dict(logN=14, p=257, nQ=8, bitsQ=50, nP=4, bitsP=50, dnum=2),
          15: dict(logN=15, p=257, nQ=14, bitsQ=50, nP=5, bitsP=50, dnum=3)}


def rotate(a):
    """Slot rotations (automorphism + key switch) of a batch of top-level
    ciphertexts at N=2^15: rotations/s."""
    import numpy as np
    import torch

    import paper_2407_07308_amd as bc
    import synth

    torch.cuda.set_device(0)
    prm = CHAINS[15]
    dev = bc.Context(**prm)
    steps_rot = (1, bc.BC_ROW_SWAP)
    rnd = synth.keygen_randomness(SEED + 7, dev.N, prm["nQ"], prm["nP"], prm["dnum"], len(steps_rot))
    keys = dev.keygen(rnd["s"], rnd["a"], rnd["e"], steps_rot)
    dev.autotune()
    G = 3 * a.groups  # the comparison batch's ciphertext count
    vals = synth.slot_values(SEED + 8, G, dev.M, 0, prm["p"])
    r = synth.encrypt_randomness(SEED + 9, G, dev.N)
    x = dev.encrypt(keys, vals, r["u"], r["e"])
    y = dev.rotate(keys, x, 1)  # warm-up
    half = dev.M // 2
    want = np.concatenate([np.roll(vals[:, :half], -1, axis=1), np.roll(vals[:, half:], -1, axis=1)], axis=1)
    if not np.array_equal(dev.decrypt(keys, y), want):
        print("bench: rotated slots are wrong", file=sys.stderr)
        sys.exit(3)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(a.steps):
        dev.rotate(keys, x, 1)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / a.steps
    print(json.dumps({"metric": "ciphertext rotations/s at N=2^15", "value": G / (ms / 1e3), "unit": "rotations/s",
                      "n_gpus": 1, "steps": a.steps, "warmup": 1, "ms_per_step": ms, "higher_is_better": True,
                      "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
                      "slot_rotations_per_s": G * dev.M / (ms / 1e3),
                      "config": {"workload": f"rotation by one slot of {G} top-level ciphertexts, BGV N=2^15 "
                                             f"p=257 Q=14x50b P=5x50b dnum=3, batched", "ciphertexts": G}}))


def mixed(a):
    """256 single-digit LT pairs, N i.i.d. uniform on {2^13, 2^14, 2^15}, uniform
    slot values in [0, 257): the whole group as one persistent launch per step
    (queue reset + persistent kernel, replayed as a graph), timed beside the
    fork/join graph of ordinary launches."""
    import numpy as np
    import torch

    import paper_2407_07308_amd as bc
    import synth

    torch.cuda.set_device(0)
    seed = 104
    pick = synth.generator(seed, "schedule").integers(13, 16, size=256)
    members, reqs, truth = [], [], []
    for j, L in enumerate((13, 14, 15)):
        G = int((pick == L).sum())
        dev = bc.Context(**CHAINS[L])
        rnd = synth.keygen_randomness(seed + L, dev.N, dev.nQ, dev.nP, dev.dnum, 0)
        dk = dev.keygen(rnd["s"], rnd["a"], rnd["e"], ())
        dev.autotune()
        x = synth.slot_values(seed, G, dev.M, 0, 257, index=L)
        y = synth.slot_values(seed, G, dev.M, 0, 257, index=100 + L)
        rx, ry = synth.encrypt_randomness(seed + 10 * L, G, dev.N), synth.encrypt_randomness(seed + 10 * L + 1, G, dev.N)
        A, B = [dev.encrypt(dk, x, rx["u"], rx["e"])], [dev.encrypt(dk, y, ry["u"], ry["e"])]
        members.append(dev)
        reqs.append((dk, A, B))
        truth.append(((x.astype(np.int64) - y) % 257 >= 129).astype(np.uint32))
    grp = bc.Group(members)
    outs = None

    def timed(mode):
        """ms per step of the group in `mode` (graph replays after warm-up),
        decryptions checked afterwards; None when the mode is unavailable."""
        nonlocal outs
        try:
            grp.set_mode(mode)
        except bc.BoostcomError as e:
            print(f"bench: mixed, mode {mode} unavailable: {e}", file=sys.stderr)
            return None
        outs = grp.compare_max_min(reqs, outs=outs, want_max=False, want_min=False)
        for _ in range(max(0, a.warmup - 1)):
            grp.compare_max_min(reqs, outs=outs, want_max=False, want_min=False)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(a.steps):
            grp.compare_max_min(reqs, outs=outs, want_max=False, want_min=False)
        e1.record()
        torch.cuda.synchronize()
        for dev, (dk, _, _), o, t in zip(members, reqs, outs, truth):
            if not np.array_equal(dev.decrypt(dk, o[0]), t):
                print(f"bench: mixed decryptions are wrong (mode {mode})", file=sys.stderr)
                sys.exit(3)
        for o in outs:
            o[0].tensor.zero_()
        return e0.elapsed_time(e1) / a.steps

    fj = timed(bc.BC_GROUP_FORK_JOIN)
    ps = timed(bc.BC_GROUP_PERSISTENT)
    shape = grp.mode()
    ms = min(x for x in (fj, ps) if x is not None)
    comps = 256 * members[0].M
    return ({"metric": "encrypted LT slot comparisons/s, mixed N", "value": comps / (ms / 1e3),
                      "unit": "comparisons/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms,
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
                      "data": "synthetic",
                      "config": {"workload": "256 single-digit LT pairs, N uniform on {2^13,2^14,2^15}, p=257",
                                 "pairs_per_N": {str(1 << L): int((pick == L).sum()) for L in (13, 14, 15)}},
                      "mode": "persistent" if ms == ps else "fork/join",
                      "persistent": None if ps is None else {
                          "ms_per_step": ps, "stages": shape[1], "tickets": shape[2], "workgroups": shape[3],
                          "launches_per_step": 2},
                      "fork_join_ms_per_step": fj})


def bivariate(a):
    """uint16 as two base-257 digits (full-range digits of F_257) compared by
    the bivariate circuit at N = 2^15: LT + max + min of a.biv_groups groups
    of 128 pairs, checked against the plaintext answers."""
    import numpy as np
    import torch

    import paper_2407_07308_amd as bc
    import synth

    torch.cuda.set_device(0)
    prm = dict(logN=15, p=257, nQ=14, bitsQ=50, nP=5, bitsP=50, dnum=3)
    dev = bc.Context(**prm)
    rnd = synth.keygen_randomness(SEED + 1, dev.N, prm["nQ"], prm["nP"], prm["dnum"], 0)
    keys = dev.keygen(rnd["s"], rnd["a"], rnd["e"], ())
    dev.autotune()
    if getattr(a, "no_mfma", False):
        dev.set_tuning(bc.BC_TUNE_MFMA, 0)
    G, nd, base = a.biv_groups, 2, 257
    xs = synth.integers(SEED + 2, (G, dev.M), 0, 65536)
    ys = synth.integers(SEED + 2, (G, dev.M), 0, 65536, index=1)
    A = [dev.encrypt(keys, pl, *synth.encrypt_randomness(SEED + 30 + d, G, dev.N).values())
         for d, pl in enumerate(digits(xs, base, nd))]
    B = [dev.encrypt(keys, pl, *synth.encrypt_randomness(SEED + 40 + d, G, dev.N).values())
         for d, pl in enumerate(digits(ys, base, nd))]
    outs = dev.compare_max_min(keys, A, B, circuit=bc.BC_CIRCUIT_BIVARIATE)  # warm-up
    steps = max(1, min(a.steps, 3))
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        dev.compare_max_min(keys, A, B, outs=outs, circuit=bc.BC_CIRCUIT_BIVARIATE)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    lt, mx, mn = outs
    val = lambda planes: sum(dev.decrypt(keys, p).astype(np.int64) * base ** (nd - 1 - i) for i, p in enumerate(planes))
    if not (np.array_equal(dev.decrypt(keys, lt), (xs < ys).astype(np.uint32))
            and np.array_equal(val(mx), np.maximum(xs, ys)) and np.array_equal(val(mn), np.minimum(xs, ys))):
        print("bench: bivariate decryptions are wrong", file=sys.stderr)
        sys.exit(3)
    return {"metric": "encrypted uint16 comparisons/s, bivariate circuit", "value": G * dev.M / (ms / 1e3),
            "unit": "comparisons/s", "n_gpus": 1, "steps": steps, "ms_per_step": ms, "higher_is_better": True,
            "dtype": "u64", "data": "synthetic",
            "config": {"workload": f"uint16 as 2 base-257 digits, LT+max+min, bivariate circuit, {G} groups x "
                                   f"{dev.M} slots, BGV N=2^15 p=257 Q=14x50b P=5x50b dnum=3",
                       "multiplications_per_group": nd * 518 + nd - 1 + 2 * nd,
                       "scalar_combinations": "fp64 vector units" if getattr(a, "no_mfma", False)
                       else "int8 matrix cores"}}


def packed(a):
    """uint16 packed into slots (three base-129 digits under a zero digit, four
    consecutive slots per integer, 32 integers per ciphertext) at N = 2^15:
    per-slot LT and EQ by the univariate circuit, then two rounds of rotation
    and multiply-accumulate; plus the tournament minimum over pairs of slots
    of the same batch.  Checked against the plaintext answers."""
    import numpy as np
    import torch

    import paper_2407_07308_amd as bc
    import synth

    torch.cuda.set_device(0)
    prm = dict(logN=15, p=257, nQ=14, bitsQ=50, nP=5, bitsP=50, dnum=3)
    dev = bc.Context(**prm)
    steps_rot = (1, 2)
    rnd = synth.keygen_randomness(SEED + 3, dev.N, prm["nQ"], prm["nP"], prm["dnum"], len(steps_rot))
    keys = dev.keygen(rnd["s"], rnd["a"], rnd["e"], steps_rot)
    dev.autotune()
    G, l, nd, base, M = a.packed_cts, 4, 3, 129, dev.M
    per = M // l
    xs = synth.integers(SEED + 4, (G, per), 0, 65536)
    ys = synth.integers(SEED + 4, (G, per), 0, 65536, index=1)

    def pack(vals):
        out = np.zeros((G, M), dtype=np.uint32)
        h = M // 2
        for i, pl in enumerate(digits(vals, base, l)):  # digit i of every integer
            for k in range(per):
                r, j = divmod(k, h // l)
                out[:, r * h + j * l + i] = pl[:, k]
        return out
    A = dev.encrypt(keys, pack(xs), *synth.encrypt_randomness(SEED + 50, G, dev.N).values())
    B = dev.encrypt(keys, pack(ys), *synth.encrypt_randomness(SEED + 51, G, dev.N).values())
    lt = dev.compare_packed(keys, A, B, l)  # warm-up
    steps = max(1, min(a.steps, 3))
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        dev.compare_packed(keys, A, B, l, out=lt)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    h = M // 2
    first = [r * h + j * l for r in range(2) for j in range(h // l)]
    if not np.array_equal(dev.decrypt(keys, lt)[:, first], (xs < ys).astype(np.uint32)):
        print("bench: packed decryptions are wrong", file=sys.stderr)
        sys.exit(3)
    # the tournament over pairs of slots (single base-129 digits per slot)
    x1 = synth.slot_values(SEED + 52, G, M, 0, 129)
    X = dev.encrypt(keys, x1, *synth.encrypt_randomness(SEED + 53, G, dev.N).values())
    mn = dev.tournament(keys, X, 2)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        dev.tournament(keys, X, 2, out=mn)
    e1.record()
    torch.cuda.synchronize()
    t_ms = e0.elapsed_time(e1) / steps
    rows = x1.reshape(G, 2, h).astype(np.int64)
    want = np.minimum(rows, np.roll(rows, -1, axis=2)).reshape(G, M)
    if not np.array_equal(dev.decrypt(keys, mn).astype(np.int64), want):
        print("bench: tournament decryptions are wrong", file=sys.stderr)
        sys.exit(3)
    return {"metric": "encrypted uint16 comparisons/s, slot-packed digits", "value": G * per / (ms / 1e3),
            "unit": "comparisons/s", "n_gpus": 1, "steps": steps, "ms_per_step": ms, "higher_is_better": True,
            "dtype": "u64", "data": "synthetic",
            "config": {"workload": f"uint16 as 3 base-129 digits in 4 consecutive slots, LT by the univariate "
                                   f"circuit + 2 rounds of rotation and multiply-accumulate, {G} ciphertexts x "
                                   f"{per} integers, BGV N=2^15 p=257 Q=14x50b P=5x50b dnum=3",
                       "multiplications_per_ciphertext": 30 + 3, "rotations_per_ciphertext": 3},
            "tournament": {"ms_per_call": t_ms, "window": 2, "ciphertexts": G,
                           "min_pairs_per_s": G * M / (t_ms / 1e3)}}


def fpd_bench(a):
    """uint16 values as two coordinates of the F_{257^256} slots of a
    ciphertext at N = 2^15 (128 values per ciphertext): both F_p digits
    extracted by the mod-extract step (monomial product, eight Frobenius
    doublings, the scalar 1/d) for a batch of ciphertexts, checked against the
    plaintext coordinates."""
    import numpy as np
    import torch

    import paper_2407_07308_amd as bc
    import synth

    torch.cuda.set_device(0)
    prm = dict(logN=15, p=257, nQ=14, bitsQ=50, nP=5, bitsP=50, dnum=3)
    dev = bc.Context(**prm)
    d, steps_f = dev.fpd_info()
    rnd = synth.keygen_randomness(SEED + 7, dev.N, prm["nQ"], prm["nP"], prm["dnum"], len(steps_f))
    keys = dev.keygen(rnd["s"], rnd["a"], rnd["e"], steps_f)
    dev.autotune()
    G, M, p = a.fpd_cts, dev.M, prm["p"]
    xs = synth.integers(SEED + 8, (G, M), 0, 65536)
    E = np.zeros((G, M, d), dtype=np.uint32)
    E[:, :, 1], E[:, :, 0] = xs // p, xs % p
    X = dev.encrypt_poly(keys, dev.encode_fpd(E), *synth.encrypt_randomness(SEED + 9, G, dev.N).values())
    out = dev.extract_digits(keys, X, [1, 0])  # warm-up
    steps = max(1, min(a.steps, 3))
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        dev.extract_digits(keys, X, [1, 0], out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    planes = out.split(2)
    if not (np.array_equal(dev.decrypt(keys, planes[0]), E[:, :, 1]) and
            np.array_equal(dev.decrypt(keys, planes[1]), E[:, :, 0])):
        print("bench: extracted digits are wrong", file=sys.stderr)
        sys.exit(3)
    return {"metric": "F_{p^d} digit extractions/s", "value": 2 * G / (ms / 1e3), "unit": "digit planes/s",
            "n_gpus": 1, "steps": steps, "ms_per_step": ms, "higher_is_better": True, "dtype": "u64",
            "data": "synthetic", "values_per_s": G * M / (ms / 1e3),
            "config": {"workload": f"uint16 as coordinates 1 and 0 of the F_257^{d} slots, {G} ciphertexts x {M} "
                                   f"values, both digits extracted (x^-k product, {len(steps_f)} Frobenius "
                                   f"doublings, scalar 1/d), BGV N=2^15 p=257 Q=14x50b P=5x50b dnum=3",
                       "rotations_per_call": 2 * G * len(steps_f)}}


def bluestein_bench(a):
    """Transforms of the non-power-of-two ring Z_q[X]/(Phi_m), m = 18157
    (n = phi(m) = 17820, convolution length 2^16), on 16 polynomials of 14
    primes each (a ciphertext's worth of limbs): forward and inverse timed
    separately, checked by the round trip."""
    import numpy as np
    import torch

    import paper_2407_07308_amd as bc
    import synth

    torch.cuda.set_device(0)
    m, nprimes, count = 18157, 14, 16
    plan = bc.Bluestein(m, nprimes, 50)
    g = synth.generator(SEED + 7, "poly")
    x = np.stack([np.stack([g.integers(0, q, plan.n, dtype=np.uint64) for q in plan.moduli]) for _ in range(count)])
    xd = torch.from_numpy(x).cuda()
    fx = plan.forward(xd)
    back = plan.inverse(fx)
    torch.cuda.synchronize()
    if not torch.equal(back, xd):
        print("bench: Bluestein round trip failed", file=sys.stderr)
        sys.exit(3)
    steps = max(3, min(a.steps, 10))
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record()
    for _ in range(steps):
        plan.forward(xd, out=fx)
    e1.record()
    for _ in range(steps):
        plan.inverse(fx, out=back)
    e2.record()
    torch.cuda.synchronize()
    fwd, inv = e0.elapsed_time(e1) / steps, e1.elapsed_time(e2) / steps
    limbs = count * nprimes
    return {"metric": "non-power-of-two ring transforms (forward + inverse), limbs/s", "value": limbs / ((fwd + inv) / 1e3),
            "unit": "limbs/s", "n_gpus": 1, "steps": steps, "higher_is_better": True, "dtype": "u64",
            "data": "synthetic",
            "config": {"workload": f"Z_q[X]/(Phi_m), m={m} (n={plan.n}), convolution length {plan.conv_len}, "
                                   f"{count} polynomials x {nprimes} primes of 50 bits, Bluestein forward and inverse"},
            "forward_ms": fwd, "inverse_ms": inv,
            "forward_us_per_limb": 1e3 * fwd / limbs, "inverse_us_per_limb": 1e3 * inv / limbs,
            "forward_algorithmic_GBs": 16.0 * plan.n * limbs / (fwd / 1e3) / 1e9}


def serve(a):
    """Poisson arrivals of LT / max / argmax requests over uint16 vectors of
    length n (log-uniform on 64..4096), N uniform on {2^14, 2^15}."""
    import numpy as np
    import torch

    import paper_2407_07308_amd as bc
    import synth
    from paper_2407_07308_amd import serving

    torch.cuda.set_device(0)
    seed = 105
    members = {}
    for L in (14, 15):
        prm = dict(CHAINS[15])
        prm["logN"] = L
        dev = bc.Context(**prm)
        rnd = synth.keygen_randomness(seed + L, dev.N, dev.nQ, dev.nP, dev.dnum, 0)
        members[dev.N] = (dev, dev.keygen(rnd["s"], rnd["a"], rnd["e"], ()))
        dev.autotune()
    g = synth.generator(seed, "schedule")
    # Requests draw their encrypted operands from a pool of POOL distinct
    # payloads per (N, groups), encrypted up front: the server's work does not
    # depend on the values, and a long window would not fit in HBM otherwise.
    POOL = 4
    pool = {}

    def payload(N, groups, k):
        key = (N, groups, k)
        if key not in pool:
            dev, dk = members[N]
            s0 = 1000 + 97 * len(pool)
            xs = synth.integers(s0, (groups, dev.M), 0, 65536)
            ys = synth.integers(s0, (groups, dev.M), 0, 65536, index=1)
            enc = lambda vals, s: [dev.encrypt(dk, pl, *synth.encrypt_randomness(s + d, groups, dev.N).values())
                                   for d, pl in enumerate(digits(vals, BASE, NDIG))]
            pool[key] = (xs, ys, enc(xs, s0 + 11), enc(ys, s0 + 31))
        return pool[key]

    reqs, t = [], 0.0
    while True:
        t += float(g.exponential(1.0 / a.rate))
        if t > a.window:
            break
        N = 1 << int(g.integers(14, 16))
        n = 1 << int(g.integers(6, 13))
        kind = ["lt", "max", "argmax"][int(g.integers(0, 3))]
        groups = -(-n // members[N][0].M)
        rid = len(reqs)
        xs, ys, pa, pb = payload(N, groups, rid % POOL)
        r = serving.Request(rid, kind, N, groups, t, pa, pb)
        r.xs, r.ys = xs, ys
        reqs.append(r)
    torch.cuda.synchronize()
    srv = serving.Server(members, max_batch_groups=a.serve_max_groups, streams=a.serve_streams)
    step = max(1, len(reqs) // 20)
    checked = reqs[:: max(1, len(reqs) // 8)]
    keep = {id(r) for r in checked}

    def hand_on(r):
        # results leave the server (as if sent to the client); the checked ones stay
        if id(r) not in keep:
            r.result = None

    srv.run(reqs, progress=lambda d, n: print(f"served {d}/{n}", file=sys.stderr, flush=True)
            if d // step != (d - 1) // step or d == n else None, on_complete=hand_on)
    for r in checked:
        dev, dk = members[r.N]
        if not np.array_equal(dev.decrypt(dk, r.result[0]), (r.xs < r.ys).astype(np.uint32)):
            print("bench: served decryptions are wrong", file=sys.stderr)
            sys.exit(3)
    s = serving.latency_summary(reqs)
    groups = sum(r.groups for r in reqs)
    span = max(r.done_at for r in reqs)
    return ({"metric": "serving latency p50/p99 and throughput", "value": s["throughput_req_s"],
                      "unit": "requests/s", "n_gpus": 1, "higher_is_better": True, "dtype": "u64",
                      "data": "synthetic", "p50_ms": s["p50_ms"], "p99_ms": s["p99_ms"], "mean_ms": s["mean_ms"],
                      "uint16_comparisons_per_s": groups * 128 / span, "batches": srv.stats["batches"],
                      "oom_retries": srv.stats.get("oom_retries", 0),
                      "max_workspace_gb": srv.stats.get("max_pool_bytes", 0) / 1e9,
                      "budget_gb": srv.budget / 1e9,
                      "group_gb": {f"{N}x{nd}": b / 1e9 for (N, nd), b in srv.bpg.items()},
                      "config": {"workload": f"Poisson {a.rate:.0f} req/s for {a.window} s, LT/max/argmax, "
                                             f"n log-uniform 64..4096, N in {{2^14,2^15}}, p=257",
                                 "requests": len(reqs), "groups": groups,
                                 "distinct_payloads": len(pool)}})


if __name__ == "__main__":
    main()
