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
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-op", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-int", action="store_true", help="skip the integer-arithmetic comparison run")
    ap.add_argument("--workload", choices=["uint16", "mixed", "serving", "rotate"], default="uint16",
                    help="uint16: LT+max+min at N=2^15 (default); mixed: 256 single-digit pairs over "
                         "N in {2^13,2^14,2^15} in one graph; serving: Poisson request stream; "
                         "rotate: slot rotations of 192 ciphertexts at N=2^15")
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
        return mixed(a)
    if a.workload == "serving":
        return serve(a)
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
    tuned = dev.autotune()
    # the groups run as SPLIT concurrent slices on library streams (two timed
    # fastest: 1, 2 and 4 slices gave 165, 159-160 and 164-166 ms a step)
    dev.set_tuning(bc.BC_TUNE_SPLIT_STREAMS, a.split)
    tuned["split_streams"] = a.split
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
            rec = {name: dev.profile_read(kind) for name, kind in (
                ("forward", bc.BC_PROF_NTT_FWD), ("inverse", bc.BC_PROF_NTT_INV),
                ("forward_part", bc.BC_PROF_NTT_FWD_PART), ("inverse_part", bc.BC_PROF_NTT_INV_PART),
                ("forward_combine", bc.BC_PROF_NTT_FWD_COMBINE))}
        dev.profile_enable(False)
        return e0.elapsed_time(e1) / a.steps, wall, rec

    if a.split > 1:
        # throughput with the slices concurrent; the per-launch transform
        # figures then come from a second pass with the slices one after
        # another, where launches do not overlap (an overlapped launch's
        # duration includes the other slice's kernels)
        ms_step, wall_step, _ = timed(False)
        dev.set_tuning(bc.BC_TUNE_SPLIT_STREAMS, 1)
        dev.compare_max_min(keys, A, B, outs=outs)  # warms the unsplit workspace
        unsplit_ms, _, prof = timed(True)
        dev.set_tuning(bc.BC_TUNE_SPLIT_STREAMS, a.split)
    else:
        ms_step, wall_step, prof = timed(True)
        unsplit_ms = ms_step
    # the roofline kernel: the key-switching forward transform (part-limb
    # blocks when the producers fold its first stages, else whole limbs)
    rk = "forward_part" if prof["forward_part"][1] > 0 else "forward"
    fwd_ms, fwd_n, fwd_bytes = prof[rk]

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
    traffic = measured_traffic()

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
                               f"BGV N=2^{prm['logN']} p={prm['p']} Q={prm['nQ']}x{prm['bitsQ']}b "
                               f"P={prm['nP']}x{prm['bitsP']}b dnum={prm['dnum']}, batched "
                               f"({a.split} concurrent slices)",
                   "groups": G, "slots": M, "planes": NDIG, "N": N},
        "slot_comparisons_per_s": value * NDIG,
        "wall_ms_per_step": wall_step,
        "unsplit_ms_per_step": unsplit_ms,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "measured_in": ("the same step with the slices one after another (launches do not overlap)"
                                     if a.split > 1 else "the timed steps"),
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_note": "HBM bytes per launch from FETCH_SIZE/WRITE_SIZE, copy-calibrated",
                     "kernel": ("forward NTT of the key-switching limbs, "
                                + ("2^13-word part-limb blocks (first stages folded into modulus raising)"
                                   if rk == "forward_part" else
                                   "single pass" if tuned["single_pass"] else "column pass + row pass")
                                + (", fp64" if tuned.get("fp64") else ", integer") + " arithmetic, 16 N bytes per limb"),
                     "ntt_schedule": tuned,
                     "launches": fwd_n, "avg_launch_us": 1e3 * fwd_ms / max(1, fwd_n),
                     "avg_launch_MB": fwd_bytes / max(1, fwd_n) / 1e6,
                     "transforms": {k: {"GBs": b / (ms / 1e3) / 1e9, "launches": n, "avg_launch_us": 1e3 * ms / n}
                                    for k, (ms, n, b) in prof.items() if n > 0 and ms > 0}},
        "graph_replay_ms_per_step": graph_ms,
        "integer_arithmetic": int_path,
        "per_op_launch": None if per_op is None else {"ms_per_step": per_op, "batched_speedup": per_op / ms_step},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "ntt_forward_traffic_n15.txt")
NTT_SOURCES = [os.path.join(ROOT, "paper_2407_07308_amd", "csrc", f) for f in ("ntt.hip", "bc_internal.h")]


def ntt_source_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in NTT_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def is_forward_ntt(name: str, parts: bool) -> str | None:
    """The roofline kernel's launches: with part-limb transforms, 'a' for each
    forward part-limb launch; else 'a' for the first pass (or the single pass)
    of a forward transform and 'b' for the second."""
    import re

    if parts:
        return "a" if re.search(r"ntt_part<\d+, [^,]+, \d+(, false)?>", name) else None
    m = re.search(r"ntt_(cols|rows|full)<\d+, false[,>]", name)
    if not m:
        return None
    return "b" if m.group(1) == "rows" else "a"


def pmc_summary(fetch_csv: str, write_csv: str, command: str):
    """Per-launch HBM bytes of the forward NTT from two rocprofv3 --pmc runs.
    FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are scaled by what they read
    for the 1 GiB device copy the profiled run performs first."""
    import csv

    out = {}
    for path, counter in ((fetch_csv, "FETCH_SIZE"), (write_csv, "WRITE_SIZE")):
        rows = [r for r in csv.DictReader(open(path)) if r.get("Counter_Name", counter) == counter]
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
        # the calibration copy is the first copy dispatched after the 1 GiB fill
        fill = max((i for i, r in enumerate(rows) if "Fill" in r["Kernel_Name"]),
                   key=lambda i: int(rows[i]["Grid_Size"]))
        ref = next(float(r["Counter_Value"]) for r in rows[fill + 1:] if "copyBuffer" in r["Kernel_Name"])
        scale = (1 << 20) / ref  # KiB the copy should have counted / KiB counted
        # only the comparison steps (they start with the plane subtraction),
        # as in the timed region; set-up transforms (tuning, encryption) excluded
        first = next(i for i, r in enumerate(rows) if "k_addsub" in r["Kernel_Name"])
        parts = any("ntt_part<" in r["Kernel_Name"] for r in rows[first:])
        tot, launches = 0.0, 0
        for r in rows[first:]:
            kind = is_forward_ntt(r["Kernel_Name"], parts)
            if kind:
                tot += float(r["Counter_Value"]) * 1024 * scale
                launches += kind == "a"
        out[counter] = {"scale": scale, "bytes": tot, "launches": launches}
    per_launch = (out["FETCH_SIZE"]["bytes"] + out["WRITE_SIZE"]["bytes"]) / max(1, out["FETCH_SIZE"]["launches"])
    rec = {"kernel": "forward NTT" + (", part-limb blocks" if parts else ""), "source_hash": ntt_source_hash(),
           "traffic_bytes_per_launch": per_launch,
           "fetch_scale": out["FETCH_SIZE"]["scale"], "write_scale": out["WRITE_SIZE"]["scale"],
           "launches": out["FETCH_SIZE"]["launches"], "command": command}
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


def measured_traffic():
    """Forward-NTT bytes per launch from the committed counter summary, if the
    transform source is unchanged since the counters were taken."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    return rec["traffic_bytes_per_launch"] if rec.get("source_hash") == ntt_source_hash() else None


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
    slot values in [0, 257): one recorded fork/join graph per step."""
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
    outs = grp.compare_max_min(reqs, want_max=False, want_min=False)
    for _ in range(max(0, a.warmup - 1)):
        grp.compare_max_min(reqs, outs=outs, want_max=False, want_min=False)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(a.steps):
        grp.compare_max_min(reqs, outs=outs, want_max=False, want_min=False)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / a.steps
    for dev, (dk, _, _), o, t in zip(members, reqs, outs, truth):
        if not np.array_equal(dev.decrypt(dk, o[0]), t):
            print("bench: mixed decryptions are wrong", file=sys.stderr)
            sys.exit(3)
    comps = 256 * members[0].M
    print(json.dumps({"metric": "encrypted LT slot comparisons/s, mixed N in one graph", "value": comps / (ms / 1e3),
                      "unit": "comparisons/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms,
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
                      "data": "synthetic",
                      "config": {"workload": "256 single-digit LT pairs, N uniform on {2^13,2^14,2^15}, p=257",
                                 "pairs_per_N": {str(1 << L): int((pick == L).sum()) for L in (13, 14, 15)}}}))


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
    srv = serving.Server(members, max_batch_groups=32, streams=2)
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
    print(json.dumps({"metric": "serving latency p50/p99 and throughput", "value": s["throughput_req_s"],
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
                                 "distinct_payloads": len(pool)}}))


if __name__ == "__main__":
    main()
