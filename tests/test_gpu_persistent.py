"""The persistent executor: a group of ring sizes N = 2^13, 2^14, 2^15 as one
persistent launch draining a device work queue.

Its results must be byte-identical to each member's own comparison call (the
ordinary launches of the same kernels) and to the group's fork/join mode, on
the eager call and on graph replays with other device work between them; one
sampled pair is compared with the oracle's evaluation of the same request on
the same seeded inputs, and decryptions are checked against the plaintext
semantics.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import CtEvaluator, Oracle, Params

pytestmark = pytest.mark.gpu

BASE, ND = 129, 3
CHAINS = {13: Params(13, 257, 8, 50, 4, 50, 2), 14: Params(14, 257, 8, 50, 4, 50, 2),
          15: Params(15, 257, 14, 50, 5, 50, 3)}


def member(prm, seed):
    import paper_2407_07308_amd as bc

    dev = bc.Context.from_params(prm)
    rnd = synth.keygen_randomness(seed, prm.N, prm.nQ, prm.nP, prm.dnum, 0)
    return dev, dev.keygen(rnd["s"], rnd["a"], rnd["e"], ())


def same(dev, x, y):
    return np.array_equal(dev.export(x), dev.export(y))


def build_requests(G):
    """N = 2^13 and 2^14: single-digit LT over slot values in [0, 257);
    N = 2^15: uint16 as three base-129 planes (LT, max and min)."""
    members, reqs, truth = [], [], []
    for L, prm in CHAINS.items():
        print(f"persistent: member N=2^{L}, {G} groups", flush=True)
        dev, dk = member(prm, 150 + L)
        if L < 15:
            x = synth.slot_values(160 + L, G, dev.M, 0, 257)
            y = synth.slot_values(170 + L, G, dev.M, 0, 257)
            rx, ry = synth.encrypt_randomness(180 + L, G, dev.N), synth.encrypt_randomness(190 + L, G, dev.N)
            A, B = [dev.encrypt(dk, x, rx["u"], rx["e"])], [dev.encrypt(dk, y, ry["u"], ry["e"])]
            truth.append((((x.astype(np.int64) - y) % 257 >= 129).astype(np.uint32), None))
        else:
            xs = synth.integers(160 + L, (G, dev.M), 0, 65536)
            ys = synth.integers(170 + L, (G, dev.M), 0, 65536)
            A, B = [], []
            for d, (px, py) in enumerate(zip(oracle.to_digits(xs, BASE, ND), oracle.to_digits(ys, BASE, ND))):
                rx = synth.encrypt_randomness(180 + L + 2 * d, G, dev.N)
                ry = synth.encrypt_randomness(181 + L + 2 * d, G, dev.N)
                A.append(dev.encrypt(dk, px, rx["u"], rx["e"]))
                B.append(dev.encrypt(dk, py, ry["u"], ry["e"]))
            truth.append(((xs < ys).astype(np.uint32), (np.maximum(xs, ys), np.minimum(xs, ys))))
        members.append((dev, dk))
        reqs.append((dk, A, B))
    return members, reqs, truth


def check(members, outs, refs, truth, tag):
    for (dev, dk), o, ref, (lt, mm) in zip(members, outs, refs, truth):
        assert same(dev, o[0], ref[0]), f"{tag}: LT at N = {dev.N}"
        for x, y in zip(o[1] + o[2], ref[1] + ref[2]):
            assert same(dev, x, y), f"{tag}: max/min at N = {dev.N}"
        assert np.array_equal(dev.decrypt(dk, o[0]), lt), f"{tag}: LT decryption at N = {dev.N}"
        if mm is not None:
            mx = sum(dev.decrypt(dk, p).astype(np.int64) * BASE ** (ND - 1 - d) for d, p in enumerate(o[1]))
            mn = sum(dev.decrypt(dk, p).astype(np.int64) * BASE ** (ND - 1 - d) for d, p in enumerate(o[2]))
            assert np.array_equal(mx, mm[0]) and np.array_equal(mn, mm[1]), f"{tag}: max/min decryption"


def test_persistent_group_matches_separate_calls_fork_join_and_oracle():
    import torch

    import paper_2407_07308_amd as bc

    G = 3
    members, reqs, truth = build_requests(G)
    refs = []
    for (dev, dk), (_, A, B) in zip(members, reqs):
        if len(A) == 1:
            refs.append((dev.compare_lt(dk, A, B), [], []))
        else:
            lt, mx, mn = dev.compare_max_min(dk, A, B)
            refs.append((lt, mx, mn))
    # oracle parity of pair 1 of the N = 2^13 member
    prm, pi = CHAINS[13], 1
    orc = Oracle(prm)
    orc.keygen(synth.keygen_randomness(150 + 13, prm.N, prm.nQ, prm.nP, prm.dnum, 0))
    x = synth.slot_values(160 + 13, G, orc.M, 0, 257)
    y = synth.slot_values(170 + 13, G, orc.M, 0, 257)
    rx, ry = synth.encrypt_randomness(180 + 13, G, orc.N), synth.encrypt_randomness(190 + 13, G, orc.N)
    ox = orc.encrypt(x[pi], rx["u"][pi], rx["e"][pi])
    oy = orc.encrypt(y[pi], ry["u"][pi], ry["e"][pi])
    o_lt = oracle.compare_lt(CtEvaluator(orc), [ox], [oy], 257)
    assert np.array_equal(members[0][0].export(refs[0][0])[pi], o_lt.data)

    grp = bc.Group([m[0] for m in members])
    assert grp.mode()[0] == bc.BC_GROUP_FORK_JOIN  # the default
    grp.set_mode(bc.BC_GROUP_PERSISTENT)

    # LT for the single-digit members, LT + max + min for the uint16 member
    outs = []
    for (dev, dk), (_, A, B) in zip(members, reqs):
        ltl, mml = dev.compare_levels(A[0].level, len(A))
        if len(A) == 1:
            outs.append((dev.new_batch(G, ltl), [], []))
        else:
            outs.append((dev.new_batch(G, ltl), [dev.new_batch(G, mml) for _ in A], [dev.new_batch(G, mml) for _ in A]))

    def run(o):
        arg = [(lt, mx or None, mn or None) for lt, mx, mn in o]
        grp.compare_max_min(reqs, outs=arg)
        return o

    print("persistent: eager call", flush=True)
    run(outs)
    mode, stages, tickets, wgs = grp.mode()
    assert mode == bc.BC_GROUP_PERSISTENT and stages > 100 and tickets >= stages and wgs >= 256
    check(members, outs, refs, truth, "eager")
    for rep in range(3):
        for o in outs:
            for x in [o[0]] + o[1] + o[2]:
                x.tensor.zero_()
        torch.cuda.synchronize()
        print(f"persistent: replay {rep}", flush=True)
        run(outs)  # graph replay
        # other device work between replays
        dev, dk = members[1]
        dev.compare_lt(dk, reqs[1][1], reqs[1][2])
        check(members, outs, refs, truth, f"replay {rep}")

    # fork/join mode gives the same bytes
    grp.set_mode(bc.BC_GROUP_FORK_JOIN)
    print("persistent: fork/join comparison", flush=True)
    for o in outs:
        for x in [o[0]] + o[1] + o[2]:
            x.tensor.zero_()
    check_fj = run(outs)
    check(members, check_fj, refs, truth, "fork/join")
    grp.set_mode(bc.BC_GROUP_PERSISTENT)


def test_persistent_mode_needs_supported_members():
    import paper_2407_07308_amd as bc

    dev, _ = member(Params(10, 257, 8, 50, 4, 50, 2), 3)
    grp = bc.Group([dev])
    assert grp.mode()[0] == bc.BC_GROUP_FORK_JOIN
    with pytest.raises(bc.BoostcomError) as ei:  # N = 2^10: no 2^13-word transform blocks
        grp.set_mode(bc.BC_GROUP_PERSISTENT)
    assert ei.value.code == bc.BC_ERR_ARG


def test_context_comparison_as_one_persistent_launch():
    """bc_compare_max_min with BC_TUNE_PERSISTENT: the split slices of the
    groups are the lanes of one persistent launch; the same bytes as the
    ordinary launches, uneven slices included, in batched and graph mode."""
    import torch

    import paper_2407_07308_amd as bc

    prm = CHAINS[15]
    dev, dk = member(prm, 177)
    G = 5
    xs = synth.integers(178, (G, dev.M), 0, 65536)
    ys = synth.integers(179, (G, dev.M), 0, 65536)
    A, B = [], []
    for d, (px, py) in enumerate(zip(oracle.to_digits(xs, BASE, ND), oracle.to_digits(ys, BASE, ND))):
        rx, ry = synth.encrypt_randomness(180 + 2 * d, G, dev.N), synth.encrypt_randomness(181 + 2 * d, G, dev.N)
        A.append(dev.encrypt(dk, px, rx["u"], rx["e"]))
        B.append(dev.encrypt(dk, py, ry["u"], ry["e"]))
    ref = dev.compare_max_min(dk, A, B)
    for split in (1, 2, 3):
        for mode in (bc.BC_EXEC_BATCHED, bc.BC_EXEC_GRAPH):
            print(f"persistent context: split {split}, mode {mode}", flush=True)
            dev.set_tuning(bc.BC_TUNE_SPLIT_STREAMS, split)
            dev.set_tuning(bc.BC_TUNE_PERSISTENT, 1)
            dev.set_exec_mode(mode)
            got = dev.compare_max_min(dk, A, B)
            for rep in range(2):
                for x, y in zip([got[0]] + got[1] + got[2], [ref[0]] + ref[1] + ref[2]):
                    assert same(dev, x, y), (split, mode, rep)
                for x in [got[0]] + got[1] + got[2]:
                    x.tensor.zero_()
                torch.cuda.synchronize()
                dev.compare_max_min(dk, A, B, outs=got)
            # the last call's outputs, then one more call, whose set-up reports
            # whether the last launch stalled; its own outputs checked after it
            torch.cuda.synchronize()
            last_ok = [same(dev, x, y) for x, y in zip([got[0]] + got[1] + got[2], [ref[0]] + ref[1] + ref[2])]
            dev.compare_max_min(dk, A, B, outs=got)
            assert all(last_ok), (split, mode, "last", last_ok)
            dev.set_tuning(bc.BC_TUNE_PERSISTENT, 0)
            dev.set_exec_mode(bc.BC_EXEC_BATCHED)
            torch.cuda.synchronize()
            for x, y in zip([got[0]] + got[1] + got[2], [ref[0]] + ref[1] + ref[2]):
                assert same(dev, x, y), (split, mode, "extra")
    assert np.array_equal(dev.decrypt(dk, got[0]), (xs < ys).astype(np.uint32))
