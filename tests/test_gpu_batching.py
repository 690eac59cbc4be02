"""Mixed ring sizes in one recorded graph, and the continuous-batching server.

Both are scheduling layers: their results must be byte-identical to the plain
per-context comparison of the same inputs, and sampled results are compared
with the oracle's evaluation of the same request on the same seeded inputs
(one served request's LT and max planes, one N = 2^13 pair of the mixed
group); decryptions are checked against the plaintext semantics.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import CtEvaluator, Oracle, Params

pytestmark = pytest.mark.gpu

BASE, ND = 129, 3


def member(prm, seed):
    import paper_2407_07308_amd as bc

    dev = bc.Context.from_params(prm)
    rnd = synth.keygen_randomness(seed, prm.N, prm.nQ, prm.nP, prm.dnum, 0)
    return dev, dev.keygen(rnd["s"], rnd["a"], rnd["e"], ())


def planes(dev, dk, vals, seed):
    out = []
    for d, pl in enumerate(oracle.to_digits(vals, BASE, ND)):
        r = synth.encrypt_randomness(seed + d, pl.shape[0], dev.N)
        out.append(dev.encrypt(dk, pl, r["u"], r["e"]))
    return out


def same(dev, x, y):
    return np.array_equal(dev.export(x), dev.export(y))


def test_group_equals_separate_calls_and_replays():
    import paper_2407_07308_amd as bc

    members = [member(Params(10, 257, 12, 50, 4, 50, 3), 1), member(Params(11, 257, 12, 50, 4, 50, 3), 2)]
    reqs, refs, vals = [], [], []
    for i, (dev, dk) in enumerate(members):
        G = 2 + i
        xs = synth.integers(10 + i, (G, dev.M), 0, 65536)
        ys = synth.integers(10 + i, (G, dev.M), 0, 65536, index=1)
        a, b = planes(dev, dk, xs, 20 + 10 * i), planes(dev, dk, ys, 40 + 10 * i)
        reqs.append((dk, a, b))
        refs.append(dev.compare_max_min(dk, a, b))
        vals.append((xs, ys))
    grp = bc.Group([m[0] for m in members])
    outs = grp.compare_max_min(reqs)  # eager + record
    for rep in range(3):
        for (dev, dk), o, ref, (xs, ys) in zip(members, outs, refs, vals):
            assert same(dev, o[0], ref[0])
            for x, y in zip(o[1] + o[2], ref[1] + ref[2]):
                assert same(dev, x, y)
            assert np.array_equal(dev.decrypt(dk, o[0]), (xs < ys).astype(np.uint32))
        for o in outs:
            for x in [o[0]] + o[1] + o[2]:
                x.tensor.zero_()
        grp.compare_max_min(reqs, outs=outs)  # replay


def test_server_results_equal_alone_and_in_the_mix():
    from paper_2407_07308_amd import serving

    members = {1 << 10: member(Params(10, 257, 12, 50, 4, 50, 3), 3),
               1 << 11: member(Params(11, 257, 12, 50, 4, 50, 3), 4)}
    # (N, groups, kind, arrival s): a burst at t = 0 whose three N = 2^10
    # requests fit one batch (so coalescing must happen), then later arrivals
    specs = [(1 << 10, 1, "lt", 0.0), (1 << 11, 2, "max", 0.0), (1 << 10, 1, "argmax", 0.0),
             (1 << 10, 2, "max", 0.0), (1 << 11, 1, "lt", 0.002), (1 << 11, 3, "argmax", 0.004),
             (1 << 10, 1, "max", 0.006), (1 << 11, 1, "lt", 0.006), (1 << 10, 3, "lt", 0.008)]
    reqs = []
    for rid, (N, groups, kind, t) in enumerate(specs):
        dev, dk = members[N]
        xs = synth.integers(100 + rid, (groups, dev.M), 0, 65536)
        ys = synth.integers(100 + rid, (groups, dev.M), 0, 65536, index=1)
        xs[0, :3] = ys[0, :3]
        r = serving.Request(rid, kind, N, groups, t, planes(dev, dk, xs, 300 + 10 * rid),
                            planes(dev, dk, ys, 600 + 10 * rid))
        r.xs, r.ys = xs, ys
        reqs.append(r)
    # a budget of four of the larger groups: the 3-group N = 2^11 request has
    # to wait for memory while the first batches are in flight
    bpg = {(N, ND): 2 * 40 * 3 * 8 * m[0].ct_words(m[0].nQ - 1) for N, m in members.items()}
    srv = serving.Server(members, max_batch_groups=4, mem_budget_bytes=4 * max(bpg.values()), streams=2,
                         bytes_per_group=bpg)
    srv.run(reqs)
    assert all(r.done_at is not None for r in reqs)
    assert srv.stats["batches"] < len(reqs)  # the burst's N = 2^10 requests shared a batch
    assert srv.stats["max_inflight_bytes"] <= 4 * max(bpg.values())
    for r in reqs:
        dev, dk = members[r.N]
        lt, mx, _ = dev.compare_max_min(dk, r.a, r.b, True, r.kind == "max", False)
        assert same(dev, r.result[0], lt)
        assert np.array_equal(dev.decrypt(dk, r.result[0]), (r.xs < r.ys).astype(np.uint32))
        if r.kind == "max":
            for x, y in zip(r.result[1], mx):
                assert same(dev, x, y)
            val = sum(dev.decrypt(dk, p).astype(np.int64) * BASE ** (ND - 1 - i) for i, p in enumerate(r.result[1]))
            assert np.array_equal(val, np.maximum(r.xs, r.ys))
    summ = serving.latency_summary(reqs)
    assert summ["p99_ms"] >= summ["p50_ms"] > 0
    # oracle parity of one served request (request 1: N = 2^11, 2 groups,
    # max), group 1 of its batch slice: LT and every max plane
    r = reqs[1]
    assert r.kind == "max" and r.N == 1 << 11
    prm = Params(11, 257, 12, 50, 4, 50, 3)
    orc = Oracle(prm)
    orc.keygen(synth.keygen_randomness(4, prm.N, prm.nQ, prm.nP, prm.dnum, 0))
    gi = 1
    oa = oracle_planes(orc, r.xs, 300 + 10 * r.rid, gi)
    ob = oracle_planes(orc, r.ys, 600 + 10 * r.rid, gi)
    ev = CtEvaluator(orc)
    o_lt = oracle.compare_lt(ev, oa, ob, prm.p)
    o_mx, _ = oracle.max_min(ev, oa, ob, o_lt)
    dev = members[r.N][0]
    assert np.array_equal(dev.export(r.result[0])[gi], o_lt.data)
    for d in range(ND):
        assert np.array_equal(dev.export(r.result[1][d])[gi], o_mx[d].data), f"max plane {d}"


def oracle_planes(orc, vals, seed, gi):
    """The oracle's ciphertexts of group gi of `planes(dev, dk, vals, seed)`."""
    out = []
    for d, pl in enumerate(oracle.to_digits(vals, BASE, ND)):
        r = synth.encrypt_randomness(seed + d, pl.shape[0], orc.N)
        out.append(orc.encrypt(pl[gi], r["u"][gi], r["e"][gi]))
    return out


def test_server_measures_group_bytes_and_bounds_pools():
    """Without given sizes the server measures a shape's workspace once (the
    pool is empty again afterwards) and bounds each context's pool by its
    share of the budget."""
    import paper_2407_07308_amd as bc
    from paper_2407_07308_amd import serving

    members = {1 << 10: member(Params(10, 257, 12, 50, 4, 50, 3), 5),
               1 << 11: member(Params(11, 257, 12, 50, 4, 50, 3), 6)}
    srv = serving.Server(members, max_batch_groups=4, mem_budget_bytes=3 << 30, streams=1)
    limits = {N: m[0].get_tuning(bc.BC_TUNE_POOL_LIMIT_BYTES) for N, m in members.items()}
    assert sum(limits.values()) <= 3 << 30 and limits[1 << 11] > limits[1 << 10] > 0
    one, three = srv._group_bytes(1 << 11, 1), srv._group_bytes(1 << 11, ND)
    assert three > one > 0
    assert srv._group_bytes(1 << 11, ND) == three  # measured once
    assert members[1 << 11][0].pool_bytes() == 0


def test_mixed_ring_sizes_at_workload_sizes_concurrently():
    """The three workload chains (N = 2^13, 2^14, 2^15) in one fork/join graph,
    batches large enough that many workgroups of different members run at
    once: every member's LT equals its own single-context call, byte for
    byte, after the eager call and after a replay."""
    import paper_2407_07308_amd as bc

    chains = {13: Params(13, 257, 8, 50, 4, 50, 2), 14: Params(14, 257, 8, 50, 4, 50, 2),
              15: Params(15, 257, 14, 50, 5, 50, 3)}
    members, reqs, truth = [], [], []
    for L, prm in chains.items():
        dev, dk = member(prm, 50 + L)
        dev.autotune()
        G = 24
        x = synth.slot_values(60 + L, G, dev.M, 0, 257)
        y = synth.slot_values(70 + L, G, dev.M, 0, 257)
        rx, ry = synth.encrypt_randomness(80 + L, G, dev.N), synth.encrypt_randomness(90 + L, G, dev.N)
        A, B = [dev.encrypt(dk, x, rx["u"], rx["e"])], [dev.encrypt(dk, y, ry["u"], ry["e"])]
        members.append((dev, dk))
        reqs.append((dk, A, B))
        truth.append(((x.astype(np.int64) - y) % 257 >= 129).astype(np.uint32))
    refs = [dev.compare_lt(dk, A, B) for (dev, dk), (_, A, B) in zip(members, reqs)]
    # oracle parity of pair 5 of the N = 2^13 member
    prm, pi = chains[13], 5
    orc = Oracle(prm)
    orc.keygen(synth.keygen_randomness(50 + 13, prm.N, prm.nQ, prm.nP, prm.dnum, 0))
    x = synth.slot_values(60 + 13, 24, orc.M, 0, 257)
    y = synth.slot_values(70 + 13, 24, orc.M, 0, 257)
    rx, ry = synth.encrypt_randomness(80 + 13, 24, orc.N), synth.encrypt_randomness(90 + 13, 24, orc.N)
    ox = orc.encrypt(x[pi], rx["u"][pi], rx["e"][pi])
    oy = orc.encrypt(y[pi], ry["u"][pi], ry["e"][pi])
    o_lt = oracle.compare_lt(CtEvaluator(orc), [ox], [oy], 257)
    assert np.array_equal(members[0][0].export(refs[0])[pi], o_lt.data)
    grp = bc.Group([m[0] for m in members])
    outs = grp.compare_max_min(reqs, want_max=False, want_min=False)
    for rep in range(2):
        for (dev, dk), o, ref, t in zip(members, outs, refs, truth):
            assert same(dev, o[0], ref), f"N = {dev.N}, pass {rep}"
            assert np.array_equal(dev.decrypt(dk, o[0]), t)
        for o in outs:
            o[0].tensor.zero_()
        grp.compare_max_min(reqs, outs=outs, want_max=False, want_min=False)  # replay


@pytest.mark.parametrize("mode", ["batched", "graph"])
def test_split_streams_give_the_same_bytes(mode):
    """A comparison whose groups run as concurrent slices on library streams
    (uneven slices: 7 groups over 3 streams) equals the one-stream result,
    eagerly and under graph replay."""
    import paper_2407_07308_amd as bc

    prm = Params(10, 257, 12, 50, 4, 50, 3)  # 12 primes: depth for three planes, LT and max
    dev, dk = member(prm, 12)
    G = 7
    xs = synth.integers(81, (G, dev.M), 0, 65536)
    ys = synth.integers(81, (G, dev.M), 0, 65536, index=1)
    xs[0, :5] = ys[0, :5]
    A, B = planes(dev, dk, xs, 820), planes(dev, dk, ys, 830)
    lt1, mx1, mn1 = dev.compare_max_min(dk, A, B)
    assert np.array_equal(dev.decrypt(dk, lt1), (xs < ys).astype(np.uint32))
    ref = [dev.export(x) for x in [lt1] + mx1 + mn1]
    dev.set_tuning(bc.BC_TUNE_SPLIT_STREAMS, 3)
    assert dev.get_tuning(bc.BC_TUNE_SPLIT_STREAMS) == 3
    if mode == "graph":
        dev.set_exec_mode(bc.BC_EXEC_GRAPH)
    outs = dev.compare_max_min(dk, A, B)
    for rep in range(3):  # eager (graph mode: the recording run), then replays
        got = [dev.export(x) for x in [outs[0]] + outs[1] + outs[2]]
        assert all(np.array_equal(g, r) for g, r in zip(got, ref)), f"pass {rep}"
        for x in [outs[0]] + outs[1] + outs[2]:
            x.tensor.zero_()
        dev.compare_max_min(dk, A, B, outs=outs)
    dev.set_exec_mode(bc.BC_EXEC_BATCHED)
    assert np.array_equal(dev.decrypt(dk, outs[0]), (xs < ys).astype(np.uint32))


def test_workspace_cache_limit_keeps_results():
    """With a workspace cache limit the pool gives its cached blocks back
    whenever it must grow past the limit; results are the same bytes."""
    import paper_2407_07308_amd as bc

    prm = Params(10, 257, 8, 50, 4, 50, 2)
    dev, dk = member(prm, 9)
    x = synth.slot_values(71, 2, dev.M, 0, 129)
    y = synth.slot_values(72, 2, dev.M, 0, 129)
    rx, ry = synth.encrypt_randomness(73, 2, dev.N), synth.encrypt_randomness(74, 2, dev.N)
    A, B = [dev.encrypt(dk, x, rx["u"], rx["e"])], [dev.encrypt(dk, y, ry["u"], ry["e"])]
    ref = dev.export(dev.compare_lt(dk, A, B))
    dev.trim()
    dev.set_tuning(bc.BC_TUNE_POOL_LIMIT_BYTES, 1 << 20)
    assert dev.get_tuning(bc.BC_TUNE_POOL_LIMIT_BYTES) == 1 << 20
    for _ in range(2):
        assert np.array_equal(dev.export(dev.compare_lt(dk, A, B)), ref)
    assert np.array_equal(dev.decrypt(dk, dev.compare_lt(dk, A, B)), (x < y).astype(np.uint32))
