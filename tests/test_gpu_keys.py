"""Key sets: device key generation equals the oracle's keys (coefficient
domain, residue for residue), export/import round trips (checkpoint and
resume), and recorded comparison graphs never outlive their key set."""
import numpy as np
import pytest

import oracle
import synth
from oracle import Oracle, Params

pytestmark = pytest.mark.gpu


def split_blob(blob, prm, nrot):
    N, nm = prm.N, prm.nQ + prm.nP
    off = 40 + 4 * nrot
    s = np.frombuffer(blob, dtype=np.int8, count=N, offset=off)
    off += (N + 7) // 8 * 8
    words = np.frombuffer(blob, dtype=np.uint64, offset=off)
    pk = words[: 2 * prm.nQ * N].reshape(2, prm.nQ, N)
    rest = words[2 * prm.nQ * N:]
    kw = prm.dnum * 2 * nm * N
    assert rest.size == (1 + nrot) * kw
    rlk = rest[:kw].reshape(prm.dnum, 2, nm, N)
    gks = [rest[(1 + r) * kw:(2 + r) * kw].reshape(prm.dnum, 2, nm, N) for r in range(nrot)]
    return s, pk, rlk, gks


@pytest.mark.parametrize("prm", [Params(10, 257, 8, 50, 4, 50, 2), Params(11, 17, 6, 36, 1, 60, 3)])
def test_keygen_matches_oracle_and_round_trips(prm):
    import paper_2407_07308_amd as bc

    steps = (1, bc.BC_ROW_SWAP)
    dev = bc.Context.from_params(prm)
    rnd = synth.keygen_randomness(21, prm.N, prm.nQ, prm.nP, prm.dnum, len(steps))
    dk = dev.keygen(rnd["s"], rnd["a"], rnd["e"], steps)
    orc = Oracle(prm)
    ok = orc.keygen(rnd, rot_steps=steps)
    blob = dev.export_keys(dk)
    s, pk, rlk, gks = split_blob(blob, prm, len(steps))
    assert np.array_equal(s, rnd["s"].astype(np.int8))
    assert np.array_equal(pk, ok["pk"])
    assert np.array_equal(rlk, ok["rlk"])
    for st, gk in zip(steps, gks):
        assert np.array_equal(gk, ok["gk"][st]), f"rotation key {st}"
    # resume from the blob: same keys, same results
    k2 = dev.import_keys(blob)
    assert k2.rot_steps == steps
    assert dev.export_keys(k2) == blob
    vals = synth.slot_values(22, 2, dev.M, 0, prm.p)
    r = synth.encrypt_randomness(23, 2, prm.N)
    x1, x2 = dev.encrypt(dk, vals, r["u"], r["e"]), dev.encrypt(k2, vals, r["u"], r["e"])
    assert np.array_equal(dev.export(x1), dev.export(x2))
    assert np.array_equal(dev.export(dev.mul_relin(dk, x1, x1)), dev.export(dev.mul_relin(k2, x2, x2)))
    assert np.array_equal(dev.export(dev.rotate(dk, x1, 1)), dev.export(dev.rotate(k2, x2, 1)))
    assert np.array_equal(dev.decrypt(k2, x1), vals)
    # malformed blobs are refused
    with pytest.raises(bc.BoostcomError) as e:
        dev.import_keys(blob[:-8])
    assert e.value.code == bc.BC_ERR_ARG
    other = bc.Context.from_params(Params(prm.logN, prm.p, prm.nQ - 1, prm.bitsQ, prm.nP, prm.bitsP, prm.dnum))
    with pytest.raises(bc.BoostcomError) as e:
        other.import_keys(blob)
    assert e.value.code == bc.BC_ERR_PARAM


def test_graph_cache_never_replays_with_freed_keys():
    """Graph mode records per key set.  Destroying the keys drops their
    graphs; a new key set (possibly at the same host address) records its
    own graph, whose replays equal the eager results."""
    import gc

    import torch

    import paper_2407_07308_amd as bc

    prm = Params(10, 257, 8, 50, 4, 50, 2)
    dev = bc.Context.from_params(prm)
    G = 2
    x = synth.slot_values(31, G, dev.M, 0, 129)
    y = synth.slot_values(32, G, dev.M, 0, 129)
    # the same input and output buffers every round: only the key set differs
    A = dev.new_batch(G, prm.nQ - 1)
    B = dev.new_batch(G, prm.nQ - 1)
    outs = None
    for seed in (41, 42, 43):
        rnd = synth.keygen_randomness(seed, prm.N, prm.nQ, prm.nP, prm.dnum, 0)
        dk = dev.keygen(rnd["s"], rnd["a"], rnd["e"], ())
        rx, ry = synth.encrypt_randomness(seed + 100, G, prm.N), synth.encrypt_randomness(seed + 200, G, prm.N)
        dev.encrypt(dk, x, rx["u"], rx["e"], out=A)
        dev.encrypt(dk, y, ry["u"], ry["e"], out=B)
        ref = dev.export(dev.compare_lt(dk, [A], [B]))
        dev.set_exec_mode(bc.BC_EXEC_GRAPH)
        if outs is None:
            outs = dev.compare_max_min(dk, [A], [B], True, False, False)  # eager + record
        else:
            outs[0].tensor.zero_()
            dev.compare_max_min(dk, [A], [B], True, False, False, outs=outs)  # eager + record
        for _ in range(2):
            assert np.array_equal(dev.export(outs[0]), ref), f"key seed {seed}"
            outs[0].tensor.zero_()
            dev.compare_max_min(dk, [A], [B], True, False, False, outs=outs)  # replay
        assert np.array_equal(dev.export(outs[0]), ref)
        assert np.array_equal(dev.decrypt(dk, outs[0]), (x < y).astype(np.uint32))
        dev.set_exec_mode(bc.BC_EXEC_BATCHED)
        torch.cuda.synchronize()
        del dk
        gc.collect()


def test_handles_can_be_released_in_any_order():
    """A key set or group released after its context's handle still finds the
    context (the context lives until its last owner goes), so garbage
    collection may finalise the Python objects in any order."""
    import paper_2407_07308_amd as bc

    prm = Params(10, 257, 8, 50, 4, 50, 2)
    for order in (("ctx", "group", "keys"), ("ctx", "keys", "group"), ("keys", "ctx", "group")):
        dev = bc.Context.from_params(prm)
        rnd = synth.keygen_randomness(23, prm.N, prm.nQ, prm.nP, prm.dnum, 0)
        dk = dev.keygen(rnd["s"], rnd["a"], rnd["e"], ())
        vals = synth.slot_values(24, 1, dev.M, 0, prm.p)
        r = synth.encrypt_randomness(25, 1, prm.N)
        x = dev.encrypt(dk, vals, r["u"], r["e"])
        assert np.array_equal(dev.decrypt(dk, dev.mul_relin(dk, x, x)), vals.astype(np.int64) ** 2 % prm.p)
        grp = bc.Group([dev])
        L = dev.L
        objs = {"ctx": (dev, L.bc_ctx_destroy), "group": (grp, L.bc_group_destroy), "keys": (dk, L.bc_keys_destroy)}
        for name in order:
            obj, destroy = objs[name]
            assert destroy(obj.handle) == 0, name
            obj.handle = None
    # the library is still usable afterwards
    dev = bc.Context.from_params(prm)
    rnd = synth.keygen_randomness(26, prm.N, prm.nQ, prm.nP, prm.dnum, 0)
    dk = dev.keygen(rnd["s"], rnd["a"], rnd["e"], ())
    vals = synth.slot_values(27, 2, dev.M, 0, prm.p)
    r = synth.encrypt_randomness(28, 2, prm.N)
    assert np.array_equal(dev.decrypt(dk, dev.encrypt(dk, vals, r["u"], r["e"])), vals)
