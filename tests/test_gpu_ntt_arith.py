"""Transform arithmetic and schedules at the workload ring sizes.

With every prime below 2^50 the transforms run in fp64 arithmetic; the
integer butterflies remain selectable.  Both must give the same bytes under
every schedule (single-pass with or without part-limb transforms, two-pass
whole or chunked; with the key-switching kernels handing their intermediate
limbs over as reduced fp64 patterns or as canonical words), and the
ciphertexts must equal the oracle's.  With the single-pass schedule the last
steps of a multiplication and of a modulus switch run inside the forward
transform's store; the other schedules run them as separate kernels, so the
comparison covers both.  Sizes: N = 2^12 .. 2^15, the range of the
single-pass kernel, with two-digit key switching so special-prime limbs are
transformed too.
"""
import numpy as np
import pytest

import synth
from oracle import Oracle, Params

pytestmark = pytest.mark.gpu

SCHEDULES = [  # (fp64, single pass, chunk bytes, part-limb transforms, fp64 hand-off, modulus raising on MFMA)
    (1, 1, 0, 1, 1, 0), (1, 1, 0, 1, 0, 0), (1, 1, 0, 0, 1, 0), (1, 0, 0, 1, 1, 0), (1, 0, 1 << 20, 1, 1, 0),
    (1, 1, 0, 1, 1, 1), (1, 1, 0, 1, 0, 1), (1, 1, 0, 0, 1, 1), (1, 0, 0, 1, 1, 1),
    (0, 1, 0, 1, 1, 0), (0, 1, 0, 0, 1, 0), (0, 0, 0, 1, 1, 0), (0, 0, 1 << 20, 1, 1, 0)]


def run_all(dev, dk, slots, r):
    import paper_2407_07308_amd as bc

    outs = []
    for fp, single, chunk, parts, raw, mfma in SCHEDULES:
        dev.set_tuning(bc.BC_TUNE_MFMA_MODUP, 0)
        dev.set_tuning(bc.BC_TUNE_RAW_HANDOFF, raw)
        dev.set_tuning(bc.BC_TUNE_FP64, fp)
        dev.set_tuning(bc.BC_TUNE_NTT_SINGLE_PASS, single)
        dev.set_tuning(bc.BC_TUNE_NTT_CHUNK_BYTES, chunk)
        dev.set_tuning(bc.BC_TUNE_NTT_PARTS, parts)
        # the key-switching producers fold 1 (N = 2^14) or 2 (N = 2^15) stages
        logN = dev.N.bit_length() - 1
        folded = logN - 13 if (single and parts and logN >= 14) else 0
        assert dev.get_tuning(bc.BC_TUNE_NTT_PARTS) == folded
        dev.set_tuning(bc.BC_TUNE_MFMA_MODUP, mfma)
        ct = dev.encrypt(dk, slots, r["u"], r["e"])
        prod = dev.mul_relin(dk, ct, ct)
        ms = dev.mod_switch(ct)
        outs.append((dev.export(ct), dev.export(prod), dev.decrypt(dk, prod), dev.export(ms)))
    return outs


@pytest.mark.parametrize("logN", [12, 13, 14, 15])
def test_fp64_and_integer_transforms_agree(logN):
    import paper_2407_07308_amd as bc

    prm = Params(logN, 257, 4, 50, 2, 50, 2)
    print(f"\n[ntt arith] logN {logN}", flush=True)
    dev = bc.Context.from_params(prm)
    assert dev.get_tuning(bc.BC_TUNE_FP64) == 1
    rnd = synth.keygen_randomness(31, prm.N, prm.nQ, prm.nP, prm.dnum, 0)
    dk = dev.keygen(rnd["s"], rnd["a"], rnd["e"], ())
    count = 3
    slots = synth.slot_values(32, count, dev.M, 0, prm.p)
    r = synth.encrypt_randomness(33, count, prm.N)
    outs = run_all(dev, dk, slots, r)
    dev.set_tuning(bc.BC_TUNE_MFMA_MODUP, 0)
    dev.set_tuning(bc.BC_TUNE_RAW_HANDOFF, 1)
    want = (slots.astype(np.int64) ** 2 % prm.p).astype(np.uint32)
    for i, (ct, prod, dec, ms) in enumerate(outs):
        assert np.array_equal(ct, outs[0][0]), SCHEDULES[i]
        assert np.array_equal(prod, outs[0][1]), SCHEDULES[i]
        assert np.array_equal(dec, want), SCHEDULES[i]
        assert np.array_equal(ms, outs[0][3]), SCHEDULES[i]
    if logN <= 13:  # the oracle's ciphertexts (seconds at these sizes)
        orc = Oracle(prm)
        orc.keygen(rnd)
        o = [orc.encrypt(slots[i], r["u"][i], r["e"][i]) for i in range(count)]
        assert np.array_equal(outs[0][0], np.stack([c.data for c in o]))
        op = [orc.mul(c, c) for c in o]
        assert np.array_equal(outs[0][1], np.stack([c.data for c in op]))
        om = [orc.mod_switch(c) for c in o]
        assert np.array_equal(outs[0][3], np.stack([c.data for c in om]))


def test_integer_only_context_reports_no_fp64():
    import paper_2407_07308_amd as bc

    dev = bc.Context.from_params(Params(12, 257, 4, 50, 1, 60, 4))
    assert dev.get_tuning(bc.BC_TUNE_FP64) == 0


def test_autotune_mul_keeps_the_bytes():
    """The multiplication autotuner times every schedule and form the context
    allows and keeps one; the products are the same bytes before and after."""
    import paper_2407_07308_amd as bc

    prm = Params(14, 257, 4, 50, 2, 50, 2)
    print("\n[ntt arith] autotune_mul at N=2^14", flush=True)
    dev = bc.Context.from_params(prm)
    rnd = synth.keygen_randomness(34, prm.N, prm.nQ, prm.nP, prm.dnum, 0)
    dk = dev.keygen(rnd["s"], rnd["a"], rnd["e"], ())
    slots = synth.slot_values(35, 2, dev.M, 0, prm.p)
    r = synth.encrypt_randomness(36, 2, prm.N)
    ct = dev.encrypt(dk, slots, r["u"], r["e"])
    before = dev.export(dev.mul_relin(dk, ct, ct))
    tuned = dev.autotune_mul(dk)
    assert set(tuned) == {"single_pass", "chunk_bytes", "fp64", "parts_log", "raw_handoff", "mfma_modup"}
    assert tuned["fp64"] in (0, 1) and tuned["parts_log"] in (0, 1)
    assert not tuned["raw_handoff"] or (tuned["fp64"] and tuned["parts_log"])
    assert np.array_equal(dev.export(dev.mul_relin(dk, ct, ct)), before)
    print("[ntt arith] tuned", tuned, flush=True)
