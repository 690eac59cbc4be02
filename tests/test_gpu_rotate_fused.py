"""The rotation's key switch with its last step (base + ACC P^-1 - TH p P^-1,
hybrid key switching) stored by TH's forward transform: the single-pass
kernels (N = 2^12, 2^13, and 2^14 with the part-limb transforms off), the
part-limb kernels (2^14, 2^15), fp64 and integer arithmetic.  Each gives the
bytes of the separate transform + combine path (the context with the
single-pass transforms off) at the top level and after modulus switches;
decryptions are the rotated slots; at N = 2^12 one level down and at 2^15
the top level against the oracle.  A level-0 product, whose key switch has a
base in both components, across schedules."""
import numpy as np
import pytest

import synth
from oracle import Oracle, Params

pytestmark = pytest.mark.gpu

P12 = Params(12, 257, 13, 50, 4, 50, 4)
P13 = Params(13, 257, 8, 50, 4, 50, 2)
P14 = Params(14, 257, 8, 50, 4, 50, 2)
P15 = Params(15, 257, 14, 50, 5, 50, 3)
STEPS = (1, 5)


def rotations(prm, tune, levels=3, seed=71):
    """Rotations by each step at the top level and `levels - 1` switches
    down; returns (context, keys, randomness, inputs, {(level, step): bytes})."""
    import paper_2407_07308_amd as bc

    dev = bc.Context.from_params(prm)
    for k, v in tune:
        dev.set_tuning(k, v)
    rnd = synth.keygen_randomness(seed, prm.N, prm.nQ, prm.nP, prm.dnum, len(STEPS))
    dk = dev.keygen(rnd["s"], rnd["a"], rnd["e"], STEPS)
    vals = synth.slot_values(seed + 1, 2, dev.M, 0, prm.p)
    r = synth.encrypt_randomness(seed + 2, 2, prm.N)
    x = dev.encrypt(dk, vals, r["u"], r["e"])
    out = {}
    h = dev.M // 2
    for _ in range(levels):
        for s in STEPS:
            y = dev.rotate(dk, x, s)
            want = np.concatenate([np.roll(vals[:, :h], -s, axis=1), np.roll(vals[:, h:], -s, axis=1)], axis=1)
            assert np.array_equal(dev.decrypt(dk, y), want), (prm.logN, x.level, s)
            out[(x.level, s)] = dev.export(y)
        x = dev.mod_switch(x)
    return dev, dk, rnd, (vals, r), out


@pytest.mark.parametrize("prm,parts", [(P12, 1), (P13, 1), (P14, 1), (P14, 0), (P15, 1)])
@pytest.mark.parametrize("fp64", [1, 0])
def test_fused_matches_separate_combine(prm, parts, fp64):
    import paper_2407_07308_amd as bc

    print(f"rotate fused: N=2^{prm.logN} parts {parts} fp64 {fp64}", flush=True)
    base = [(bc.BC_TUNE_FP64, fp64)]
    _, _, _, _, got = rotations(prm, base + [(bc.BC_TUNE_NTT_PARTS, parts)])
    _, _, _, _, ref = rotations(prm, base + [(bc.BC_TUNE_NTT_SINGLE_PASS, 0)])
    assert got.keys() == ref.keys()
    for key in got:
        assert np.array_equal(got[key], ref[key]), key


def test_fused_matches_oracle():
    print("rotate fused: N=2^12 one level down, N=2^15 top, against the oracle", flush=True)
    for prm, down in ((P12, 1), (P15, 0)):
        dev, dk, rnd, (vals, r), got = rotations(prm, (), levels=down + 1)
        o = Oracle(prm)
        o.keygen(rnd, rot_steps=STEPS)
        oc = o.encrypt(vals[1], r["u"][1], r["e"][1])
        for _ in range(down):
            oc = o.mod_switch(oc)
        for s in STEPS:
            assert np.array_equal(got[(oc.level, s)][1], o.rotate(oc, s).data), (prm.logN, s)


@pytest.mark.parametrize("prm,parts", [(P12, 1), (P14, 1), (P14, 0)])
def test_level0_relinearisation_with_two_bases(prm, parts):
    """A product at level 0 relinearises without a modulus switch: a key
    switch with a base in both components (d0, d1), which keeps the separate
    transform and combine; the same bytes under every transform schedule."""
    import paper_2407_07308_amd as bc

    print(f"relinearise at level 0: N=2^{prm.logN} parts {parts}", flush=True)

    def run(tune):
        dev = bc.Context.from_params(prm)
        for k, v in tune:
            dev.set_tuning(k, v)
        rnd = synth.keygen_randomness(81, prm.N, prm.nQ, prm.nP, prm.dnum, 0)
        dk = dev.keygen(rnd["s"], rnd["a"], rnd["e"], ())
        vals = synth.slot_values(82, 3, dev.M, 0, prm.p)
        r = synth.encrypt_randomness(83, 3, prm.N)
        x = dev.encrypt(dk, vals, r["u"], r["e"])
        while x.level > 0:
            x = dev.mod_switch(x)
        y = dev.mul_relin(dk, x, x)
        assert y.level == 0
        assert np.array_equal(dev.decrypt(dk, y), (vals.astype(np.int64) ** 2) % prm.p)
        return dev.export(y)

    got = run([(bc.BC_TUNE_NTT_PARTS, parts)])
    ref = run([(bc.BC_TUNE_NTT_SINGLE_PASS, 0)])
    assert np.array_equal(got, ref)
