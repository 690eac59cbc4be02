"""Device path vs the CPU oracle, operation by operation (bit-exact).

Both sides consume the same seeded randomness (``synth``): the device library
builds its own primes, tables and keys from it, the oracle builds its own.
Ciphertexts are compared in the coefficient domain (``bc_export``), so the
two NTT orderings never meet.  Sizes: N = 2^10 and 2^11 (several NTT tiles in
both passes), batch counts that are not multiples of anything (3, 5), every
level of the chain for modulus switching, digits of uneven size.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import Ct, Oracle, Params

pytestmark = pytest.mark.gpu

SETS = {
    "p17": Params(10, 17, 6, 36, 1, 60, 3),
    "p257": Params(10, 257, 8, 50, 3, 60, 2),
    "p257_uneven": Params(11, 257, 7, 50, 4, 60, 3),  # digits of 3, 3 and 1 primes
    # every prime below 2^50: the transforms run in fp64 arithmetic
    "p257_fp64": Params(11, 257, 7, 50, 3, 50, 3),
}
ROT = (1, 2, -1)


class Pair:
    """A device context and an oracle on the same parameters and keys."""

    def __init__(self, prm, seed=7):
        import paper_2407_07308_amd as bc

        self.prm = prm
        self.dev = bc.Context.from_params(prm)
        self.orc = Oracle(prm)
        rnd = synth.keygen_randomness(seed, prm.N, prm.nQ, prm.nP, prm.dnum, len(ROT))
        self.dk = self.dev.keygen(rnd["s"], rnd["a"], rnd["e"], ROT)
        self.orc.keygen(rnd, rot_steps=ROT)
        self.N, self.M, self.p = prm.N, self.orc.M, prm.p

    def enc_both(self, count, seed, lo=0, hi=None):
        hi = self.p if hi is None else hi
        slots = synth.slot_values(seed, count, self.M, lo, hi)
        r = synth.encrypt_randomness(seed + 1000, count, self.N)
        d = self.dev.encrypt(self.dk, slots, r["u"], r["e"])
        o = [self.orc.encrypt(slots[i], r["u"][i], r["e"][i]) for i in range(count)]
        return slots, d, o

    def to_dev(self, cts):
        host = np.stack([c.data for c in cts])
        return self.dev.import_(host, cts[0].level, cts[0].ncomp)

    def check(self, d, o, what):
        got = self.dev.export(d)
        want = np.stack([c.data for c in o])
        assert got.shape == want.shape, (what, got.shape, want.shape)
        bad = np.argwhere(got != want)
        assert bad.size == 0, f"{what}: {len(bad)} residues differ, first at {bad[:3].tolist()}"


@pytest.fixture(scope="module", params=sorted(SETS))
def pair(request):
    print(f"\n[gpu parity] params {request.param}", flush=True)
    return Pair(SETS[request.param])


def test_moduli_match(pair):
    assert pair.dev.moduli == pair.orc.moduli
    assert pair.dev.M == pair.orc.M


def test_encrypt_bit_exact_and_decrypt(pair):
    slots, d, o = pair.enc_both(3, 11)
    pair.check(d, o, "encrypt")
    assert np.array_equal(pair.dev.decrypt(pair.dk, d), slots)


def test_import_export_round_trip(pair):
    _, _, o = pair.enc_both(2, 12)
    d = pair.to_dev(o)
    pair.check(d, o, "import/export")
    assert np.array_equal(pair.dev.decrypt(pair.dk, d), np.stack([pair.orc.decrypt(c) for c in o]))


def test_add_sub_scalar_const(pair):
    _, da, oa = pair.enc_both(3, 13)
    _, db, ob = pair.enc_both(3, 14)
    o, p = pair.orc, pair.p
    pair.check(pair.dev.add(da, db), [o.add(x, y) for x, y in zip(oa, ob)], "add")
    pair.check(pair.dev.sub(da, db), [o.sub(x, y) for x, y in zip(oa, ob)], "sub")
    for c in (0, 1, p - 1, (p + 1) // 2, 5):
        pair.check(pair.dev.mul_scalar(da, c), [o.mul_scalar(x, c) for x in oa], f"scalar {c}")
        pair.check(pair.dev.add_const(da, c), [o.add_const(x, c) for x in oa], f"const {c}")


def test_mod_switch_every_level(pair):
    _, d, o = pair.enc_both(2, 15)
    for _ in range(pair.prm.nQ - 1):
        d = pair.dev.mod_switch(d)
        o = [pair.orc.mod_switch(c) for c in o]
        pair.check(d, o, f"mod_switch to level {d.level}")


def test_tensor_relin_mul(pair):
    sa, da, oa = pair.enc_both(5, 16)
    sb, db, ob = pair.enc_both(5, 17)
    t = pair.dev.tensor(da, db)
    ot = [pair.orc.tensor(x, y) for x, y in zip(oa, ob)]
    pair.check(t, ot, "tensor")
    r = pair.dev.relin(pair.dk, t)
    pair.check(r, [pair.orc.relin(x) for x in ot], "relin")
    m = pair.dev.mul_relin(pair.dk, da, db)
    om = [pair.orc.mul(x, y) for x, y in zip(oa, ob)]
    pair.check(m, om, "mul_relin")
    assert np.array_equal(pair.dev.decrypt(pair.dk, m), (sa.astype(np.int64) * sb % pair.p))


def test_mul_at_every_level_and_mixed_levels(pair):
    _, d, o = pair.enc_both(3, 18)
    _, e, oe = pair.enc_both(3, 19)
    while d.level > 0:
        d = pair.dev.mul_relin(pair.dk, d, e)  # e stays at the top level: aligned each time
        o = [pair.orc.mul(x, y) for x, y in zip(o, oe)]
        pair.check(d, o, f"mul chain at level {d.level}")
    d = pair.dev.mul_relin(pair.dk, d, d)  # level 0: no modulus switch
    o = [pair.orc.mul(x, x) for x in o]
    pair.check(d, o, "mul at level 0")


def test_broadcast_operand(pair):
    _, da, oa = pair.enc_both(4, 20)
    _, db, ob = pair.enc_both(1, 21)
    pair.check(pair.dev.mul_relin(pair.dk, da, db), [pair.orc.mul(x, ob[0]) for x in oa], "broadcast mul")
    pair.check(pair.dev.add(da, db), [pair.orc.add(x, ob[0]) for x in oa], "broadcast add")


@pytest.mark.parametrize("step", ROT)
def test_rotate(pair, step):
    s, d, o = pair.enc_both(3, 22)
    r = pair.dev.rotate(pair.dk, d, step)
    pair.check(r, [pair.orc.rotate(c, step) for c in o], f"rotate {step}")
    h = pair.M // 2
    dec = pair.dev.decrypt(pair.dk, r)
    for i in range(3):
        v = s[i]
        want = np.concatenate([v[h:], v[:h]]) if step == -1 else np.concatenate(
            [np.roll(v[:h], -step), np.roll(v[h:], -step)])
        assert np.array_equal(dec[i], want)
    # rotation at a lower level
    d2 = pair.dev.mod_switch(d)
    pair.check(pair.dev.rotate(pair.dk, d2, step), [pair.orc.rotate(pair.orc.mod_switch(c), step) for c in o],
               f"rotate {step} below the top level")


def test_decrypt_poly_matches_oracle(pair):
    _, d, o = pair.enc_both(2, 23)
    m = pair.dev.mul_relin(pair.dk, d, d)
    got = pair.dev.decrypt_poly(pair.dk, m)
    want = np.stack([pair.orc.decrypt_poly(pair.orc.mul(c, c)) for c in o])
    assert np.array_equal(got, want)


def test_batch_equals_single_calls(pair):
    """The same ciphertext gives the same bytes alone and inside a batch."""
    _, d, o = pair.enc_both(3, 24)
    full = pair.dev.export(pair.dev.mul_relin(pair.dk, d, d))
    for i in range(3):
        one = pair.to_dev([o[i]])
        single = pair.dev.export(pair.dev.mul_relin(pair.dk, one, one))
        assert np.array_equal(single[0], full[i])
