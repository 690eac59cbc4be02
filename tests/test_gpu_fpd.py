"""F_{p^d} slots and the mod-extract step on the device (bc_fpd_info,
bc_encode_fpd / bc_decode_fpd, bc_encrypt_poly, bc_extract_digits).

Byte-identical to the oracle on the same seeded inputs: the encoding, the
encryption of a polynomial, and every extracted digit ciphertext, at N = 2^10
(p = 17: d = 128, seven Frobenius doublings; p = 257: d = 8, three) and at the
workload's N = 2^15 (p = 257, d = 256, eight doublings; one digit of one
ciphertext sampled).  Decryptions of every extracted digit against the
coordinates that were encoded; uint16 values held as two coordinates of one
F_{257^256} slot, extracted and compared by the bivariate circuit against
integer '<'; the argument and key errors."""
import numpy as np
import pytest

import oracle
import synth
from oracle import CtEvaluator, Oracle, Params

pytestmark = pytest.mark.gpu


def setup(prm, seed, extra_steps=()):
    import paper_2407_07308_amd as bc

    dev = bc.Context.from_params(prm)
    d, steps = dev.fpd_info()
    assert d == oracle.fpd_degree(prm.p, prm.N)
    assert steps == oracle.frobenius_steps(prm.p, prm.N)
    steps = list(steps) + list(extra_steps)
    rnd = synth.keygen_randomness(seed, prm.N, prm.nQ, prm.nP, prm.dnum, len(steps))
    return dev, dev.keygen(rnd["s"], rnd["a"], rnd["e"], steps), rnd, steps


def random_elems(seed, G, M, d, p, ncols=None):
    g = synth.generator(seed, "fpd")
    E = g.integers(0, p, (G, M, d), dtype=np.int64)
    if ncols is not None:
        E[:, :, ncols:] = 0
    return E


@pytest.mark.parametrize("prm", [Params(10, 17, 6, 36, 1, 60, 3), Params(10, 257, 8, 50, 4, 50, 2)])
def test_extract_matches_oracle_small(prm):
    p, N = prm.p, prm.N
    print(f"fpd: N=2^{prm.logN} p={p} oracle parity", flush=True)
    dev, dk, rnd, steps = setup(prm, 51)
    d = N // dev.M
    G = 2
    E = random_elems(52, G, dev.M, d, p)
    coeffs = dev.encode_fpd(E)
    for g in range(G):
        assert np.array_equal(coeffs[g], oracle.encode_fpd(E[g], p, N)), g
    assert np.array_equal(dev.decode_fpd(coeffs), E)
    r = synth.encrypt_randomness(53, G, N)
    ct = dev.encrypt_poly(dk, coeffs, r["u"], r["e"])
    digits = sorted({0, 1, 5 % d, d - 1})
    out = dev.extract_digits(dk, ct, digits)
    assert out.count == G * len(digits) and out.level == ct.level
    planes = out.split(len(digits))
    for i, k in enumerate(digits):
        assert np.array_equal(dev.decrypt(dk, planes[i]), E[:, :, k]), k
    # ciphertext 1 through the oracle (same keys, same encryption randomness)
    o = Oracle(prm)
    o.keygen(rnd, rot_steps=steps)
    oc = o.encrypt_poly(oracle.encode_fpd(E[1], p, N), r["u"][1], r["e"][1])
    assert np.array_equal(dev.export(ct)[1], oc.data)
    ev = CtEvaluator(o)
    for i, k in enumerate(digits):
        oz = oracle.extract_digit(ev, o, oc, k, p)
        assert np.array_equal(dev.export(planes[i])[1], oz.data), k


def test_extract_full_size_and_compare():
    """N = 2^15, p = 257: uint16 values as coordinates 1 (high) and 0 (low)
    of one F_{257^256} slot; extraction, then the bivariate comparison of
    the two digit planes; ciphertext 0's coordinate 1 against the oracle."""
    import paper_2407_07308_amd as bc

    prm = Params(15, 257, 14, 50, 5, 50, 3)
    p, N = prm.p, prm.N
    print("fpd: N=2^15 extraction", flush=True)
    dev, dk, rnd, steps = setup(prm, 54)
    d = N // dev.M
    G = 2
    xs = synth.integers(55, (G, dev.M), 0, 1 << 16)
    ys = synth.integers(55, (G, dev.M), 0, 1 << 16, index=1)
    xs[0, :3], ys[0, :3] = [0, 65535, 77], [65535, 0, 77]

    def elems(v):
        E = np.zeros((G, dev.M, d), np.int64)
        E[:, :, 1], E[:, :, 0] = v // p, v % p
        return E

    EX, EY = elems(xs), elems(ys)
    rx, ry = synth.encrypt_randomness(56, G, N), synth.encrypt_randomness(57, G, N)
    cx = dev.encrypt_poly(dk, dev.encode_fpd(EX), rx["u"], rx["e"])
    cy = dev.encrypt_poly(dk, dev.encode_fpd(EY), ry["u"], ry["e"])
    X = dev.extract_digits(dk, cx, [1, 0]).split(2)
    Y = dev.extract_digits(dk, cy, [1, 0]).split(2)
    for i, k in enumerate((1, 0)):
        assert np.array_equal(dev.decrypt(dk, X[i]), EX[:, :, k]), k
        assert np.array_equal(dev.decrypt(dk, Y[i]), EY[:, :, k]), k
    lt = dev.compare_max_min(dk, X, Y, True, False, False, circuit=bc.BC_CIRCUIT_BIVARIATE)[0]
    assert np.array_equal(dev.decrypt(dk, lt), (xs < ys).astype(np.uint32))
    # the same through the packed comparison helper, with the maximum
    lt2, mx, _ = dev.compare_fpd(dk, cx, cy, 2, want_max=True)
    assert np.array_equal(dev.export(lt2), dev.export(lt))
    assert np.array_equal(dev.decrypt(dk, mx[0]).astype(np.int64) * p + dev.decrypt(dk, mx[1]), np.maximum(xs, ys))
    print("fpd: N=2^15 oracle sample", flush=True)
    o = Oracle(prm)
    o.keygen(rnd, rot_steps=steps)
    oc = o.encrypt_poly(oracle.encode_fpd(EX[0], p, N), rx["u"][0], rx["e"][0])
    oz = oracle.extract_digit(CtEvaluator(o), o, oc, 1, p)
    assert np.array_equal(dev.export(X[0])[0], oz.data)


def test_extract_errors():
    import paper_2407_07308_amd as bc

    prm = Params(10, 257, 8, 50, 4, 50, 2)
    dev, dk, _, steps = setup(prm, 58)
    d = prm.N // dev.M
    r = synth.encrypt_randomness(59, 1, prm.N)
    ct = dev.encrypt_poly(dk, np.zeros((1, prm.N), np.uint32), r["u"], r["e"])

    def code(f):
        with pytest.raises(bc.BoostcomError) as ei:
            f()
        return ei.value.code

    assert code(lambda: dev.extract_digits(dk, ct, [d])) == bc.BC_ERR_ARG
    assert code(lambda: dev.extract_digits(dk, ct, [-1])) == bc.BC_ERR_ARG
    assert code(lambda: dev.extract_digits(dk, ct, [])) == bc.BC_ERR_ARG
    assert code(lambda: dev.extract_digits(dk, ct, [0], out=ct)) == bc.BC_ERR_ARG  # in place
    assert code(lambda: dev.extract_digits(dk, ct, [0, 1], out=dev.new_batch(1, ct.level, 2))) == bc.BC_ERR_ARG
    # an output that overlaps the input in part
    big = dev.new_batch(3, ct.level, 2)
    big.split(3)[1].tensor.copy_(ct.tensor)
    w = big.tensor.numel() // 3
    src = bc.Batch(big.tensor[w:2 * w], 1, ct.level, 2, ct.noise)
    dst = bc.Batch(big.tensor[:2 * w], 2, ct.level, 2)
    assert code(lambda: dev.extract_digits(dk, src, [0, 1], out=dst)) == bc.BC_ERR_ARG
    # keys without the last Frobenius step
    rnd = synth.keygen_randomness(60, prm.N, prm.nQ, prm.nP, prm.dnum, len(steps) - 1)
    k2 = dev.keygen(rnd["s"], rnd["a"], rnd["e"], steps[:-1])
    ct2 = dev.encrypt_poly(k2, np.zeros((1, prm.N), np.uint32), r["u"], r["e"])
    assert code(lambda: dev.extract_digits(k2, ct2, [0])) == bc.BC_ERR_KEY
    # steps at or beyond N/2 are not rotations
    rnd1 = synth.keygen_randomness(61, prm.N, prm.nQ, prm.nP, prm.dnum, 1)
    assert code(lambda: dev.keygen(rnd1["s"], rnd1["a"], rnd1["e"], [prm.N // 2])) == bc.BC_ERR_ARG
