"""The oracle's timing helpers compute what the timed operations compute: the
key inner product with given digits equals the hoisted rotation, and the
thread count of its loops does not change a residue."""
import numpy as np

from paper_2305_17341_amd import inputs as I


def test_hoisted_rotation_with_given_digits(oracle_mod):
    ch = I.TOY2
    o = oracle_mod.Oracle(ch.log_n, ch.q_bits, ch.p_bits, seed=4)
    o.keygen(rot_steps=[5])
    ct = o.encrypt(np.random.default_rng(1).uniform(-1, 1, o.slots), nonce=2)
    digits = o.decompose(ct.data()[1], ct.level)
    assert np.array_equal(o.hoisted_rotate_digits(ct, digits, 5).data(), o.hoisted_rotate(ct, 5).data())


def test_thread_count_keeps_residues(oracle_mod):
    ch = I.TOY2
    o = oracle_mod.Oracle(ch.log_n, ch.q_bits, ch.p_bits, seed=4)
    o.keygen(rot_steps=[5])
    ct = o.encrypt(np.random.default_rng(1).uniform(-1, 1, o.slots), nonce=2)
    before = oracle_mod.get_threads()
    try:
        oracle_mod.set_threads(1)
        assert oracle_mod.get_threads() == 1
        one = o.rotate(ct, 5).data()
        oracle_mod.set_threads(4)
        assert np.array_equal(o.rotate(ct, 5).data(), one)
    finally:
        oracle_mod.set_threads(before)
