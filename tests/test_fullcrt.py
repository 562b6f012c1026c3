"""The full-limb decryption used by the full-size GPU tests, checked on the
CPU: equal to the oracle's exact big-integer CRT decryption, and a residue
changed in any limb is caught."""
import numpy as np
import pytest

from paper_2305_17341_amd import inputs as I
from tests.fullcrt import FullDecryptor


class _AsGpu:
    """an oracle ciphertext behind the two attributes the decryptor reads"""

    def __init__(self, data, scale):
        self._d, self.scale = data, scale

    def export(self):
        return self._d.copy()


def test_full_decryption_equals_exact_crt(oracle_mod):
    ch = I.TOY2
    o = oracle_mod.Oracle(ch.log_n, ch.q_bits, ch.p_bits, seed=9)
    o.keygen(rot_steps=[3])
    z = np.random.default_rng(2).uniform(-1, 1, o.slots)
    ct = o.rotate(o.rescale(o.mult(o.encrypt(z, nonce=1), o.encrypt(z, nonce=2))), 3)
    fd = FullDecryptor(oracle_mod, ch, 9)
    coeffs = fd.coefficients(_AsGpu(ct.data(), ct.scale))
    assert [int(v) for v in coeffs] == o.decrypt_coeffs(ct)
    got = fd.decrypt(_AsGpu(ct.data(), ct.scale))
    assert np.max(np.abs(got - np.roll(z * z, -3))) < 2.0 ** -15

    for limb in range(1, ct.level + 1):
        bad = ct.data()
        bad[0, limb, 17] = (int(bad[0, limb, 17]) + 1) % o.q[limb]
        with pytest.raises(AssertionError, match=f"limb {limb}"):
            fd.coefficients(_AsGpu(bad, ct.scale))
