"""Decryption of a GPU ciphertext through every limb, by the CPU oracle.

The library's own decryption reads the residue mod q_0 only, which cannot see
a wrong residue in any other limb.  Here the GPU residues are imported into an
oracle context built from the same seed (only its secret key is generated,
which the seed fixes), the oracle forms c_0 + c_1 s limb by limb, and the
message m is reconstructed by CRT over all l + 1 limbs: with |m| < q_0 / 2
(the CKKS correctness condition at any level) the CRT value equals the centred
residue mod q_0, so m is taken from limb 0 and every other limb must hold
m mod q_i exactly.  A limb that does not raises; otherwise m is decoded
(canonical embedding, FP64).
"""
from __future__ import annotations

import numpy as np


class FullDecryptor:
    def __init__(self, oracle_mod, chain, seed):
        self.O = oracle_mod
        self.o = oracle_mod.Oracle(chain.log_n, chain.q_bits, chain.p_bits, seed=seed)
        self.o.keygen(rot_steps=(), relin=False)

    def coefficients(self, gpu_ct):
        """exact integer coefficients of the plaintext (int64), checked in every limb"""
        data = gpu_ct.export()
        level = data.shape[1] - 1
        ct = self.o.ct_import(data, level, False, gpu_ct.scale)
        res = self.o.decrypt_residues(ct)
        q0 = self.o.q[0]
        r0 = res[0].astype(np.uint64)
        half = np.uint64(q0 // 2)
        m = np.where(r0 > half, r0.astype(np.int64) - np.int64(q0), r0.astype(np.int64))
        for k in range(1, level + 1):
            qk = np.int64(self.o.q[k])
            want = np.mod(m, qk).astype(np.uint64)
            bad = np.nonzero(want != res[k])[0]
            if bad.size:
                raise AssertionError(f"limb {k}: {bad.size} coefficients inconsistent with limb 0 "
                                     f"(first at {int(bad[0])})")
        return m

    def decrypt(self, gpu_ct, n=None):
        m = self.coefficients(gpu_ct)
        z = self.O.decode_float([int(v) for v in m], gpu_ct.scale, self.o.N)
        return z if n is None else z[:n]
