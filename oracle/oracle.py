"""ctypes wrapper around the plain CPU oracle (ckks_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py, never by the product path.  Nothing here imports
the HIP package; the two sides share only the seeded input generators.

Decryption is finished here with exact Python integers: the oracle returns
coefficient residues of c0 + c1*s, this module centres them by CRT (a plain
big-integer reconstruction) and decodes the canonical embedding with a
float64 FFT (decoding is only ever compared within a tolerance).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ckks_oracle.c")
LIB = os.path.join(HERE, "libckks_oracle.so")

u64p = C.POINTER(C.c_uint64)
i64p = C.POINTER(C.c_int64)
intp = C.POINTER(C.c_int)
dblp = C.POINTER(C.c_double)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, OpenMP across independent limbs)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fPIC",
               "-shared", SRC, "-o", LIB + ".tmp", "-lquadmath", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        L.oc_create.restype = C.c_void_p
        L.oc_create.argtypes = [C.c_int, intp, C.c_int, intp, C.c_int, C.c_double, C.c_double, C.c_uint64]
        L.oc_destroy.argtypes = [C.c_void_p]
        L.oc_nmods.argtypes = [C.c_void_p]
        L.oc_moduli.argtypes = [C.c_void_p, u64p]
        L.oc_psi.restype = C.c_uint64
        L.oc_psi.argtypes = [C.c_void_p, C.c_int]
        L.oc_L.argtypes = [C.c_void_p]
        L.oc_alpha.argtypes = [C.c_void_p]
        L.oc_cdt.argtypes = [C.c_void_p, u64p]
        L.oc_cdt_table.argtypes = [C.c_double, u64p]
        L.oc_philox4x64.argtypes = [u64p, u64p, u64p]
        L.oc_ntt.argtypes = [C.c_void_p, C.c_int, u64p]
        L.oc_intt.argtypes = [C.c_void_p, C.c_int, u64p]
        L.oc_ntt_direct.argtypes = [C.c_void_p, C.c_int, u64p, u64p]
        L.oc_automorph_ntt.argtypes = [C.c_void_p, C.c_uint64, u64p, u64p]
        L.oc_automorph_coef.argtypes = [C.c_void_p, C.c_int, C.c_uint64, u64p, u64p]
        L.oc_galois_of_step.restype = C.c_uint64
        L.oc_galois_of_step.argtypes = [C.c_void_p, C.c_int64]
        L.oc_encode.argtypes = [C.c_void_p, dblp, C.c_int, C.c_double, i64p]
        L.oc_encode_direct.argtypes = [C.c_void_p, dblp, C.c_int, C.c_double, i64p]
        L.oc_keygen_secret.argtypes = [C.c_void_p]
        L.oc_keygen_relin.argtypes = [C.c_void_p]
        L.oc_keygen_rot.argtypes = [C.c_void_p, C.c_int64]
        L.oc_secret.argtypes = [C.c_void_p, C.POINTER(C.c_int8)]
        L.oc_encrypt.restype = C.c_void_p
        L.oc_encrypt.argtypes = [C.c_void_p, dblp, C.c_int, C.c_int, C.c_uint64]
        L.oc_encrypt_poly.restype = C.c_void_p
        L.oc_encrypt_poly.argtypes = [C.c_void_p, i64p, C.c_int, C.c_double, C.c_uint64]
        L.oc_decrypt_residues.argtypes = [C.c_void_p, C.c_void_p, u64p]
        L.oc_ct_free.argtypes = [C.c_void_p]
        L.oc_free.argtypes = [C.c_void_p]
        L.oc_ct_level.argtypes = [C.c_void_p]
        L.oc_ct_scale.restype = C.c_double
        L.oc_ct_scale.argtypes = [C.c_void_p]
        L.oc_ct_nlimbs.argtypes = [C.c_void_p]
        L.oc_ct_data.restype = u64p
        L.oc_ct_data.argtypes = [C.c_void_p]
        L.oc_ct_import.restype = C.c_void_p
        L.oc_ct_import.argtypes = [C.c_void_p, u64p, C.c_int, C.c_int, C.c_double]
        for name in ("oc_add", "oc_sub"):
            f = getattr(L, name)
            f.restype = C.c_void_p
            f.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.oc_pmult.restype = C.c_void_p
        L.oc_pmult.argtypes = [C.c_void_p, C.c_void_p, i64p, C.c_double]
        L.oc_padd.restype = C.c_void_p
        L.oc_padd.argtypes = [C.c_void_p, C.c_void_p, i64p]
        L.oc_mul_int.restype = C.c_void_p
        L.oc_mul_int.argtypes = [C.c_void_p, C.c_void_p, C.c_int64]
        L.oc_tensor.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, u64p]
        L.oc_mult.restype = C.c_void_p
        L.oc_mult.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.oc_rescale.restype = C.c_void_p
        L.oc_rescale.argtypes = [C.c_void_p, C.c_void_p]
        L.oc_drop.restype = C.c_void_p
        L.oc_drop.argtypes = [C.c_void_p, C.c_void_p, C.c_int]
        L.oc_beta_at.argtypes = [C.c_void_p, C.c_int]
        L.oc_decompose.restype = u64p
        L.oc_decompose.argtypes = [C.c_void_p, u64p, C.c_int]
        L.oc_moddown.restype = C.c_void_p
        L.oc_moddown.argtypes = [C.c_void_p, C.c_void_p]
        L.oc_moddown_rescale.restype = C.c_void_p
        L.oc_moddown_rescale.argtypes = [C.c_void_p, C.c_void_p]
        L.oc_hoisted_rotate.restype = C.c_void_p
        L.oc_hoisted_rotate.argtypes = [C.c_void_p, C.c_void_p, C.c_int64]
        L.oc_hoisted_rotate_digits.restype = C.c_void_p
        L.oc_hoisted_rotate_digits.argtypes = [C.c_void_p, C.c_void_p, u64p, C.c_int64]
        L.oc_set_threads.argtypes = [C.c_int]
        L.oc_get_threads.argtypes = []
        L.oc_rotate.restype = C.c_void_p
        L.oc_rotate.argtypes = [C.c_void_p, C.c_void_p, C.c_int64]
        for name in ("oc_lt_sigma", "oc_lt_tau"):
            f = getattr(L, name)
            f.restype = C.c_void_p
            f.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_int, intp]
        L.oc_lt_dcd.restype = C.c_void_p
        L.oc_lt_dcd.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, intp]
        L.oc_lt_smpkeysub.restype = C.c_void_p
        L.oc_lt_smpkeysub.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, intp]
        L.oc_lt_transpose.restype = C.c_void_p
        L.oc_lt_transpose.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_double, intp]
        L.oc_matmul.restype = C.c_void_p
        L.oc_matmul.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int, intp]
        L.oc_matmul_ex.restype = C.c_void_p
        L.oc_matmul_ex.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int,
                                   C.c_int, intp]
        L.oc_matmul_lazy.restype = C.c_void_p
        L.oc_matmul_lazy.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int,
                                     C.c_int, C.c_int, intp]
        L.oc_covariance_lazy.argtypes = [C.c_void_p, C.POINTER(C.c_void_p), C.c_int, C.c_int, C.c_int, C.c_uint64,
                                         C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                         C.POINTER(C.c_void_p)]
        L.oc_dcd_factors.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, intp, C.POINTER(C.c_longlong), C.c_int]
        L.oc_covariance.argtypes = [C.c_void_p, C.POINTER(C.c_void_p), C.c_int, C.c_int, C.c_int, C.c_uint64,
                                    C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_void_p)]
        L.oc_perm.argtypes = [C.c_int, C.c_int, intp]
        L.oc_perm_phi_sigma.argtypes = [C.c_int, C.c_int, intp]
        L.oc_counts_reset.argtypes = []
        L.oc_counts_get.argtypes = [intp]
        _lib = L
    return _lib


def set_threads(n):
    """OpenMP threads of the oracle's loops (for timing)"""
    lib().oc_set_threads(int(n))


def get_threads():
    return int(lib().oc_get_threads())


def _u64(a):
    a = np.ascontiguousarray(a, dtype=np.uint64)
    return a, a.ctypes.data_as(u64p)


def philox4x64(ctr, key):
    c = (C.c_uint64 * 4)(*[int(x) for x in ctr])
    k = (C.c_uint64 * 2)(*[int(x) for x in key])
    o = (C.c_uint64 * 4)()
    lib().oc_philox4x64(c, k, o)
    return [int(x) for x in o]


def cdt_table(sigma=3.2):
    o = (C.c_uint64 * 38)()
    lib().oc_cdt_table(sigma, o)
    return [int(x) for x in o]


class Ct:
    """Owning handle to an oracle ciphertext."""

    def __init__(self, ctx: "Oracle", ptr):
        if not ptr:
            raise RuntimeError("oracle operation failed")
        self.ctx = ctx
        self.ptr = C.c_void_p(ptr)

    def __del__(self):
        if getattr(self, "ptr", None) and _lib is not None:
            _lib.oc_ct_free(self.ptr)
            self.ptr = None

    @property
    def level(self):
        return lib().oc_ct_level(self.ptr)

    @property
    def scale(self):
        return lib().oc_ct_scale(self.ptr)

    @property
    def nlimbs(self):
        return lib().oc_ct_nlimbs(self.ptr)

    def data(self) -> np.ndarray:
        """Residues as u64[2][nlimbs][N] (a copy)."""
        n = 2 * self.nlimbs * self.ctx.N
        p = lib().oc_ct_data(self.ptr)
        return np.ctypeslib.as_array(p, shape=(n,)).copy().reshape(2, self.nlimbs, self.ctx.N)


class Oracle:
    """One CKKS context of the oracle."""

    def __init__(self, log_n, q_bits, p_bits, log2_scale=40.0, sigma=3.2, seed=1):
        L = lib()
        qb = (C.c_int * len(q_bits))(*q_bits)
        pb = (C.c_int * len(p_bits))(*p_bits)
        self.ptr = C.c_void_p(L.oc_create(log_n, qb, len(q_bits), pb, len(p_bits), log2_scale, sigma, seed))
        if not self.ptr:
            raise ValueError("oracle: invalid parameters")
        self.log_n = log_n
        self.N = 1 << log_n
        self.slots = self.N // 2
        self.nq = len(q_bits)
        self.L = len(q_bits) - 1
        self.alpha = len(p_bits)
        self.delta = 2.0 ** log2_scale
        m = (C.c_uint64 * L.oc_nmods(self.ptr))()
        L.oc_moduli(self.ptr, m)
        self.moduli = [int(x) for x in m]
        self.q = self.moduli[: self.nq]
        self.p = self.moduli[self.nq:]

    def __del__(self):
        if getattr(self, "ptr", None) and _lib is not None:
            _lib.oc_destroy(self.ptr)
            self.ptr = None

    # -- arithmetic pieces -------------------------------------------------
    def psi(self, m):
        return int(lib().oc_psi(self.ptr, m))

    def ntt(self, m, a):
        a, p = _u64(np.array(a, dtype=np.uint64).copy())
        lib().oc_ntt(self.ptr, m, p)
        return a

    def intt(self, m, a):
        a, p = _u64(np.array(a, dtype=np.uint64).copy())
        lib().oc_intt(self.ptr, m, p)
        return a

    def ntt_direct(self, m, a):
        a, p = _u64(a)
        out = np.zeros(self.N, dtype=np.uint64)
        lib().oc_ntt_direct(self.ptr, m, p, out.ctypes.data_as(u64p))
        return out

    def automorph_ntt(self, g, a):
        a, p = _u64(a)
        out = np.zeros(self.N, dtype=np.uint64)
        lib().oc_automorph_ntt(self.ptr, g, p, out.ctypes.data_as(u64p))
        return out

    def automorph_coef(self, m, g, a):
        a, p = _u64(a)
        out = np.zeros(self.N, dtype=np.uint64)
        lib().oc_automorph_coef(self.ptr, m, g, p, out.ctypes.data_as(u64p))
        return out

    def galois(self, step):
        return int(lib().oc_galois_of_step(self.ptr, step))

    def encode(self, z, delta=None, direct=False):
        z = np.ascontiguousarray(z, dtype=np.float64)
        out = np.zeros(self.N, dtype=np.int64)
        f = lib().oc_encode_direct if direct else lib().oc_encode
        rc = f(self.ptr, z.ctypes.data_as(dblp), len(z), self.delta if delta is None else delta,
               out.ctypes.data_as(i64p))
        if rc:
            raise ValueError("encode: message length must divide N/2")
        return out

    # -- keys --------------------------------------------------------------
    def keygen(self, rot_steps=(), relin=True):
        L = lib()
        L.oc_keygen_secret(self.ptr)
        if relin:
            L.oc_keygen_relin(self.ptr)
        for s in rot_steps:
            if L.oc_keygen_rot(self.ptr, int(s)) != 0:
                raise RuntimeError("rotation keygen failed")

    def add_rot_keys(self, rot_steps):
        for s in rot_steps:
            lib().oc_keygen_rot(self.ptr, int(s))

    def secret(self):
        out = np.zeros(self.N, dtype=np.int8)
        lib().oc_secret(self.ptr, out.ctypes.data_as(C.POINTER(C.c_int8)))
        return out

    # -- encryption --------------------------------------------------------
    def encrypt(self, z, level=None, nonce=0):
        z = np.ascontiguousarray(z, dtype=np.float64).ravel()
        level = self.L if level is None else level
        return Ct(self, lib().oc_encrypt(self.ptr, z.ctypes.data_as(dblp), len(z), level, nonce))

    def encrypt_poly(self, m, level, scale, nonce=0):
        m = np.ascontiguousarray(m, dtype=np.int64)
        return Ct(self, lib().oc_encrypt_poly(self.ptr, m.ctypes.data_as(i64p), level, scale, nonce))

    def decrypt_residues(self, ct: Ct) -> np.ndarray:
        out = np.zeros((ct.level + 1) * self.N, dtype=np.uint64)
        if lib().oc_decrypt_residues(self.ptr, ct.ptr, out.ctypes.data_as(u64p)):
            raise RuntimeError("decrypt failed")
        return out.reshape(ct.level + 1, self.N)

    def decrypt_coeffs(self, ct: Ct):
        """Centred integer coefficients of c0 + c1 s mod Q_l (exact CRT)."""
        res = self.decrypt_residues(ct)
        return crt_centred(res, self.q[: ct.level + 1])

    def decrypt(self, ct: Ct, n=None):
        coeffs = self.decrypt_coeffs(ct)
        z = decode_float(coeffs, ct.scale, self.N)
        return z if n is None else z[:n]

    def ct_import(self, data, level, qp, scale):
        a, p = _u64(np.asarray(data, dtype=np.uint64).ravel())
        return Ct(self, lib().oc_ct_import(self.ptr, p, level, 1 if qp else 0, scale))

    # -- evaluation ----------------------------------------------------------
    def add(self, a, b):
        return Ct(self, lib().oc_add(self.ptr, a.ptr, b.ptr))

    def sub(self, a, b):
        return Ct(self, lib().oc_sub(self.ptr, a.ptr, b.ptr))

    def pmult(self, a, m, pt_scale):
        m = np.ascontiguousarray(m, dtype=np.int64)
        return Ct(self, lib().oc_pmult(self.ptr, a.ptr, m.ctypes.data_as(i64p), pt_scale))

    def padd(self, a, m):
        m = np.ascontiguousarray(m, dtype=np.int64)
        return Ct(self, lib().oc_padd(self.ptr, a.ptr, m.ctypes.data_as(i64p)))

    def mul_int(self, a, k):
        return Ct(self, lib().oc_mul_int(self.ptr, a.ptr, int(k)))

    def tensor(self, a, b):
        out = np.zeros(3 * a.nlimbs * self.N, dtype=np.uint64)
        if lib().oc_tensor(self.ptr, a.ptr, b.ptr, out.ctypes.data_as(u64p)):
            raise RuntimeError("tensor failed")
        return out.reshape(3, a.nlimbs, self.N)

    def mult(self, a, b):
        return Ct(self, lib().oc_mult(self.ptr, a.ptr, b.ptr))

    def rescale(self, a):
        return Ct(self, lib().oc_rescale(self.ptr, a.ptr))

    def drop(self, a, level):
        return Ct(self, lib().oc_drop(self.ptr, a.ptr, level))

    def beta_at(self, level):
        return lib().oc_beta_at(self.ptr, level)

    def decompose(self, d, level):
        d, p = _u64(np.asarray(d, dtype=np.uint64).ravel())
        beta = self.beta_at(level)
        nqp = level + 1 + self.alpha
        r = lib().oc_decompose(self.ptr, p, level)
        out = np.ctypeslib.as_array(r, shape=(beta * nqp * self.N,)).copy()
        lib().oc_free(C.cast(r, C.c_void_p))
        return out.reshape(beta, nqp, self.N)

    def moddown(self, a):
        return Ct(self, lib().oc_moddown(self.ptr, a.ptr))

    def moddown_rescale(self, a):
        """round(x / (P q_l)): ModDown and the Rescale after it as one rounding"""
        return Ct(self, lib().oc_moddown_rescale(self.ptr, a.ptr))

    def hoisted_rotate(self, a, step):
        return Ct(self, lib().oc_hoisted_rotate(self.ptr, a.ptr, step))

    def hoisted_rotate_digits(self, a, digits, step):
        """hoisted rotation with the digits Decompose(c1) given (as from decompose())"""
        d, p = _u64(np.asarray(digits, dtype=np.uint64).ravel())
        return Ct(self, lib().oc_hoisted_rotate_digits(self.ptr, a.ptr, p, step))

    def rotate(self, a, step):
        return Ct(self, lib().oc_rotate(self.ptr, a.ptr, step))

    def _lt(self, f, *args):
        err = C.c_int(0)
        r = f(self.ptr, *args, C.byref(err))
        if not r:
            raise RuntimeError(f"linear transform failed ({err.value})")
        return Ct(self, r)

    def lt_sigma(self, a, n, n1):
        return self._lt(lib().oc_lt_sigma, a.ptr, n, n1)

    def lt_tau(self, a, n, n1):
        return self._lt(lib().oc_lt_tau, a.ptr, n, n1)

    def lt_dcd(self, a, kind, n, n1, nprime):
        """Z (kind 0) or T (kind 1), decomposed when 0 < nprime < n - 1"""
        return self._lt(lib().oc_lt_dcd, a.ptr, kind, n, n1, nprime)

    def lt_smpkeysub(self, a, kind, n, n1, n1p):
        """Z (kind 0) or T (kind 1) by dh-BSGS whose baby steps use only the keys
        of the prefix a j', 0 < j' < n1p (simple key substitution, section 4.2.1)"""
        return self._lt(lib().oc_lt_smpkeysub, a.ptr, kind, n, n1, n1p)

    def lt_transpose(self, a, n, n1, weight=1.0):
        return self._lt(lib().oc_lt_transpose, a.ptr, n, n1, weight)

    def matmul(self, a, b, n, n1z, n1t, npz=None, npt=None, lazy=False, fused_rescale=False, folded=False):
        """lazy: relinearise once after summing the n tensors; fused_rescale:
        the A side's ModDown and Rescale as one rounding by P q_l (both
        variants; the paper's order relinearises every product and rounds
        twice); folded: the masks of C^k folded into Z, so the product takes
        two levels instead of three"""
        npz = n - 1 if npz is None else npz
        npt = n - 1 if npt is None else npt
        flags = (1 if lazy else 0) | (2 if fused_rescale else 0) | (4 if folded else 0)
        return self._lt(lib().oc_matmul_lazy, a.ptr, b.ptr, n, n1z, n1t, npz, npt, flags)

    def covariance(self, blocks, rb, k, n, n_samples, n1z, n1t, n1g, npz=None, npt=None, lazy=False,
                   fused_rescale=False):
        npz = n - 1 if npz is None else npz
        npt = n - 1 if npt is None else npt
        px = (C.c_void_p * len(blocks))(*[b.ptr for b in blocks])
        out = (C.c_void_p * (k * k))()
        flags = (1 if lazy else 0) | (2 if fused_rescale else 0)
        rc = lib().oc_covariance_lazy(self.ptr, px, rb, k, n, n_samples, n1z, n1t, npz, npt, n1g, flags, out)
        if rc:
            raise RuntimeError(f"covariance failed ({rc})")
        return [Ct(self, out[i]) for i in range(k * k)]


DCD_KIND = {"Z1": 0, "Z2": 1, "T": 2}


def dcd_factors(n, which, nprime, n1):
    """Factors of the diagonal convergence decomposition in application order:
    list of (perm, (a, n1, i_lo, i_hi)); perm[t] = input of output t or -1."""
    maxf = 64
    perms = np.zeros(maxf * n * n, dtype=np.int32)
    geom = np.zeros(maxf * 4, dtype=np.int64)
    nf = lib().oc_dcd_factors(n, DCD_KIND[which], nprime, n1, perms.ctypes.data_as(intp),
                              geom.ctypes.data_as(C.POINTER(C.c_longlong)), maxf)
    if nf < 0:
        raise ValueError("decomposition is not a product of partial permutations")
    return [(perms[j * n * n:(j + 1) * n * n].copy(), tuple(int(v) for v in geom[4 * j:4 * j + 4]))
            for j in range(nf)]


def perm_phi_sigma(n: int, k: int) -> np.ndarray:
    """the folded A side's permutation: output (i, j) takes A[i, (i + j + k) mod n]"""
    out = np.zeros(n * n, dtype=np.int32)
    lib().oc_perm_phi_sigma(n, k, out.ctypes.data_as(intp))
    return out


def perm(which: str, n: int) -> np.ndarray:
    out = np.zeros(n * n, dtype=np.int32)
    lib().oc_perm({"sigma": 0, "tau": 1, "transpose": 2}[which], n, out.ctypes.data_as(intp))
    return out


def crt_centred(res, primes):
    """Exact CRT of residues u64[k][N] to centred Python ints in (-Q/2, Q/2]."""
    Q = 1
    for q in primes:
        Q *= q
    coeffs = [0] * res.shape[1]
    terms = []
    for q in primes:
        Qi = Q // q
        terms.append((Qi * pow(Qi, -1, q)) % Q)
    rows = [[int(v) for v in r] for r in res]
    for i in range(res.shape[1]):
        x = 0
        for t, row in zip(terms, rows):
            x += row[i] * t
        x %= Q
        if x > Q // 2:
            x -= Q
        coeffs[i] = x
    return coeffs


def decode_float(coeffs, scale, N):
    """Slots z_j = (1/scale) sum_i m_i zeta^(5^j i), real parts (float64 FFT)."""
    m = np.array([float(v) for v in coeffs], dtype=np.float64)
    zeta = np.exp(1j * np.pi * np.arange(N) / N)
    y = N * np.fft.ifft(m * zeta)
    S = N // 2
    e = np.empty(S, dtype=np.int64)
    g = 1
    for j in range(S):
        e[j] = g
        g = (g * 5) % (2 * N)
    return (y[(e - 1) // 2].real / scale)
