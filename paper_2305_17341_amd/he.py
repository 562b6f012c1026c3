"""Thin ctypes binding of the C ABI in include/he_mi355x.h.

Argument marshalling only: every step runs in the HIP library
(libhe_mi355x.so, built in-tree by paper_2305_17341_amd.build).  There is no
fallback: if the library is missing or no HIP device is present, calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libhe_mi355x.so")

HE_OK = 0
# bytes of the per-GPU workspace of the allocation-free entry points (HE_NOALLOC_WS_BYTES)
NOALLOC_WS_BYTES = 64 << 20
STATUS = {0: "HE_OK", -1: "HE_EINVAL", -2: "HE_ELEVEL", -3: "HE_ESCALE", -4: "HE_EKEY", -5: "HE_ENOMEM",
          -6: "HE_EDEVICE", -7: "HE_EBUSY", -8: "HE_ENEEDREFRESH"}

# every symbol the header declares (checked by the CPU test-suite)
EXPORTS = [
    "he_ctx_create", "he_ctx_destroy", "he_ctx_moduli", "he_keygen", "he_matmul_rot_steps",
    "he_transpose_rot_steps", "he_encode", "he_encrypt_slots", "he_encrypt_matrix", "he_decrypt", "he_ct_info",
    "he_ct_export", "he_ct_import", "he_ct_free", "he_add", "he_sub", "he_mult", "he_rescale", "he_rotate",
    "he_drop_level", "he_pmult_slots", "he_lintrans", "he_lintrans_dcd", "he_lintrans_smpkeysub", "he_matmul", "he_matmul_batch", "he_covariance", "he_sync",
    "he_mem_info", "he_trim", "he_device_memory", "he_ntt_limbs", "he_automorph_limbs", "he_hoisted_rotate_export", "he_last_op_ms",
    "he_profile_enable", "he_profile_read", "he_op_counts", "he_lintrans_rot_steps", "he_smpkeysub_rot_steps", "he_refresh",
    "he_power_rot_steps", "he_power_step", "he_eigen_shift", "he_knob_set", "he_knob_get", "he_last_error",
    "he_rotate_noalloc", "he_rotate_workspace_bytes", "he_modmul_peak", "he_profile_read_ops", "he_rotate_many", "he_params_moduli",
    "he_covariance_begin", "he_covariance_add", "he_covariance_end", "he_covariance_free",
]

# he_refresh_fn: status (he_ct*, void* user)
REFRESH_FN = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_void_p)

u64p = C.POINTER(C.c_uint64)
i64p = C.POINTER(C.c_int64)
dblp = C.POINTER(C.c_double)
vp = C.c_void_p


class HeError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class he_params(C.Structure):
    _fields_ = [("log_n", C.c_uint32), ("q_bits", C.POINTER(C.c_uint32)), ("n_q", C.c_uint32),
                ("p_bits", C.POINTER(C.c_uint32)), ("n_p", C.c_uint32), ("log2_scale", C.c_double),
                ("sigma", C.c_double)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class he_device(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("release", RELEASE_FN), ("user", C.c_void_p), ("hip_stream", C.c_void_p)]


class DeviceHooks:
    """A caller's device allocator and HIP stream for a context (he_device):
    alloc(nbytes) -> device address (int, 0 on failure), release(address),
    stream = a HIP stream handle (int) or None.  The callbacks stay alive
    with this object, which must outlive the context."""

    def __init__(self, alloc=None, release=None, stream=None):
        self._alloc = ALLOC_FN(lambda n, user: alloc(n) or None) if alloc else ALLOC_FN()
        self._release = RELEASE_FN(lambda ptr, user: release(ptr)) if release else RELEASE_FN()
        self.struct = he_device(self._alloc, self._release, None, stream)


class he_matmul_opts(C.Structure):
    _fields_ = [("n1_z", C.c_uint32), ("n1_t", C.c_uint32), ("nprime_z", C.c_uint32), ("nprime_t", C.c_uint32),
                ("flags", C.c_uint32)]


_lib = None


def load():
    """Load the built library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} (run paper_2305_17341_amd.build.build())")
    L = C.CDLL(LIB_PATH)
    sig = {
        "he_ctx_create": [C.POINTER(he_params), vp, C.c_uint64, C.POINTER(vp)],
        "he_ctx_destroy": [vp],
        "he_ctx_moduli": [vp, u64p, C.c_size_t, C.POINTER(C.c_size_t)],
        "he_keygen": [vp, C.POINTER(C.c_int32), C.c_size_t],
        "he_matmul_rot_steps": [vp, C.c_uint32, C.POINTER(he_matmul_opts), C.POINTER(C.c_int32), C.c_size_t,
                                C.POINTER(C.c_size_t)],
        "he_transpose_rot_steps": [vp, C.c_uint32, C.c_uint32, C.POINTER(C.c_int32), C.c_size_t,
                                   C.POINTER(C.c_size_t)],
        "he_encode": [vp, dblp, C.c_size_t, C.c_double, i64p],
        "he_encrypt_slots": [vp, dblp, C.c_size_t, C.c_uint32, C.c_uint64, C.POINTER(vp)],
        "he_encrypt_matrix": [vp, dblp, C.c_uint32, C.c_uint32, C.c_uint64, C.POINTER(vp)],
        "he_decrypt": [vp, vp, dblp, C.c_size_t],
        "he_ct_info": [vp, C.POINTER(C.c_uint32), dblp],
        "he_ct_export": [vp, u64p, C.c_size_t, C.POINTER(C.c_uint32), dblp],
        "he_ct_import": [vp, u64p, C.c_size_t, C.c_uint32, C.c_double, C.POINTER(vp)],
        "he_ct_free": [vp],
        "he_add": [vp, vp, vp, C.POINTER(vp)],
        "he_sub": [vp, vp, vp, C.POINTER(vp)],
        "he_mult": [vp, vp, vp, C.POINTER(vp)],
        "he_rescale": [vp, vp, C.POINTER(vp)],
        "he_rotate": [vp, vp, C.c_int32, C.POINTER(vp)],
        "he_drop_level": [vp, vp, C.c_uint32, C.POINTER(vp)],
        "he_rotate_noalloc": [vp, vp, C.c_int32, vp],
        "he_rotate_many": [vp, C.POINTER(vp), C.c_size_t, C.POINTER(C.c_int32), C.c_size_t, C.POINTER(vp)],
        "he_modmul_peak": [C.c_uint32, C.c_uint64, C.c_uint32, dblp, dblp],
        "he_params_moduli": [C.POINTER(he_params), u64p, u64p, C.c_size_t],
        "he_profile_read_ops": [vp, C.c_char_p, dblp, dblp, dblp],
        "he_rotate_workspace_bytes": [vp, C.c_uint32, C.POINTER(C.c_size_t)],
        "he_pmult_slots": [vp, vp, dblp, C.c_size_t, C.c_double, C.POINTER(vp)],
        "he_lintrans": [vp, vp, C.c_uint32, C.c_uint32, C.c_uint32, C.c_double, C.POINTER(vp)],
        "he_lintrans_dcd": [vp, vp, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.POINTER(vp)],
        "he_lintrans_smpkeysub": [vp, vp, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.POINTER(vp)],
        "he_matmul": [vp, vp, vp, C.c_uint32, C.POINTER(he_matmul_opts), C.POINTER(vp)],
        "he_matmul_batch": [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(C.c_uint32), C.c_size_t,
                            C.POINTER(he_matmul_opts), C.POINTER(vp)],
        "he_covariance": [vp, C.POINTER(vp), C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64,
                          C.POINTER(he_matmul_opts), C.POINTER(vp)],
        "he_covariance_begin": [vp, C.c_uint32, C.c_uint32, C.c_uint64, C.POINTER(he_matmul_opts), C.POINTER(vp)],
        "he_covariance_add": [vp, C.POINTER(vp), C.c_uint32],
        "he_covariance_end": [vp, C.POINTER(vp)],
        "he_covariance_free": [vp],
        "he_sync": [vp],
        "he_mem_info": [vp, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)],
        "he_trim": [vp],
        "he_device_memory": [C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)],
        "he_ntt_limbs": [vp, u64p, u64p, C.c_size_t, C.POINTER(C.c_int32), C.c_int],
        "he_automorph_limbs": [vp, u64p, u64p, C.c_size_t, C.c_uint64],
        "he_hoisted_rotate_export": [vp, vp, C.c_int32, u64p, C.c_size_t],
        "he_last_op_ms": [vp, dblp],
        "he_profile_enable": [vp, C.c_int],
        "he_profile_read": [vp, C.c_char_p, dblp, u64p, dblp],
        "he_op_counts": [vp, u64p, u64p, u64p],
        "he_lintrans_rot_steps": [C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.POINTER(C.c_int32), C.c_size_t,
                                  C.POINTER(C.c_size_t)],
        "he_smpkeysub_rot_steps": [C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.POINTER(C.c_int32),
                                   C.c_size_t, C.POINTER(C.c_size_t)],
        "he_refresh": [vp, vp, C.c_uint64],
        "he_knob_set": [C.c_char_p, C.c_int32],
        "he_knob_get": [C.c_char_p, C.POINTER(C.c_int32)],
        "he_power_rot_steps": [C.c_uint32, C.POINTER(C.c_int32), C.c_size_t, C.POINTER(C.c_size_t)],
        "he_power_step": [vp, C.POINTER(vp), C.c_uint32, C.c_uint32, C.POINTER(vp), C.c_uint32, C.c_uint32,
                          C.c_double, C.c_uint32, C.c_int, C.c_uint32, REFRESH_FN, vp, C.POINTER(vp),
                          C.POINTER(C.c_uint32), C.POINTER(vp), C.POINTER(vp)],
        "he_eigen_shift": [vp, C.POINTER(vp), C.c_uint32, C.c_uint32, vp, C.POINTER(vp), C.POINTER(vp), C.c_uint32,
                           REFRESH_FN, vp, C.POINTER(vp)],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int
    L.he_last_error.restype = C.c_char_p
    L.he_last_error.argtypes = []
    _lib = L
    return L


def _check(st):
    if st != HE_OK:
        raise HeError(st, load().he_last_error().decode())


def _opts(opts):
    if opts is None:
        return None
    o = he_matmul_opts()
    for k, v in opts.items():
        setattr(o, k, int(v))
    return C.byref(o)


class CovarianceParts:
    """State of he_covariance_begin/add/end (see Context.covariance_begin)."""

    def __init__(self, ctx, ptr, k):
        self.ctx, self.ptr, self.k = ctx, ptr, k

    def add(self, blocks, row_blocks):
        px = (vp * (row_blocks * self.k))(*[x.ptr for x in blocks])
        _check(load().he_covariance_add(self.ptr, px, row_blocks))

    def end(self):
        out = (vp * (self.k * self.k))()
        _check(load().he_covariance_end(self.ptr, out))
        return [Ciphertext(self.ctx, vp(out[i])) for i in range(self.k * self.k)]

    def free(self):
        if self.ptr and self.ptr.value:
            _check(load().he_covariance_free(self.ptr))
            self.ptr = vp()

    def __del__(self):
        try:
            if _lib is not None and self.ptr and self.ptr.value and self.ctx.ptr and self.ctx.ptr.value:
                _lib.he_covariance_free(self.ptr)
                self.ptr = vp()
        except Exception:
            pass


class Ciphertext:
    def __init__(self, ctx: "Context", ptr):
        self.ctx = ctx
        self.ptr = vp(ptr) if not isinstance(ptr, vp) else ptr

    def free(self):
        if self.ptr and self.ptr.value:
            _check(load().he_ct_free(self.ptr))
            self.ptr = vp()

    def __del__(self):
        # a ciphertext keeps its context alive; skip if the context is gone already
        try:
            if _lib is not None and self.ptr and self.ptr.value and self.ctx.ptr and self.ctx.ptr.value:
                _lib.he_ct_free(self.ptr)
                self.ptr = vp()
        except Exception:
            pass

    @property
    def level(self):
        lv = C.c_uint32()
        _check(load().he_ct_info(self.ptr, C.byref(lv), None))
        return lv.value

    @property
    def scale(self):
        s = C.c_double()
        _check(load().he_ct_info(self.ptr, None, C.byref(s)))
        return s.value

    def export(self) -> np.ndarray:
        """Residues u64[2][level+1][N] (synchronises)."""
        lv = self.level
        out = np.zeros(2 * (lv + 1) * self.ctx.N, dtype=np.uint64)
        _check(load().he_ct_export(self.ptr, out.ctypes.data_as(u64p), out.size, None, None))
        return out.reshape(2, lv + 1, self.ctx.N)


class Context:
    """One CKKS parameter set on the current HIP device."""

    def __init__(self, log_n, q_bits, p_bits, log2_scale=40.0, sigma=3.2, seed=1, hooks=None):
        L = load()
        self._qb = (C.c_uint32 * len(q_bits))(*q_bits)
        self._pb = (C.c_uint32 * len(p_bits))(*p_bits)
        prm = he_params(log_n, self._qb, len(q_bits), self._pb, len(p_bits), log2_scale, sigma)
        ptr = vp()
        self._hooks = hooks
        dev = C.cast(C.pointer(hooks.struct), vp) if hooks is not None else None
        _check(L.he_ctx_create(C.byref(prm), dev, seed, C.byref(ptr)))
        self.ptr = ptr
        self.log_n = log_n
        self.N = 1 << log_n
        self.slots = self.N // 2
        self.L = len(q_bits) - 1
        self.alpha = len(p_bits)
        n = C.c_size_t()
        buf = (C.c_uint64 * 128)()
        _check(L.he_ctx_moduli(ptr, buf, 128, C.byref(n)))
        self.moduli = [int(buf[i]) for i in range(n.value)]

    def close(self):
        if getattr(self, "ptr", None) and self.ptr.value:
            _check(load().he_ctx_destroy(self.ptr))
            self.ptr = vp()

    def __del__(self):
        # device memory (keys, caches, pool) goes back when the last reference
        # (every ciphertext holds one) is dropped
        try:
            if _lib is not None:
                self.close()
        except Exception:
            pass

    def _ct(self, f, *args):
        out = vp()
        _check(f(self.ptr, *args, C.byref(out)))
        return Ciphertext(self, out)

    # keys
    def keygen(self, rot_steps=()):
        steps = (C.c_int32 * max(1, len(rot_steps)))(*[int(s) for s in rot_steps])
        _check(load().he_keygen(self.ptr, steps, len(rot_steps)))

    def matmul_rot_steps(self, d, opts=None):
        n = C.c_size_t()
        buf = (C.c_int32 * 4096)()
        _check(load().he_matmul_rot_steps(self.ptr, d, _opts(opts), buf, 4096, C.byref(n)))
        return [int(buf[i]) for i in range(n.value)]

    def transpose_rot_steps(self, d, n1=0):
        n = C.c_size_t()
        buf = (C.c_int32 * 4096)()
        _check(load().he_transpose_rot_steps(self.ptr, d, n1, buf, 4096, C.byref(n)))
        return [int(buf[i]) for i in range(n.value)]

    # encoding / encryption
    def encode(self, z, delta):
        z = np.ascontiguousarray(z, dtype=np.float64).ravel()
        out = np.zeros(self.N, dtype=np.int64)
        _check(load().he_encode(self.ptr, z.ctypes.data_as(dblp), len(z), delta, out.ctypes.data_as(i64p)))
        return out

    def encrypt(self, z, level=None, nonce=0):
        z = np.ascontiguousarray(z, dtype=np.float64).ravel()
        level = self.L if level is None else level
        return self._ct(load().he_encrypt_slots, z.ctypes.data_as(dblp), len(z), level, nonce)

    def encrypt_matrix(self, A, level=None, nonce=0):
        A = np.ascontiguousarray(A, dtype=np.float64)
        level = self.L if level is None else level
        return self._ct(load().he_encrypt_matrix, A.ctypes.data_as(dblp), A.shape[0], level, nonce)

    def decrypt(self, ct, n=None):
        n = self.slots if n is None else n
        out = np.zeros(n, dtype=np.float64)
        _check(load().he_decrypt(self.ptr, ct.ptr, out.ctypes.data_as(dblp), n))
        return out

    def ct_import(self, data, level, scale):
        d = np.ascontiguousarray(data, dtype=np.uint64).ravel()
        return self._ct(load().he_ct_import, d.ctypes.data_as(u64p), d.size, level, scale)

    # operations
    def add(self, a, b):
        return self._ct(load().he_add, a.ptr, b.ptr)

    def sub(self, a, b):
        return self._ct(load().he_sub, a.ptr, b.ptr)

    def mult(self, a, b):
        return self._ct(load().he_mult, a.ptr, b.ptr)

    def rescale(self, a):
        return self._ct(load().he_rescale, a.ptr)

    def rotate(self, a, step):
        return self._ct(load().he_rotate, a.ptr, int(step))

    def rotate_many(self, cts, steps):
        """hoisted rotations of every ciphertext by every step: result[i][r] = Rot(cts[i], steps[r])"""
        a = (vp * len(cts))(*[c.ptr.value for c in cts])
        st = (C.c_int32 * len(steps))(*[int(x) for x in steps])
        out = (vp * (len(cts) * len(steps)))()
        _check(load().he_rotate_many(self.ptr, a, len(cts), st, len(steps), out))
        return [[Ciphertext(self, vp(out[i * len(steps) + r])) for r in range(len(steps))]
                for i in range(len(cts))]

    def rotate_noalloc(self, a, step, out):
        """Rotation into the existing ciphertext `out` (a's level) with no
        device allocation: temporaries in the library's per-GPU workspace."""
        _check(load().he_rotate_noalloc(self.ptr, a.ptr, int(step), out.ptr))
        return out

    def rotate_workspace_bytes(self, level):
        n = C.c_size_t()
        _check(load().he_rotate_workspace_bytes(self.ptr, level, C.byref(n)))
        return n.value

    def drop(self, a, level):
        return self._ct(load().he_drop_level, a.ptr, level)

    def pmult(self, a, z, pt_scale):
        z = np.ascontiguousarray(z, dtype=np.float64).ravel()
        return self._ct(load().he_pmult_slots, a.ptr, z.ctypes.data_as(dblp), len(z), pt_scale)

    def lintrans(self, a, kind, d, n1=0, weight=1.0):
        k = {"sigma": 0, "tau": 1, "transpose": 2}[kind] if isinstance(kind, str) else kind
        return self._ct(load().he_lintrans, a.ptr, k, d, n1, weight)

    def lintrans_dcd(self, a, kind, d, n1=0, nprime=0):
        """Z (kind 0 / "sigma") or T (1 / "tau"), decomposed when 0 < nprime < d - 1"""
        k = {"sigma": 0, "tau": 1}[kind] if isinstance(kind, str) else kind
        return self._ct(load().he_lintrans_dcd, a.ptr, k, d, n1, nprime)

    def lintrans_smpkeysub(self, a, kind, d, n1=0, n1p=0):
        """Z or T by dh-BSGS with the simple key substitution of the baby steps
        (keys of the prefix a j', j' < n1p, only)"""
        k = {"sigma": 0, "tau": 1}[kind] if isinstance(kind, str) else kind
        return self._ct(load().he_lintrans_smpkeysub, a.ptr, k, d, n1, n1p)

    def matmul(self, a, b, d, opts=None):
        return self._ct(load().he_matmul, a.ptr, b.ptr, d, _opts(opts))

    def matmul_batch(self, As, Bs, ds, opts=None):
        n = len(As)
        pa = (vp * n)(*[x.ptr for x in As])
        pb = (vp * n)(*[x.ptr for x in Bs])
        dd = (C.c_uint32 * n)(*ds)
        out = (vp * n)()
        _check(load().he_matmul_batch(self.ptr, pa, pb, dd, n, _opts(opts), out))
        return [Ciphertext(self, vp(out[i])) for i in range(n)]

    def covariance(self, blocks, row_blocks, k, d, n_samples, opts=None):
        n = row_blocks * k
        px = (vp * n)(*[x.ptr for x in blocks])
        out = (vp * (k * k))()
        _check(load().he_covariance(self.ptr, px, row_blocks, k, d, n_samples, _opts(opts), out))
        return [Ciphertext(self, vp(out[i])) for i in range(k * k)]

    def covariance_begin(self, k, d, n_samples, opts=None):
        """the covariance in parts: a state taking row blocks (add) and
        returning the k*k blocks (end), with he_covariance's residues"""
        st = vp()
        _check(load().he_covariance_begin(self.ptr, k, d, n_samples, _opts(opts), C.byref(st)))
        return CovarianceParts(self, st, k)

    def refresh(self, ct, nonce):
        """in place: ct becomes a top-level encryption of its message"""
        _check(load().he_refresh(self.ptr, ct.ptr, nonce))

    def power_step(self, cov, k, d, V, axis, tau, x0, last, refresher=None, goldschmidt=False, pack=False):
        """One HPowerMethod round.  Returns (V', axis') or, for the last
        round, (V, axis, lambda, V^T).  goldschmidt: the inverse square root
        by Goldschmidt's form of the Newton iterates (HE_PM_GOLDSCHMIDT); pack:
        a low vector refreshed through one ciphertext (HE_PM_PACK_REFRESH).
        Entries of V may be replaced in place by refreshes."""
        pc = (vp * (k * k))(*[c.ptr for c in cov])
        pv = (vp * k)(*[x.ptr for x in V])
        vo = (vp * k)()
        vto = (vp * k)()
        lam = vp()
        ax = C.c_uint32()
        fn = refresher.fn if refresher is not None else REFRESH_FN()
        _check(load().he_power_step(self.ptr, pc, k, d, pv, axis, tau, x0, 1, 1 if last else 0,
                                    (1 if goldschmidt else 0) | (2 if pack else 0), fn, None, vo, C.byref(ax),
                                    C.byref(lam), vto))
        if last:
            return V, ax.value, Ciphertext(self, lam), [Ciphertext(self, vp(vto[i])) for i in range(k)]
        return [Ciphertext(self, vp(vo[i])) for i in range(k)], ax.value

    def eigen_shift(self, cov, k, d, lam, V, VT, axis, refresher=None):
        pc = (vp * (k * k))(*[c.ptr for c in cov])
        pv = (vp * k)(*[x.ptr for x in V])
        pvt = (vp * k)(*[x.ptr for x in VT])
        out = (vp * (k * k))()
        fn = refresher.fn if refresher is not None else REFRESH_FN()
        _check(load().he_eigen_shift(self.ptr, pc, k, d, lam.ptr, pv, pvt, axis, fn, None, out))
        return [Ciphertext(self, vp(out[i])) for i in range(k * k)]

    def sync(self):
        _check(load().he_sync(self.ptr))

    def mem_info(self):
        a, b, c = C.c_size_t(), C.c_size_t(), C.c_size_t()
        _check(load().he_mem_info(self.ptr, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def trim(self):
        _check(load().he_trim(self.ptr))

    def last_op_ms(self):
        ms = C.c_double()
        _check(load().he_last_op_ms(self.ptr, C.byref(ms)))
        return ms.value

    def profile_enable(self, on=True):
        _check(load().he_profile_enable(self.ptr, 1 if on else 0))

    def profile_read(self, family):
        """(device ms, launches, algorithmic bytes) of a kernel family since enabling."""
        ms, n, b = C.c_double(), C.c_uint64(), C.c_double()
        _check(load().he_profile_read(self.ptr, family.encode(), C.byref(ms), C.byref(n), C.byref(b)))
        return ms.value, n.value, b.value

    def profile_read_ops(self, family):
        """(FP64 modular products, integer modular products, bytes in the key
        switch's unit of work) of a kernel family since enabling."""
        f, i, u = C.c_double(), C.c_double(), C.c_double()
        _check(load().he_profile_read_ops(self.ptr, family.encode(), C.byref(f), C.byref(i), C.byref(u)))
        return f.value, i.value, u.value

    def op_counts(self):
        a, b, c = C.c_uint64(), C.c_uint64(), C.c_uint64()
        _check(load().he_op_counts(self.ptr, C.byref(a), C.byref(b), C.byref(c)))
        return {"decompose": a.value, "multsum": b.value, "moddown": c.value}

    # raw pieces for parity checks
    def ntt_limbs(self, limbs, mod_idx, inverse=False):
        a = np.ascontiguousarray(limbs, dtype=np.uint64)
        out = np.zeros_like(a)
        mi = (C.c_int32 * len(mod_idx))(*mod_idx)
        _check(load().he_ntt_limbs(self.ptr, a.ctypes.data_as(u64p), out.ctypes.data_as(u64p), len(mod_idx), mi,
                                   1 if inverse else 0))
        return out

    def automorph_limbs(self, limbs, galois):
        a = np.ascontiguousarray(limbs, dtype=np.uint64)
        out = np.zeros_like(a)
        nl = a.size // self.N
        _check(load().he_automorph_limbs(self.ptr, a.ctypes.data_as(u64p), out.ctypes.data_as(u64p), nl, galois))
        return out

    def hoisted_rotate_export(self, a, step):
        lv = a.level
        out = np.zeros(2 * (lv + 1 + self.alpha) * self.N, dtype=np.uint64)
        _check(load().he_hoisted_rotate_export(self.ptr, a.ptr, int(step), out.ctypes.data_as(u64p), out.size))
        return out.reshape(2, lv + 1 + self.alpha, self.N)


def params_moduli(log_n, q_bits, p_bits):
    """Host only: (moduli, psi) a context with these prime sizes uses."""
    qb = (C.c_uint32 * len(q_bits))(*q_bits)
    pb = (C.c_uint32 * len(p_bits))(*p_bits)
    prm = he_params(log_n, qb, len(q_bits), pb, len(p_bits), 40.0, 3.2)
    n = len(q_bits) + len(p_bits)
    m, psi = (C.c_uint64 * n)(), (C.c_uint64 * n)()
    _check(load().he_params_moduli(C.byref(prm), m, psi, n))
    return [int(x) for x in m], [int(x) for x in psi]


MODMUL_KINDS = {"f64_lazy": 0, "shoup": 1, "barrett": 2, "f64_butterfly": 3}


def modmul_peak(kind, iters=4096, blocks=8192):
    """Measured rate (products/s) of one kind of modular product on the
    current device (he_modmul_peak); returns (rate, ms)."""
    r, ms = C.c_double(), C.c_double()
    _check(load().he_modmul_peak(MODMUL_KINDS[kind], iters, blocks, C.byref(r), C.byref(ms)))
    return r.value, ms.value


def lintrans_rot_steps(kind, d, n1, nprime=0):
    """Planner (host only): rotation steps of one transform ("Z", "T", "G")."""
    k = {"Z": 0, "T": 1, "G": 2}[kind]
    n = C.c_size_t()
    buf = (C.c_int32 * 8192)()
    _check(load().he_lintrans_rot_steps(k, d, n1, nprime, buf, 8192, C.byref(n)))
    return [int(buf[i]) for i in range(n.value)]


def smpkeysub_rot_steps(kind, d, n1, n1p):
    """Planner (host only): rotation steps of Z or T with the simple key
    substitution of the baby steps (prefix n1p)."""
    k = {"Z": 0, "T": 1}[kind]
    n = C.c_size_t()
    buf = (C.c_int32 * 8192)()
    _check(load().he_smpkeysub_rot_steps(k, d, n1, n1p, buf, 8192, C.byref(n)))
    return [int(buf[i]) for i in range(n.value)]


class Refresher:
    """Client-side refresh for he_power_step / he_eigen_shift: re-encrypts
    the ciphertext it is handed at the top level with the next nonce."""

    def __init__(self, ctx: "Context", nonce0: int = 1 << 40):
        self.ctx = ctx
        self.nonce = nonce0
        self.count = 0

        def cb(ct_ptr, user):
            st = load().he_refresh(self.ctx.ptr, ct_ptr, self.nonce)
            self.nonce += 1
            self.count += 1
            return st

        self.fn = REFRESH_FN(cb)


def power_rot_steps(d):
    n = C.c_size_t()
    buf = (C.c_int32 * 256)()
    _check(load().he_power_rot_steps(d, buf, 256, C.byref(n)))
    return [int(buf[i]) for i in range(n.value)]


def knob_set(name, value):
    _check(load().he_knob_set(name.encode(), int(value)))


def knob_get(name):
    v = C.c_int32()
    _check(load().he_knob_get(name.encode(), C.byref(v)))
    return v.value


def device_memory():
    """(free, total) bytes of the current device"""
    a, b = C.c_size_t(), C.c_size_t()
    _check(load().he_device_memory(C.byref(a), C.byref(b)))
    return a.value, b.value


def chain_context(chain, seed=1) -> Context:
    return Context(chain.log_n, chain.q_bits, chain.p_bits, chain.log2_scale, chain.sigma, seed)
