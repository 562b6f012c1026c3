"""A context driven through the boundary's device hooks (he_device): device
memory from the caller's allocator and work on the caller's HIP stream.  The
caller here is plain HIP (hipMalloc / hipFree / hipStreamCreate of the same
HIP runtime the library links).  The residues equal those of a context on
its own pool and stream; every block the library took goes back through the
release hook when the context closes."""
import ctypes as C
import os

import numpy as np
import pytest

from paper_2305_17341_amd import inputs as I

pytestmark = pytest.mark.gpu

CH = I.MID


def _hip():
    from paper_2305_17341_amd import he
    he.load()   # the runtime the library links, already loaded: same handle
    hip = C.CDLL(os.path.join("/opt/rocm/lib", "libamdhip64.so.7"))
    hip.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
    hip.hipFree.argtypes = [C.c_void_p]
    hip.hipStreamCreate.argtypes = [C.POINTER(C.c_void_p)]
    hip.hipStreamDestroy.argtypes = [C.c_void_p]
    hip.hipStreamSynchronize.argtypes = [C.c_void_p]
    return hip


def test_context_on_callers_allocator_and_stream():
    from paper_2305_17341_amd import he
    hip = _hip()
    stream = C.c_void_p()
    assert hip.hipStreamCreate(C.byref(stream)) == 0
    live = {}

    def alloc(n):
        p = C.c_void_p()
        if hip.hipMalloc(C.byref(p), n) != 0:
            return 0
        live[p.value] = n
        return p.value

    def release(p):
        assert p in live, "release of a block the allocator did not hand out"
        del live[p]
        assert hip.hipFree(p) == 0

    hooks = he.DeviceHooks(alloc, release, stream.value)
    n = 16
    A, B = I.uniform_matrix(61, n), I.uniform_matrix(62, n)
    results = []
    try:
        for h in (hooks, None):
            ctx = he.Context(CH.log_n, CH.q_bits, CH.p_bits, seed=57, hooks=h)
            ctx.keygen(ctx.matmul_rot_steps(n))
            r = ctx.matmul(ctx.encrypt_matrix(A, nonce=1), ctx.encrypt_matrix(B, nonce=2), n)
            results.append(r.export())
            assert np.max(np.abs(ctx.decrypt(r, n * n) - (A @ B).ravel())) < 2.0 ** -15
            del r
            if h is not None:
                assert live, "the library allocated nothing through the hook"
            ctx.close()
        assert np.array_equal(results[0], results[1])
        assert not live, f"{len(live)} blocks not released"
    finally:
        hip.hipStreamSynchronize(stream)
        hip.hipStreamDestroy(stream)
