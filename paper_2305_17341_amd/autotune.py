"""Launch-shape autotuner: times the batched product under each value of the
library's knobs (members and rotations per launch, the order in which the
block passes and the plaintext sums visit limbs, the NTT's stage split
between its column and block passes) and keeps the fastest.
The knobs only regroup or reorder work, so every choice gives the same
residues; the timing decides."""
from __future__ import annotations

import time

from . import he

CANDIDATES = {
    "mr_members": (2, 4, 8),
    "mr_rotations": (4, 8, 16, 32, 64),
    "ms_members": (4, 8),
    "ntt_interleave": (0, 1),
    "ew_interleave": (0, 1),
    "mr_group": (1, 2, 4),
    "mr_int_split": (0, 1),
    "mr_int_pass": (4, 8),
    "mr_int_chunk": (4, 16, 64),
    "mr_int_concurrent": (0, 1),
    "sum_streams": (1, 2, 4),
    "mr_pair": (0, 1),
}


# the NTT's stage split, per ring size that has an alternative (tuned on a
# product of that ring size)
NTT_SPLIT_LOG_N = (13, 14, 15)


def autotune_ntt_split(ctx, cA, cB, d, opts=None, log=None, margin=0.01):
    """the stage split of the register-blocked NTT for ctx's ring size"""
    if ctx.log_n not in NTT_SPLIT_LOG_N:
        return {}, {}
    return autotune(ctx, cA, cB, d, opts=opts, candidates={f"ntt_split_{ctx.log_n}": (0, 1)}, log=log,
                    margin=margin)


def autotune(ctx, cA, cB, d, opts=None, candidates=CANDIDATES, log=None, margin=0.01):
    """Coordinate descent over the knobs, one batched step per candidate
    value (the plaintext caches must be warm).  A knob leaves its current
    value only for one at least `margin` faster, so that timing noise does
    not flip it.  Leaves the chosen values set and returns (best, timings in
    ms)."""
    best = {k: he.knob_get(k) for k in candidates}
    timings = {}
    for name, values in candidates.items():
        res = {}
        for v in values:
            he.knob_set(name, v)
            ctx.sync()
            t0 = time.perf_counter()
            outs = ctx.matmul_batch(cA, cB, [d] * len(cA), opts=opts)
            ctx.sync()
            res[v] = 1e3 * (time.perf_counter() - t0)
            del outs
        fastest = min(res, key=res.get)
        if best[name] not in res or res[fastest] < (1.0 - margin) * res[best[name]]:
            best[name] = fastest
        he.knob_set(name, best[name])
        timings[name] = {str(k): round(v, 2) for k, v in res.items()}
        if log:
            log(f"[autotune] {name}: " + ", ".join(f"{k}={v:.1f} ms" for k, v in res.items()) + f" -> {best[name]}")
    return best, timings
