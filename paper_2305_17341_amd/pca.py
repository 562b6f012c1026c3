"""Privacy-preserving PCA driver (section 6.2, Algorithm Privacy-Preserving
PCA) over the library's calls: block covariance (he_covariance), then for
each of l_E components l_P + 1 rounds of he_power_step (Lazy Normalization
schedule for the Newton counts, the eigenvalue in the last round) and
he_eigen_shift.  Refreshes are the client's (Refresher)."""
from __future__ import annotations

import time

import numpy as np

from . import he


def taylor_point(B2: float) -> float:
    """TaylorInit expands x^-1/2 at the midpoint B^2/2 + 1 of (0, B^2]"""
    return B2 / 2.0 + 1.0


def lazy_schedule(l_p: int, S: float = 0.5, e: float = 1e-5, precision: float = 1e-3, B2: float = 2.0 ** 16,
                  max_tau: int = 200):
    """Newton counts per PowerMethod round (Lazy Normalization, section
    6.1.2): a unit length shrunk by S each round is normalised with the
    fewest Newton steps that keep (l S' S)^2 >= precision, and in the last
    round also 1 - l S' < e."""
    x0 = taylor_point(B2)
    length = 1.0
    out = []
    for t in range(l_p):
        length *= S
        x = length * length
        y = 1.5 * x0 ** -0.5 - 0.5 * x0 ** -1.5 * x
        tau = 0
        while True:
            good = (length * y * S) ** 2 >= precision
            if t == l_p - 1:
                good = good and 1.0 - length * y < e
            if good:
                break
            if tau == max_tau:
                raise ValueError("Lazy Normalization: no Newton count meets the bounds")
            y = y * (1.5 + (-0.5 * x) * (y * y))
            tau += 1
        out.append(tau)
        length *= y
    return out


def replicate(v, k, d, axis):
    """blocks of a replicated vector: axis 0 repeats segments as rows, 1 as columns"""
    blocks = []
    for i in range(k):
        seg = np.asarray(v[i * d:(i + 1) * d], dtype=np.float64)
        blocks.append(np.tile(seg, (d, 1)) if axis == 0 else np.tile(seg[:, None], (1, d)))
    return blocks


def read_vector(ctx, V, d, axis):
    """client side: decrypt a replicated vector"""
    parts = []
    for ct in V:
        b = ctx.decrypt(ct, d * d).reshape(d, d)
        parts.append(b[0, :] if axis == 0 else b[:, 0])
    return np.concatenate(parts)


def power_method(ctx, cov, k, d, V0, axis, taus, x0, refresher):
    """HPowerMethod: len(taus) normalising rounds, then the eigenvalue round.
    Returns (V, axis, lambda, V^T)."""
    V = V0
    for tau in taus:
        V, axis = ctx.power_step(cov, k, d, V, axis, tau, x0, False, refresher)
    return ctx.power_step(cov, k, d, V, axis, 0, x0, True, refresher)


def pppca(ctx, cov, k, d, l_e, l_p, seed=0, B2=2.0 ** 16, nonce0=1 << 40, on_component=None):
    """Algorithm Privacy-Preserving PCA from an encrypted covariance: l_E
    (eigenvalue, eigenvector) pairs by PowerMethod and EigenShift.  The
    random unit start vectors are encrypted by the client (axis 1)."""
    refresher = he.Refresher(ctx, nonce0)
    taus = lazy_schedule(l_p, B2=B2)
    x0 = taylor_point(B2)
    g = np.random.default_rng(seed)
    out = []
    for m in range(l_e):
        v0 = g.standard_normal(k * d)
        v0 /= np.linalg.norm(v0)
        V0 = [ctx.encrypt_matrix(b, nonce=(1 << 50) + m * k + i) for i, b in enumerate(replicate(v0, k, d, 1))]
        t0 = time.perf_counter()
        V, axis, lam, VT = power_method(ctx, cov, k, d, V0, 1, taus, x0, refresher)
        cov = ctx.eigen_shift(cov, k, d, lam, V, VT, axis, refresher)
        ctx.sync()
        out.append((lam, V, VT, axis))
        if on_component is not None:
            on_component(m, time.perf_counter() - t0)
    return out, refresher.count


def pca_bench(l_e=8, l_p=14, seed=3, log=print):
    """The PCA configuration at N = 2^16: a 256 x 256 dataset in [0, 1] with a
    planted spectrum, centred by the client, encrypted as 2 x 2 blocks of
    128 x 128; covariance (HCovMtrx), then l_e components by l_p + 1 power
    rounds each and the eigen-shift.  Decrypted results are compared with
    the same algorithm replayed in FP64 and with numpy's eigh."""
    from . import inputs as I
    ch = I.LARGE
    n, k, rb = 128, 2, 2
    ctx = he.chain_context(ch, seed=seed)
    steps = set(ctx.matmul_rot_steps(n)) | set(ctx.transpose_rot_steps(n)) | set(he.power_rot_steps(n))
    ctx.keygen(sorted(steps))
    X = I.centre(I.pca_dataset(seed, rb * n, k * n))
    blk = I.blocks(X, n)
    cts = [ctx.encrypt_matrix(blk[r, c], nonce=10 + r * k + c) for r in range(rb) for c in range(k)]
    ctx.sync()
    t0 = time.perf_counter()
    cov_ct = ctx.covariance(cts, rb, k, n, X.shape[0])
    ctx.sync()
    t_cov = time.perf_counter() - t0
    comp_s = []
    t0 = time.perf_counter()
    res, refreshes = pppca(ctx, cov_ct, k, n, l_e, l_p, seed=seed,
                           on_component=lambda m, s: (comp_s.append(s), log(f"[pca] component {m}: {s:.2f} s")))
    t_pca = time.perf_counter() - t0
    # client side: decrypt, FP64 replay of the same rounds, eigh
    cov = X.T @ X / X.shape[0]
    taus = lazy_schedule(l_p)
    x0 = taylor_point(2.0 ** 16)
    g = np.random.default_rng(seed)
    shifted = cov.copy()
    err_v, err_l, eig_l, eig_cos = 0.0, 0.0, [], []
    w, U = np.linalg.eigh(cov)
    w, U = w[::-1], U[:, ::-1]
    for m, (lam, V, VT, axis) in enumerate(res):
        v = g.standard_normal(k * n)
        v /= np.linalg.norm(v)
        for tau in taus:
            y = shifted @ v
            x = float(y @ y)
            s = 1.5 * x0 ** -0.5 - 0.5 * x0 ** -1.5 * x
            for _ in range(tau):
                s = s * (1.5 + (-0.5 * x) * (s * s))
            v = y * s
        lf = float((shifted @ v) @ v)
        shifted = shifted - lf * np.outer(v, v)
        got_v = read_vector(ctx, V, n, axis)
        got_l = float(ctx.decrypt(lam, 4)[0])
        err_v = max(err_v, float(np.max(np.abs(got_v - v))))
        err_l = max(err_l, abs(got_l - lf) / max(1.0, abs(lf)))
        eig_l.append(abs(got_l - w[m]) / w[m])
        eig_cos.append(abs(float(got_v @ U[:, m])) / float(np.linalg.norm(got_v)))
    return {
        "workload": f"PCA of a 256x256 [0,1] dataset with planted spectrum at N=2^16: covariance (2x2 blocks of "
                    f"128), {l_e} components x ({l_p} + 1) power rounds, Lazy Normalization schedule {taus}",
        "covariance_s": round(t_cov, 3),
        "pca_s": round(t_pca, 3),
        "s_per_component": [round(x, 3) for x in comp_s],
        "power_rounds_per_s": round(l_e * (l_p + 1) / t_pca, 3),
        "refreshes": refreshes,
        "max_abs_err_vs_fp64_replay": {"eigenvector": err_v, "eigenvalue_rel": err_l},
        "vs_eigh": {"eigenvalue_rel_err": [round(x, 6) for x in eig_l],
                    "abs_cos_to_eigenvector": [round(x, 6) for x in eig_cos],
                    "top_eigenvalues": [round(float(x), 4) for x in w[:l_e]]},
    }
