"""Privacy-preserving PCA driver (section 6.2, Algorithm Privacy-Preserving
PCA) over the library's calls: block covariance (he_covariance), then for
each of l_E components l_P + 1 rounds of he_power_step (Lazy Normalization
schedule for the Newton counts, the eigenvalue in the last round) and
he_eigen_shift.  Refreshes are the client's (Refresher)."""
from __future__ import annotations

import time

import numpy as np

from . import he, packing


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


def power_method(ctx, cov, k, d, V0, axis, taus, x0, refresher, goldschmidt=False, pack=False):
    """HPowerMethod: len(taus) normalising rounds, then the eigenvalue round.
    Returns (V, axis, lambda, V^T).  goldschmidt: Goldschmidt's form of the
    inverse square root (the same iterates, fewer levels); pack: a low output
    vector refreshed through one ciphertext (Appendix C)."""
    V = V0
    for tau in taus:
        V, axis = ctx.power_step(cov, k, d, V, axis, tau, x0, False, refresher, goldschmidt=goldschmidt, pack=pack)
    return ctx.power_step(cov, k, d, V, axis, 0, x0, True, refresher)


def pppca(ctx, cov, k, d, l_e, l_p, seed=0, B2=2.0 ** 16, nonce0=1 << 40, on_component=None, start_nonce=1 << 50,
          goldschmidt=False, pack=False):
    """Algorithm Privacy-Preserving PCA from an encrypted covariance: l_E
    (eigenvalue, eigenvector) pairs by PowerMethod and EigenShift.  The
    random unit start vectors are encrypted by the client (axis 1, nonces
    from start_nonce; refreshes take theirs from nonce0)."""
    refresher = he.Refresher(ctx, nonce0)
    taus = lazy_schedule(l_p, B2=B2)
    x0 = taylor_point(B2)
    g = np.random.default_rng(seed)
    out = []
    for m in range(l_e):
        v0 = g.standard_normal(k * d)
        v0 /= np.linalg.norm(v0)
        V0 = [ctx.encrypt_matrix(b, nonce=start_nonce + m * k + i) for i, b in enumerate(replicate(v0, k, d, 1))]
        t0 = time.perf_counter()
        V, axis, lam, VT = power_method(ctx, cov, k, d, V0, 1, taus, x0, refresher, goldschmidt, pack)
        cov = ctx.eigen_shift(cov, k, d, lam, V, VT, axis, refresher)
        ctx.sync()
        out.append((lam, V, VT, axis))
        if on_component is not None:
            on_component(m, time.perf_counter() - t0)
    return out, refresher.count


def fp64_replay(cov, l_e, l_p, seed=0, B2=2.0 ** 16):
    """Client-side reference: the same PowerMethod rounds, Newton counts,
    start vectors and eigen-shifts as pppca, in FP64 on the plaintext
    covariance.  Returns the eigenvalues and the (unit-length) vectors."""
    taus = lazy_schedule(l_p, B2=B2)
    x0 = taylor_point(B2)
    g = np.random.default_rng(seed)
    shifted = np.array(cov, dtype=np.float64)
    lams, vecs = [], []
    for _ in range(l_e):
        v = g.standard_normal(shifted.shape[0])
        v /= np.linalg.norm(v)
        for tau in taus:
            y = shifted @ v
            x = float(y @ y)
            s = 1.5 * x0 ** -0.5 - 0.5 * x0 ** -1.5 * x
            for _ in range(tau):
                s = s * (1.5 + (-0.5 * x) * (s * s))
            v = y * s
        lam = float((shifted @ v) @ v)
        shifted = shifted - lam * np.outer(v, v)
        lams.append(lam)
        vecs.append(v)
    return np.array(lams), np.stack(vecs, axis=1)


# Accuracy metrics of section 7.2 (client side, on decrypted results)
def r2_score(y_true, y_pred):
    """Coefficient of determination of every column, 1 - (residual sum of
    squares) / (sum of squares about the column's mean), averaged over the
    columns with equal weights"""
    y_true = np.asarray(y_true, dtype=np.float64)
    y_pred = np.asarray(y_pred, dtype=np.float64)
    if y_true.ndim == 1:
        y_true, y_pred = y_true[:, None], y_pred[:, None]
    ss_res = np.sum((y_true - y_pred) ** 2, axis=0)
    ss_tot = np.sum((y_true - y_true.mean(axis=0)) ** 2, axis=0)
    return float(np.mean(1.0 - ss_res / ss_tot))


def r2_x(X, V):
    """R2(X): the dataset against its reconstruction from the components
    (columns of V, used as they are): mu + (X - mu) V V^T"""
    X = np.asarray(X, dtype=np.float64)
    mu = X.mean(axis=0, keepdims=True)
    return r2_score(X, mu + (X - mu) @ V @ V.T)


def r2_v(U, V):
    """R2(V): computed components (columns of V) against reference
    eigenvectors (columns of U), each computed vector first given the sign of
    its reference (an eigenvector is defined up to sign)"""
    U = np.asarray(U, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    sign = np.where(np.sum(U * V, axis=0) < 0, -1.0, 1.0)
    return r2_score(U, V * sign)


# Synthetic stand-ins for the accuracy table's rows (section 7.2): 16 x 16
# pixel-like features in [0, 1] (t = 256) with a planted spectrum; s samples,
# l_E components, l_P normalising rounds.
ACCURACY_CASES = [("s200_lE4_lP4", 200, 4, 4), ("s200_lE4_lP14", 200, 4, 14), ("s165_lE6_lP14", 165, 6, 14)]


def accuracy_bench(cases=None, seed=7, log=print, ctx=None):
    """The whole PPPCA pipeline from a raw (uncentred) dataset: homomorphic
    means and covariance (HE_COV_UNCENTRED), then PowerMethod and EigenShift;
    R2(X) and R2(V) of the decrypted components against numpy's eigenvectors
    of the FP64 covariance, beside the same metrics for the FP64 replay of the
    same algorithm and for exact PCA (the R2(X) ceiling)."""
    from . import inputs as I
    cases = ACCURACY_CASES if cases is None else cases
    n, k, t = 128, 2, 256
    own = ctx is None
    if own:
        ctx = he.chain_context(I.LARGE, seed=seed)
        steps = set(ctx.matmul_rot_steps(n)) | set(ctx.transpose_rot_steps(n)) | set(he.power_rot_steps(n))
        ctx.keygen(sorted(steps))
    rows = []
    for ci, (name, s, l_e, l_p) in enumerate(cases):
        X = I.pca_dataset(seed + ci, s, t)
        rb = -(-s // n)
        blk = packing.blocks(X, n)
        cts = [ctx.encrypt_matrix(blk[r, c], nonce=(ci << 20) + r * k + c) for r in range(rb) for c in range(k)]
        ctx.sync()
        t0 = time.perf_counter()
        cov_ct = ctx.covariance(cts, rb, k, n, s, {"flags": 2 | 4 | 16})   # lazy relin, one rounding, uncentred
        ctx.sync()
        t_cov = time.perf_counter() - t0
        t0 = time.perf_counter()
        res, refreshes = pppca(ctx, cov_ct, k, n, l_e, l_p, seed=seed + ci, nonce0=(1 << 40) + (ci << 32),
                               start_nonce=(1 << 50) + (ci << 32))
        t_pca = time.perf_counter() - t0
        V = np.stack([read_vector(ctx, Vc, n, axis) for _, Vc, _, axis in res], axis=1)
        lam = np.array([float(ctx.decrypt(l, 4)[0]) for l, _, _, _ in res])
        cov = np.cov(X, rowvar=False, bias=True)
        w, U = np.linalg.eigh(cov)
        w, U = w[::-1][:l_e], U[:, ::-1][:, :l_e]
        lam_r, V_r = fp64_replay(cov, l_e, l_p, seed=seed + ci)
        taus = lazy_schedule(l_p)
        row = {"case": name, "s": s, "t": t, "l_E": l_e, "l_P": l_p, "l_N": round(float(np.mean(taus)), 2),
               "covariance_s": round(t_cov, 3), "pca_s": round(t_pca, 3), "refreshes": refreshes,
               "r2_x": round(r2_x(X, V), 4), "r2_v": round(r2_v(U, V), 4),
               "r2_x_fp64_replay": round(r2_x(X, V_r), 4), "r2_v_fp64_replay": round(r2_v(U, V_r), 4),
               "r2_x_exact_pca": round(r2_x(X, U), 4),
               "max_abs_err_vs_replay": float(np.max(np.abs(V - V_r))),
               "eigenvalue_rel_err_vs_eigh": [round(float(x), 6) for x in np.abs(lam - w) / w]}
        rows.append(row)
        if log:
            log(f"[accuracy] {row}")
        del res, cov_ct, cts
    if own:
        ctx.close()
    return {"workload": "PPPCA from raw synthetic [0,1] data (t = 256 features, planted spectrum) at N=2^16: "
                        "homomorphic means and covariance, PowerMethod + EigenShift; R2 against numpy's eigenvectors",
            "rows": rows}


def covariance_bench(s=60000, t=256, seed=13, stacked=(4, 8), log=print, n1=64):
    """The serving workload's large covariance job on its own: an s x t
    uniform[0,1] dataset, centred by the client, encrypted as ceil(s/128) x
    ceil(t/128) blocks of 128 x 128 at N = 2^16; X^T X / s accumulated
    homomorphically over the row blocks (lazy relinearisation, one rounding
    for ModDown and Rescale), with `stacked` row blocks per batch in turn
    (the "cov_row_blocks" knob).  Reports the client's encryption time, each
    covariance's time and device peak, and the largest error of the
    decrypted blocks against FP64.  n1: baby steps of Z and T and the shift
    blocks of the products (0: the library's default)."""
    from . import inputs as I
    n = 128
    k, rb = -(-t // n), -(-s // n)
    geo = {"n1_z": n1, "n1_t": n1} if n1 else {}
    ctx = he.chain_context(I.LARGE, seed=seed)
    ctx.keygen(sorted(set(ctx.matmul_rot_steps(n, dict(geo) or None)) | set(ctx.transpose_rot_steps(n))))
    X = I.centre(I.dataset(seed, s, t))
    blk = packing.blocks(X, n)
    t0 = time.perf_counter()
    cts = [ctx.encrypt_matrix(blk[r, c], nonce=(1 << 30) + r * k + c) for r in range(rb) for c in range(k)]
    ctx.sync()
    t_enc = time.perf_counter() - t0
    del blk
    P = np.zeros((rb * n, k * n))
    P[:s, :t] = X
    ref = P.T @ P / s
    old = he.knob_get("cov_row_blocks")
    runs = []
    try:
        for g in stacked:
            he.knob_set("cov_row_blocks", g)
            ctx.trim()
            live0, _, _ = ctx.mem_info()
            t0 = time.perf_counter()
            cov = ctx.covariance(cts, rb, k, n, s, {"flags": 2 | 4, **geo})
            ctx.sync()
            t_cov = time.perf_counter() - t0
            _, _, peak = ctx.mem_info()
            err = 0.0
            for i, c in enumerate(cov):
                a, b = divmod(i, k)
                got = ctx.decrypt(c, n * n).reshape(n, n)
                err = max(err, float(np.max(np.abs(got - ref[a * n:(a + 1) * n, b * n:(b + 1) * n]))))
            run = {"row_blocks_per_batch": g, "n1": n1 or None, "covariance_s": round(t_cov, 2),
                   "products_per_s": round(rb * k * (k + 1) / 2 / t_cov, 2),
                   "device_peak_gib": round((peak - live0) / 2**30, 1), "max_abs_err": err}
            runs.append(run)
            if log:
                log(f"[covariance] {run}")
            del cov
    finally:
        he.knob_set("cov_row_blocks", old)
    ctx.close()
    return {"workload": f"covariance of a {s}x{t} uniform[0,1] dataset (centred by the client) at N=2^16: {rb} row "
                        f"blocks x {k} feature blocks of 128 x 128 = {rb * k} ciphertexts, "
                        f"{rb * k * (k + 1) // 2} block products",
            "encrypt_s": round(t_enc, 2), "input_gib": round(rb * k * 2 * 31 * (1 << 16) * 8 / 2**30, 1),
            "runs": runs}


def pca_bench(l_e=8, l_p=14, seed=3, log=print, goldschmidt=False, pack=False):
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
    blk = packing.blocks(X, n)
    cts = [ctx.encrypt_matrix(blk[r, c], nonce=10 + r * k + c) for r in range(rb) for c in range(k)]
    ctx.sync()
    # the first call also finds and encodes the transforms' diagonals (then
    # cached by the context) and loads the kernels; the second is timed warm
    times = []
    for _ in range(2):
        t0 = time.perf_counter()
        cov_ct = ctx.covariance(cts, rb, k, n, X.shape[0])
        ctx.sync()
        times.append(time.perf_counter() - t0)
    t_cov_cold, t_cov = times
    comp_s = []
    t0 = time.perf_counter()
    res, refreshes = pppca(ctx, cov_ct, k, n, l_e, l_p, seed=seed, goldschmidt=goldschmidt, pack=pack,
                           on_component=lambda m, s: (comp_s.append(s), log(f"[pca] component {m}: {s:.2f} s")))
    t_pca = time.perf_counter() - t0
    # client side: decrypt, FP64 replay of the same rounds, eigh
    cov = X.T @ X / X.shape[0]
    taus = lazy_schedule(l_p)
    lam_r, V_r = fp64_replay(cov, l_e, l_p, seed=seed)
    err_v, err_l, eig_l, eig_cos = 0.0, 0.0, [], []
    w, U = np.linalg.eigh(cov)
    w, U = w[::-1], U[:, ::-1]
    for m, (lam, V, VT, axis) in enumerate(res):
        v, lf = V_r[:, m], float(lam_r[m])
        got_v = read_vector(ctx, V, n, axis)
        got_l = float(ctx.decrypt(lam, 4)[0])
        err_v = max(err_v, float(np.max(np.abs(got_v - v))))
        err_l = max(err_l, abs(got_l - lf) / max(1.0, abs(lf)))
        eig_l.append(abs(got_l - w[m]) / w[m])
        eig_cos.append(abs(float(got_v @ U[:, m])) / float(np.linalg.norm(got_v)))
    del res, cov_ct, cts
    ctx.close()
    return {
        "workload": f"PCA of a 256x256 [0,1] dataset with planted spectrum at N=2^16: covariance (2x2 blocks of "
                    f"128), {l_e} components x ({l_p} + 1) power rounds, Lazy Normalization schedule {taus}, "
                    f"inverse square root by {'Goldschmidt' if goldschmidt else 'Newton'}"
                    f"{', low vectors refreshed packed' if pack else ''}",
        "covariance_s": round(t_cov, 3),
        "covariance_cold_s": round(t_cov_cold, 3),
        "pca_s": round(t_pca, 3),
        "s_per_component": [round(x, 3) for x in comp_s],
        "power_rounds_per_s": round(l_e * (l_p + 1) / t_pca, 3),
        "refreshes": refreshes,
        "max_abs_err_vs_fp64_replay": {"eigenvector": err_v, "eigenvalue_rel": err_l},
        "vs_eigh": {"eigenvalue_rel_err": [round(x, 6) for x in eig_l],
                    "abs_cos_to_eigenvector": [round(x, 6) for x in eig_cos],
                    "top_eigenvalues": [round(float(x), 4) for x in w[:l_e]]},
    }
