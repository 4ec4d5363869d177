"""Tolerance scales for barrier parity at large sizes (test helper)."""
import numpy as np

import oracle


def abs_scale(S, x, pt, ee, P, keys):
    """Summation-order-invariant tolerance scales (vectorised form of the
    per-pair loop in the small-scene parity tests, for states with
    hundreds of thousands of active pairs): gradients per entry
    sum_pairs |J|^T |g_loc|; Hessian blocks per entry sum_pairs
    |H_pair|_max (|J_k|^T 1 |J_l|).  With J_k = [I | I (x) xbar_k^T],
    |J_k|^T 1 |J_l| = c_k c_l^T where c_k = (1,1,1, |xbar_k|, |xbar_k|,
    |xbar_k|), so per (pair, k, l) only the 4x4 outer product of
    u_k = (1, |xbar_k|) is summed and expanded at the end."""
    r = oracle.barrier(S, x, pt, ee, P, keys, project=True, local=True)
    ru = oracle.barrier(S, x, pt, ee, P, keys, project=False, local=True)
    nb = len(S["body_fixed"])
    fixed = S["body_fixed"] != 0
    kcode = keys[:, 0].astype(np.int64) * (1 << 32) + keys[:, 1].astype(np.int64)
    nblk = nb + len(keys)
    gs_cols = np.zeros((nb, 12))
    W = np.zeros((nblk, 16))
    for name, pairs in (("pt", pt), ("ee", ee)):
        if len(pairs) == 0:
            continue
        lg, lH = r["local"][name]
        _, lHu = ru["local"][name]
        act = np.any(lHu != 0.0, axis=1)
        if not act.any():
            continue
        pairs = np.asarray(pairs)[act]
        lg, lH, lHu = lg[act], lH[act], lHu[act]
        if name == "pt":
            vid = np.concatenate([pairs[:, :1], S["tris"][pairs[:, 1]]], 1)
        else:
            vid = np.concatenate([S["edges"][pairs[:, 0]], S["edges"][pairs[:, 1]]], 1)
        bod = S["vert_body"][vid]                       # (n, 4)
        hmax = np.maximum(np.abs(lHu).max(1), np.abs(lH).max(1))
        u = np.concatenate([np.ones(vid.shape + (1,)), np.abs(S["xbar"][vid])], 2)   # (n, 4, 4)
        ag = np.abs(lg).reshape(-1, 4, 3)               # (n, 4, 3)
        for k in range(4):
            bk = bod[:, k]
            ok = ~fixed[bk]
            # |J_k|^T |g_k|: p_i -> |g_i|; a_ij -> |g_i| |xbar_j|
            contrib = np.concatenate([ag[:, k, :], (ag[:, k, :, None] * u[:, k, None, 1:]).reshape(-1, 9)], 1)
            for c in range(12):
                gs_cols[:, c] += np.bincount(bk[ok], weights=contrib[ok, c], minlength=nb)
            for l in range(4):
                bl = bod[:, l]
                okl = ok & ~fixed[bl]
                same = okl & (bk == bl)
                up = okl & (bk < bl)
                blk = np.full(len(bk), -1, np.int64)
                blk[same] = bk[same]
                if up.any():
                    code = bk[up].astype(np.int64) * (1 << 32) + bl[up].astype(np.int64)
                    pos = np.searchsorted(kcode, code)
                    assert np.all(kcode[pos] == code)
                    blk[up] = nb + pos
                sel = blk >= 0
                val = hmax[sel, None, None] * u[sel, k, :, None] * u[sel, l, None, :]
                val = val.reshape(-1, 16)
                for c in range(16):
                    W[:, c] += np.bincount(blk[sel], weights=val[:, c], minlength=nblk)
    m = np.array([0, 0, 0] + [1 + j for i in range(3) for j in range(3)])
    full = W.reshape(nblk, 4, 4)[:, m][:, :, m].reshape(nblk, 144)
    return r, gs_cols, full[:nb], full[nb:]
