"""Shared helpers of the GPU parity tests: device transfer and band-aware flag comparison."""
import sys

import numpy as np

BAND = 1e-4          # near-contact band: |oracle minimum clearance| <= 1e-4 m
CENTRE_TOL = 1e-5    # sphere-centre tolerance (Euclidean, metres)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda")


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def state_mismatches(gpu_flags, cmin):
    """(mismatches outside the band, near-contact count).  A NaN clearance (non-finite input)
    is a definite collision."""
    gpu = np.asarray(gpu_flags).astype(bool)
    nan = np.isnan(cmin)
    truth = nan | (cmin < 0.0)
    definite = nan | (np.abs(cmin) > BAND)
    bad = definite & (gpu != truth)
    return int(bad.sum()), int((~definite).sum())


def edge_mismatches(gpu_flags, cls):
    """Edge classes from the oracle: 0 clearly free, 1 clearly colliding, 2 near contact."""
    gpu = np.asarray(gpu_flags).astype(np.int64)
    bad = ((cls == 0) & (gpu != 0)) | ((cls == 1) & (gpu != 1))
    return int(bad.sum()), int((cls == 2).sum())


def knn_against_exact(x, gidx, gd2, k, rows=None):
    """Compare GPU k-nearest lists (gidx, gd2 for the queried rows) with the FP64 definition
    (oracle.roadmap.knn_exact).  Every listed FP32 distance must lie within the FP32 rounding
    bound of the exact distance of the listed sample; a list position whose exact distance is
    separated from its neighbours in the exact order by more than that bound must hold the
    exact neighbour; a near-tie position must hold a sample whose exact distance is within
    twice the bound of the exact one there; when the k-th and (k+1)-th exact distances are
    separated the sets are equal.  Returns (rows checked, rows with a near tie)."""
    from oracle import roadmap
    x = np.asarray(x, np.float32)
    n, dim = x.shape
    q = np.arange(n) if rows is None else np.asarray(rows)
    ridx, rd2, rnext = roadmap.knn_exact(x, k, rows=q)
    g = roadmap.fp32_rel_bound(dim)
    floor = 1e-37 * dim                      # FP32 underflow of tiny squared differences
    near_rows = 0
    for r, i in enumerate(q):
        S = np.concatenate([rd2[r], [rnext[r]]])
        gi, gd = np.asarray(gidx[r]), np.asarray(gd2[r], np.float64)
        have = int((ridx[r] >= 0).sum())
        assert np.all(gi[have:] == -1) and np.all(np.isinf(gd[have:])), (i, gi, ridx[r])
        assert np.all(gi[:have] >= 0) and np.all(gi[:have] < n), (i, gi)
        assert len(set(gi[:have].tolist())) == have and i not in gi[:have], (i, gi)
        s_g = roadmap.dist2_exact(x[i:i + 1], x[gi[:have]])[0]
        assert np.all(np.abs(gd[:have] - s_g) <= g * s_g + floor), (i, gd[:have], s_g)
        tie = False
        for m in range(have):
            lo_ok = m == 0 or S[m] - S[m - 1] > g * (S[m] + S[m - 1]) + floor
            hi_ok = not np.isfinite(S[m + 1]) or S[m + 1] - S[m] > g * (S[m + 1] + S[m]) + floor
            if lo_ok and hi_ok:
                assert gi[m] == ridx[r, m], (i, m, gi, ridx[r])
            else:
                tie = True
                assert abs(s_g[m] - S[m]) <= 2 * g * max(s_g[m], S[m]) + floor, (i, m)
        if have == k and (not np.isfinite(S[k]) or S[k] - S[k - 1] > g * (S[k] + S[k - 1]) + floor):
            assert set(gi.tolist()) == set(ridx[r].tolist()), (i, gi, ridx[r])
        near_rows += tie
    return len(q), near_rows


def nearest_against_exact(target, cands, got):
    """GPU nearest-node index `got` among rows of cands [m][d] for one target, against the FP64
    definition: the exact argmin when its gap to the second-nearest exceeds the FP32 rounding
    bound, else a node within twice the bound of the exact minimum.  Returns True at a near tie."""
    from oracle import roadmap
    s = roadmap.dist2_exact(np.asarray(target, np.float32)[None, :], cands)[0]
    g = roadmap.fp32_rel_bound(cands.shape[1])
    order = np.lexsort((np.arange(len(s)), s))
    best = s[order[0]]
    second = s[order[1]] if len(s) > 1 else np.inf
    if not np.isfinite(second) or second - best > g * (second + best):
        assert got == order[0], (got, order[0])
        return False
    assert abs(s[got] - best) <= 2 * g * max(s[got], best), (got, s[got], best)
    return True
