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
