"""Shared helpers of the GPU parity tests."""
import numpy as np

import oracle
from paper_2203_14354_amd._lib import RECORD_DTYPE


def agreement(gpu, orc):
    """Per-photon agreement: same terminal flag, final triangle, sensor and step count."""
    return ((gpu["flag"] == orc["flag"]) & (gpu["last_tri"] == orc["last_tri"]) &
            (gpu["steps"] == orc["steps"]) & (gpu["sensor"] == orc["sensor"]))


def chi2_ndf(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    m = (a + b) > 0
    return float(((a[m] - b[m]) ** 2 / (a[m] + b[m])).sum() / max(int(m.sum()), 1))


def hist_of_detected(rec, n_events, n_channels, channel=None):
    det = (rec["flag"] & 0xFF) == oracle.F_DETECT
    ch = rec["sensor"][det] if channel is None else channel[rec["sensor"][det]]
    cell = rec["event"][det].astype(np.int64) * n_channels + ch
    return np.bincount(cell, minlength=n_events * n_channels).reshape(n_events, n_channels)


def to_records(t):
    return t.cpu().numpy().view(RECORD_DTYPE).reshape(-1)
