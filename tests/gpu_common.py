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


def detected_scores(rec, mats, gm=0):
    """Score-function weights of each detected photon (zero for the others):
    (L/L_a^2, L/L_R^2 - N_sca/L_R, sum 1/R, sum 1/T) with the tables in FP32."""
    # the tables reach the kernel in FP32
    L_a = float(np.float32(mats[gm].abs_length))
    L_r = float(np.float32(mats[gm].rayleigh_length))
    det = (rec["flag"] & 0xFF) == 1
    s = np.zeros((len(rec), 4))
    L = rec["path_len"].astype(np.float64)
    s[:, 0] = L / L_a ** 2
    s[:, 1] = L / L_r ** 2 - rec["n_scatter"].astype(np.float64) / L_r
    s[:, 2] = rec["sum_inv_r"].astype(np.float64)
    s[:, 3] = rec["sum_inv_t"].astype(np.float64)
    return s * det[:, None]
