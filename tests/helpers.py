"""Statistics and closed-form helpers for the tests (independent of the oracle
and of the HIP path: plain numpy / scipy)."""
import math

import numpy as np
from scipy import stats


def chi2_pvalue(observed, expected_prob):
    """Pearson chi-square p-value of a histogram against bin probabilities."""
    observed = np.asarray(observed, dtype=np.float64)
    p = np.asarray(expected_prob, dtype=np.float64)
    n = observed.sum()
    exp = n * p / p.sum()
    keep = exp > 0
    chi2 = float((((observed - exp) ** 2)[keep] / exp[keep]).sum())
    ndf = int(keep.sum()) - 1
    return float(stats.chi2.sf(chi2, ndf)), chi2 / max(ndf, 1)


def binom_sigma(p, n):
    return math.sqrt(max(p * (1 - p), 1e-300) / n)


def triangle_solid_angle(a, b, c):
    """Solid angle of triangles (a, b, c) seen from the origin (Van Oosterom and
    Strackee, IEEE Trans. Biomed. Eng. 1983).  Arrays (..., 3)."""
    la, lb, lc = (np.linalg.norm(x, axis=-1) for x in (a, b, c))
    num = np.abs(np.einsum("...i,...i->...", a, np.cross(b, c)))
    den = (la * lb * lc + np.einsum("...i,...i->...", a, b) * lc
           + np.einsum("...i,...i->...", a, c) * lb + np.einsum("...i,...i->...", b, c) * la)
    return 2.0 * np.arctan2(num, den)


def face_average(vertices, triangles, source, g, m=6):
    """(1/4 pi) * integral over the directions that hit the given faces of
    g(distance), by subdividing each face into m^2 sub-triangles, weighting each
    with its exact solid angle and evaluating g at its centroid."""
    v = np.asarray(vertices, dtype=np.float64) - np.asarray(source, dtype=np.float64)
    t = np.asarray(triangles)
    A, B, C = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    total = 0.0
    for i in range(m):
        for j in range(m - i):
            for up in (0, 1):
                if up == 0:
                    bary = [(i, j), (i + 1, j), (i, j + 1)]
                else:
                    if i + j + 2 > m:
                        continue
                    bary = [(i + 1, j), (i + 1, j + 1), (i, j + 1)]
                pts = []
                for (bi, bj) in bary:
                    wa, wb = bi / m, bj / m
                    pts.append(A * (1 - wa - wb) + B * wa + C * wb)
                om = triangle_solid_angle(*pts)
                cen = (pts[0] + pts[1] + pts[2]) / 3.0
                total += float((om * g(np.linalg.norm(cen, axis=1))).sum())
    return total / (4 * math.pi)


def fresnel_sine_tangent(theta_i, n1, n2):
    """Fresnel's reflection amplitudes in the sine/tangent form
    r_s = -sin(ti - tt)/sin(ti + tt), r_p = tan(ti - tt)/tan(ti + tt)
    (Hecht, Optics, ch. 4), for 0 < theta_i < critical angle.  Returns (R_s, R_p)."""
    st = n1 * math.sin(theta_i) / n2
    tt = math.asin(st)
    rs = -math.sin(theta_i - tt) / math.sin(theta_i + tt)
    rp = math.tan(theta_i - tt) / math.tan(theta_i + tt)
    return rs * rs, rp * rp


def closed_edges_ok(triangles, oriented=True):
    """True if every undirected edge of the triangle set is used exactly twice
    (a closed surface) and, if ``oriented``, each time in opposite directions
    (consistently oriented)."""
    t = np.asarray(triangles, dtype=np.int64)
    e = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]], 0)
    if not oriented:
        lo, hi = e.min(axis=1), e.max(axis=1)
        _, cnt = np.unique(lo * (1 << 32) + hi, return_counts=True)
        return bool(np.all(cnt == 2))
    key_dir = e[:, 0] * (1 << 32) + e[:, 1]
    key_rev = e[:, 1] * (1 << 32) + e[:, 0]
    if len(np.unique(key_dir)) != len(key_dir):
        return False
    return bool(np.isin(key_rev, key_dir).all())
