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


def plane_wave_boundary(d, e, N, n1, n_sub, layers=(), lam_nm=174.8):
    """Reflected and transmitted plane waves of a linearly polarized plane wave
    meeting a planar stack, from Maxwell's boundary conditions alone: the
    tangential components of E and of H (proportional to kappa x E in
    non-magnetic media, kappa the refractive wave vector with
    kappa . kappa = n^2) are continuous at every interface.  The linear system
    of those conditions is solved numerically; no Fresnel or Airy formula is
    used.

    d: unit incident direction, e: incident field (unit, perpendicular to d),
    N: unit normal pointing back into the incident medium (real index n1);
    layers: (complex index, thickness in nm) of films from the top down, on a
    substrate of complex index n_sub.  Returns (d_r, E_r, d_t, E_t): the
    reflected direction and complex field (incident amplitude 1), and the
    substrate's (complex) refractive wave vector divided by |n_sub| and field
    at its top interface."""
    d, e, N = (np.asarray(x, dtype=np.float64) for x in (d, e, N))
    z = N / np.linalg.norm(N)
    dt = d - np.dot(d, z) * z
    if np.linalg.norm(dt) > 1e-12:
        x = dt / np.linalg.norm(dt)
    else:
        a = np.array([1.0, 0, 0]) if abs(z[0]) < 0.9 else np.array([0, 1.0, 0])
        x = np.cross(a, z)
        x /= np.linalg.norm(x)
    y = np.cross(z, x)
    F = np.stack([x, y, z])           # world -> frame rows
    df, ef = F @ d, F @ e
    beta = n1 * df[0]                 # conserved tangential wave number
    k0 = 2 * math.pi / lam_nm
    media = [complex(n1)] + [complex(n) for n, _ in layers] + [complex(n_sub)]
    thick = [0.0] + [float(t) for _, t in layers]
    zs = np.cumsum([0.0] + [-t for t in thick[1:]])  # interface heights z_0 = 0, z_1, ...
    qs = [np.sqrt(complex(n * n - beta * beta)) for n in media]  # principal branch
    L = len(layers)
    n_unk = 4 * (L + 1)
    yv = np.array([0, 1.0, 0], dtype=complex)

    def waves(j):
        """(kappa, unknown index of A or None, z_ref) of the waves of medium j."""
        up = np.array([beta, 0, qs[j]], dtype=complex)
        down = np.array([beta, 0, -qs[j]], dtype=complex)
        if j == 0:
            return [(down, None, 0.0), (up, 0, 0.0)]
        if j == L + 1:
            return [(down, 2 + 4 * L, zs[j - 1])]
        b = 2 + 4 * (j - 1)
        return [(down, b, zs[j - 1]), (up, b + 2, zs[j - 1])]

    M = np.zeros((n_unk, n_unk), dtype=complex)
    rhs = np.zeros(n_unk, dtype=complex)
    for m in range(L + 1):
        rows = slice(4 * m, 4 * m + 4)
        for j, sign in ((m, 1.0), (m + 1, -1.0)):
            for kap, idx, zref in waves(j):
                ph = np.exp(1j * k0 * kap[2] * (zs[m] - zref))
                if idx is None:  # the known incident wave
                    E = ef.astype(complex) * ph
                    H = np.cross(n1 * df.astype(complex), E)
                    rhs[rows] -= sign * np.array([E[0], E[1], H[0], H[1]])
                    continue
                for col, vec in ((idx, yv), (idx + 1, np.cross(yv, kap))):
                    E = vec * ph
                    H = np.cross(kap, E)
                    M[rows, col] += sign * np.array([E[0], E[1], H[0], H[1]])
    sol = np.linalg.solve(M, rhs)
    kr = np.array([beta, 0, qs[0]], dtype=complex)
    kt = np.array([beta, 0, -qs[-1]], dtype=complex)
    Er = sol[0] * yv + sol[1] * np.cross(yv, kr)
    Et = sol[2 + 4 * L] * yv + sol[3 + 4 * L] * np.cross(yv, kt)
    d_r = F.T @ (kr.real / np.linalg.norm(kr.real))
    return d_r, F.T @ Er, F.T @ (kt / abs(media[-1])), F.T @ Et


def poynting_z(kappa, E, N):
    """Normal component (along N) of the time-averaged energy flux of a plane
    wave, up to the constant common to all non-magnetic media: Re(E x conj(H))
    with H = kappa x E."""
    H = np.cross(kappa, E)
    return float(np.real(np.dot(np.cross(E, np.conj(H)), N)))
