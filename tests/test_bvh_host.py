"""The host BVH builder, inspected without a device (xp_bvh_build_host).

The transport kernels trust the structure in three ways: every point of every
triangle lies inside the box of some leaf that references it (also after
reference splitting cut long triangles into pieces), the leaf ranges and the
three rotated record copies are consistent, and the host's worst-case stack
bound covers the traversal the kernel runs.  These tests check each on meshes
with long fan wedges (the shape the splitting targets): the first two
directly, the last by running the kernel's traversal order (the nearest child hit is
followed, or held if it is a leaf, and the other hits are pushed) in Python
over random rays, and comparing its closest hits with a brute-force FP64
intersection of every triangle.
"""
import numpy as np
import pytest

from paper_2203_14354_amd import _lib
from paper_2203_14354_amd import runtime as R
from paper_2203_14354_amd import workloads as W


def fan_drum(n_seg=96, radius=1.0, height=0.6):
    """A closed drum: two end disks triangulated as fans from their centres
    (n_seg wedges each, every wedge as long as the radius) and a side wall of
    n_seg quads."""
    a = 2 * np.pi * np.arange(n_seg) / n_seg
    ring = np.stack([radius * np.cos(a), radius * np.sin(a)], 1)
    v = np.concatenate([np.c_[ring, np.zeros(n_seg)], np.c_[ring, np.full(n_seg, height)],
                        [[0, 0, 0], [0, 0, height]]]).astype(np.float32)
    i = np.arange(n_seg)
    j = (i + 1) % n_seg
    c0, c1 = 2 * n_seg, 2 * n_seg + 1
    bottom = np.stack([np.full(n_seg, c0), j, i], 1)
    top = np.stack([np.full(n_seg, c1), n_seg + i, n_seg + j], 1)
    wall = np.concatenate([np.stack([i, j, n_seg + j], 1), np.stack([i, n_seg + j, n_seg + i], 1)])
    return v, np.concatenate([bottom, top, wall]).astype(np.int32)


MESHES = {
    "fan_drum": fan_drum,
    "tpc1_plane": lambda: (W.tpc1(plane=True).vertices, W.tpc1(plane=True).triangles),
}


def leaf_boxes(nodes, n_refs):
    """Box (lo[3], hi[3]) of the leaf holding each reference, and how many
    leaves hold it."""
    lo = np.full((n_refs, 3), np.nan)
    hi = np.full((n_refs, 3), np.nan)
    held = np.zeros(n_refs, dtype=np.int64)
    for k in range(4):
        ch = nodes["child"][:, k]
        leaf = (ch < 0) & (ch != _lib.EMPTY_CHILD)
        e = ~ch[leaf]
        first, count = e >> 3, (e & 7) + 1
        box_lo = np.stack([nodes["lo_x"][leaf, k], nodes["lo_y"][leaf, k], nodes["lo_z"][leaf, k]], 1)
        box_hi = np.stack([nodes["hi_x"][leaf, k], nodes["hi_y"][leaf, k], nodes["hi_z"][leaf, k]], 1)
        for f, c, bl, bh in zip(first, count, box_lo, box_hi):
            lo[f:f + c] = bl
            hi[f:f + c] = bh
            held[f:f + c] += 1
    return lo, hi, held


def default_budget(nt):
    """The builder's default split budget: extra references up to 2 % of the
    triangles, at least 2,048 pieces, at most 4 per triangle."""
    return min(4.0, max(0.02, 2048.0 / nt))


@pytest.fixture(scope="module", params=[("fan_drum", 0.0), ("fan_drum", 1.0), ("fan_drum", -1.0),
                                        ("tpc1_plane", 0.0), ("tpc1_plane", 0.5)],
                ids=lambda p: f"{p[0]}-split{p[1]}")
def built(request):
    name, split = request.param
    v, t = MESHES[name]()
    info, nodes, recs = R.bvh_build_host(v, t, split_budget=split)
    return dict(v=np.asarray(v, np.float32), t=np.asarray(t, np.int32), split=split, info=info,
                nodes=nodes, recs=recs)


def test_sizes_and_reference_budget(built):
    info, nt = built["info"], len(built["t"])
    n_refs = info["n_references"]
    assert info["n_triangles"] == nt
    assert len(built["nodes"]) == info["n_nodes"] and info["node_bytes"] == 128 * info["n_nodes"]
    assert len(built["recs"]) == 3 * n_refs and info["triangle_bytes"] == 3 * 48 * n_refs
    budget = default_budget(nt) if built["split"] == 0.0 else max(built["split"], 0.0)
    assert nt <= n_refs <= nt + int(budget * nt) + 1
    if built["split"] < 0:
        assert n_refs == nt
    else:  # the fan wedges waste most of their boxes: the budget is used
        assert n_refs > nt


def test_leaves_and_records_are_consistent(built):
    info, recs, v, t = built["info"], built["recs"], built["v"], built["t"]
    n = info["n_references"]
    lo, hi, held = leaf_boxes(built["nodes"], n)
    assert np.all(held == 1)  # every record sits in exactly one leaf
    assert np.all(built["nodes"]["reserved"] == 0)
    # empty slots hold inverted boxes, which every slab test misses
    empty = built["nodes"]["child"] == _lib.EMPTY_CHILD
    for ax in "xyz":
        assert np.all(np.isposinf(built["nodes"]["lo_" + ax][empty]))
        assert np.all(np.isneginf(built["nodes"]["hi_" + ax][empty]))
        assert np.all(built["nodes"]["lo_" + ax][~empty] <= built["nodes"]["hi_" + ax][~empty])
    inner = built["nodes"]["child"][built["nodes"]["child"] >= 0]
    assert inner.min() >= 1 and inner.max() < info["n_nodes"]
    assert len(np.unique(inner)) == len(inner) == info["n_nodes"] - 1  # a tree
    base = recs[:n]
    ids = base["tri"]
    assert ids.min() >= 0 and ids.max() < len(t)
    assert np.array_equal(np.unique(ids), np.arange(len(t)))  # every triangle referenced
    # copy 0 holds the mesh's own vertices in the mesh's order
    for key, col in (("v0", 0), ("v1", 1), ("v2", 2)):
        assert np.array_equal(base[key], v[t[ids, col]])
    assert np.all(base["packed"] == (0 | 0 << 8 | 0 << 16)) and np.all(base["sensor"] == -1)
    # copy c holds the coordinates rotated to (k + 1, k + 2, k), k = (c + 2) % 3
    for c in (1, 2):
        k = (c + 2) % 3
        cp = recs[c * n:(c + 1) * n]
        assert np.array_equal(cp["tri"], ids)
        for key in ("v0", "v1", "v2"):
            assert np.array_equal(cp[key], base[key][:, [(k + 1) % 3, (k + 2) % 3, k]])


def test_every_triangle_point_lies_in_a_referencing_leaf(built):
    """Coverage after splitting: vertices, edge midpoints and random interior
    points of every triangle (FP64) lie inside the box of at least one of the
    leaves that reference the triangle."""
    info, v, t = built["info"], built["v"].astype(np.float64), built["t"]
    n = info["n_references"]
    lo, hi, _ = leaf_boxes(built["nodes"], n)
    ids = built["recs"]["tri"][:n]
    order = np.argsort(ids, kind="stable")
    counts = np.bincount(ids, minlength=len(t))
    kmax = counts.max()
    starts = np.concatenate([[0], np.cumsum(counts)[:-1]])
    refs = np.full((len(t), kmax), -1)
    for q in range(kmax):
        has = counts > q
        refs[has, q] = order[starts[has] + q]
    rng = np.random.default_rng(1)
    bary = np.concatenate([np.eye(3), [[0.5, 0.5, 0], [0, 0.5, 0.5], [0.5, 0, 0.5]],
                           rng.dirichlet([1, 1, 1], size=24)])
    P = np.einsum("sk,tkd->tsd", bary, v[t])  # [tri, sample, 3]
    inside = np.zeros(P.shape[:2], dtype=bool)
    for q in range(kmax):
        r = refs[:, q]
        ok = r >= 0
        b_lo, b_hi = lo[np.maximum(r, 0)][:, None, :], hi[np.maximum(r, 0)][:, None, :]
        inside |= ok[:, None] & np.all((P >= b_lo) & (P <= b_hi), axis=2)
    assert inside.all(), np.argwhere(~inside)[:5]


# -- the kernel's traversal order, in Python ----------------------------------

def brute_closest(v, t, o, d):
    """FP64 closest hit of one ray over every triangle (Moller-Trumbore);
    ties to the lower index.  Returns (triangle, distance)."""
    a, b, c = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    e1, e2 = b - a, c - a
    p = np.cross(d, e2)
    det = np.einsum("ij,ij->i", e1, p)
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / det
        s = o - a
        u = np.einsum("ij,ij->i", s, p) * inv
        q = np.cross(s, e1)
        w = (q @ d) * inv
        dist = np.einsum("ij,ij->i", e2, q) * inv
    hit = (np.abs(det) > 1e-15) & (u >= 0) & (w >= 0) & (u + w <= 1) & (dist > 1e-9)
    if not hit.any():
        return -1, np.inf
    dist = np.where(hit, dist, np.inf)
    m = dist.min()
    return int(np.nonzero(dist == m)[0][0]), m


def traverse(nodes, recs, n_refs, v, t, o, d):
    """The kernel's node visits and stack use for one ray, with FP64 box and
    triangle tests.  Returns (closest triangle, the largest stack depth seen)."""
    with np.errstate(divide="ignore"):
        inv = np.where(d != 0, 1.0 / d, np.copysign(np.inf, d))
    best_t, best_tri = np.inf, -1
    stack, max_depth = [], 0
    node, leaf = 0, None
    ids = recs["tri"][:n_refs]
    while True:
        if leaf is not None:
            first, count = leaf
            for r in range(first, first + count):
                tri, dist = brute_closest(v, t[ids[r]:ids[r] + 1], o, d)
                if tri >= 0 and (dist < best_t or (dist == best_t and ids[r] < best_tri)):
                    best_t, best_tri = dist, int(ids[r])
            leaf = None
        if node is None:
            if not stack:
                break
            e = stack.pop()
            if e >= 0:
                node = e
            else:
                leaf = ((~e) >> 3, ((~e) & 7) + 1)
            continue
        nd = nodes[node]
        lo = np.stack([nd["lo_x"], nd["lo_y"], nd["lo_z"]], 1).astype(np.float64)
        hi = np.stack([nd["hi_x"], nd["hi_y"], nd["hi_z"]], 1).astype(np.float64)
        with np.errstate(invalid="ignore"):
            t0, t1 = (lo - o) * inv, (hi - o) * inv
        tn = np.nanmax(np.minimum(t0, t1), axis=1).clip(min=0.0)
        tf = np.minimum(np.nanmin(np.maximum(t0, t1), axis=1), best_t)
        key = [tn[k] if nd["child"][k] != _lib.EMPTY_CHILD and tn[k] <= tf[k] else np.inf
               for k in range(4)]
        ent = [int(nd["child"][k]) for k in range(4)]
        # the nearest hit (ties to the lower slot) is followed, or held if it is
        # a leaf; every other hit is pushed, slot 3 first
        j = int(np.argmin(key)) if min(key) != np.inf else -1
        node = None
        stack.extend(ent[k] for k in (3, 2, 1, 0) if k != j and key[k] != np.inf)
        if j >= 0:
            if ent[j] < 0:
                leaf = ((~ent[j]) >> 3, ((~ent[j]) & 7) + 1)
            else:
                node = ent[j]
        max_depth = max(max_depth, len(stack) + (1 if leaf is not None else 0))
    return best_tri, max_depth


@pytest.mark.parametrize("name,split", [("fan_drum", 1.0), ("tpc1_plane", 0.0)])
def test_traversal_matches_brute_force_within_the_stack_bound(name, split):
    v, t = MESHES[name]()
    v = np.asarray(v, np.float64)
    info, nodes, recs = R.bvh_build_host(v, t, split_budget=split)
    lo, hi = v.min(0), v.max(0)
    rng = np.random.default_rng(7)
    n = 300
    o = lo + (hi - lo) * rng.uniform(0.05, 0.95, size=(n, 3))
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    deepest = 0
    for i in range(n):
        tri, depth = traverse(nodes, recs, info["n_references"], v, t, o[i], d[i])
        ref, _ = brute_closest(v, t, o[i], d[i])
        assert tri == ref, (i, tri, ref)
        deepest = max(deepest, depth)
    assert deepest <= info["max_stack"]


def test_build_is_deterministic():
    v, t = fan_drum()
    a = R.bvh_build_host(v, t, split_budget=0.5)
    b = R.bvh_build_host(v, t, split_budget=0.5)
    assert a[1].tobytes() == b[1].tobytes() and a[2].tobytes() == b[2].tobytes()


def test_host_build_rejects_bad_input():
    v, t = fan_drum()
    bad_t = t.copy()
    bad_t[0, 0] = len(v)
    degenerate = t.copy()
    degenerate[0] = [0, 0, 1]
    nan_v = v.copy()
    nan_v[3, 1] = np.nan
    for vv, tt, kw in ((v, bad_t, {}), (v, degenerate, {}), (nan_v, t, {}),
                       (v, t, dict(split_budget=5.0)), (v, t, dict(split_budget=float("nan"))),
                       (v, t, dict(max_leaf_size=9)), (v, t, dict(sah_bins=2))):
        with pytest.raises(_lib.XpError):
            R.bvh_build_host(vv, tt, **kw)
    # buffers too small for the result
    import ctypes
    lib = _lib.load()
    info = _lib.BvhInfo()
    opts = _lib.BvhOptions(1, 32, 0.0)
    vv = np.ascontiguousarray(v, np.float32)
    tt = np.ascontiguousarray(t, np.int32)
    P = ctypes.c_void_p
    args = (vv.ctypes.data_as(P), len(vv), tt.ctypes.data_as(P), len(tt), ctypes.byref(opts),
            ctypes.byref(info))
    assert lib.xp_bvh_build_host(*args, None, 0, None, 0) == _lib.XP_OK
    small = np.zeros(info.n_nodes - 1, dtype=_lib.NODE_DTYPE)
    assert lib.xp_bvh_build_host(*args, small.ctypes.data_as(P), len(small), None, 0) != _lib.XP_OK


@pytest.mark.parametrize("split", [-1.0, 0.0, 1.0, 4.0])
def test_tiny_meshes(split):
    """One sliver triangle and two, at every budget: at most budget x n extra
    references, every point still covered, and the root of a one-leaf tree
    holds the leaf."""
    sliver = (np.array([[0, 0, 0], [3.0, 2.9, 0], [3.0, 3.0, 0.1]], np.float32),
              np.array([[0, 1, 2]], np.int32))
    pair = (np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [5, 5, 5]], np.float32),
            np.array([[0, 1, 2], [1, 3, 2]], np.int32))
    for v, t in (sliver, pair):
        info, nodes, recs = R.bvh_build_host(v, t, split_budget=split)
        nt, n = len(t), info["n_references"]
        budget = default_budget(nt) if split == 0.0 else max(split, 0.0)
        assert nt <= n <= nt + int(budget * nt)
        lo, hi, held = leaf_boxes(nodes, n)
        assert np.all(held == 1)
        ids = recs["tri"][:n]
        assert np.array_equal(np.unique(ids), np.arange(nt))
        rng = np.random.default_rng(0)
        for k in range(nt):
            P = rng.dirichlet([1, 1, 1], size=200) @ v[t[k]].astype(np.float64)
            mine = np.nonzero(ids == k)[0]
            ok = np.zeros(len(P), bool)
            for r in mine:
                ok |= np.all((P >= lo[r]) & (P <= hi[r]), axis=1)
            assert ok.all()


def test_split_depth_limit():
    """A single long sliver with a budget far beyond what it can use stops at
    the depth limit (at most 2^10 pieces) and stays covered."""
    v = np.array([[0, 0, 0], [100.0, 99.9, 0], [100.0, 100.0, 0.01]], np.float32)
    t = np.array([[0, 1, 2]], np.int32)
    info, nodes, recs = R.bvh_build_host(v, t, split_budget=4.0)
    assert info["n_references"] <= 5  # the budget: 4 x 1 triangle
    v2 = np.concatenate([v, v + np.float32(200)])
    t2 = np.array([[0, 1, 2], [3, 4, 5]], np.int32)
    info2, _, _ = R.bvh_build_host(v2, t2, split_budget=4.0)
    assert info2["n_references"] <= 2 + 8
    assert info2["max_stack"] >= info2["depth"]


def test_meshes_of_2_24_triangles_are_rejected():
    """The kernels address the three triangle-record copies by 32-bit byte
    offsets (record index x 48 by a 24-bit multiply), so the builder refuses
    2^24 triangles and stops reference splitting below 2^24 references."""
    v = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]], np.float32)
    t = np.zeros((1 << 24, 3), np.int32)
    t[:, 1], t[:, 2] = 1, 2
    with pytest.raises(_lib.XpError, match="2\\^24"):
        R.bvh_build_host(v, t)
    info, _, _ = R.bvh_build_host(v, t[:1000], split_budget=4.0)
    assert info["n_references"] < 1 << 24


def test_default_split_budget_scales_with_the_mesh():
    """The default budget adds at least 2,048 pieces on a small mesh (the
    4,256-triangle TPC with its plane: its fan wedges take them all) and 2 % of
    the triangles on a large one; an explicit budget overrides it."""
    v, t = MESHES["tpc1_plane"]()
    nt = len(t)
    info, _, _ = R.bvh_build_host(v, t)
    assert info["n_references"] == nt + 2048
    info, _, _ = R.bvh_build_host(v, t, split_budget=0.02)
    assert info["n_references"] == nt + int(0.02 * nt)
    big_v, big_t = MESHES["fan_drum"]()
    reps = max(1, 120_000 // len(big_t))  # ~1.2e5 triangles: 2 % is more than 2,048
    vv = np.concatenate([np.asarray(big_v, np.float32) + np.float32(3.0 * k) for k in range(reps)])
    tt = np.concatenate([np.asarray(big_t, np.int32) + k * len(big_v) for k in range(reps)])
    info, _, _ = R.bvh_build_host(vv, tt)
    assert len(tt) * 0.02 > 2048
    assert len(tt) < info["n_references"] <= len(tt) + int(0.02 * len(tt))
