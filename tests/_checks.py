"""Property checks written directly in numpy/scipy (independent of both the
oracle and the GPU library): triangulation validity, local Delaunay property,
Euler counts and brute-force overlap detection."""
import numpy as np
from scipy.spatial import ConvexHull, cKDTree


def orient(a, b, c):
    return (b[..., 0] - a[..., 0]) * (c[..., 1] - a[..., 1]) - (b[..., 1] - a[..., 1]) * (c[..., 0] - a[..., 0])


def incircle(a, b, c, d):
    ad, bd, cd = a - d, b - d, c - d
    al = (ad ** 2).sum(-1)
    bl = (bd ** 2).sum(-1)
    cl = (cd ** 2).sum(-1)
    return (al * (bd[..., 0] * cd[..., 1] - cd[..., 0] * bd[..., 1])
            - bl * (ad[..., 0] * cd[..., 1] - cd[..., 0] * ad[..., 1])
            + cl * (ad[..., 0] * bd[..., 1] - bd[..., 0] * ad[..., 1]))


def tri_set(tris):
    return {tuple(sorted(map(int, t))) for t in tris}


def check_delaunay(xy, tris):
    """Asserts: every triangle CCW, Euler count 2n-2-h, every interior edge locally Delaunay.
    Returns the largest in-circle value over interior edges (<= 0 for Delaunay)."""
    n = xy.shape[0]
    tris = np.asarray(tris, dtype=np.int64)
    P = xy[tris]
    assert np.all(orient(P[:, 0], P[:, 1], P[:, 2]) > 0), "non-positive triangle"
    h = len(ConvexHull(xy).vertices)
    assert len(tris) == 2 * n - 2 - h, (len(tris), 2 * n - 2 - h)
    a = np.concatenate([tris[:, 0], tris[:, 1], tris[:, 2]])
    b = np.concatenate([tris[:, 1], tris[:, 2], tris[:, 0]])
    c = np.concatenate([tris[:, 2], tris[:, 0], tris[:, 1]])
    key = np.minimum(a, b) * (n + 1) + np.maximum(a, b)
    order = np.argsort(key, kind="stable")
    ks = key[order]
    same = np.nonzero(ks[1:] == ks[:-1])[0]
    i1, i2 = order[same], order[same + 1]
    assert len(i1) == 3 * n - 3 - h - h, "interior edge count"
    # edge i1: a->b with opposite c; the other side has opposite c[i2]
    val = incircle(xy[a[i1]], xy[b[i1]], xy[c[i1]], xy[c[i2]])
    assert np.all(val <= 0), f"non-Delaunay edge, max in-circle {val.max()}"
    return float(val.max()) if len(val) else 0.0


def count_overlaps(xy, radius=1.0, tol=1e-9):
    pairs = cKDTree(xy).query_pairs(2 * radius * (1 - tol))
    return len(pairs)


def rel_err(a, b):
    """Largest |a - b| / max(|b|, 1) over all components (position metric)."""
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1.0)))
