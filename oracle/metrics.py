"""Float64 reference of the surface evaluation (test infrastructure only, like
the rest of this package): the zero-level surface of a grid field, points
sampled uniformly on it, and the HD / CD / CS metrics of Section 4
(Evaluation Metric).

Readings (the paper's extraction method is an external one):
- the surface of a grid field is extracted by marching tetrahedra on the
  cell-centred grid: each cube of eight neighbouring points is split into six
  tetrahedra around its main diagonal (corner 0 to corner 7, corner c at
  offsets (c & 1, c >> 1 & 1, c >> 2)); a tetrahedron whose corners straddle
  the iso value gives one triangle (one corner apart) or two (two and two),
  with vertices interpolated linearly along the straddling edges (on the
  finite corner when the other corner's value is infinite); cubes in
  point order (x fastest), tetrahedra and triangles in a fixed order;
- the network's normalised output is taken back to a signed distance by
  inverting eq. 3-10 on its branch S >= m, and its surface is that field's
  zero set;
- points are sampled uniformly by area: a triangle chosen with probability
  proportional to its area (cumulative areas in float64),
  then a uniform point on it; the normal is the triangle's unit normal (the
  metric uses |cos|, so orientation does not matter);
- HD, CD and CS as printed, with closest points by Euclidean distance.
"""

import math

import numpy as np

# the six tetrahedra of a cube around the diagonal 0-7 (corner c: x = c & 1,
# y = c >> 1 & 1, z = c >> 2)
TETS = ((0, 1, 3, 7), (0, 3, 2, 7), (0, 2, 6, 7), (0, 6, 4, 7), (0, 4, 5, 7), (0, 5, 1, 7))


def sdf_from_targets(t: np.ndarray, m: float) -> np.ndarray:
    """Inverse of eq. 3-10 on the branch S >= m: S = m + sqrt(ln(2 / t) / h),
    h = ln 2 / m^2; t >= 2 gives m, t <= 0 gives +inf."""
    t = np.asarray(t, np.float64)
    h = math.log(2.0) / (m * m)
    with np.errstate(divide="ignore", invalid="ignore"):
        arg = np.where(t > 0.0, np.log(2.0 / np.where(t > 0.0, t, 1.0)), np.inf)
    return m + np.sqrt(np.maximum(arg, 0.0) / h)


def marching_tets(F: np.ndarray, axis: np.ndarray, iso: float = 0.0) -> np.ndarray:
    """Triangles (T, 3, 3) of the iso-surface of the grid field F (n^3, x
    fastest) on the cell-centred axis, in the fixed order described above.
    A corner is inside when F < iso."""
    a = np.asarray(axis, np.float64)
    n = a.size
    V = np.asarray(F, np.float64).reshape(n, n, n)          # [z, y, x]
    corners = [V[(c >> 2):n - 1 + (c >> 2), ((c >> 1) & 1):n - 1 + ((c >> 1) & 1), (c & 1):n - 1 + (c & 1)]
               for c in range(8)]
    inside = sum((cv < iso).astype(np.int64) for cv in corners)
    tris = []
    # straddling cubes in point order (z slowest, x fastest)
    for k, j, i in np.argwhere((inside > 0) & (inside < 8)):
        cv = [V[k + (c >> 2), j + ((c >> 1) & 1), i + (c & 1)] for c in range(8)]
        cp = [np.array([a[i + (c & 1)], a[j + ((c >> 1) & 1)], a[k + (c >> 2)]]) for c in range(8)]
        for tet in TETS:
            tris.extend(_tet_triangles([cp[c] for c in tet], [cv[c] for c in tet], iso))
    return np.array(tris, np.float64).reshape(-1, 3, 3)


def _edge(p, v, a, b, iso):
    # an infinite corner value (the inverse of eq. 3-10 where the network
    # gives t <= 0) is infinitely far outside: the vertex sits on the other
    # corner
    if math.isinf(v[b]):
        t = 0.0
    elif math.isinf(v[a]):
        t = 1.0
    else:
        t = (iso - v[a]) / (v[b] - v[a])
    return p[a] + t * (p[b] - p[a])


def _tet_triangles(p, v, iso):
    inside = [x < iso for x in v]
    ins = [q for q in range(4) if inside[q]]
    outs = [q for q in range(4) if not inside[q]]
    if len(ins) in (0, 4):
        return []
    if len(ins) == 1 or len(ins) == 3:
        lone, others = (ins[0], outs) if len(ins) == 1 else (outs[0], ins)
        return [[_edge(p, v, lone, others[0], iso), _edge(p, v, lone, others[1], iso),
                 _edge(p, v, lone, others[2], iso)]]
    a, b = ins
    c, d = outs
    # quad a-c, a-d, b-d, b-c split along a-c .. b-d
    e0, e1, e2, e3 = (_edge(p, v, a, c, iso), _edge(p, v, a, d, iso), _edge(p, v, b, d, iso),
                      _edge(p, v, b, c, iso))
    return [[e0, e1, e2], [e0, e2, e3]]


def triangle_areas(tris: np.ndarray) -> np.ndarray:
    T = np.asarray(tris, np.float64)
    cr = np.cross(T[:, 1] - T[:, 0], T[:, 2] - T[:, 0])
    return 0.5 * np.sqrt(np.sum(cr * cr, axis=1))


def sample_surface(tris: np.ndarray, u: np.ndarray):
    """Points uniform by area on the triangles, from uniform numbers u
    (S, 3) in [0, 1): u0 picks the triangle by cumulative area (the first
    whose running sum exceeds u0 times the total), u1, u2 place the point
    (1 - sqrt(u1)) A + sqrt(u1) (1 - u2) B + sqrt(u1) u2 C.  Returns points,
    unit normals and the triangle of each sample."""
    T = np.asarray(tris, np.float64)
    u = np.asarray(u, np.float64).reshape(-1, 3)
    csum = np.cumsum(triangle_areas(T))
    tri = np.searchsorted(csum, u[:, 0] * csum[-1], side="right")
    tri = np.minimum(tri, T.shape[0] - 1)
    r1 = np.sqrt(u[:, 1])[:, None]
    r2 = u[:, 2][:, None]
    A, B, C = T[tri, 0], T[tri, 1], T[tri, 2]
    pts = (1.0 - r1) * A + r1 * (1.0 - r2) * B + r1 * r2 * C
    nr = np.cross(B - A, C - A)
    nr /= np.linalg.norm(nr, axis=1, keepdims=True)
    return pts, nr, tri


def surface_metrics(Pt, Nt, Pr, Nr):
    """HD, CD and CS (Section 4) between point sets sampled on the ground-truth
    surface (Pt, normals Nt) and on the reconstructed one (Pr, Nr); closest
    points by a k-d tree."""
    from scipy.spatial import cKDTree
    Pt, Pr = np.asarray(Pt, np.float64), np.asarray(Pr, np.float64)
    Nt, Nr = np.asarray(Nt, np.float64), np.asarray(Nr, np.float64)
    d_tr, i_tr = cKDTree(Pr).query(Pt)
    d_rt, i_rt = cKDTree(Pt).query(Pr)
    hd = max(d_tr.max(), d_rt.max())
    cd = 0.5 * d_tr.mean() + 0.5 * d_rt.mean()
    cs = 0.5 * np.abs(np.sum(Nt * Nr[i_tr], axis=1)).mean() + 0.5 * np.abs(np.sum(Nr * Nt[i_rt], axis=1)).mean()
    return float(hd), float(cd), float(cs)
