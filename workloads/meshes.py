"""Triangle meshes for the synthetic scenes (float32 vertices, int32 indices).

Shapes follow the paper's workloads: an extracted triangle mesh of one object
(57k-2M triangles in the paper's mesh-size table), here a tessellated
sphere-like surface plus occluders, or a dense lattice inside a closed room.
"""

import numpy as np


def _icosahedron():
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = np.array([
        [-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
        [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
        [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)
    return v, f


def geodesic_sphere(freq):
    """Class-I geodesic sphere: each icosahedron face split into freq^2
    triangles, vertices projected to the unit sphere.  20*freq^2 triangles,
    outward (counter-clockwise) winding."""
    v0, f0 = _icosahedron()
    pts = []
    faces = []
    base = 0
    # per-face barycentric lattice; shared vertices are merged afterwards
    ij = [(i, j) for i in range(freq + 1) for j in range(freq + 1 - i)]
    index = {p: k for k, p in enumerate(ij)}
    ij = np.array(ij, dtype=np.float64)
    local_faces = []
    for i in range(freq):
        for j in range(freq - i):
            a = index[(i, j)]
            b = index[(i + 1, j)]
            c = index[(i, j + 1)]
            local_faces.append((a, b, c))
            if i + j + 1 < freq:
                d = index[(i + 1, j + 1)]
                local_faces.append((b, d, c))
    local_faces = np.array(local_faces, dtype=np.int64)
    for (ia, ib, ic) in f0:
        A, B, C = v0[ia], v0[ib], v0[ic]
        w1 = ij[:, 0:1] / freq
        w2 = ij[:, 1:2] / freq
        p = A * (1.0 - w1 - w2) + B * w1 + C * w2
        pts.append(p)
        faces.append(local_faces + base)
        base += p.shape[0]
    pts = np.concatenate(pts, axis=0)
    faces = np.concatenate(faces, axis=0)
    pts /= np.linalg.norm(pts, axis=1, keepdims=True)
    # merge duplicated edge/corner vertices
    key = np.round(pts * 1e9).astype(np.int64)
    _, first, inv = np.unique(key, axis=0, return_index=True, return_inverse=True)
    pts = pts[first]
    faces = inv.reshape(-1)[faces]
    # orient outward
    a, b, c = pts[faces[:, 0]], pts[faces[:, 1]], pts[faces[:, 2]]
    nrm = np.cross(b - a, c - a)
    flip = (nrm * (a + b + c)).sum(axis=1) < 0
    faces[flip] = faces[flip][:, ::-1]
    return pts, faces


def icosphere(level):
    """Loop-style icosphere: 20 * 4^level triangles on the unit sphere."""
    return geodesic_sphere(2 ** level)


def quad(p0, p1, p2, p3):
    """Two triangles for the planar quad p0-p1-p2-p3 (in order)."""
    v = np.array([p0, p1, p2, p3], dtype=np.float64)
    f = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int64)
    return v, f


def box(center, half, yaw=0.0):
    """Closed box (12 triangles), rotated by `yaw` about +Y."""
    hx, hy, hz = half
    c = np.array(center, dtype=np.float64)
    corners = np.array([[sx * hx, sy * hy, sz * hz]
                        for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)], dtype=np.float64)
    cy, sy = np.cos(yaw), np.sin(yaw)
    rot = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
    v = corners[:, 0, None] * rot.T[0] + corners[:, 1, None] * rot.T[1] + corners[:, 2, None] * rot.T[2] + c
    # corner index = 4*ix + 2*iy + iz
    f = np.array([
        [0, 1, 3], [0, 3, 2],   # -x
        [4, 6, 7], [4, 7, 5],   # +x
        [0, 4, 5], [0, 5, 1],   # -y
        [2, 3, 7], [2, 7, 6],   # +y
        [0, 2, 6], [0, 6, 4],   # -z
        [1, 5, 7], [1, 7, 3],   # +z
    ], dtype=np.int64)
    return v, f


def merge(parts):
    vs, fs, base = [], [], 0
    for v, f in parts:
        vs.append(np.asarray(v, dtype=np.float64))
        fs.append(np.asarray(f, dtype=np.int64) + base)
        base += len(v)
    return np.concatenate(vs, 0), np.concatenate(fs, 0)


def to_device_layout(v, f):
    return (np.ascontiguousarray(v, dtype=np.float32),
            np.ascontiguousarray(f, dtype=np.int32))


def wall_with_window(axis, sign, half, win_w, win_h, win_center_y=0.0):
    """A square wall of the room [-half, half]^3 on plane axis=sign*half, with a
    rectangular window (win_w wide, win_h tall) cut out; 8 triangles."""
    h = half
    ww, wh = win_w / 2.0, win_h / 2.0
    y0, y1 = win_center_y - wh, win_center_y + wh
    # coordinates along the wall: s (horizontal), y (vertical)
    rects = [(-h, h, y1, h), (-h, h, -h, y0), (-h, -ww, y0, y1), (ww, h, y0, y1)]
    parts = []
    for (s0, s1, ya, yb) in rects:
        def P(s, y):
            if axis == 0:
                return [sign * h, y, s]
            return [s, y, sign * h]
        parts.append(quad(P(s0, ya), P(s1, ya), P(s1, yb), P(s0, yb)))
    return merge(parts)
