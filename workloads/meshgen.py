"""Deterministic linear-tetrahedron mesh generators.

* ``cube_kuhn``  -- unit cube split into n^3 cubes of 6 Kuhn tetrahedra.
* ``pipe``       -- straight pipe: polar-ring disk triangulation extruded to
                    prisms, each prism cut into 3 tets with a diagonal rule
                    that keeps shared quad faces conforming.
* ``junction``   -- synthetic cross junction (two inlet tubes along z, two
                    outlet tubes along x) cut out of a voxel Kuhn grid.

All generators return positively oriented tets, with nodes and elements in
Morton order for memory locality.  Boundary faces are classified by a label
function.
"""
from __future__ import annotations

import dataclasses
import numpy as np


@dataclasses.dataclass
class Mesh:
    xyz: np.ndarray            # (n_nodes, 3) float64
    tets: np.ndarray           # (n_tets, 4) int32, positive orientation
    faces: dict                # label -> (nf, 3) int32 boundary triangles, outward (b-a)x(c-a)

    @property
    def n_nodes(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_tets(self) -> int:
        return int(self.tets.shape[0])


def _signed_vol(xyz, tets):
    a = xyz[tets[:, 0]]
    d1 = xyz[tets[:, 1]] - a
    d2 = xyz[tets[:, 2]] - a
    d3 = xyz[tets[:, 3]] - a
    return np.einsum("ij,ij->i", d1, np.cross(d2, d3)) / 6.0


def orient_positive(xyz, tets):
    tets = tets.copy()
    neg = _signed_vol(xyz, tets) < 0
    tets[neg, 2], tets[neg, 3] = tets[neg, 3].copy(), tets[neg, 2].copy()
    return tets


def _morton_key(p, bits=20):
    lo = p.min(axis=0)
    span = np.maximum(p.max(axis=0) - lo, 1e-300)
    q = np.clip(((p - lo) / span * ((1 << bits) - 1)).astype(np.int64), 0, (1 << bits) - 1)
    key = np.zeros(p.shape[0], dtype=np.int64)
    for b in range(bits):
        for d in range(3):
            key |= ((q[:, d] >> b) & 1) << (3 * b + d)
    return key


def morton_order_elements(xyz, tets):
    """Renumber nodes and elements along a Morton (Z-order) curve."""
    nkey = _morton_key(xyz)
    nperm = np.argsort(nkey, kind="stable")
    inv = np.empty_like(nperm)
    inv[nperm] = np.arange(nperm.size)
    xyz2 = xyz[nperm]
    tets2 = inv[tets]
    ekey = _morton_key(xyz2[tets2].mean(axis=1))
    eperm = np.argsort(ekey, kind="stable")
    return xyz2, tets2[eperm].astype(np.int32), inv


_LOCAL_FACES = np.array([[1, 2, 3], [0, 3, 2], [0, 1, 3], [0, 2, 1]])


def boundary_faces(xyz, tets):
    """Triangles that belong to exactly one tet, oriented outward."""
    f = tets[:, _LOCAL_FACES].reshape(-1, 3)
    key = np.sort(f, axis=1)
    _, idx, cnt = np.unique(key, axis=0, return_index=True, return_counts=True)
    bf = f[idx[cnt == 1]]
    # outward orientation: the opposite vertex must lie behind the face
    e = idx[cnt == 1] // 4
    loc = idx[cnt == 1] % 4
    opp = tets[e, loc]
    a, b, c = xyz[bf[:, 0]], xyz[bf[:, 1]], xyz[bf[:, 2]]
    nrm = np.cross(b - a, c - a)
    flip = np.einsum("ij,ij->i", nrm, xyz[opp] - a) > 0
    bf[flip, 1], bf[flip, 2] = bf[flip, 2].copy(), bf[flip, 1].copy()
    return bf.astype(np.int32)


def _finish(xyz, tets, label_fn):
    tets = orient_positive(xyz, tets)
    xyz, tets, _ = morton_order_elements(xyz, tets)
    bf = boundary_faces(xyz, tets)
    labels = label_fn(xyz[bf].mean(axis=1), xyz[bf])
    faces = {}
    for lab in np.unique(labels):
        faces[str(lab)] = bf[labels == lab]
    return Mesh(xyz=np.ascontiguousarray(xyz, dtype=np.float64),
                tets=np.ascontiguousarray(tets, dtype=np.int32), faces=faces)


# Kuhn subdivision of the unit cube: 6 tets along the main diagonal, one per
# permutation of the axes.  The same split in every cube keeps faces conforming.
_KUHN_PATHS = []
for perm in ([0, 1, 2], [0, 2, 1], [1, 0, 2], [1, 2, 0], [2, 0, 1], [2, 1, 0]):
    v = [0, 0, 0]
    path = [tuple(v)]
    for ax in perm:
        v = list(v)
        v[ax] = 1
        path.append(tuple(v))
    _KUHN_PATHS.append(path)


def _kuhn_grid(nx, ny, nz, keep_cell=None):
    """Tets of an nx*ny*nz cell grid, node (i,j,k) -> i + (nx+1)*(j + (ny+1)*k)."""
    ii, jj, kk = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ii, jj, kk = ii.ravel(), jj.ravel(), kk.ravel()
    if keep_cell is not None:
        m = keep_cell(ii, jj, kk)
        ii, jj, kk = ii[m], jj[m], kk[m]

    def nid(a, b, c):
        return a + (nx + 1) * (b + (ny + 1) * c)

    tets = []
    for path in _KUHN_PATHS:
        tets.append(np.stack([nid(ii + p[0], jj + p[1], kk + p[2]) for p in path], axis=1))
    return np.concatenate(tets, axis=0)


def cube_kuhn(n: int, length: float = 1.0) -> Mesh:
    """Unit cube [0,L]^3, 6 n^3 tets; all boundary faces labelled 'wall'."""
    g = np.linspace(0.0, length, n + 1)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    xyz = np.stack([X.ravel(order="F"), Y.ravel(order="F"), Z.ravel(order="F")], axis=1)
    tets = _kuhn_grid(n, n, n)
    return _finish(xyz, tets, lambda c, t: np.array(["wall"] * c.shape[0]))


def _disk(n_rings: int, radius: float):
    """Polar-ring disk: centre + ring r with 8r nodes; 8 n_rings^2 triangles."""
    pts = [(0.0, 0.0)]
    rings = [[0]]
    for r in range(1, n_rings + 1):
        m = 8 * r
        th = 2 * np.pi * np.arange(m) / m
        ids = list(range(len(pts), len(pts) + m))
        pts.extend(zip(radius * r / n_rings * np.cos(th), radius * r / n_rings * np.sin(th)))
        rings.append(ids)
    tris = []
    for r in range(1, n_rings + 1):
        outer = rings[r]
        if r == 1:
            for j in range(8):
                tris.append((0, outer[j], outer[(j + 1) % 8]))
            continue
        inner = rings[r - 1]
        mo, mi = len(outer), len(inner)
        # advancing merge of the two angle-sorted rings
        io = ii = 0
        while io < mo or ii < mi:
            ao = (io + 1) / mo
            ai = (ii + 1) / mi
            if ii >= mi or (io < mo and ao <= ai):
                tris.append((inner[ii % mi], outer[io % mo], outer[(io + 1) % mo]))
                io += 1
            else:
                tris.append((inner[ii % mi], outer[io % mo], inner[(ii + 1) % mi]))
                ii += 1
    return np.array(pts), np.array(tris, dtype=np.int64)


def pipe(n_rings: int = 4, n_layers: int = 16, radius: float = 1.0, length: float = 4.0) -> Mesh:
    """Pipe along +z from z=0 (label 'inlet') to z=length ('outlet'), wall 'wall'."""
    p2, tri = _disk(n_rings, radius)
    nd = p2.shape[0]
    z = np.linspace(0.0, length, n_layers + 1)
    xyz = np.concatenate([np.column_stack([p2, np.full(nd, zk)]) for zk in z])
    tets = []
    for layer in range(n_layers):
        t = np.sort(tri, axis=1)  # a < b < c by in-layer index
        a, b, c = t[:, 0] + layer * nd, t[:, 1] + layer * nd, t[:, 2] + layer * nd
        a1, b1, c1 = a + nd, b + nd, c + nd
        # quad (a,b) split a-b1, (b,c) split b-c1, (a,c) split a-c1
        tets.append(np.stack([a, b, c, c1], axis=1))
        tets.append(np.stack([a, b, b1, c1], axis=1))
        tets.append(np.stack([a, a1, b1, c1], axis=1))
    tets = np.concatenate(tets)

    def label(cen, tri_xyz):
        lab = np.array(["wall"] * cen.shape[0], dtype=object)
        zz = tri_xyz[:, :, 2]
        lab[np.all(np.abs(zz) < 1e-12, axis=1)] = "inlet"
        lab[np.all(np.abs(zz - length) < 1e-12, axis=1)] = "outlet"
        return lab.astype(str)

    return _finish(xyz, tets, label)


# Junction geometry: inlet tube 'in1' (radius r_in1) along z from z=-arm to 0,
# inlet tube 'in2' (radius r_in2) along z from 0 to +arm, outlet tube along x
# (radius r_out) from -arm to +arm; outlets 'out1' at x=-arm and 'out2' at x=+arm.
JUNCTION_DEFAULT = dict(r_in1=0.8, r_in2=0.6, r_out=0.5, arm=4.0)


def junction_inside(p, r_in1=0.8, r_in2=0.6, r_out=0.5, arm=4.0):
    x, y, z = p[:, 0], p[:, 1], p[:, 2]
    rz2 = x * x + y * y
    rx2 = y * y + z * z
    in1 = (z <= 0) & (z >= -arm) & (rz2 <= r_in1 ** 2)
    in2 = (z >= 0) & (z <= arm) & (rz2 <= r_in2 ** 2)
    out = (np.abs(x) <= arm) & (rx2 <= r_out ** 2)
    return in1 | in2 | out


def junction(h: float, r_in1=0.8, r_in2=0.6, r_out=0.5, arm=4.0) -> Mesh:
    """Voxel Kuhn grid of spacing ~h; tets whose centroid lies in the tubes."""
    ncell = int(round(2 * arm / h))
    hh = 2 * arm / ncell
    rmax = max(r_in1, r_in2, r_out)
    jy0 = int(np.floor((arm - rmax) / hh)) - 1
    jy1 = int(np.ceil((arm + rmax) / hh)) + 1
    ny = jy1 - jy0
    nx = nz = ncell
    gx = -arm + hh * np.arange(nx + 1)
    gy = -arm + hh * (jy0 + np.arange(ny + 1))
    gz = -arm + hh * np.arange(nz + 1)

    def coord(n):
        i = n % (nx + 1)
        r = n // (nx + 1)
        j = r % (ny + 1)
        k = r // (ny + 1)
        return np.stack([gx[i], gy[j], gz[k]], axis=1)

    def keep_cell(i, j, k):
        c = np.stack([gx[i] + hh / 2, gy[j] + hh / 2, gz[k] + hh / 2], axis=1)
        # cells near the tubes; individual tets are filtered below
        return junction_inside(c, r_in1 + hh, r_in2 + hh, r_out + hh, arm)

    tets = _kuhn_grid(nx, ny, nz, keep_cell)
    cen = coord(tets.ravel()).reshape(-1, 4, 3).mean(axis=1)
    tets = tets[junction_inside(cen, r_in1, r_in2, r_out, arm)]
    used, inv = np.unique(tets.ravel(), return_inverse=True)
    xyz = coord(used)
    tets = inv.reshape(-1, 4)

    def label(cen, tri_xyz):
        lab = np.array(["wall"] * cen.shape[0], dtype=object)
        tol = 1e-9
        lab[np.all(np.abs(tri_xyz[:, :, 2] + arm) < tol, axis=1)] = "in1"
        lab[np.all(np.abs(tri_xyz[:, :, 2] - arm) < tol, axis=1)] = "in2"
        lab[np.all(np.abs(tri_xyz[:, :, 0] + arm) < tol, axis=1)] = "out1"
        lab[np.all(np.abs(tri_xyz[:, :, 0] - arm) < tol, axis=1)] = "out2"
        return lab.astype(str)

    return _finish(xyz, tets, label)
