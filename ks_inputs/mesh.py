"""Structured tetrahedral meshes of a cube [-L, L]^3.

The cube is cut into n^3 hexahedra; each hexahedron is split into the six
Kuhn (Freudenthal) tetrahedra {v, v+e_p0, v+e_p0+e_p1, v+(1,1,1)}, one per
permutation p of the axes.  Every tetrahedron is stored with positive
orientation (the last two vertices are swapped where needed).

P1 nodes are the (n+1)^3 lattice vertices; P2 nodes are the (2n+1)^3
half-lattice points (vertices plus the midpoint of every mesh edge), numbered
lexicographically with x fastest.  The local node order of an element is
v0, v1, v2, v3 followed (P2 only) by the edge midpoints of the edges
01, 02, 03, 12, 13, 23.

The finite element spaces of the paper (Sec. 2) are defined on such a
shape-regular tetrahedral decomposition; the paper's own meshes come from an
anisotropic remesher, which the seeded node-moving map below stands in for
(it clusters nodes near the nuclei while keeping the boundary fixed).
"""
from dataclasses import dataclass, field
import numpy as np

# the six Kuhn tetrahedra of a unit cube, one per axis permutation
_PERMS = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
# local edges of a P2 element, in storage order
EDGES = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]


@dataclass
class Mesh:
    order: int                 # 1 (P1) or 2 (P2)
    n: int                     # hexahedra per side
    L: float                   # half side of the cube
    coords: np.ndarray         # [n_nodes][3] float64 (Bohr)
    elems: np.ndarray          # [n_elems][4 or 10] int32, positively oriented
    dirichlet: np.ndarray      # [n_nodes] uint8, 1 on the cube's boundary
    moved: bool = False
    info: dict = field(default_factory=dict)

    @property
    def n_nodes(self):
        return self.coords.shape[0]

    @property
    def n_elems(self):
        return self.elems.shape[0]

    @property
    def n_loc(self):
        return self.elems.shape[1]

    @property
    def interior(self):
        """Node ids of the non-Dirichlet nodes, ascending (the DOF order)."""
        return np.flatnonzero(self.dirichlet == 0).astype(np.int64)


def _kuhn_local_vertices():
    """Per permutation: the four lattice offsets, orientation-corrected."""
    out = []
    for p in _PERMS:
        e = np.eye(3, dtype=np.int64)
        v0 = np.zeros(3, np.int64)
        v1 = v0 + e[p[0]]
        v2 = v1 + e[p[1]]
        v3 = np.ones(3, np.int64)
        vs = [v0, v1, v2, v3]
        d = np.linalg.det(np.stack([vs[1] - vs[0], vs[2] - vs[0], vs[3] - vs[0]], 1).astype(float))
        if d < 0:
            vs[2], vs[3] = vs[3], vs[2]
        out.append(np.stack(vs))
    return np.stack(out)  # [6][4][3]


def _vertex_positions(n, L, idx):
    """Lattice index (..., 3) -> Cartesian position of an unmoved vertex."""
    return -L + 2.0 * L * idx.astype(np.float64) / n


def freudenthal_mesh(n: int, L: float, order: int = 1) -> Mesh:
    if order not in (1, 2):
        raise ValueError("order must be 1 or 2")
    kuhn = _kuhn_local_vertices()                      # [6][4][3]
    hi = np.arange(n)
    hx, hy, hz = np.meshgrid(hi, hi, hi, indexing="ij")
    # hexes ordered x fastest
    base = np.stack([hx.transpose(2, 1, 0).ravel(), hy.transpose(2, 1, 0).ravel(),
                     hz.transpose(2, 1, 0).ravel()], 1)   # [n^3][3]
    # lattice vertices of every element: [n^3][6][4][3] -> [n_e][4][3]
    verts = (base[:, None, None, :] + kuhn[None]).reshape(-1, 4, 3)
    if order == 1:
        s = n + 1
        ids = verts[..., 0] + s * (verts[..., 1] + s * verts[..., 2])
        elems = ids.astype(np.int32)
        g = np.arange(s)
        gx, gy, gz = np.meshgrid(g, g, g, indexing="ij")
        lat = np.stack([gx.transpose(2, 1, 0).ravel(), gy.transpose(2, 1, 0).ravel(),
                        gz.transpose(2, 1, 0).ravel()], 1)
        coords = _vertex_positions(n, L, lat)
        dirich = np.any((lat == 0) | (lat == n), axis=1).astype(np.uint8)
        info = {"lattice": lat, "lat_scale": 1}
    else:
        s = 2 * n + 1
        half = 2 * verts                                   # vertex half-lattice coords
        cols = [half]
        for a, b in EDGES:
            cols.append((verts[:, a] + verts[:, b])[:, None, :])
        hl = np.concatenate(cols, axis=1)                  # [n_e][10][3]
        ids = hl[..., 0] + s * (hl[..., 1] + s * hl[..., 2])
        elems = ids.astype(np.int32)
        g = np.arange(s)
        gx, gy, gz = np.meshgrid(g, g, g, indexing="ij")
        lat = np.stack([gx.transpose(2, 1, 0).ravel(), gy.transpose(2, 1, 0).ravel(),
                        gz.transpose(2, 1, 0).ravel()], 1)
        coords = -L + L * lat.astype(np.float64) / n
        dirich = np.any((lat == 0) | (lat == 2 * n), axis=1).astype(np.uint8)
        info = {"lattice": lat, "lat_scale": 2}
    return Mesh(order=order, n=n, L=float(L), coords=coords, elems=elems,
                dirichlet=dirich, moved=False, info=info)


def _signed_volumes6(coords, elems):
    p = coords[elems[:, :4]]
    d1, d2, d3 = p[:, 1] - p[:, 0], p[:, 2] - p[:, 0], p[:, 3] - p[:, 0]
    return np.einsum("ij,ij->i", d1, np.cross(d2, d3))


def _phi(x, L, R, a, s):
    """Smooth map that pulls points toward the nuclei R and fixes the boundary."""
    b = np.prod(1.0 - (x / L) ** 8, axis=1)
    disp = np.zeros_like(x)
    for r in R:
        d = r[None, :] - x
        disp += a * d * np.exp(-np.sum(d * d, axis=1) / (s * s))[:, None]
    return x + b[:, None] * disp


def move_nodes_toward_nuclei(mesh: Mesh, R, a: float = 0.5, s: float = 2.0,
                             min_ratio: float = 1e-3) -> Mesh:
    """Apply the seeded moving map to the vertices; P2 edge nodes are placed
    at the straight midpoint of their moved end vertices.  The amplitude is
    halved until every element keeps at least min_ratio of its unmoved
    volume."""
    R = np.asarray(R, dtype=np.float64).reshape(-1, 3)
    n, L = mesh.n, mesh.L
    lat = mesh.info["lattice"]
    scale = mesh.info["lat_scale"]
    vol0 = _signed_volumes6(mesh.coords, mesh.elems)
    amp = a
    for _ in range(30):
        if scale == 1:
            new = _phi(mesh.coords, L, R, amp, s)
        else:
            lo = lat // 2
            hi = (lat + 1) // 2
            pl = _phi(_vertex_positions(n, L, lo), L, R, amp, s)
            ph = _phi(_vertex_positions(n, L, hi), L, R, amp, s)
            new = 0.5 * (pl + ph)
        vol = _signed_volumes6(new, mesh.elems)
        if np.all(vol > min_ratio * vol0):
            info = dict(mesh.info)
            info["move_amplitude"] = amp
            return Mesh(order=mesh.order, n=n, L=L, coords=new, elems=mesh.elems,
                        dirichlet=mesh.dirichlet, moved=True, info=info)
        amp *= 0.5
    raise RuntimeError("could not find a valid moving-map amplitude")


def jittered_coarse_mesh(n_H: int, L: float, amp: float = 0.25, seed: int = 7) -> Mesh:
    """A P1 Kuhn mesh of the box with n_H hexahedra per side whose interior
    vertices are moved by seeded uniform offsets of up to amp * h per axis
    (h = 2L / n_H; amp < 0.5 keeps every element positively oriented, which is
    checked): a coarse mesh that is not nested in any fine lattice mesh."""
    base = freudenthal_mesh(n_H, L, 1)
    rng = np.random.default_rng(seed)
    h = 2.0 * L / n_H
    off = rng.uniform(-amp * h, amp * h, size=base.coords.shape)
    off[base.dirichlet == 1] = 0.0
    coords = base.coords + off
    if np.any(_signed_volumes6(coords, base.elems) <= 0.0):
        raise RuntimeError("jitter inverted an element; use a smaller amp")
    info = dict(base.info)
    info["jitter"] = amp
    return Mesh(order=1, n=n_H, L=L, coords=coords, elems=base.elems, dirichlet=base.dirichlet,
                moved=True, info=info)
