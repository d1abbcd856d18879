"""Structured n x n x n hexahedral meshes of the unit cube of order p.

Node numbering.  The order-p mesh has a lattice of (n*p+1)^3 nodes.  Lattice
node (ix, iy, iz) has global id ``(ix*(n*p+1) + iy)*(n*p+1) + iz``.  Element
(ex, ey, ez) has id ``(ex*n + ey)*n + ez`` and its local node (i, j, k),
0 <= i, j, k <= p, sits at local position ``(p+1)^2*i + (p+1)*j + k`` of its
row of ``l2g`` -- the tensor ordering of the paper's appendix (hexahedral
dof ordering, i along x, j along y, k along z).

Modal ordering (basis="modal").  The hierarchical modal basis of the
paper's appendix numbers the 1-D modes 0 = (1-a)/2, 1 = (1+a)/2, then the
bubbles 2..p.  A mode's global id is the lattice id of its position: mode 0
at position 0, mode 1 at position p, bubble m at position m - 1.  Vertex
modes are then shared between neighbouring elements exactly as nodal end
nodes are, bubbles stay inside their element along that axis, and every
element has the same orientation, so face and edge modes match across
elements.  ``coords`` is the same lattice; only vertex-mode positions carry
geometry.

Geometry.  Mesh vertices form an (n+1)^3 grid with spacing h = 1/n.  Interior
vertices (not on the cube's boundary) are moved by independent
U(-perturb*h, +perturb*h) offsets per coordinate, drawn from numpy's PCG64
with the given seed, in vertex order (x slowest, then y, then z; for each
vertex the x, y, z offsets in that order).  Only the coordinates of element
corner nodes carry geometry: an element is the trilinear image of its eight
corners.  Non-corner nodes are placed by trilinear interpolation at the
equispaced reference positions i/p, j/p, k/p -- a display placement that no
solver reads.
"""
from dataclasses import dataclass

import numpy as np


@dataclass
class HexMesh:
    n: int                 # elements per direction
    p: int                 # polynomial order
    coords: np.ndarray     # float64 [n_nodes, 3]
    l2g: np.ndarray        # int32 [n_elem, (p+1)^3]
    vertices: np.ndarray   # float64 [(n+1)^3, 3], the corner grid

    @property
    def n_nodes(self) -> int:
        return self.coords.shape[0]

    @property
    def n_elem(self) -> int:
        return self.l2g.shape[0]


def _vertex_grid(n: int, perturb: float, seed) -> np.ndarray:
    h = 1.0 / n
    t = np.arange(n + 1, dtype=np.float64) * h
    vx, vy, vz = np.meshgrid(t, t, t, indexing="ij")
    v = np.stack([vx.ravel(), vy.ravel(), vz.ravel()], axis=1)
    if perturb > 0.0:
        rng = np.random.Generator(np.random.PCG64(seed))
        off = rng.uniform(-perturb * h, perturb * h, size=v.shape)
        idx = np.arange(n + 1)
        interior = (idx > 0) & (idx < n)
        mask = (interior[:, None, None] & interior[None, :, None]
                & interior[None, None, :]).ravel()
        v[mask] += off[mask]
    return v


def modal_positions(p: int) -> np.ndarray:
    """Lattice position (0..p) of each 1-D modal index in an element."""
    pos = np.arange(p + 1) - 1
    pos[0], pos[1] = 0, p
    return pos


def hex_mesh(n: int, p: int, perturb: float = 0.0, seed=None, basis: str = "nodal") -> HexMesh:
    """Build the order-p structured mesh of n^3 hexahedra on the unit cube;
    ``basis`` picks the local ordering of l2g ("nodal" or "modal")."""
    if n < 1 or p < 1:
        raise ValueError("n and p must be >= 1")
    if basis not in ("nodal", "modal"):
        raise ValueError("basis must be 'nodal' or 'modal'")
    L = n * p + 1
    verts = _vertex_grid(n, perturb, seed)
    V = verts.reshape(n + 1, n + 1, n + 1, 3)

    # lattice node coordinates: trilinear interpolation between the vertices
    lat = np.arange(L)
    e = np.minimum(lat // p, n - 1)          # owning element index per axis
    f = (lat - e * p) / float(p)             # equispaced fraction in [0, 1]
    ex, ey, ez = np.meshgrid(e, e, e, indexing="ij")
    fx, fy, fz = np.meshgrid(f, f, f, indexing="ij")
    coords = np.zeros((L, L, L, 3), dtype=np.float64)
    for cx in (0, 1):
        wx = fx if cx else 1.0 - fx
        for cy in (0, 1):
            wy = fy if cy else 1.0 - fy
            for cz in (0, 1):
                wz = fz if cz else 1.0 - fz
                coords += (wx * wy * wz)[..., None] * V[ex + cx, ey + cy, ez + cz]
    coords = coords.reshape(-1, 3)

    # element -> node map in the (p+1)^2 i + (p+1) j + k ordering
    el = np.arange(n)
    EX, EY, EZ = np.meshgrid(el, el, el, indexing="ij")
    loc = np.arange(p + 1) if basis == "nodal" else modal_positions(p)
    I, J, K = np.meshgrid(loc, loc, loc, indexing="ij")
    gx = EX.ravel()[:, None] * p + I.ravel()[None, :]
    gy = EY.ravel()[:, None] * p + J.ravel()[None, :]
    gz = EZ.ravel()[:, None] * p + K.ravel()[None, :]
    l2g = ((gx * L + gy) * L + gz).astype(np.int32)
    return HexMesh(n=n, p=p, coords=coords, l2g=np.ascontiguousarray(l2g),
                   vertices=verts)
