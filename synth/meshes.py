"""Hexahedral mesh generators and coefficient-vector size bookkeeping.

Conventions shared by every consumer:

* ``vertices`` is float64 ``[n_vertices, 3]``.
* ``hexes`` is int64 ``[n_elements, 8]``; local vertex ``v = b0 + 2*b1 + 4*b2``
  sits at reference corner ``(b0, b1, b2)`` of the unit cube (x-hat fastest).
* ``p`` (spatial degree) and ``q`` (temporal degree) are int32 per element,
  ``eps`` and ``mu`` float64 per element.
* Coefficient vectors are element-major.  Per element, the full trial vector
  holds ``6*(q+1)*(p+1)**3`` scalars, the unknown / residual vector
  ``6*q*(p+1)**3`` scalars.
"""
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Mesh:
    vertices: np.ndarray            # [nv, 3] float64
    hexes: np.ndarray               # [ne, 8] int64
    p: np.ndarray                   # [ne] int32
    q: np.ndarray                   # [ne] int32
    eps: np.ndarray                 # [ne] float64
    mu: np.ndarray                  # [ne] float64
    shape: tuple = None             # (nx, ny, nz) for lattice meshes, else None
    meta: dict = field(default_factory=dict)
    nsub: np.ndarray = None         # [ne] temporal sub-intervals (local time steps), None = 1

    @property
    def n_elements(self):
        return int(self.hexes.shape[0])

    def levels(self):
        """Temporal degree times sub-intervals: the test levels per element."""
        return self.q if self.nsub is None else np.asarray(self.q) * np.asarray(self.nsub)

    def trial_size(self):
        return int(trial_sizes(self.p, self.levels()).sum())

    def unknown_size(self):
        return int(unknown_sizes(self.p, self.levels()).sum())

    def state_size(self):
        a = self.p.astype(np.int64) + 1
        return int((6 * a ** 3).sum())


def trial_sizes(p, q):
    a = np.asarray(p, dtype=np.int64) + 1
    return 6 * (np.asarray(q, dtype=np.int64) + 1) * a ** 3


def unknown_sizes(p, q):
    a = np.asarray(p, dtype=np.int64) + 1
    return 6 * np.asarray(q, dtype=np.int64) * a ** 3


def offsets(sizes):
    sizes = np.asarray(sizes, dtype=np.int64)
    off = np.zeros(sizes.size + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    return off


def box_mesh(shape, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)):
    """Lattice of ``nx*ny*nz`` axis-aligned hexahedra filling the box [lo, hi].

    Element ``(ex, ey, ez)`` has index ``ex + nx*(ey + ny*ez)``.
    Returns ``(vertices, hexes)``.
    """
    nx, ny, nz = (int(s) for s in shape)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    xs = np.linspace(lo[0], hi[0], nx + 1)
    ys = np.linspace(lo[1], hi[1], ny + 1)
    zs = np.linspace(lo[2], hi[2], nz + 1)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    vertices = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)

    def vid(i, j, k):
        return i + (nx + 1) * (j + (ny + 1) * k)

    ez, ey, ex = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ex, ey, ez = ex.ravel(), ey.ravel(), ez.ravel()
    hexes = np.empty((ex.size, 8), dtype=np.int64)
    for v in range(8):
        b0, b1, b2 = v & 1, (v >> 1) & 1, (v >> 2) & 1
        hexes[:, v] = vid(ex + b0, ey + b1, ez + b2)
    return vertices, hexes


def hanging_mesh(n=2, split=1, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)):
    """A box of n^3 axis-aligned cells in which every cell with x index >=
    ``split`` is refined into 2 x 2 x 2 halves: the faces between cells at x
    index split - 1 and split are 2:1 hanging faces (one coarse face against
    four fine faces).  Vertices are shared by position.  Returns
    ``(vertices, hexes)``; cells in x-fastest order, each refined cell's eight
    children in place of it (x fastest)."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    h = (hi - lo) / n
    index = {}
    verts = []

    def vid(x):
        key = tuple(np.round(x, 12))
        if key not in index:
            index[key] = len(verts)
            verts.append(np.array(x, dtype=np.float64))
        return index[key]

    corners = np.array([[v & 1, (v >> 1) & 1, (v >> 2) & 1] for v in range(8)], dtype=np.float64)
    hexes = []
    for k in range(n):
        for j in range(n):
            for i in range(n):
                x0 = lo + h * np.array([i, j, k], dtype=np.float64)
                if i >= split:
                    for c in range(8):
                        y0 = x0 + 0.5 * h * corners[c]
                        hexes.append([vid(y0 + 0.5 * h * corners[v]) for v in range(8)])
                else:
                    hexes.append([vid(x0 + h * corners[v]) for v in range(8)])
    return np.array(verts), np.array(hexes, dtype=np.int64)


def perturb_interior(vertices, shape, frac, seed, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)):
    """Shift every coordinate of every interior lattice vertex by an independent
    U(-frac*h_d, +frac*h_d) draw (h_d = lattice spacing along axis d).
    Boundary vertices stay fixed so boundary faces stay planar."""
    nx, ny, nz = (int(s) for s in shape)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    h = (hi - lo) / np.array([nx, ny, nz], dtype=np.float64)
    rng = np.random.default_rng(seed)
    out = vertices.copy()
    k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    interior = ((i > 0) & (i < nx) & (j > 0) & (j < ny) & (k > 0) & (k < nz)).ravel()
    shift = rng.uniform(-1.0, 1.0, size=(vertices.shape[0], 3)) * (frac * h)[None, :]
    out[interior] += shift[interior]
    return out


def affine_transform(vertices, A, b=(0.0, 0.0, 0.0)):
    """x -> A x + b applied to every vertex (used to build sheared meshes)."""
    A = np.asarray(A, dtype=np.float64)
    return vertices @ A.T + np.asarray(b, dtype=np.float64)[None, :]


def centroids(vertices, hexes):
    """Arithmetic mean of the 8 vertices of every element."""
    return vertices[hexes].mean(axis=1)


def cube_rotations():
    """The 24 proper rotations of the reference cube as permutations of its 8
    corners: perm[v_new] = v_old, i.e. relabelling an element's vertices with
    hexes[e] = hexes[e][perm] turns it without inverting it (each rotation is
    a signed permutation of the centred axes with determinant +1)."""
    import itertools
    out = []
    for axes in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            R = np.zeros((3, 3), dtype=np.int64)
            for i in range(3):
                R[i, axes[i]] = signs[i]
            if round(np.linalg.det(R)) != 1:
                continue
            perm = []
            for v in range(8):
                s_new = np.array([2 * ((v >> d) & 1) - 1 for d in range(3)])
                s_old = R @ s_new
                perm.append(int(sum(((s_old[d] + 1) // 2) << d for d in range(3))))
            out.append(perm)
    return out


def reorient(hexes, seed, frac=1.0):
    """Relabel the vertices of a random fraction of the elements by random
    cube rotations (seeded): the same physical mesh with faces met in every
    orientation (axes swapped and reversed between neighbours)."""
    rots = cube_rotations()
    rng = np.random.default_rng(seed)
    out = np.array(hexes, dtype=np.int64, copy=True)
    for e in range(out.shape[0]):
        if rng.random() < frac:
            out[e] = out[e][rots[rng.integers(len(rots))]]
    return out
