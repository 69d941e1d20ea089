"""Element maps and face topology (oracle step O2).

Section 2.3: F_K maps the unit cube [0, 1]^3 onto the hexahedron K; here F_K
is the trilinear map through the 8 vertices (local vertex v = b0 + 2 b1 + 4 b2
at reference corner (b0, b1, b2)).  Section 2.4: faces are interior (shared by
two elements) or boundary.

Local face numbering: face 2*alpha + side lies on x-hat_alpha = side.
"""
import numpy as np

CORNERS = np.array([[v & 1, (v >> 1) & 1, (v >> 2) & 1] for v in range(8)], dtype=np.float64)


def shape_functions(xh):
    """Trilinear shape functions N_v(x-hat) and their gradients.
    xh: [..., 3] -> N [..., 8], dN [..., 8, 3]."""
    xh = np.asarray(xh, dtype=np.float64)
    f = np.where(CORNERS[None, :, :] > 0.5, xh[..., None, :].reshape(-1, 1, 3),
                 1.0 - xh[..., None, :].reshape(-1, 1, 3))          # [P, 8, 3]
    df = np.where(CORNERS[None, :, :] > 0.5, 1.0, -1.0) * np.ones_like(f)
    N = f[:, :, 0] * f[:, :, 1] * f[:, :, 2]
    dN = np.stack([df[:, :, 0] * f[:, :, 1] * f[:, :, 2],
                   f[:, :, 0] * df[:, :, 1] * f[:, :, 2],
                   f[:, :, 0] * f[:, :, 1] * df[:, :, 2]], axis=-1)
    shp = xh.shape[:-1]
    return N.reshape(shp + (8,)), dN.reshape(shp + (8, 3))


def map_point(X, xh):
    """F(x-hat) for vertex array X [8, 3]."""
    N, _ = shape_functions(xh)
    return N @ X


def jacobian(X, xh):
    """DF[..., i, m] = dF_i / dx-hat_m."""
    _, dN = shape_functions(xh)
    return np.einsum("...vm,vi->...im", dN, X)


def second_derivatives(X, xh):
    """H[..., i, m, n] = d^2 F_i / (dx-hat_m dx-hat_n) of the trilinear map."""
    xh = np.asarray(xh, dtype=np.float64)
    shp = xh.shape[:-1]
    P = xh.reshape(-1, 3)
    out = np.zeros((P.shape[0], 3, 3, 3))
    for v in range(8):
        b = CORNERS[v]
        f = np.where(b > 0.5, P, 1.0 - P)           # [P, 3]
        s = np.where(b > 0.5, 1.0, -1.0)            # [3]
        for m in range(3):
            for n in range(3):
                if m == n:
                    continue
                k = 3 - m - n
                val = s[m] * s[n] * f[:, k]
                out[:, :, m, n] += val[:, None] * X[v][None, :]
    return out.reshape(shp + (3, 3, 3))


def face_vertices(hexrow, face):
    """The 4 global vertex ids of local face (alpha, side), ordered by the
    tangential reference coordinates (u, v) = the two remaining axes in
    increasing order, u fastest."""
    alpha, side = divmod(face, 2)
    tang = [d for d in range(3) if d != alpha]
    ids = []
    for bv in range(2):
        for bu in range(2):
            b = [0, 0, 0]
            b[alpha] = side
            b[tang[0]] = bu
            b[tang[1]] = bv
            ids.append(int(hexrow[b[0] + 2 * b[1] + 4 * b[2]]))
    return ids


def face_topology(hexes):
    """Neighbour table nb[e, f] (-1 on the boundary) and the neighbour's local
    face nbf[e, f], found by matching the sorted vertex ids of the 6 faces of
    every element.  Also reports whether each interior face is in canonical
    orientation (neighbour face = same axis, opposite side, same (u, v)
    vertex order)."""
    ne = hexes.shape[0]
    table = {}
    for e in range(ne):
        for f in range(6):
            key = tuple(sorted(face_vertices(hexes[e], f)))
            table.setdefault(key, []).append((e, f))
    nb = -np.ones((ne, 6), dtype=np.int64)
    nbf = -np.ones((ne, 6), dtype=np.int64)
    canonical = np.ones((ne, 6), dtype=bool)
    for key, lst in table.items():
        if len(lst) == 1:
            continue
        if len(lst) != 2:
            raise ValueError("non-manifold face shared by %d elements" % len(lst))
        (e1, f1), (e2, f2) = lst
        nb[e1, f1], nbf[e1, f1] = e2, f2
        nb[e2, f2], nbf[e2, f2] = e1, f1
        ok = (f1 // 2 == f2 // 2) and (f1 % 2 != f2 % 2) and \
            face_vertices(hexes[e1], f1) == face_vertices(hexes[e2], f2)
        canonical[e1, f1] = canonical[e2, f2] = ok
    return nb, nbf, canonical


def face_map(hexrow, face, hexrow_o, face_o):
    """Map between the reference coordinates of a shared face: (u', v') =
    A (u, v) + b takes the tangential coordinates (u, v) of local face `face`
    of one element (the two remaining axes in increasing order) to those of
    local face `face_o` of its neighbour, found from the shared vertex ids.
    On a conforming face it is a symmetry of the unit square (A a signed
    permutation); canonical orientation is A = I, b = 0."""
    mine = face_vertices(hexrow, face)
    theirs = face_vertices(hexrow_o, face_o)
    corner = {}
    for j, g in enumerate(theirs):
        corner[g] = np.array([j & 1, j >> 1], dtype=np.int64)
    p00, p10, p01 = corner[mine[0]], corner[mine[1]], corner[mine[2]]
    A = np.stack([p10 - p00, p01 - p00], axis=1)
    b = p00.copy()
    if sorted(np.abs(A).sum(axis=0).tolist()) != [1, 1] or abs(round(np.linalg.det(A))) != 1 or \
            not np.array_equal(A @ np.array([1, 1]) + b, corner[mine[3]]):
        raise ValueError("faces do not match as quadrilaterals")
    return A, b


def is_affine(X, tol=1e-12):
    """True when the trilinear map is affine (the hexahedron is a parallelepiped)."""
    x0 = X[0]
    A = np.stack([X[1] - x0, X[2] - x0, X[4] - x0], axis=1)
    pred = x0[None, :] + CORNERS @ A.T
    scale = max(1.0, np.abs(X).max())
    return bool(np.abs(pred - X).max() <= tol * scale)


def hanging_faces(vertices, hexes, nb, tol=1e-9):
    """2:1 nonconforming faces (Section 5.2 sums the flux terms of a face over
    the neighbours that share parts of it): a face without a conforming
    partner whose four quarters are whole faces of four other elements.

    The quarter corners are mesh vertices at the face's corners, edge
    midpoints and centre (the bilinear face map at (i/2, j/2)); a quarter
    matches the face of another element with the same four vertex ids.
    Returns a dict keyed by (element, local face) with, for the coarse side,
    four entries (k, f_k, A, b, (u0, v0)): own face coordinates (u, v) in the
    quarter [u0, u0 + 1/2] x [v0, v0 + 1/2] map to the fine face's by
    (u', v') = A (u, v) + b (A = 2 times a signed permutation); and for each
    fine side one entry (k, f_k, A, b, None): its whole face maps into the
    coarse face by (u', v') = A (u, v) + b (A = 1/2 times a signed
    permutation).  Faces with a conforming partner (nb >= 0) are skipped."""
    vertices = np.asarray(vertices, dtype=np.float64)
    scale = max(1.0, float(np.abs(vertices).max()))
    key_of = lambda x: tuple(np.round(np.asarray(x) / (tol * scale)).astype(np.int64))
    vid = {}
    for i, x in enumerate(vertices):
        vid.setdefault(key_of(x), i)
    ne = hexes.shape[0]
    free = {}
    for e in range(ne):
        for f in range(6):
            if nb[e, f] < 0:
                free[tuple(sorted(face_vertices(hexes[e], f)))] = (e, f)
    out = {}
    for e in range(ne):
        for f in range(6):
            if nb[e, f] >= 0:
                continue
            ids = face_vertices(hexes[e], f)                 # (0,0), (1,0), (0,1), (1,1) in (u, v)
            P = vertices[ids]
            grid = {}
            ok = True
            for i in range(3):
                for j in range(3):
                    s, t = 0.5 * i, 0.5 * j
                    x = (1 - s) * (1 - t) * P[0] + s * (1 - t) * P[1] + (1 - s) * t * P[2] + s * t * P[3]
                    g = vid.get(key_of(x))
                    if g is None:
                        ok = False
                        break
                    grid[(i, j)] = g
                if not ok:
                    break
            if not ok:
                continue
            where = {g: np.array([0.5 * i, 0.5 * j]) for (i, j), g in grid.items()}
            quarters = []
            for iv in range(2):
                for iu in range(2):
                    qids = tuple(sorted(grid[(iu + du, iv + dv)] for du in (0, 1) for dv in (0, 1)))
                    if qids not in free:
                        break
                    quarters.append(((iu, iv), free[qids]))
            if len(quarters) != 4:
                continue
            entries = []
            for (iu, iv), (k, fk) in quarters:
                fine = face_vertices(hexes[k], fk)
                p00, p10, p01, p11 = (where[g] for g in fine)
                Af = np.stack([p10 - p00, p01 - p00], axis=1)   # fine (u', v') -> coarse (u, v)
                bf = p00.copy()
                if not np.allclose(Af @ np.array([1.0, 1.0]) + bf, p11) or \
                        sorted(np.abs(Af).sum(axis=0).tolist()) != [0.5, 0.5]:
                    raise ValueError("hanging face: a quarter does not match as a quadrilateral")
                Ac = np.linalg.inv(Af)
                entries.append((k, fk, np.round(Ac), -np.round(Ac) @ bf, (0.5 * iu, 0.5 * iv)))
                out[(k, fk)] = [(e, f, Af, bf, None)]
            out[(e, f)] = entries
    return out
