"""Dense local matrices, slab blocks, residual, load, energy and slab solves
(oracle steps O3-O6).

Everything follows the slab bilinear form of the paper:

  C_h(U, V) = (eps d_t E, v) + (mu d_t H, w) - (H, curl_h v) + (curl_h E, w)
              + sum_f ({H}, [v]_T)_f - sum_f ([E]_T, {w})_f          (Section 2.5, eq. bilinearform:C)
  S_h(U, V) = stabilisation of eq. bilinearform:S (Section 4.1)
  B_h = C_h + S_h                                                    (eq. weakform_stabilized)
  D_h(U, V) = dissipative upwind-type face terms (remark closing Section 4),
              added to B_h when c_diss > 0
  R_h(V) = B_h(U_h, V) - L(V),  L(V) = (J, v) - (n x g, w)_{F_b}      (Section 5, eq. residual)

with centred fluxes ({v} = v and [v]_T = n x v on boundary faces; g = 0 here:
PEC walls), the covariant map E = DF^{-T} E-hat (Section 2.3) and the tensor
bases of Section 5.1.  The space-time integrals factor into a time integral
times a space integral because every basis function is a product of a
temporal and a spatial factor (Section 5.2, first display); the oracle uses that
factorisation and nothing else from Section 5.2.

Readings where the paper is silent or garbled (each pinned by a test):
* time tables: D[i, m] = int L_i l_m', N[i, m] = int L_i l_m on [0, 1]; the
  time-derivative term carries no dt factor, the curl and flux terms carry dt.
* reference-space curl and flux: for covariant maps (curl E, w)_K equals the
  reference integral of curl-hat E-hat . w-hat, and on a conforming face with
  matching orientation (H, n x v)_f equals the reference integral of
  v-hat . (H-hat x n-hat); so only the mass and the load see the geometry
  (checked against the physical-space assembler in ``brute``).
* boundary faces (PEC): weight 1 for the self terms; interior faces 1/2.
* S_h with one temporal element per slab: pi-tilde truncates the orthonormal
  Legendre test modes to i < min(q_K, q_K'); only the neighbour coupling is
  truncated.  The derivation from eq. bilinearform:S is checked by ``brute``.
* local time steps (Section 2.2): element K's slab interval is bisected into
  n_K equal sub-intervals, n_K a power of two, so the partitions of two
  neighbours nest; the common temporal test space of S_h is then piecewise
  P_{min(q_K, q_K') - 1} on the coarser of the two partitions, and S_h again
  reduces to the neighbour coupling with the own test function projected
  onto it (the self terms keep weight 1/2, unprojected).  Test functions of
  sub-interval j are L_i(n_K s - j), s the unit slab coordinate; the trial
  levels are flattened as in basis.trial_level (slab start and end values at
  levels 0 and 1).
* D_h with local time steps: the same projection on the test function.
* mass quadrature: n_q = p + 2 Gauss points per direction (exact on affine
  elements); the same rule is used by the library.
* load quadrature: p + 3 points per space direction, q + 3 in time per
  sub-interval.
* D_h: the projection on interior faces acts on the test function (rows
  i >= min(q_K, q_K') vanish for own and neighbour trial), the trial jump is
  not projected; on PEC faces nothing is projected and g = 0; {.} of the
  impedances is the plain mean of the two sides, on PEC faces the element's own.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import basis
from .geometry import face_map, face_topology, hanging_faces, jacobian, map_point

LEVI = np.zeros((3, 3, 3))
LEVI[0, 1, 2] = LEVI[1, 2, 0] = LEVI[2, 0, 1] = 1.0
LEVI[0, 2, 1] = LEVI[2, 1, 0] = LEVI[1, 0, 2] = -1.0
EYE3 = np.eye(3)


# ----------------------------------------------------------------------------
# reference tensor-product basis on quadrature grids
# ----------------------------------------------------------------------------

def tensor_points(n):
    """n^3 Gauss points on [0,1]^3, ordered g = gx + n (gy + n gz), and weights."""
    x, w = basis.gauss01(n)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    WZ, WY, WX = np.meshgrid(w, w, w, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    return pts, (WX * WY * WZ).ravel()


def basis_at(a, pts):
    """phi_s(x-hat) for s = j + a (k + a l): Phi [P, a^3] and the reference
    gradient dPhi [P, a^3, 3]."""
    Vx = basis.legendre_matrix(a, pts[:, 0])
    Vy = basis.legendre_matrix(a, pts[:, 1])
    Vz = basis.legendre_matrix(a, pts[:, 2])
    dVx = basis.dlegendre_matrix(a, pts[:, 0])
    dVy = basis.dlegendre_matrix(a, pts[:, 1])
    dVz = basis.dlegendre_matrix(a, pts[:, 2])
    P = pts.shape[0]
    Phi = np.einsum("pl,pk,pj->plkj", Vz, Vy, Vx).reshape(P, a ** 3)
    g0 = np.einsum("pl,pk,pj->plkj", Vz, Vy, dVx).reshape(P, a ** 3)
    g1 = np.einsum("pl,pk,pj->plkj", Vz, dVy, Vx).reshape(P, a ** 3)
    g2 = np.einsum("pl,pk,pj->plkj", dVz, Vy, Vx).reshape(P, a ** 3)
    return Phi, np.stack([g0, g1, g2], axis=-1)


def face_points(face, n):
    """n^2 Gauss points on local face (alpha, side) of the unit cube, with the
    tangential coordinates (the remaining axes in increasing order) on the grid,
    and weights."""
    alpha, side = divmod(face, 2)
    tang = [d for d in range(3) if d != alpha]
    x, w = basis.gauss01(n)
    V, U = np.meshgrid(x, x, indexing="ij")
    WV, WU = np.meshgrid(w, w, indexing="ij")
    pts = np.zeros((n * n, 3))
    pts[:, alpha] = float(side)
    pts[:, tang[0]] = U.ravel()
    pts[:, tang[1]] = V.ravel()
    return pts, (WU * WV).ravel()


def opposite(face):
    return face ^ 1


# ----------------------------------------------------------------------------
# spatial matrices (rows (c, s) test, cols (d, t) trial; index = c * a^3 + s)
# ----------------------------------------------------------------------------

def mass_matrix(X, a, coef, nq):
    """M[(c,s),(d,t)] = int_K coef (DF^{-T} e_c phi_s) . (DF^{-T} e_d phi_t) dx
    = int_Khat coef G_cd phi_s phi_t, G = |J| DF^{-1} DF^{-T}, by an nq^3 Gauss rule."""
    pts, w = tensor_points(nq)
    DF = jacobian(X, pts)
    det = np.linalg.det(DF)
    if np.any(det <= 0):
        raise ValueError("inverted element")
    Dinv = np.linalg.inv(DF)
    G = det[:, None, None] * np.einsum("pcm,pdm->pcd", Dinv, Dinv)
    Phi, _ = basis_at(a, pts)
    n3 = a ** 3
    M = np.zeros((3, n3, 3, n3))
    for c in range(3):
        for d in range(3):
            M[c, :, d, :] = (Phi * (w * coef * G[:, c, d])[:, None]).T @ Phi
    return M.reshape(3 * n3, 3 * n3)


def curl_matrix(a):
    """C[(c,s),(d,t)] = int_Khat phi_s e_c . curl-hat(phi_t e_d)
    = sum_m levi(c, m, d) int phi_s d_m phi_t  (exact with a+1 points)."""
    pts, w = tensor_points(a + 1)
    Phi, dPhi = basis_at(a, pts)
    n3 = a ** 3
    C = np.zeros((3, n3, 3, n3))
    for m in range(3):
        Gm = (Phi * w[:, None]).T @ dPhi[:, :, m]
        for c in range(3):
            for d in range(3):
                if LEVI[c, m, d] != 0.0:
                    C[c, :, d, :] += LEVI[c, m, d] * Gm
    return C.reshape(3 * n3, 3 * n3)


def face_matrices(a, face, a_other=None, neighbour=False):
    """Reference face matrices on local face (alpha, side) of K with outward
    reference normal n-hat = (2 side - 1) e_alpha.

    FE[(c,s),(d,t)] = int_f phi_s e_c . (psi_t e_d x n-hat)      (E-test, H-trial: v . (H x n))
    FH[(c,s),(d,t)] = -int_f phi_s e_c . (n-hat x psi_t e_d)     (H-test, E-trial: -w . (n x E))

    psi is K's own basis (neighbour=False) or the neighbour's basis of degree
    a_other evaluated on the neighbour's opposite face at the same tangential
    coordinates (canonical orientation)."""
    alpha, side = divmod(face, 2)
    ao = a if a_other is None else a_other
    n = max(a, ao) + 1
    pts, w = face_points(face, n)
    Phi, _ = basis_at(a, pts)
    if neighbour:
        pts_o, _ = face_points(opposite(face), n)
        Psi, _ = basis_at(ao, pts_o)
    else:
        Psi, _ = basis_at(a, pts)
    nhat = (2.0 * side - 1.0) * EYE3[alpha]
    Sface = (Phi * w[:, None]).T @ Psi                     # int phi_s psi_t
    n3, m3 = a ** 3, ao ** 3
    FE = np.zeros((3, n3, 3, m3))
    FH = np.zeros((3, n3, 3, m3))
    for c in range(3):
        for d in range(3):
            ed_x_n = np.cross(EYE3[d], nhat)[c]
            n_x_ed = np.cross(nhat, EYE3[d])[c]
            if ed_x_n != 0.0:
                FE[c, :, d, :] = ed_x_n * Sface
            if n_x_ed != 0.0:
                FH[c, :, d, :] = -n_x_ed * Sface
    return FE.reshape(3 * n3, 3 * m3), FH.reshape(3 * n3, 3 * m3)


def face_matrices_oriented(a, face, ao, face_o, A, b, sub=None):
    """The neighbour face matrices of ``face_matrices`` for a neighbour met in
    any orientation: its basis is evaluated on its own face ``face_o`` at the
    points (u', v') = A (u, v) + b matched to K's face points, and its
    covariant reference components are carried into K's frame along the
    face, E-hat_{tau_i} = sum_j A[j, i] E-hat'_{tau'_j} (chain rule for the
    tangent vectors of the shared face; the normal components do not enter
    the fluxes).  Geometry-free like the canonical case; exact quadrature.

    ``sub = (u0, v0)`` restricts the integral to the quarter
    [u0, u0 + 1/2] x [v0, v0 + 1/2] of K's face (a 2:1 hanging face seen
    from the coarse side, the neighbour covering that quarter; then A holds
    2 times a signed permutation, and 1/2 times one seen from the fine side)."""
    alpha, side = divmod(face, 2)
    tang = [d for d in range(3) if d != alpha]
    alpha_o, side_o = divmod(face_o, 2)
    tang_o = [d for d in range(3) if d != alpha_o]
    n = max(a, ao) + 1
    pts, w = face_points(face, n)
    if sub is not None:
        pts = pts.copy()
        pts[:, tang[0]] = sub[0] + 0.5 * pts[:, tang[0]]
        pts[:, tang[1]] = sub[1] + 0.5 * pts[:, tang[1]]
        w = 0.25 * w
    Phi, _ = basis_at(a, pts)
    uv = pts[:, tang]
    uvo = uv @ A.T + b[None, :]
    pts_o = np.zeros_like(pts)
    pts_o[:, alpha_o] = float(side_o)
    pts_o[:, tang_o[0]] = uvo[:, 0]
    pts_o[:, tang_o[1]] = uvo[:, 1]
    Psi, _ = basis_at(ao, pts_o)
    Cmap = np.zeros((3, 3))                      # K-frame component d <- neighbour component d'
    for i in range(2):
        for j in range(2):
            Cmap[tang[i], tang_o[j]] = A[j, i]
    nhat = (2.0 * side - 1.0) * EYE3[alpha]
    Sface = (Phi * w[:, None]).T @ Psi
    n3, m3 = a ** 3, ao ** 3
    FE = np.zeros((3, n3, 3, m3))
    FH = np.zeros((3, n3, 3, m3))
    for c in range(3):
        for d in range(3):
            ed_x_n = np.cross(EYE3[d], nhat)[c]
            n_x_ed = np.cross(nhat, EYE3[d])[c]
            for dp in range(3):
                if Cmap[d, dp] == 0.0:
                    continue
                FE[c, :, dp, :] += Cmap[d, dp] * ed_x_n * Sface
                FH[c, :, dp, :] -= Cmap[d, dp] * n_x_ed * Sface
    return FE.reshape(3 * n3, 3 * m3), FH.reshape(3 * n3, 3 * m3)


def dissipation_matrices(X, a, face, Xo=None, ao=None, nq=None, face_o=None, fmap=None):
    """Face matrices of the dissipative stabilisation (the upwind-type remark
    after Section 4): with covariant basis functions u = DF^{-T} e_c phi_s,
      Dself[(c,s),(d,t)] = int_f (n x u_(c,s)) . (n x u_(d,t)) dS      (K's own trial)
      Dnb[(c,s),(d,t)]   = int_f (n x u_(c,s)) . (n x u'_(d,t)) dS     (neighbour trial)
    in physical space on local face (alpha, side) of K, n the unit normal,
    u' the neighbour's basis of degree ao on its face at the same physical
    points (its opposite face at the same tangential coordinates, or face_o
    through the face map fmap = (A, b) for other orientations).  The face rule has
    max(a, ao) + 2 Gauss points per direction unless nq is given: exact on
    affine elements, a quadrature of the rational integrand on trilinear ones."""
    alpha, side = divmod(face, 2)
    tang = [d for d in range(3) if d != alpha]
    n = (max(a, ao or a) + 2) if nq is None else nq
    pts, w = face_points(face, n)
    DF = jacobian(X, pts)                                   # [P, 3, 3], DF[:, :, m] = dx / dxhat_m
    nv = np.cross(DF[:, :, tang[0]], DF[:, :, tang[1]])
    dS = np.linalg.norm(nv, axis=1)
    nrm = nv / dS[:, None] * (2.0 * side - 1.0) * np.sign(np.einsum("pi,pi->p", nv, DF[:, :, alpha]))[:, None]
    wS = w * dS

    def nx_basis(Xe, ae, fpts):
        Dinv = np.linalg.inv(jacobian(Xe, fpts))            # rows: DF^{-1}; DF^{-T} e_c = Dinv[c, :]
        Phi, _ = basis_at(ae, fpts)
        vecs = np.cross(nrm[:, None, :], Dinv)              # [P, c, 3]: n x DF^{-T} e_c
        return np.einsum("pck,ps->pcsk", vecs, Phi).reshape(len(fpts), 3 * ae ** 3, 3)

    A = nx_basis(X, a, pts)
    Aw = A * wS[:, None, None]
    Dself = np.tensordot(Aw, A, axes=([0, 2], [0, 2]))      # sum_p,k w A[p,a,k] A[p,b,k]
    if Xo is None:
        return Dself, None
    if fmap is None:
        pts_o, _ = face_points(opposite(face), n)
    else:
        Am, bm = fmap
        alpha_o, side_o = divmod(face_o, 2)
        tang_o = [d for d in range(3) if d != alpha_o]
        uvo = pts[:, tang] @ Am.T + bm[None, :]
        pts_o = np.zeros_like(pts)
        pts_o[:, alpha_o] = float(side_o)
        pts_o[:, tang_o[0]] = uvo[:, 0]
        pts_o[:, tang_o[1]] = uvo[:, 1]
    B = nx_basis(Xo, ao, pts_o)
    Dnb = np.tensordot(Aw, B, axes=([0, 2], [0, 2]))
    return Dself, Dnb


# ----------------------------------------------------------------------------
# discretisation of one mesh
# ----------------------------------------------------------------------------

class Discretisation:
    """Slab discretisation of a hexahedral mesh with per-element (p, q, eps, mu).

    Coefficient layouts (element-major, canonical):
      full trial U : per element [field E,H][comp x,y,z][m = 0..n q][s]
      unknowns  x  : per element [field][comp][m = 1..n q][s]
      residual  y  : per element [field][comp][i = 0..n q-1][s]
      state        : per element [field][comp][s]   (fields at one time)
    with s = j + a (k + a l), j the x-hat index, and n the element's number of
    temporal sub-intervals (``nk``, a power of two, default 1; Section 2.2):
    trial level m is the flattened level of basis.trial_level (level 0 the
    slab start, level 1 the slab end), test level j q + i the test function
    L_i of sub-interval j."""

    def __init__(self, vertices, hexes, p, q, eps, mu, mass_nq=None, c_diss=0.0, nk=None):
        self.vertices = np.asarray(vertices, dtype=np.float64)
        self.hexes = np.asarray(hexes, dtype=np.int64)
        self.p = np.asarray(p, dtype=np.int64)
        self.q = np.asarray(q, dtype=np.int64)
        self.a = self.p + 1
        self.eps = np.asarray(eps, dtype=np.float64)
        self.mu = np.asarray(mu, dtype=np.float64)
        self.ne = self.hexes.shape[0]
        self.nb, self.nbf, self.canon = face_topology(self.hexes)
        # face maps of the interior faces met in another orientation
        self.fmap = {}
        for e in range(self.hexes.shape[0]):
            for f in range(6):
                if self.nb[e, f] >= 0 and not self.canon[e, f]:
                    self.fmap[(e, f)] = face_map(self.hexes[e], f, self.hexes[self.nb[e, f]], int(self.nbf[e, f]))
        # 2:1 hanging faces (four neighbours on a coarse face, one coarse
        # neighbour on each fine face): interior faces without a conforming partner
        self.hang = hanging_faces(self.vertices, self.hexes, self.nb)
        self.interior = self.nb >= 0
        for (e, f) in self.hang:
            self.interior[e, f] = True
        self.mass_nq = mass_nq
        self.c_diss = float(c_diss)  # dissipative stabilisation D_h, c >= 0 (0 = off)
        if self.c_diss > 0.0 and self.hang:
            raise ValueError("D_h on meshes with hanging faces is not supported")
        self.nk = np.ones(self.ne, dtype=np.int64) if nk is None else np.asarray(nk, dtype=np.int64)
        if self.nk.shape != (self.ne,) or np.any(self.nk < 1) or np.any(self.nk & (self.nk - 1)):
            raise ValueError("nk: one power of two >= 1 per element (temporal bisection)")
        self.nt = self.nk * self.q           # test levels per element; trial levels nt + 1
        a3 = self.a ** 3
        self.trial_size = 6 * (self.nt + 1) * a3
        self.unk_size = 6 * self.nt * a3
        self.state_size = 6 * a3
        self.trial_off = np.concatenate([[0], np.cumsum(self.trial_size)])
        self.unk_off = np.concatenate([[0], np.cumsum(self.unk_size)])
        self.state_off = np.concatenate([[0], np.cumsum(self.state_size)])
        self._cache = {}

    # -- cached pieces ------------------------------------------------------
    def X(self, e):
        return self.vertices[self.hexes[e]]

    def nq(self, e):
        return int(self.a[e] + 1) if self.mass_nq is None else int(self.mass_nq)

    def mass(self, e, which):
        coef = self.eps[e] if which == "eps" else self.mu[e]
        X = self.X(e)
        key = ("M", int(self.a[e]), self.nq(e), float(coef),
               tuple(np.round((X - X[0]).ravel(), 14)))
        if key not in self._cache:
            self._cache[key] = mass_matrix(X, int(self.a[e]), coef, self.nq(e))
        return self._cache[key]

    def curl(self, a):
        key = ("C", int(a))
        if key not in self._cache:
            self._cache[key] = curl_matrix(int(a))
        return self._cache[key]

    def face(self, a, f, ao=None, neighbour=False):
        key = ("F", int(a), int(f), None if ao is None else int(ao), neighbour)
        if key not in self._cache:
            self._cache[key] = face_matrices(int(a), f, ao, neighbour)
        return self._cache[key]

    def tables(self, qt, qr):
        key = ("T", int(qt), int(qr))
        if key not in self._cache:
            self._cache[key] = basis.time_tables(int(qt), int(qr))
        return self._cache[key]

    def own_tables(self, e):
        """(D, N) of element e's own terms over the slab: D[I, M] = int L_I
        d_s phi_M and N[I, M] = int L_I phi_M (s the unit slab coordinate;
        with n sub-intervals the blocks of each sub-interval are D and N / n)."""
        qe, ne_ = int(self.q[e]), int(self.nk[e])
        if ne_ == 1:
            return self.tables(qe, qe)
        key = ("TO", qe, ne_)
        if key not in self._cache:
            self._cache[key] = (basis.subinterval_time_table(qe, ne_, qe, ne_, deriv=True),
                                basis.subinterval_time_table(qe, ne_, qe, ne_))
        return self._cache[key]

    def coupling_table(self, e, k, trial=None):
        """Time factor of the neighbour coupling of S_h (Section 4.1, eq.
        bilinearform:S): C[I, M] = int (pi L_I) phi_M over the slab, test
        function I of e projected onto the common temporal test space of e and
        k (piecewise degree < min(q_e, q_k) on the coarser of the two
        partitions), against the trial levels of ``trial`` (default k).
        With one sub-interval on both sides the projection keeps the test
        levels i < min(q_e, q_k) and removes the others."""
        trial = k if trial is None else trial
        qe, qk, qt = int(self.q[e]), int(self.q[k]), int(self.q[trial])
        ne_, nk_, nt_ = int(self.nk[e]), int(self.nk[k]), int(self.nk[trial])
        r, npj = min(qe, qk), min(ne_, nk_)
        if ne_ == 1 and nk_ == 1 and nt_ == 1:
            _, Nc = self.tables(qe, qt)
            Nc = Nc.copy()
            Nc[r:, :] = 0.0
            return Nc
        key = ("TC", qe, ne_, qt, nt_, r, npj)
        if key not in self._cache:
            self._cache[key] = basis.subinterval_time_table(qe, ne_, qt, nt_, proj=(r, npj))
        return self._cache[key]

    # -- spatial pieces of element e's own block ------------------------------
    def self_spatial(self, e):
        """(SE, SH): E-rows/H-cols and H-rows/E-cols spatial matrices of the
        diagonal block: -C^T + sum_f w_f FE_self and C + sum_f w_f FH_self with
        w_f = 1/2 on interior faces and 1 on boundary faces."""
        key = ("S", int(self.a[e]), tuple(self.interior[e]))
        if key not in self._cache:
            a = int(self.a[e])
            C = self.curl(a)
            SE = -C.T.copy()
            SH = C.copy()
            for f in range(6):
                FE, FH = self.face(a, f)
                wgt = 0.5 if self.interior[e, f] else 1.0
                SE += wgt * FE
                SH += wgt * FH
            self._cache[key] = (SE, SH)
        return self._cache[key]

    # -- blocks as lists of (time matrix, spatial matrix, row field, col field)
    def blocks(self, e, dt):
        """Terms of block row e: list of (col element, T, S, row field, col field)
        meaning rows [field_r][c][i][s] of e receive (T kron S) applied to the
        trial coefficients [field_c][d][m][t] of the column element."""
        a = int(self.a[e])
        D, N = self.own_tables(e)
        SE, SH = self.self_spatial(e)
        out = [(e, D, self.mass(e, "eps"), 0, 0),
               (e, dt * N, SE, 0, 1),
               (e, dt * N, SH, 1, 0),
               (e, D, self.mass(e, "mu"), 1, 1)]
        for f in range(6):
            for (k, fk, A, b, sub) in self.hang.get((e, f), ()):
                # a 2:1 hanging face: each neighbour couples over its part of the face
                ak = int(self.a[k])
                Nc = self.coupling_table(e, k)
                key = ("FH", a, f, ak, int(fk), tuple(np.ravel(A)), tuple(np.ravel(b)), sub)
                if key not in self._cache:
                    self._cache[key] = face_matrices_oriented(a, f, ak, int(fk), np.asarray(A, float),
                                                              np.asarray(b, float), sub)
                FE, FH = self._cache[key]
                out.append((k, dt * Nc, 0.5 * FE, 0, 1))
                out.append((k, dt * Nc, -0.5 * FH, 1, 0))
            k = int(self.nb[e, f])
            if k < 0:
                continue
            ak = int(self.a[k])
            Nc = self.coupling_table(e, k)       # S_h: neighbour coupling on the common test space
            if (e, f) in self.fmap:
                A, b = self.fmap[(e, f)]
                key = ("FO", a, f, ak, int(self.nbf[e, f]), tuple(A.ravel()), tuple(b))
                if key not in self._cache:
                    self._cache[key] = face_matrices_oriented(a, f, ak, int(self.nbf[e, f]), A, b)
                FE, FH = self._cache[key]
            else:
                FE, FH = self.face(a, f, ak, neighbour=True)
            out.append((k, dt * Nc, 0.5 * FE, 0, 1))
            out.append((k, dt * Nc, -0.5 * FH, 1, 0))
        if self.c_diss > 0.0:
            out += self.dissipation_blocks(e, dt)
        return out

    def dissipation_blocks(self, e, dt):
        """D_h (the dissipative remark after Section 4): on interior faces
        (alpha_E [E]_T, [pi v]_T) + (alpha_H [H]_T, [pi w]_T), the test function
        projected in time onto the common test space (levels i < min(q, q'),
        so rows i >= min(q, q') vanish for own and neighbour trial alike); on
        PEC faces (alpha_E [E]_T, [v]_T) with g = 0.  alpha_E = c / {sqrt(mu/eps)},
        alpha_H = c / {sqrt(eps/mu)}."""
        a = int(self.a[e])
        Xe = self.X(e)
        out = []
        ze, zh = np.sqrt(self.mu[e] / self.eps[e]), np.sqrt(self.eps[e] / self.mu[e])

        def face_mats(f, k):
            # cached by the shape of the pair (translation invariant)
            Xk = None if k < 0 else self.X(k)
            ak = None if k < 0 else int(self.a[k])
            fm = self.fmap.get((e, f))
            key = ("D", a, ak, f, tuple(np.round((Xe - Xe[0]).ravel(), 14)),
                   None if Xk is None else tuple(np.round((Xk - Xe[0]).ravel(), 14)),
                   None if fm is None else (int(self.nbf[e, f]), tuple(fm[0].ravel()), tuple(fm[1])))
            if key not in self._cache:
                self._cache[key] = dissipation_matrices(Xe, a, f, Xk, ak, nq=self.mass_nq,
                                                        face_o=None if fm is None else int(self.nbf[e, f]),
                                                        fmap=fm)
            return self._cache[key]

        for f in range(6):
            k = int(self.nb[e, f])
            if k < 0:
                _, N = self.own_tables(e)
                Ds, _ = face_mats(f, -1)
                out.append((e, dt * N, (self.c_diss / ze) * Ds, 0, 0))
                continue
            ak = int(self.a[k])
            aE = self.c_diss / (0.5 * (ze + np.sqrt(self.mu[k] / self.eps[k])))
            aH = self.c_diss / (0.5 * (zh + np.sqrt(self.eps[k] / self.mu[k])))
            Ds, Dn = face_mats(f, k)
            Ns = self.coupling_table(e, k, trial=e)
            Nk = self.coupling_table(e, k)
            out.append((e, dt * Ns, aE * Ds, 0, 0))
            out.append((e, dt * Ns, aH * Ds, 1, 1))
            out.append((k, dt * Nk, -aE * Dn, 0, 0))
            out.append((k, dt * Nk, -aH * Dn, 1, 1))
        return out

    # -- layout helpers ---------------------------------------------------------
    def split_trial(self, U, e):
        """[2][3 a^3][q+1] view-friendly reshape of element e's trial block ->
        array T[field, (d,t), m]."""
        a3 = int(self.a[e]) ** 3
        te = int(self.nt[e])
        blk = U[self.trial_off[e]:self.trial_off[e + 1]].reshape(2, 3, te + 1, a3)
        return blk.transpose(0, 1, 3, 2).reshape(2, 3 * a3, te + 1)

    def embed_unknowns(self, x, l0_state=None, elements=None):
        """Full trial vector from unknowns (m = 1..q) and an optional l_0 state.
        With ``elements`` only those blocks are filled (others left 0)."""
        U = np.zeros(self.trial_off[-1])
        for e in (range(self.ne) if elements is None else elements):
            e = int(e)
            a3 = int(self.a[e]) ** 3
            te = int(self.nt[e])
            blk = U[self.trial_off[e]:self.trial_off[e + 1]].reshape(2, 3, te + 1, a3)
            blk[:, :, 1:, :] = x[self.unk_off[e]:self.unk_off[e + 1]].reshape(2, 3, te, a3)
            if l0_state is not None:
                blk[:, :, 0, :] = l0_state[self.state_off[e]:self.state_off[e + 1]].reshape(2, 3, a3)
        return U

    def unknowns_of(self, U):
        x = np.zeros(self.unk_off[-1])
        for e in range(self.ne):
            a3 = int(self.a[e]) ** 3
            te = int(self.nt[e])
            blk = U[self.trial_off[e]:self.trial_off[e + 1]].reshape(2, 3, te + 1, a3)
            x[self.unk_off[e]:self.unk_off[e + 1]] = blk[:, :, 1:, :].ravel()
        return x

    def level_state(self, U, m):
        """State [field][comp][s] of trial level m of every element; m = 1 is the
        end-of-slab value (l_1(1) = 1, every other l_m(1) = 0), m = 0 the start."""
        S = np.zeros(self.state_off[-1])
        for e in range(self.ne):
            a3 = int(self.a[e]) ** 3
            te = int(self.nt[e])
            blk = U[self.trial_off[e]:self.trial_off[e + 1]].reshape(2, 3, te + 1, a3)
            S[self.state_off[e]:self.state_off[e + 1]] = blk[:, :, m, :].ravel()
        return S

    # -- residual -----------------------------------------------------------
    def apply_rows(self, U, dt, elements=None):
        """B_h(U, .) evaluated on the test functions of the listed elements
        (all by default).  Returns dict e -> residual block [field][c][i][s]."""
        if elements is None:
            elements = range(self.ne)
        res = {}
        for e in elements:
            e = int(e)
            te = int(self.nt[e])
            a3 = int(self.a[e]) ** 3
            Y = np.zeros((2, 3 * a3, te))
            for (k, T, S, fr, fc) in self.blocks(e, dt):
                Uk = self.split_trial(U, k)[fc]             # [(d,t), m]
                Y[fr] += S @ Uk @ T.T                       # (T kron S) u  =  S U T^T
            res[e] = Y.reshape(2, 3, a3, te).transpose(0, 1, 3, 2).ravel()
        return res

    def residual(self, U, dt, load=None, elements=None):
        """R_h = B_h(U, .) - L for a full trial vector U (Section 5, eq. residual).
        Returns the residual vector (all elements) or a dict for a subset."""
        rows = self.apply_rows(U, dt, elements)
        if elements is not None:
            if load is not None:
                for e in rows:
                    rows[e] = rows[e] - load[self.unk_off[e]:self.unk_off[e + 1]]
            return rows
        y = np.zeros(self.unk_off[-1])
        for e, v in rows.items():
            y[self.unk_off[e]:self.unk_off[e + 1]] = v
        if load is not None:
            y -= load
        return y

    def operator(self, x, dt, elements=None):
        """B_h applied to unknowns x (trial levels m >= 1), l_0 block zero."""
        return self.residual(self.embed_unknowns(x), dt, None, elements)

    # -- preconditioner (Section 5.4, eq. preconditioner) -----------------------
    def precond_solve(self, y, elements=None):
        """P^{-1} y with P the time-derivative terms restricted to the unknowns:
        block diagonal D_u kron the element mass matrix, D_u the columns m >= 1
        of the element's D (the identity with one sub-interval; with several,
        row (j, i) holds +1 at the level of l_{i+1} of sub-interval j, and row
        (j, 0), j > 0, also -1 at the value of node j, which is l_0 of
        sub-interval j).  With ``elements`` only those blocks are computed
        (others left 0)."""
        out = np.zeros_like(y)
        for e in (range(self.ne) if elements is None else elements):
            e = int(e)
            a3 = int(self.a[e]) ** 3
            te = int(self.nt[e])
            blk = y[self.unk_off[e]:self.unk_off[e + 1]].reshape(2, 3, te, a3)
            Du = self.own_tables(e)[0][:, 1:]
            res = np.zeros_like(blk)
            for fld, which in ((0, "eps"), (1, "mu")):
                M = self.mass(e, which)
                rhs = blk[fld].transpose(0, 2, 1).reshape(3 * a3, te)
                sol = np.linalg.solve(M, rhs)                  # [(c,s), I]
                if self.nk[e] > 1:                             # sum_m Du[I, m] x_m = z_I
                    sol = np.linalg.solve(Du, sol.T).T
                res[fld] = sol.reshape(3, a3, te).transpose(0, 2, 1)
            out[self.unk_off[e]:self.unk_off[e + 1]] = res.ravel()
        return out

    def precond_centre_solve(self, y, elements=None):
        """P_c^{-1} y with P_c the block mass taken with the metric at the element
        centre: kappa G(1/2, 1/2, 1/2) (x) I per level, G = |J| DF^{-1} DF^{-T}.
        On affine elements this is the exact P (orthonormal basis, constant
        metric); on trilinear ones it is the cheaper approximation of the block
        mass that the preconditioner may use (Section 5.4 leaves P's
        evaluation open; the converged slab solution does not depend on it)."""
        out = np.zeros_like(y)
        for e in (range(self.ne) if elements is None else elements):
            e = int(e)
            a3 = int(self.a[e]) ** 3
            te = int(self.nt[e])
            DF = jacobian(self.X(e), np.array([[0.5, 0.5, 0.5]]))[0]
            Di = np.linalg.inv(DF)
            G = np.linalg.det(DF) * Di @ Di.T
            Du = self.own_tables(e)[0][:, 1:]
            blk = y[self.unk_off[e]:self.unk_off[e + 1]].reshape(2, 3, te, a3)
            if self.nk[e] > 1:
                blk = np.einsum("mI,fcIs->fcms", np.linalg.inv(Du), blk)
            blk = blk.reshape(2, 3, te * a3)
            res = np.empty_like(blk)
            res[0] = np.linalg.solve(self.eps[e] * G, blk[0])
            res[1] = np.linalg.solve(self.mu[e] * G, blk[1])
            out[self.unk_off[e]:self.unk_off[e + 1]] = res.ravel()
        return out

    # -- inexact solve: dual norm of the residual and the iteration-error bound --
    def dual_norms(self, R, dt, elements=None):
        """(||R_E||^2, ||R_H||^2) in the dual of the test space W_h with the
        L2(I_n; L2(Omega)) norm (Section 5.3): the Riesz representor of a
        residual-layout vector R [f][c][i][s] solves (dt M_K) z_i = R_i per
        element and test level (test functions orthonormal in time on [0, 1],
        dx dt = dt dx dtau; with n sub-intervals each test function lives on
        one of length dt / n, so the factor is dt / n), M_K the unit-coefficient
        element mass; the norm is R . z."""
        out = np.zeros(2)
        for e in (range(self.ne) if elements is None else elements):
            e = int(e)
            a = int(self.a[e])
            a3 = a ** 3
            te = int(self.nt[e])
            key = ("M1", a, self.nq(e), tuple(np.round((self.X(e) - self.X(e)[0]).ravel(), 14)))
            if key not in self._cache:
                self._cache[key] = mass_matrix(self.X(e), a, 1.0, self.nq(e))
            M = self._cache[key]
            blk = R[self.unk_off[e]:self.unk_off[e + 1]].reshape(2, 3, te, a3)
            for f in range(2):
                rhs = blk[f].transpose(0, 2, 1).reshape(3 * a3, te)
                z = np.linalg.solve(M, rhs) / (dt / int(self.nk[e]))
                out[f] += float(np.sum(rhs * z))
        return out

    def eta_it_term(self, R, dt, t_final):
        """One slab's contribution to eta_it^2 (eq. a_posteriori:iteration,
        taken as printed): 4 [(2 t_N / eps_min + dt^2 / (2 t_N eps_min)) ||R_E||^2
        + (2 t_N / mu_min + dt^2 / (2 t_N mu_min)) ||R_H||^2]."""
        rE, rH = self.dual_norms(R, dt)
        em, mm = float(np.min(self.eps)), float(np.min(self.mu))
        return 4.0 * ((2 * t_final / em + dt ** 2 / (2 * t_final * em)) * rE +
                      (2 * t_final / mm + dt ** 2 / (2 * t_final * mm)) * rH)

    # -- energy (eq. stability:energydef) -------------------------------------
    def energy(self, state):
        """1/2 int (eps E.E + mu H.H) of a state [field][comp][s] per element."""
        tot = 0.0
        for e in range(self.ne):
            a3 = int(self.a[e]) ** 3
            blk = state[self.state_off[e]:self.state_off[e + 1]].reshape(2, 3 * a3)
            tot += 0.5 * (blk[0] @ self.mass(e, "eps") @ blk[0] + blk[1] @ self.mass(e, "mu") @ blk[1])
        return tot

    # -- load (eq. bilinearform:C, l_E(v) = (J, v)) ----------------------------
    def load(self, J, t0, dt, nx=None, nt=None):
        """L_E[c, i, s] = int_{I_n} int_K J . (DF^{-T} e_c phi_s) L_i dx dt by
        tensor Gauss quadrature (p + 3 points per space direction, q + 3 in
        time per sub-interval unless given); the H part is zero (g = 0).
        J(x [P,3], t) -> [P,3]."""
        L = np.zeros(self.unk_off[-1])
        for e in range(self.ne):
            L[self.unk_off[e]:self.unk_off[e + 1]] = self._load_block(e, J, t0, dt, nx, nt)
        return L

    def load_rows(self, J, t0, dt, elements, nx=None, nt=None):
        """The load blocks of the given elements only: {e: block}, each as in load()."""
        return {int(e): self._load_block(int(e), J, t0, dt, nx, nt) for e in elements}

    def _load_block(self, e, J, t0, dt, nx, nt):
        a = int(self.a[e])
        qe = int(self.q[e])
        nsub = int(self.nk[e])
        n = a + 2 if nx is None else nx
        m = qe + 3 if nt is None else nt
        pts, w = tensor_points(n)
        tx, tw = basis.gauss01(m)
        X = self.X(e)
        x = map_point(X, pts)
        DF = jacobian(X, pts)
        det = np.linalg.det(DF)
        Dinv = np.linalg.inv(DF)
        Phi, _ = basis_at(a, pts)
        acc = np.zeros((3, nsub * qe, a ** 3))
        for j in range(nsub):
            for tau, wt in zip(tx, tw):
                Jv = J(x, t0 + (j + tau) * dt / nsub)           # [P, 3]
                # J . DF^{-T} e_c = (DF^{-1} J)_c
                Jr = np.einsum("pcm,pm->pc", Dinv, Jv) * (det * w)[:, None]
                proj = Jr.T @ Phi                               # [3, a^3]
                for i in range(qe):
                    acc[:, j * qe + i, :] += (dt / nsub) * wt * basis.L(i, tau) * proj
        blk = np.zeros((2, 3, nsub * qe, a ** 3))
        blk[0] = acc
        return blk.ravel()

    # -- global sparse slab matrix (tiny meshes) --------------------------------
    def slab_matrix(self, dt):
        """Sparse B with rows = test dofs (residual layout), cols = full trial dofs."""
        rows, cols, vals = [], [], []
        for e in range(self.ne):
            te = int(self.nt[e])
            a3 = int(self.a[e]) ** 3
            for (k, T, S, fr, fc) in self.blocks(e, dt):
                tk = int(self.nt[k])
                ak3 = int(self.a[k]) ** 3
                S4 = S.reshape(3, a3, 3, ak3)
                Bk = np.einsum("im,csdt->cisdmt", T, S4).reshape(3 * te * a3, 3 * (tk + 1) * ak3)
                r0 = self.unk_off[e] + fr * 3 * te * a3
                c0 = self.trial_off[k] + fc * 3 * (tk + 1) * ak3
                ii, jj = np.nonzero(Bk)
                rows.append(r0 + ii)
                cols.append(c0 + jj)
                vals.append(Bk[ii, jj])
        rows = np.concatenate(rows)
        cols = np.concatenate(cols)
        vals = np.concatenate(vals)
        return sp.csr_matrix((vals, (rows, cols)), shape=(self.unk_off[-1], self.trial_off[-1]))

    def unknown_columns(self):
        """Boolean mask over trial dofs: True for m >= 1."""
        mask = np.zeros(self.trial_off[-1], dtype=bool)
        for e in range(self.ne):
            a3 = int(self.a[e]) ** 3
            te = int(self.nt[e])
            blk = mask[self.trial_off[e]:self.trial_off[e + 1]].reshape(2, 3, te + 1, a3)
            blk[:, :, 1:, :] = True
        return mask

    # -- slab solve (Section 3, eq. weakform / Section 4, eq. weakform_stabilized)
    def solve_direct(self, state0, dt, load=None):
        """Find U with l_0 block = state0 and B_h(U, V) = L(V) for all V, by a
        sparse direct solve.  Returns the full trial vector."""
        B = self.slab_matrix(dt)
        mask = self.unknown_columns()
        U0 = self.embed_unknowns(np.zeros(self.unk_off[-1]), state0)
        b = -(B @ U0)
        if load is not None:
            b = b + load
        Bu = B[:, mask].tocsc()
        x = spla.spsolve(Bu, b)
        return self.embed_unknowns(x, state0)

    def solve_gmres(self, state0, dt, load=None, rtol=1e-13, restart=10, maxiter=2000):
        """Same problem, right-preconditioned restarted GMRES on the oracle's own
        block apply, with P = the time-derivative terms (eq. preconditioner)."""
        n = int(self.unk_off[-1])
        U0 = self.embed_unknowns(np.zeros(n), state0)
        b = -self.residual(U0, dt)
        if load is not None:
            b = b + load
        Aop = spla.LinearOperator((n, n), matvec=lambda z: self.operator(self.precond_solve(z), dt))
        z, info = spla.gmres(Aop, b, rtol=rtol, atol=0.0, restart=restart, maxiter=maxiter)
        if info != 0:
            raise RuntimeError("oracle GMRES did not converge (info=%d)" % info)
        x = self.precond_solve(z)
        return self.embed_unknowns(x, state0)

    # -- spatial semi-discrete operators (for the time-discretisation pin) ------
    def spatial_operators(self):
        """(M, K) of the semi-discrete system M u' + K u = 0 on states
        [field][comp][s]: M = blockdiag(M_eps, M_mu) and K the curl + centred
        flux operator (uniform q only; conforming faces)."""
        if self.hang:
            raise ValueError("spatial_operators: hanging faces are not supported")
        n = int(self.state_off[-1])
        M = np.zeros((n, n))
        K = np.zeros((n, n))
        for e in range(self.ne):
            a3 = int(self.a[e]) ** 3
            r = self.state_off[e]
            M[r:r + 3 * a3, r:r + 3 * a3] = self.mass(e, "eps")
            M[r + 3 * a3:r + 6 * a3, r + 3 * a3:r + 6 * a3] = self.mass(e, "mu")
            SE, SH = self.self_spatial(e)
            K[r:r + 3 * a3, r + 3 * a3:r + 6 * a3] += SE
            K[r + 3 * a3:r + 6 * a3, r:r + 3 * a3] += SH
            for f in range(6):
                k = int(self.nb[e, f])
                if k < 0:
                    continue
                ak3 = int(self.a[k]) ** 3
                c = self.state_off[k]
                FE, FH = self.face(int(self.a[e]), f, int(self.a[k]), neighbour=True)
                K[r:r + 3 * a3, c + 3 * ak3:c + 6 * ak3] += 0.5 * FE
                K[r + 3 * a3:r + 6 * a3, c:c + 3 * ak3] += -0.5 * FH
        return M, K
