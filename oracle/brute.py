"""Physical-space brute-force assembler of the slab bilinear form (oracle step O7).

Written separately from ``dg`` to pin it: nothing here uses the reference-space
shortcuts of ``dg``.  Every entry B_h(phi_a, psi_b) of the slab matrix is
integrated in physical space-time with

* covariantly mapped basis functions v = DF^{-T}(x-hat) e_c phi_s(x-hat)
  (Section 2.3), evaluated at physical quadrature points;
* the physical curl by the chain rule, including the derivative of DF^{-T}
  (no Piola identity);
* physical face normals and surface measures from the tangent vectors of the
  trilinear map, oriented away from the element;
* neighbour traces at the same physical points, found by Newton inversion of
  the neighbour's map; faces are matched by physical centroid (2:1
  hanging faces by their quarter centroids, the coarse face integrated
  quarter by quarter);
* the average / tangential-jump operators of Section 2.4 and the terms of
  C_h (eq. bilinearform:C), S_h (eq. bilinearform:S) and the dissipative D_h
  (the remark after Section 4) as written, with the temporal L2 projection
  pi-tilde computed by quadrature from the Gram matrix of a basis of the
  common test space (piecewise polynomials on the coarser of two nested
  partitions when slab intervals are bisected, Section 2.2);
* its own Legendre evaluation by the three-term recurrence.

Only tiny meshes are feasible (dense matrices, many quadrature points).
"""
import numpy as np
from numpy.polynomial.legendre import leggauss


def _gauss(n):
    x, w = leggauss(int(n))
    return 0.5 * (x + 1.0), 0.5 * w


def _legendre_all(nmax, xi):
    """Orthonormal Legendre on [0,1] and derivatives, degrees 0..nmax, by
    Bonnet's recurrence on u = 2 xi - 1: values V[..., n], derivatives dV[..., n]."""
    u = 2.0 * np.asarray(xi, dtype=np.float64) - 1.0
    P = [np.ones_like(u), u.copy()]
    dP = [np.zeros_like(u), np.ones_like(u)]
    for n in range(1, nmax):
        P.append(((2 * n + 1) * u * P[n] - n * P[n - 1]) / (n + 1))
        dP.append(dP[n - 1] + (2 * n + 1) * P[n])
    P, dP = P[:nmax + 1], dP[:nmax + 1]
    V = np.stack([np.sqrt(2 * n + 1) * P[n] for n in range(nmax + 1)], axis=-1)
    dV = np.stack([2.0 * np.sqrt(2 * n + 1) * dP[n] for n in range(nmax + 1)], axis=-1)
    return V, dV, P


def _time_functions(q, tau):
    """Trial l_m (m = 0..q) with d/dtau, and test L_i (i = 0..q-1) at tau."""
    V, _, P = _legendre_all(max(q, 1) + 1, tau)
    u = 2.0 * tau - 1.0
    lt = [1.0 - tau, tau.copy()]
    dlt = [-np.ones_like(tau), np.ones_like(tau)]
    for m in range(2, q + 1):
        # int_0^tau sqrt(2m-1) P_{m-1}(2s-1) ds = sqrt(2m-1)/2 * (P_m(u) - P_{m-2}(u)) / (2m-1)
        lt.append(np.sqrt(2 * m - 1) * 0.5 * (P[m] - P[m - 2]) / (2 * m - 1))
        dlt.append(V[..., m - 1])
    return np.stack(lt, -1), np.stack(dlt, -1), V[..., :q]


def _level(q, n, j, m):
    """Column of local trial function l_m of sub-interval j in the flattened
    block of 1 + n q trial levels (the layout of the slab matrix's columns):
    0 = slab start, 1 = slab end, then per sub-interval its l_2..l_q and the
    value at its right end if that end is interior."""
    if m == 0:
        return 0 if j == 0 else 1 + j * q
    if m == 1:
        return 1 if j == n - 1 else 1 + (j + 1) * q
    return 2 + j * q + m - 2


def _slab_functions(q, n, tau):
    """At slab coordinates tau (inside sub-intervals of every partition in
    use): flattened trial functions [tau, 1 + n q] with d/dtau, and test
    functions [tau, n q], L_i(n tau - j) on sub-interval j."""
    j = np.minimum(np.floor(tau * n).astype(np.int64), n - 1)
    xi = tau * n - j
    lt, dlt, Lt = _time_functions(q, xi)
    trial = np.zeros((tau.size, 1 + n * q))
    dtrial = np.zeros_like(trial)
    test = np.zeros((tau.size, n * q))
    for p in range(tau.size):
        for m in range(q + 1):
            trial[p, _level(q, n, int(j[p]), m)] += lt[p, m]
            dtrial[p, _level(q, n, int(j[p]), m)] += n * dlt[p, m]
        test[p, j[p] * q:(j[p] + 1) * q] = Lt[p, :q]
    return trial, dtrial, test


class _Element:
    def __init__(self, X, a):
        self.X = np.asarray(X, dtype=np.float64)
        self.a = int(a)
        self.c = self.X.mean(axis=0)

    def _shape(self, xh):
        P = xh.shape[0]
        N = np.ones((P, 8))
        dN = np.ones((P, 8, 3))
        d2 = np.zeros((P, 8, 3, 3))
        for v in range(8):
            b = [(v >> d) & 1 for d in range(3)]
            f = [xh[:, d] if b[d] else 1.0 - xh[:, d] for d in range(3)]
            s = [1.0 if b[d] else -1.0 for d in range(3)]
            N[:, v] = f[0] * f[1] * f[2]
            dN[:, v, 0] = s[0] * f[1] * f[2]
            dN[:, v, 1] = f[0] * s[1] * f[2]
            dN[:, v, 2] = f[0] * f[1] * s[2]
            d2[:, v, 0, 1] = d2[:, v, 1, 0] = s[0] * s[1] * f[2]
            d2[:, v, 0, 2] = d2[:, v, 2, 0] = s[0] * s[2] * f[1]
            d2[:, v, 1, 2] = d2[:, v, 2, 1] = s[1] * s[2] * f[0]
        return N, dN, d2

    def geometry(self, xh):
        N, dN, d2 = self._shape(xh)
        x = N @ self.X
        DF = np.einsum("pvm,vi->pim", dN, self.X)
        HF = np.einsum("pvmn,vi->pimn", d2, self.X)        # d^2 F_i / dxm dxn
        return x, DF, HF

    def invert(self, x, iters=60):
        """Newton solve of F(x-hat) = x."""
        xh = np.full_like(x, 0.5)
        for _ in range(iters):
            xp, DF, _ = self.geometry(xh)
            r = xp - x
            xh = xh - np.linalg.solve(DF, r[..., None])[..., 0]
            if np.abs(r).max() < 1e-15:
                break
        return xh

    def fields(self, xh, with_curl=True):
        """Physical values of all spatial basis fields DF^{-T} e_c phi_s at x-hat
        -> val [P, 3 a^3, 3] (index c * a^3 + s), curl [P, 3 a^3, 3], |J| [P]."""
        a = self.a
        x, DF, HF = self.geometry(xh)
        det = np.linalg.det(DF)
        Dinv = np.linalg.inv(DF)                       # Dinv[p, m, j] = (DF^{-1})_{mj}
        DinvT = np.transpose(Dinv, (0, 2, 1))          # (DF^{-T})_{kc}
        Vx, dVx, _ = _legendre_all(a - 1, xh[:, 0])
        Vy, dVy, _ = _legendre_all(a - 1, xh[:, 1])
        Vz, dVz, _ = _legendre_all(a - 1, xh[:, 2])
        Vx, Vy, Vz = Vx[:, :a], Vy[:, :a], Vz[:, :a]
        dVx, dVy, dVz = dVx[:, :a], dVy[:, :a], dVz[:, :a]
        P = xh.shape[0]
        phi = np.einsum("pl,pk,pj->plkj", Vz, Vy, Vx).reshape(P, a ** 3)
        dphi = np.stack([np.einsum("pl,pk,pj->plkj", Vz, Vy, dVx).reshape(P, a ** 3),
                         np.einsum("pl,pk,pj->plkj", Vz, dVy, Vx).reshape(P, a ** 3),
                         np.einsum("pl,pk,pj->plkj", dVz, Vy, Vx).reshape(P, a ** 3)], -1)
        val = np.einsum("pkc,ps->pcsk", DinvT, phi).reshape(P, 3 * a ** 3, 3)
        if not with_curl:
            return x, val, None, det
        # d(DF^{-T})/dx-hat_m = -DF^{-T} (dDF/dx-hat_m)^T DF^{-T}
        dDinvT = np.zeros((P, 3, 3, 3))                # [p, m, k, c]
        for m in range(3):
            dDF_m = HF[:, :, m, :]                     # [p, i, n]
            dDinvT[:, m] = -np.einsum("pki,pni,pnc->pkc", DinvT, dDF_m, DinvT)
        # dv_k/dx-hat_m for field (c, s)
        dv = (np.einsum("pmkc,ps->pcskm", dDinvT, phi)
              + np.einsum("pkc,psm->pcskm", DinvT, dphi))   # [p, c, s, k, m]
        grad = np.einsum("pcskm,pmj->pcskj", dv, Dinv)      # dv_k / dx_j
        curl = np.stack([grad[..., 2, 1] - grad[..., 1, 2],
                         grad[..., 0, 2] - grad[..., 2, 0],
                         grad[..., 1, 0] - grad[..., 0, 1]], axis=-1)
        return x, val, curl.reshape(P, 3 * a ** 3, 3), det


def _face_param(face, uv):
    alpha, side = divmod(face, 2)
    tang = [d for d in range(3) if d != alpha]
    xh = np.zeros((uv.shape[0], 3))
    xh[:, alpha] = side
    xh[:, tang[0]] = uv[:, 0]
    xh[:, tang[1]] = uv[:, 1]
    return xh, tang


def assemble(vertices, hexes, p, q, eps, mu, dt, nvol_extra=2, nface_extra=2, nt=None, c_diss=0.0, nk=None):
    """Dense slab matrix B[test dof, trial dof] of B_h = C_h + S_h (+ D_h for
    c_diss > 0) by physical quadrature.  Element e's slab interval is bisected
    into nk[e] equal sub-intervals (powers of two, default 1; Section 2.2).
    Row layout per element [field][c][(j, i)][s] (i < q on sub-interval j);
    column layout per element [field][d][m][t] over the 1 + nk q flattened
    trial levels of ``_level``."""
    vertices = np.asarray(vertices, dtype=np.float64)
    hexes = np.asarray(hexes)
    ne = hexes.shape[0]
    a = np.asarray(p, dtype=np.int64) + 1
    q = np.asarray(q, dtype=np.int64)
    nk = np.ones(ne, dtype=np.int64) if nk is None else np.asarray(nk, dtype=np.int64)
    ntest = nk * q
    els = [_Element(vertices[hexes[e]], a[e]) for e in range(ne)]
    roff = np.concatenate([[0], np.cumsum(6 * ntest * a ** 3)])
    coff = np.concatenate([[0], np.cumsum(6 * (ntest + 1) * a ** 3)])
    B = np.zeros((roff[-1], coff[-1]))
    ntq = (int(q.max()) + 3) if nt is None else nt
    # composite Gauss rule on the finest partition (all partitions nest in it)
    nfine = int(nk.max())
    g0, w0 = _gauss(ntq)
    tg = ((np.arange(nfine)[:, None] + g0[None, :]) / nfine).ravel()
    tw = np.tile(w0, nfine) / nfine

    def time_int(er, ec, kind, proj=None):
        """Integrals over the slab (t = t0 + dt tau) of the test functions of
        element er against the trial functions of element ec: 'D' -> int L d_t l
        dt, 'N' -> int L l dt, 'Nd' -> int (pi L - L) l dt with pi the L2
        projection onto proj = (r, n_p): piecewise polynomials of degree < r
        on n_p equal sub-intervals, by its Gram matrix."""
        _, _, Lt = _slab_functions(int(q[er]), int(nk[er]), tg)
        lt, dlt, _ = _slab_functions(int(q[ec]), int(nk[ec]), tg)
        if kind == "D":
            return (Lt * (tw * dt)[:, None]).T @ (dlt / dt)
        if kind == "N":
            return (Lt * (tw * dt)[:, None]).T @ lt
        r, npj = proj
        _, _, Bp = _slab_functions(r, npj, tg)              # a basis of the projection space
        G = (Bp * tw[:, None]).T @ Bp
        piL = Bp @ np.linalg.solve(G, (Bp * tw[:, None]).T @ Lt)
        return ((piL - Lt) * (tw * dt)[:, None]).T @ lt

    def put(e_row, fr, e_col, fc, T, S):
        ar3, ac3 = int(a[e_row]) ** 3, int(a[e_col]) ** 3
        qr, qc = int(ntest[e_row]), int(ntest[e_col])
        blk = np.einsum("im,csdt->cisdmt", T, S.reshape(3, ar3, 3, ac3)).reshape(3 * qr * ar3, 3 * (qc + 1) * ac3)
        r0 = roff[e_row] + fr * 3 * qr * ar3
        c0 = coff[e_col] + fc * 3 * (qc + 1) * ac3
        B[r0:r0 + blk.shape[0], c0:c0 + blk.shape[1]] += blk

    # volume terms
    for e in range(ne):
        el = els[e]
        n = int(a[e]) + nvol_extra
        g, w = _gauss(n)
        Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
        WZ, WY, WX = np.meshgrid(w, w, w, indexing="ij")
        xh = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
        wt = (WX * WY * WZ).ravel()
        _, val, curl, det = el.fields(xh)
        dx = wt * det
        mass = np.einsum("p,pak,pbk->ab", dx, val, val)
        curl_test = np.einsum("p,pak,pbk->ab", dx, curl, val)    # int curl(v_a) . u_b
        curl_trial = np.einsum("p,pak,pbk->ab", dx, val, curl)   # int w_a . curl(u_b)
        Dt = time_int(e, e, "D")
        Nt = time_int(e, e, "N")
        put(e, 0, e, 0, Dt, eps[e] * mass)            # (eps d_t E, v)
        put(e, 1, e, 1, Dt, mu[e] * mass)             # (mu d_t H, w)
        put(e, 0, e, 1, Nt, -curl_test)               # -(H, curl v)
        put(e, 1, e, 0, Nt, curl_trial)               # (curl E, w)

    # faces, matched by physical centroid
    def fkey(e, f):
        alpha, side = divmod(f, 2)
        ids = [v for v in range(8) if ((v >> alpha) & 1) == side]
        return tuple(np.round(vertices[hexes[e][ids]].mean(axis=0), 10))

    where = {}
    for e in range(ne):
        for f in range(6):
            where.setdefault(fkey(e, f), []).append((e, f))

    # 2:1 hanging faces, matched by physical centroids as well: a face whose
    # four quarter centroids are centroids of four other faces is the coarse
    # side; a face whose centroid is a quarter centroid of another face is a
    # fine side
    def quarter_keys(e, f):
        out = []
        for iv in range(2):
            for iu in range(2):
                xh, _ = _face_param(f, np.array([[(iu + 0.5) / 2, (iv + 0.5) / 2]]))
                x, _, _ = els[e].geometry(xh)
                out.append(((0.5 * iu, 0.5 * iv), tuple(np.round(x[0], 10))))
        return out

    quarter_of = {}
    for e in range(ne):
        for f in range(6):
            for sub, key in quarter_keys(e, f):
                quarter_of.setdefault(key, []).append((e, f))

    def pieces(e, f):
        """(neighbour or -1, own-face sub-square origin or None) pieces of face f of e"""
        partners = [(k, g) for (k, g) in where[fkey(e, f)] if (k, g) != (e, f)]
        if partners:
            return [(partners[0][0], None)]
        quarters = []
        for sub, key in quarter_keys(e, f):
            fine = [(k, g) for (k, g) in where.get(key, []) if k != e]
            if len(fine) == 1:
                quarters.append((fine[0][0], sub))
        if len(quarters) == 4:
            return quarters
        coarse = [(k, g) for (k, g) in quarter_of.get(fkey(e, f), []) if k != e]
        if len(coarse) == 1:
            return [(coarse[0][0], None)]
        return [(-1, None)]

    for e in range(ne):
        el = els[e]
        for f in range(6):
          for k, sub in pieces(e, f):
            nf = max(int(a[e]), int(a[k]) if k >= 0 else 0) + nface_extra
            g1, w1 = _gauss(nf)
            V, U = np.meshgrid(g1, g1, indexing="ij")
            WV, WU = np.meshgrid(w1, w1, indexing="ij")
            uv = np.stack([U.ravel(), V.ravel()], 1)
            wuv = (WU * WV).ravel()
            if sub is not None:
                uv = np.asarray(sub)[None, :] + 0.5 * uv
                wuv = 0.25 * wuv
            xh, tang = _face_param(f, uv)
            x, DF, _ = el.geometry(xh)
            tu, tv = DF[:, :, tang[0]], DF[:, :, tang[1]]
            nv = np.cross(tu, tv)
            dS = np.linalg.norm(nv, axis=1)
            n1 = nv / dS[:, None]
            sgn = np.sign(np.einsum("pi,pi->p", n1, x - el.c[None, :]))
            n1 = n1 * sgn[:, None]
            wS = wuv * dS
            _, v1, _, _ = el.fields(xh, with_curl=False)
            n1xv1 = np.cross(n1[:, None, :], v1)
            if k < 0:
                Nt = time_int(e, e, "N")
                Pb = np.einsum("p,pbk,pak->ab", wS, v1, n1xv1)        # int u . (n x v)
                Rb = np.einsum("p,pbk,pak->ab", wS, np.cross(n1[:, None, :], v1), v1)  # int (n x u) . w
                put(e, 0, e, 1, Nt, Pb)
                put(e, 1, e, 0, Nt, -Rb)
                if c_diss > 0.0:
                    # D_h on the PEC face: (alpha_E [E]_T, [v]_T), [u]_T = n x u, g = 0
                    aE = c_diss / np.sqrt(mu[e] / eps[e])
                    put(e, 0, e, 0, Nt, aE * np.einsum("p,pak,pbk->ab", wS, n1xv1, n1xv1))
                continue
            elk = els[k]
            xh2 = elk.invert(x)
            _, v2, _, _ = elk.fields(xh2, with_curl=False)
            n2 = -n1
            # the common temporal test space of the two sides (Section 4.1)
            proj = (min(int(q[e]), int(q[k])), min(int(nk[e]), int(nk[k])))
            for side_l, (kk, ul, nl) in enumerate(((e, v1, n1), (k, v2, n2))):
                Nt = time_int(e, kk, "N")
                Nd = time_int(e, kk, "Nd", proj)
                Pl = 0.5 * np.einsum("p,pbk,pak->ab", wS, ul, n1xv1)              # 1/2 int u_l . (n1 x v1)
                Ql = 0.5 * np.einsum("p,pbk,pak->ab", wS, np.cross(nl[:, None, :], ul), v1)  # 1/2 int (n_l x u_l) . v1
                # E-row: ({H}, [v]_T) + 1/2 (({H}, [dv]_T) + ([H]_T, {dv}))
                put(e, 0, kk, 1, Nt, Pl)
                put(e, 0, kk, 1, Nd, 0.5 * (Pl + Ql))
                # H-row: -([E]_T, {w}) - 1/2 (({E}, [dw]_T) + ([E]_T, {dw}))
                put(e, 1, kk, 0, Nt, -Ql)
                put(e, 1, kk, 0, Nd, -0.5 * (Pl + Ql))
                if c_diss > 0.0:
                    # D_h: (alpha [U]_T, [pi v]_T): the time-projected test function
                    # pi L_i = L_i + (pi L_i - L_i) gives the N + Nd time factors
                    aE = c_diss / (0.5 * (np.sqrt(mu[e] / eps[e]) + np.sqrt(mu[k] / eps[k])))
                    aH = c_diss / (0.5 * (np.sqrt(eps[e] / mu[e]) + np.sqrt(eps[k] / mu[k])))
                    J = np.einsum("p,pak,pbk->ab", wS, n1xv1, np.cross(nl[:, None, :], ul))  # int (n1 x v1) . (n_l x u_l)
                    put(e, 0, kk, 0, Nt + Nd, aE * J)
                    put(e, 1, kk, 1, Nt + Nd, aH * J)
    return B
