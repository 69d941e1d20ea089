"""The five synthetic workloads, as seeded parameter sets.

Only parameters are produced here (meshes, degrees, materials, source and
initial-field parameters, arrival times, random vectors).  How a source is
integrated or an initial field projected is discretisation arithmetic and is
implemented separately by the library and by the oracle.
"""
from dataclasses import dataclass, field

import numpy as np

from .meshes import Mesh, box_mesh, perturb_interior, centroids


@dataclass
class Source:
    """Current density J(x, t) = dir * amp * exp(-|x-center|^2 / (2 sigma_x^2))
    * sin(2 pi f0 (t - t0)) * exp(-(t - t0)^2 / (2 sigma_t^2)).
    kind 0 = no source; kind 1 = the Gaussian pulse above."""
    kind: int = 0
    amp: float = 1.0
    center: tuple = (0.5, 0.5, 0.5)
    sigma_x: float = 0.05
    f0: float = 4.0
    t0: float = 0.0
    sigma_t: float = 1.0
    dir: tuple = (0.0, 0.0, 1.0)


@dataclass
class ModeSet:
    """Superposition of PEC-compatible cavity fields on the unit cube:
    E = sum_r (A_r cos(m pi x) sin(n pi y) sin(l pi z),
               B_r sin(m pi x) cos(n pi y) sin(l pi z),
               C_r sin(m pi x) sin(n pi y) cos(l pi z)),  H = 0."""
    mnl: np.ndarray = field(default_factory=lambda: np.zeros((0, 3), dtype=np.int64))
    abc: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))


CAVITY_MODES = np.array([(1, 0, 1), (0, 1, 1), (1, 1, 0), (1, 1, 1),
                         (2, 1, 1), (1, 2, 1), (1, 1, 2), (2, 2, 1)], dtype=np.int64)


def mode_superposition(seed):
    """8 cavity fields; polarisation g - (g.k)k with g ~ N(0, I3) (k the unit
    wave vector), normalised, then scaled by an N(0, 1) amplitude."""
    rng = np.random.default_rng(seed)
    abc = np.zeros((len(CAVITY_MODES), 3))
    for r, k in enumerate(CAVITY_MODES):
        kk = k / np.linalg.norm(k)
        g = rng.standard_normal(3)
        g = g - (g @ kk) * kk
        g = g / np.linalg.norm(g)
        abc[r] = g * rng.standard_normal()
    return ModeSet(mnl=CAVITY_MODES.copy(), abc=abc)


def random_vector(n, seed):
    """N(0, 1) float64 vector of length n from numpy's PCG64 with the given seed."""
    return np.random.default_rng(seed).standard_normal(int(n))


def _lattice(n):
    v, h = box_mesh((n, n, n))
    return v, h


def cavity_small():
    """PEC unit cube, 4x4x4 axis-aligned hexahedra, eps = mu = 1, p = 2, q = 1,
    one slab of dt = 0.05; initial data is the TE101 mode."""
    v, h = _lattice(4)
    ne = h.shape[0]
    mesh = Mesh(v, h, np.full(ne, 2, np.int32), np.full(ne, 1, np.int32),
                np.ones(ne), np.ones(ne), shape=(4, 4, 4))
    return dict(name="cavity 4^3 p2 q1", mesh=mesh, dt=0.05, n_slabs=1, source=Source(),
                init="te101")


def cavity_two_material(n=32, p=4, q=3, seed=0):
    """PEC unit cube, n^3 axis-aligned hexahedra, uniform p, q; eps = 1 where
    the element centroid has x < 0.5, else 4; mu = 1; 64 slabs of dt = 0.01;
    initial E a seeded superposition of 8 cavity fields, H = 0."""
    v, h = _lattice(n)
    ne = h.shape[0]
    c = centroids(v, h)
    eps = np.where(c[:, 0] < 0.5, 1.0, 4.0)
    mesh = Mesh(v, h, np.full(ne, p, np.int32), np.full(ne, q, np.int32),
                eps, np.ones(ne), shape=(n, n, n))
    return dict(name=f"cavity {n}^3 p{p} q{q} two-material", mesh=mesh, dt=0.01,
                n_slabs=64, source=Source(), init=mode_superposition(seed))


def local_time_cavity(n=32, p=4, q=3, seed=0):
    """The two-material cavity (eps = 1 for centroid x < 0.5, else 4; mu = 1)
    with local time steps in the faster material: 4 sub-intervals per slab
    where x < 0.25, 2 where 0.25 <= x < 0.5, 1 in the eps = 4 half (the
    1 / 2 / 4 local steps of the paper's local-refinement experiments);
    16 slabs of dt = 0.01 from a seeded superposition of 8 cavity fields."""
    cfg = cavity_two_material(n, p, q, seed)
    m = cfg["mesh"]
    c = centroids(m.vertices, m.hexes)
    m.nsub = np.where(c[:, 0] < 0.25, 4, np.where(c[:, 0] < 0.5, 2, 1)).astype(np.int32)
    cfg["name"] = f"cavity {n}^3 p{p} q{q} two-material, local time steps 4/2/1"
    cfg["n_slabs"] = 16
    return cfg


def graded_nonaffine(n=24, seed=0, n_slabs=40, dt=0.005):
    """Unit cube, n^3 trilinear hexahedra with interior vertices perturbed by
    U(-0.1 h, 0.1 h) per coordinate; ring k = min(3, floor(d / 0.125)) with d the
    infinity-norm distance of the unperturbed centroid from the centre; p = 6 - k,
    q = p - 2; eps = mu = 1; Gaussian-pulse J along z at the centre."""
    v0, h = _lattice(n)
    c0 = centroids(v0, h)
    d = np.abs(c0 - 0.5).max(axis=1)
    ring = np.minimum(3, np.floor(d / 0.125 + 1e-12).astype(np.int64))
    p = (6 - ring).astype(np.int32)
    q = (p - 2).astype(np.int32)
    v = perturb_interior(v0, (n, n, n), 0.1, seed)
    ne = h.shape[0]
    mesh = Mesh(v, h, p, q, np.ones(ne), np.ones(ne), shape=(n, n, n))
    T = n_slabs * dt
    src = Source(kind=1, amp=1.0, center=(0.5, 0.5, 0.5), sigma_x=0.05, f0=4.0,
                 t0=T / 2, sigma_t=T / 4, dir=(0.0, 0.0, 1.0))
    return dict(name=f"graded non-affine {n}^3 p3..6", mesh=mesh, dt=dt, n_slabs=n_slabs,
                source=src, init="zero")


def large_cavity(n=48, p=6, q=4, seed=0, n_slabs=32):
    """PEC unit cube, n^3 axis-aligned hexahedra, p = 6, q = 4, eps ~ U[1, 4] per
    element, mu = 1, dt = h / (2p + 1), dipole Gaussian-pulse J at the centre."""
    v, h = _lattice(n)
    ne = h.shape[0]
    rng = np.random.default_rng(seed)
    eps = rng.uniform(1.0, 4.0, size=ne)
    dt = (1.0 / n) / (2 * p + 1)
    T = n_slabs * dt
    mesh = Mesh(v, h, np.full(ne, p, np.int32), np.full(ne, q, np.int32),
                eps, np.ones(ne), shape=(n, n, n))
    src = Source(kind=1, amp=1.0, center=(0.5, 0.5, 0.5), sigma_x=0.05, f0=4.0,
                 t0=T / 2, sigma_t=T / 4, dir=(0.0, 0.0, 1.0))
    return dict(name=f"cavity {n}^3 p{p} q{q}", mesh=mesh, dt=dt, n_slabs=n_slabs,
                source=src, init="zero")


def serving_stream(n_requests=256, rate=50.0, seed=0, sizes=(4, 6, 8, 12, 16),
                   degrees=(2, 3, 4, 5, 6), n_slabs=20):
    """Independent PEC cavity solves arriving as a Poisson stream.

    Arrival times are the cumulative sum of Exp(1/rate) draws (seed).  Request r
    uses seed 1000 + r: n uniform in ``sizes``, p uniform in ``degrees``,
    q = p - 1, eps uniform in {1, 2, 4} per element, mu = 1, dt = h / (2p + 1),
    initial E a cavity-mode superposition with seed 1000 + r."""
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n_requests))
    reqs = []
    for r in range(n_requests):
        rr = np.random.default_rng(1000 + r)
        n = int(rr.choice(sizes))
        p = int(rr.choice(degrees))
        q = p - 1
        v, h = _lattice(n)
        ne = h.shape[0]
        eps = rr.choice(np.array([1.0, 2.0, 4.0]), size=ne)
        mesh = Mesh(v, h, np.full(ne, p, np.int32), np.full(ne, q, np.int32),
                    eps, np.ones(ne), shape=(n, n, n))
        reqs.append(dict(id=r, arrival=float(arrivals[r]), mesh=mesh,
                         dt=(1.0 / n) / (2 * p + 1), n_slabs=n_slabs,
                         init=mode_superposition(1000 + r), source=Source()))
    return reqs
