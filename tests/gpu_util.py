"""Helpers shared by the GPU tests: library context, mesh upload, apply through
the C ABI, and comparison with the oracle on the same seeded inputs."""
import sys

import numpy as np

import synth


def rel_err(got, ref):
    """The larger of the relative 2-norm error ||got - ref|| / ||ref|| and the
    largest entry error relative to the largest reference entry,
    max|got - ref| / max|ref|: every parity bar bounds both (a single wrong
    entry cannot hide in the norm of a long vector)."""
    ref = np.asarray(ref, dtype=np.float64)
    got = np.asarray(got, dtype=np.float64)
    if got.shape != ref.shape:
        raise ValueError("shapes differ: %s vs %s" % (got.shape, ref.shape))
    if not np.all(np.isfinite(got)):
        return float("inf")
    den = np.linalg.norm(ref)
    norm2 = np.linalg.norm(got - ref) / (den if den > 0 else 1.0)
    top = np.abs(ref).max() if ref.size else 0.0
    entry = (np.abs(got - ref).max() / (top if top > 0 else 1.0)) if ref.size else 0.0
    return max(norm2, entry)


def rel_err_dev(got, ref):
    """rel_err of two device tensors, computed on the device (long vectors)."""
    import torch
    g = got.double()
    r = ref.double()
    if not bool(torch.isfinite(g).all()):
        return float("inf")
    den = float(torch.linalg.vector_norm(r))
    norm2 = float(torch.linalg.vector_norm(g - r)) / (den if den > 0 else 1.0)
    top = float(r.abs().max())
    entry = float((g - r).abs().max()) / (top if top > 0 else 1.0)
    return max(norm2, entry)


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


class Lib:
    """Context + helpers around the C ABI."""

    def __init__(self):
        import torch
        import paper_1307_5310_amd as stdg
        self.torch = torch
        self.stdg = stdg
        self.ctx = stdg.stdg_init(0, 0)

    def upload(self, mesh):
        return self.stdg.stdg_mesh_upload(self.ctx, mesh.vertices, mesh.hexes, mesh.p, mesh.q,
                                          mesh.eps, mesh.mu, getattr(mesh, "nsub", None))

    def dev(self, arr, dtype):
        t = self.torch
        return t.from_numpy(np.ascontiguousarray(arr)).to(device="cuda", dtype=dtype)

    def apply(self, mh, dt, prec, mode, x, load=None):
        """Run stdg_residual_apply on host array x; returns host float64 result."""
        t = self.torch
        stdg = self.stdg
        dtype = t.float64 if prec == stdg.STDG_FP64 else t.float32
        info = stdg.stdg_mesh_info(mh)
        xd = self.dev(x, dtype)
        ld = self.dev(load, dtype) if load is not None else None
        yd = t.full((info["unknown_size"],), float("nan"), dtype=dtype, device="cuda")
        stdg.stdg_residual_apply(mh, dt, prec, mode, xd, ld, yd)
        t.cuda.synchronize()
        return yd.cpu().numpy().astype(np.float64)


def random_mixed_mesh(shape, pmax, qmax, seed, perturb=None):
    """Lattice mesh with random per-element p in 1..pmax, q in 1..qmax, eps, mu."""
    v, h = synth.box_mesh(shape)
    rng = np.random.default_rng(seed)
    ne = h.shape[0]
    p = rng.integers(1, pmax + 1, ne).astype(np.int32)
    q = rng.integers(1, qmax + 1, ne).astype(np.int32)
    eps = rng.uniform(1, 4, ne)
    mu = rng.uniform(1, 2, ne)
    return synth.Mesh(v, h, p, q, eps, mu, shape=tuple(shape))


def oracle_disc(mesh):
    from oracle.dg import Discretisation
    return Discretisation(mesh.vertices, mesh.hexes, mesh.p, mesh.q, mesh.eps, mesh.mu,
                          nk=getattr(mesh, "nsub", None))
