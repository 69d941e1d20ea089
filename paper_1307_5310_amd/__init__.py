"""stdg: MI355X-native space-time hp-DG residual for the time-dependent Maxwell
equations (Lilienthal, Schnepp, Weiland, arXiv 1307.5310).

Thin Python binding of the C ABI in include/stdg.h: the functions below have
the same names as the C entry points and only marshal arguments (numpy host
arrays, torch device tensors, torch streams).  See the header for layouts,
ownership and error behaviour.
"""
import ctypes

import numpy as np

try:
    import torch
except ImportError:  # pragma: no cover - the binding needs torch only for device tensors
    torch = None

from ._lib import (StdgError, STDG_FP32, STDG_FP64, STDG_OPERATOR, STDG_RESIDUAL,
                   STDG_OPERATOR_PRECOND, STDG_E_NOT_READY, MeshDesc, MeshInfo, Source, SolveOpts,
                   SolveInfo, ServeOpts, Request, Result, lib, check, ptr, stream_handle,
                   exported_symbols)
from . import _lib

__all__ = ["StdgError", "STDG_FP32", "STDG_FP64", "STDG_OPERATOR", "STDG_RESIDUAL",
           "STDG_OPERATOR_PRECOND", "stdg_version", "stdg_init", "stdg_finalize",
           "stdg_mesh_upload", "stdg_mesh_info", "stdg_mesh_offsets", "stdg_mesh_free", "stdg_mesh_set_dissipation",
           "stdg_mesh_set_order", "stdg_mesh_autotune", "stdg_mesh_set_launch", "stdg_mesh_group",
           "stdg_residual_apply", "stdg_residual_apply_noalloc", "stdg_noalloc_scratch_bytes",
           "stdg_stream_copy", "stdg_load_assemble", "stdg_project_modes",
           "stdg_slab_solve", "stdg_energy", "stdg_residual_dual_norm", "stdg_serve_start", "stdg_serve_submit",
           "stdg_serve_poll", "stdg_serve_clock", "stdg_serve_stop", "exported_symbols"]


def stdg_version():
    return lib().stdg_version()


def stdg_init(device=0, hbm_budget_bytes=0):
    h = ctypes.c_void_p()
    check(lib().stdg_init(int(device), int(hbm_budget_bytes), ctypes.byref(h)))
    return h


def stdg_finalize(ctx):
    check(lib().stdg_finalize(ctx))


def _mesh_desc(vertices, hexes, p, q, eps, mu, nsub=None):
    """MeshDesc over contiguous copies; returns (desc, arrays kept alive).
    ``nsub``: temporal sub-intervals per element (local time steps), or None."""
    v = np.ascontiguousarray(vertices, dtype=np.float64)
    h = np.ascontiguousarray(hexes, dtype=np.int64)
    p = np.ascontiguousarray(p, dtype=np.int32)
    q = np.ascontiguousarray(q, dtype=np.int32)
    eps = np.ascontiguousarray(eps, dtype=np.float64)
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    # the library reads n_elements entries of every per-element array and
    # 3 n_vertices / 8 n_elements of the coordinates and connectivity
    if v.ndim != 2 or v.shape[1] != 3:
        raise ValueError("vertices must have shape (n_vertices, 3), got %s" % (v.shape,))
    if h.ndim != 2 or h.shape[1] != 8:
        raise ValueError("hexes must have shape (n_elements, 8), got %s" % (h.shape,))
    ns = None if nsub is None else np.ascontiguousarray(nsub, dtype=np.int32)
    for name, a in (("p", p), ("q", q), ("eps", eps), ("mu", mu), ("nsub", ns)):
        if a is not None and a.shape != (h.shape[0],):
            raise ValueError("%s must have shape (%d,), got %s" % (name, h.shape[0], a.shape))
    d = MeshDesc(v.shape[0], v.ctypes.data, h.shape[0], h.ctypes.data, p.ctypes.data,
                 q.ctypes.data, eps.ctypes.data, mu.ctypes.data, None if ns is None else ns.ctypes.data)
    return d, (v, h, p, q, eps, mu, ns)


def stdg_mesh_upload(ctx, vertices, hexes, p, q, eps, mu, nsub=None):
    d, _keep = _mesh_desc(vertices, hexes, p, q, eps, mu, nsub)
    out = ctypes.c_void_p()
    check(lib().stdg_mesh_upload(ctx, ctypes.byref(d), ctypes.byref(out)))
    return out


def stdg_mesh_info(mesh):
    info = MeshInfo()
    check(lib().stdg_mesh_info(mesh, ctypes.byref(info)))
    return {name: getattr(info, name) for name, _ in MeshInfo._fields_}


def stdg_mesh_offsets(mesh):
    n = stdg_mesh_info(mesh)["n_elements"] + 1
    t, u, s = (np.zeros(n, dtype=np.int64) for _ in range(3))
    check(lib().stdg_mesh_offsets(mesh, t.ctypes.data, u.ctypes.data, s.ctypes.data))
    return t, u, s


_SIZES = {}


def _sizes(mesh):
    """(unknown, trial, state) sizes of a mesh handle, cached per handle."""
    key = mesh.value if isinstance(mesh, ctypes.c_void_p) else int(mesh)
    got = _SIZES.get(key)
    if got is None:
        info = stdg_mesh_info(mesh)
        got = _SIZES[key] = (info["unknown_size"], info["trial_size"], info["state_size"])
    return got


def _dev(t, n, dtype, name, optional=False):
    """Check a device vector before its address crosses the ABI: a contiguous
    CUDA tensor of the expected dtype holding at least n elements (the kernels
    index by the mesh's offsets and trust the caller for the extent)."""
    if t is None:
        if optional:
            return
        raise ValueError("%s is required" % name)
    if isinstance(t, int):
        return  # a raw device address: the caller vouches for it
    if torch is None or not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor on the GPU (or a raw device address)" % name)
    if not t.is_cuda:
        raise ValueError("%s must live on the GPU" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.dtype != dtype:
        raise ValueError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if t.numel() < n:
        raise ValueError("%s holds %d elements, the mesh needs %d" % (name, t.numel(), n))


def stdg_mesh_free(mesh):
    _SIZES.pop(mesh.value if isinstance(mesh, ctypes.c_void_p) else int(mesh), None)
    check(lib().stdg_mesh_free(mesh))


def stdg_mesh_set_dissipation(mesh, c):
    check(lib().stdg_mesh_set_dissipation(mesh, float(c)))


def stdg_mesh_set_order(mesh, order):
    check(lib().stdg_mesh_set_order(mesh, int(order)))


def _tune_key(mesh, prec):
    i = stdg_mesh_info(mesh)
    return "ne=%d,groups=%d,affine=%d,nonaffine=%d,diag=%d,pmax=%d,qmax=%d,unk=%d,prec=%d" % (
        i["n_elements"], i["n_groups"], i["n_affine"], i["n_nonaffine"], i["n_diagonal_mass"], i["p_max"],
        i["q_max"], i["unknown_size"], int(prec))


def _tune_entry_ok(v):
    return (isinstance(v, dict) and isinstance(v.get("order"), int) and isinstance(v.get("variants"), list)
            and all(isinstance(k, int) for k in v["variants"]))


def _tune_cache_read(path):
    """The cached choices in `path` ({key: {"order": int, "variants": [int per
    group]}}), or {} when the file is missing or malformed (it is then
    rewritten on the next store)."""
    import json
    try:
        with open(path) as f:
            table = json.load(f)
    except (OSError, ValueError):
        return {}
    if not isinstance(table, dict) or not all(_tune_entry_ok(v) for v in table.values()):
        return {}
    return table


def _tune_cache_write(path, table):
    """Replace `path` atomically (a temporary file of its own in the same
    directory, so concurrent writers never share one)."""
    import json
    import os
    import tempfile
    fd, tmp = tempfile.mkstemp(prefix=os.path.basename(path) + ".", dir=os.path.dirname(os.path.abspath(path)))
    try:
        with os.fdopen(fd, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except BaseException:
        if os.path.exists(tmp):
            os.remove(tmp)
        raise


def stdg_mesh_autotune(mesh, prec=STDG_FP32, dt=0.01, reps=10, cache=None, stream=None):
    """Pick the kernels' element order and each group's launch variant for
    this mesh by timing (C ABI stdg_mesh_autotune); returns
    {"order": int, "variants": [int per group]}.  With a cache file
    (argument, or the STDG_TUNE_CACHE environment variable) choices stored for
    a mesh of the same shape are applied without timing, and new choices are
    stored."""
    import os
    path = cache or os.environ.get("STDG_TUNE_CACHE")
    key = _tune_key(mesh, prec)
    table = _tune_cache_read(path) if path else {}
    n_groups = stdg_mesh_info(mesh)["n_groups"]
    if key in table and len(table[key]["variants"]) == n_groups:
        stdg_mesh_set_order(mesh, table[key]["order"])
        for g, v in enumerate(table[key]["variants"]):
            stdg_mesh_set_launch(mesh, g, v)
        return dict(table[key])
    out = ctypes.c_int32()
    check(lib().stdg_mesh_autotune(mesh, int(prec), float(dt), int(reps), ctypes.byref(out),
                                   stream_handle(stream)))
    choice = {"order": int(out.value), "variants": [stdg_mesh_group(mesh, g)["variant"] for g in range(n_groups)]}
    if path:
        table = _tune_cache_read(path)   # keep what other processes stored meanwhile
        table[key] = choice
        _tune_cache_write(path, table)
    return choice


def stdg_mesh_set_launch(mesh, group, variant):
    check(lib().stdg_mesh_set_launch(mesh, int(group), int(variant)))


def stdg_mesh_group(mesh, group):
    g = _lib.GroupInfo()
    check(lib().stdg_mesh_group(mesh, int(group), ctypes.byref(g)))
    return {name: getattr(g, name) for name, _ in _lib.GroupInfo._fields_}


def stdg_residual_apply(mesh, dt, prec, mode, x, load, y, stream=None):
    if torch is not None and mesh:
        nu, nt, _ = _sizes(mesh)
        dtype = torch.float64 if int(prec) == STDG_FP64 else torch.float32
        _dev(x, nt if int(mode) == STDG_RESIDUAL else nu, dtype, "x")
        _dev(load, nu, dtype, "load", optional=True)
        _dev(y, nu, dtype, "y")
    check(lib().stdg_residual_apply(mesh, float(dt), int(prec), int(mode), ptr(x), ptr(load),
                                    ptr(y), stream_handle(stream)))


def stdg_residual_apply_noalloc(mesh, dt, prec, mode, x, load, y, stream=None):
    """stdg_residual_apply that allocates nothing (static device scratch)."""
    if torch is not None and mesh:
        nu, nt, _ = _sizes(mesh)
        dtype = torch.float64 if int(prec) == STDG_FP64 else torch.float32
        _dev(x, nt if int(mode) == STDG_RESIDUAL else nu, dtype, "x")
        _dev(load, nu, dtype, "load", optional=True)
        _dev(y, nu, dtype, "y")
    check(lib().stdg_residual_apply_noalloc(mesh, float(dt), int(prec), int(mode), ptr(x), ptr(load),
                                            ptr(y), stream_handle(stream)))


def stdg_noalloc_scratch_bytes():
    return lib().stdg_noalloc_scratch_bytes()


def stdg_stream_copy(src, dst, stream=None):
    """dst[:] = src[:] by the library's streaming kernel (the practical HBM
    ceiling); both contiguous device tensors of the same byte size."""
    for t, name in ((src, "src"), (dst, "dst")):
        if torch is None or not isinstance(t, torch.Tensor):
            raise TypeError("%s must be a torch tensor on the GPU" % name)
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError("%s must be a contiguous tensor on the GPU" % name)
    nbytes = src.numel() * src.element_size()
    if nbytes != dst.numel() * dst.element_size():
        raise ValueError("src and dst differ in size")
    check(lib().stdg_stream_copy(ptr(src), ptr(dst), ctypes.c_size_t(nbytes), stream_handle(stream)))


def _source(src):
    s = Source()
    if src is None:
        s.kind = 0
        return s
    s.kind = int(src.kind)
    s.amp = float(src.amp)
    s.center[:] = [float(c) for c in src.center]
    s.sigma_x, s.f0, s.t0, s.sigma_t = float(src.sigma_x), float(src.f0), float(src.t0), float(src.sigma_t)
    s.dir[:] = [float(c) for c in src.dir]
    return s


def stdg_load_assemble(mesh, src, t0, dt, load, stream=None):
    if torch is not None and mesh:
        _dev(load, _sizes(mesh)[0], torch.float64, "load")
    s = _source(src)
    check(lib().stdg_load_assemble(mesh, ctypes.byref(s), float(t0), float(dt), ptr(load),
                                   stream_handle(stream)))


def stdg_project_modes(mesh, mnl, abc, state, stream=None):
    mnl = np.ascontiguousarray(mnl, dtype=np.int32).reshape(-1, 3)
    abc = np.ascontiguousarray(abc, dtype=np.float64).reshape(-1, 3)
    if torch is not None and mesh:
        _dev(state, _sizes(mesh)[2], torch.float64, "state")
    check(lib().stdg_project_modes(mesh, mnl.shape[0], mnl.ctypes.data, abc.ctypes.data,
                                   ptr(state), stream_handle(stream)))


def stdg_slab_solve(mesh, t0, dt, load, state, inner_prec=STDG_FP64, restart=10, max_iters=500,
                    max_refine=100, rtol=1e-12, inner_rtol=1e-4, slab_U=None, stream=None, krylov_prec=None,
                    eta_tol=0.0, eta_t_final=0.0, use_graph=False):
    """One slab (C ABI stdg_slab_solve).  krylov_prec None: the basis in the
    precision of the inner applies (FP32 with FP32 applies, whose refinement
    against the FP64 residual corrects it; FP64 otherwise)."""
    if krylov_prec is None:
        krylov_prec = STDG_FP32 if int(inner_prec) == STDG_FP32 else STDG_FP64
    o = SolveOpts(int(inner_prec), int(restart), int(max_iters), int(max_refine), float(rtol),
                  float(inner_rtol), int(krylov_prec), float(eta_tol), float(eta_t_final), int(bool(use_graph)))
    info = SolveInfo()
    if torch is not None and mesh:
        nu, nt, ns = _sizes(mesh)
        _dev(load, nu, torch.float64, "load", optional=True)
        _dev(state, ns, torch.float64, "state")
        _dev(slab_U, nt, torch.float64, "slab_U", optional=True)
    st = lib().stdg_slab_solve(mesh, float(t0), float(dt), ptr(load), ctypes.byref(o), ptr(state),
                               ptr(slab_U), ctypes.byref(info), stream_handle(stream))
    res = {name: getattr(info, name) for name, _ in SolveInfo._fields_}
    res["status"] = st
    if st not in (0, -5):
        check(st)
    return res


def stdg_residual_dual_norm(mesh, dt, r, stream=None):
    out = (ctypes.c_double * 2)()
    if torch is not None and mesh:
        _dev(r, _sizes(mesh)[0], torch.float64, "r")
    check(lib().stdg_residual_dual_norm(mesh, float(dt), ptr(r), out, stream_handle(stream)))
    return out[0], out[1]


def stdg_energy(mesh, state, stream=None):
    out = ctypes.c_double()
    if torch is not None and mesh:
        _dev(state, _sizes(mesh)[2], torch.float64, "state")
    check(lib().stdg_energy(mesh, ptr(state), ctypes.byref(out), stream_handle(stream)))
    return out.value


def stdg_serve_start(ctx, hbm_budget=0, max_active=0, inner_prec=STDG_FP32, restart=10, max_iters=500,
                     max_refine=100, rtol=1e-10, inner_rtol=1e-4, krylov_prec=None, eta_rel=0.0,
                     use_graph=False, batch_cycles=True):
    """Start a server (C ABI stdg_serve_start); krylov_prec None as in stdg_slab_solve."""
    if krylov_prec is None:
        krylov_prec = STDG_FP32 if int(inner_prec) == STDG_FP32 else STDG_FP64
    o = ServeOpts(int(hbm_budget), int(max_active), int(inner_prec), int(restart), int(max_iters),
                  int(max_refine), float(rtol), float(inner_rtol), int(krylov_prec), float(eta_rel),
                  int(bool(use_graph)), int(bool(batch_cycles)))
    h = ctypes.c_void_p()
    check(lib().stdg_serve_start(ctx, ctypes.byref(o), ctypes.byref(h)))
    return h


def stdg_serve_submit(server, vertices, hexes, p, q, eps, mu, t0, dt, n_slabs, source=None, mnl=None,
                      abc=None, init_state=None, c_diss=0.0, nsub=None):
    """Queue one request; every array is copied before return.  Returns the ticket.
    ``nsub``: temporal sub-intervals per element (local time steps), or None."""
    d, _keep = _mesh_desc(vertices, hexes, p, q, eps, mu, nsub)
    r = Request()
    r.mesh = d
    r.t0, r.dt, r.n_slabs = float(t0), float(dt), int(n_slabs)
    r.c_diss = float(c_diss)
    r.source = _source(source)
    keep2 = []
    if mnl is not None and len(mnl):
        mnl = np.ascontiguousarray(mnl, dtype=np.int32).reshape(-1, 3)
        abc = np.ascontiguousarray(abc, dtype=np.float64).reshape(-1, 3)
        keep2 += [mnl, abc]
        r.n_modes, r.mnl, r.abc = mnl.shape[0], mnl.ctypes.data, abc.ctypes.data
    if init_state is not None:
        init_state = np.ascontiguousarray(init_state, dtype=np.float64).ravel()
        need = int((6 * (np.asarray(p, dtype=np.int64) + 1) ** 3).sum())
        if init_state.size != need:
            raise ValueError("init_state has %d entries, the mesh's state size is %d" % (init_state.size, need))
        keep2.append(init_state)
        r.init_state = init_state.ctypes.data
        r.init_state_size = init_state.size
    t = ctypes.c_uint64()
    check(lib().stdg_serve_submit(server, ctypes.byref(r), ctypes.byref(t)))
    return t.value


def stdg_serve_poll(server, ticket, state_out=None):
    """None while the request runs; then a dict of the result (the final state
    is written into state_out, a float64 numpy array, when given)."""
    res = Result()
    if state_out is not None:
        if not (isinstance(state_out, np.ndarray) and state_out.dtype == np.float64
                and state_out.flags["C_CONTIGUOUS"] and state_out.flags["WRITEABLE"]):
            raise ValueError("state_out must be a writeable C-contiguous float64 numpy array")
        res.state = state_out.ctypes.data
        res.state_capacity = state_out.size
    st = lib().stdg_serve_poll(server, ctypes.c_uint64(int(ticket)), ctypes.byref(res))
    if st == STDG_E_NOT_READY:
        return None
    check(st)
    return {name: getattr(res, name) for name, _ in Result._fields_ if name not in ("state", "state_capacity")}


def stdg_serve_clock(server):
    return lib().stdg_serve_clock(server)


def stdg_serve_stop(server):
    check(lib().stdg_serve_stop(server))
