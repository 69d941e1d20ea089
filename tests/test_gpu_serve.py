"""GPU tests of the serving loop (stdg_serve_*): independent cavity solves
marched slab by slab (Section 2.2), admitted by device footprint and run
concurrently.

* each request's result is bitwise the same alone, in a mix, and as the plain
  stdg_slab_solve march of the same slabs, also when requests of one kernel
  group run their restart cycles batched;
* a small request matches the oracle's direct slab solves to 1e-10;
* admission waits for memory; invalid requests are refused at submit, a
  failing request reports through its result without disturbing the others;
  stop with work in flight returns."""
import time

import numpy as np
import pytest

import synth
from tests.gpu_util import Lib, note, oracle_disc, rel_err

pytestmark = pytest.mark.gpu

OPTS = dict(inner_prec=1, rtol=1e-12, max_iters=3000, max_refine=300)


@pytest.fixture(scope="module")
def lib():
    return Lib()


def _small_stream(k, sizes=(4, 6), degrees=(2, 3), n_slabs=3):
    return synth.serving_stream(n_requests=k, sizes=sizes, degrees=degrees, n_slabs=n_slabs)


def _submit(stdg, srv, rq):
    m = rq["mesh"]
    return stdg.stdg_serve_submit(srv, m.vertices, m.hexes, m.p, m.q, m.eps, m.mu, 0.0, rq["dt"], rq["n_slabs"],
                                  source=None, mnl=rq["init"].mnl, abc=rq["init"].abc)


def _wait(stdg, srv, tickets, sizes, timeout=120.0):
    out = {}
    t_end = time.time() + timeout
    while len(out) < len(tickets):
        assert time.time() < t_end, "serving requests did not finish in time"
        for t, n in zip(tickets, sizes):
            if t in out:
                continue
            st = np.zeros(n)
            r = stdg.stdg_serve_poll(srv, t, st)
            if r is not None:
                r["state"] = st
                out[t] = r
        time.sleep(0.002)
    return [out[t] for t in tickets]


def _march(lib, rq, **opts):
    """The same request through stdg_project_modes + stdg_slab_solve."""
    stdg = lib.stdg
    m = rq["mesh"]
    mh = lib.upload(m)
    info = stdg.stdg_mesh_info(mh)
    st = lib.torch.zeros(info["state_size"], dtype=lib.torch.float64, device="cuda")
    stdg.stdg_project_modes(mh, rq["init"].mnl, rq["init"].abc, st)
    for n in range(rq["n_slabs"]):
        r = stdg.stdg_slab_solve(mh, n * rq["dt"], rq["dt"], None, st, **opts)
        assert r["status"] == 0
    out = st.cpu().numpy()
    stdg.stdg_mesh_free(mh)
    return out


@pytest.mark.parametrize("krylov,graph", [(0, False), (1, False), (1, True)])
def test_serve_matches_slab_solve_alone_and_in_mix(lib, krylov, graph):
    stdg = lib.stdg
    opts = dict(OPTS, krylov_prec=krylov)
    reqs = _small_stream(10)
    sizes = [r["mesh"].state_size() for r in reqs]
    note("serve: one request alone")
    srv = stdg.stdg_serve_start(lib.ctx, hbm_budget=1 << 30, max_active=4, use_graph=graph, **opts)
    try:
        alone = _wait(stdg, srv, [_submit(stdg, srv, reqs[3])], [sizes[3]])[0]
        note("serve: ten requests in a mix")
        tickets = [_submit(stdg, srv, r) for r in reqs]
        mix = _wait(stdg, srv, tickets, sizes)
    finally:
        stdg.stdg_serve_stop(srv)
    assert alone["status"] == 0 and alone["slabs_done"] == reqs[3]["n_slabs"]
    for r in mix:
        assert r["status"] == 0, r
        assert abs(r["energy_end"] - r["energy_start"]) < 1e-10 * r["energy_start"]
    assert np.array_equal(alone["state"], mix[3]["state"])
    note("serve: plain march of request 3")
    ref = _march(lib, reqs[3], **opts)
    assert np.array_equal(ref, mix[3]["state"])


@pytest.mark.parametrize("krylov", [0, 1])
def test_batched_cycles_bitwise(lib, krylov):
    """A burst of requests of two kernel groups ((p, q) = (2, 1) and (3, 2)
    cavities with their own materials and fields): with batched restart
    cycles the requests of one group share launches (batched_cycles > 0), and
    every final state is bitwise the one of the same server without batching
    and of the plain march."""
    stdg = lib.stdg
    opts = dict(OPTS, krylov_prec=krylov)
    reqs = _small_stream(12, sizes=(4, 6), degrees=(2, 3), n_slabs=2)
    sizes = [r["mesh"].state_size() for r in reqs]
    out = {}
    for batch in (True, False):
        note("serve: burst of 12, batch_cycles=%s krylov=%d" % (batch, krylov))
        srv = stdg.stdg_serve_start(lib.ctx, hbm_budget=1 << 30, max_active=12, batch_cycles=batch, **opts)
        try:
            out[batch] = _wait(stdg, srv, [_submit(stdg, srv, r) for r in reqs], sizes)
        finally:
            stdg.stdg_serve_stop(srv)
    for r in out[True] + out[False]:
        assert r["status"] == 0, r
    assert sum(r["batched_cycles"] for r in out[True]) > 0
    assert all(r["batched_cycles"] == 0 for r in out[False])
    for a, b in zip(out[True], out[False]):
        assert np.array_equal(a["state"], b["state"])
        assert a["iters"] == b["iters"]
    k = int(np.argmax([r["batched_cycles"] for r in out[True]]))
    note("serve: plain march of request %d (%d batched cycles)" % (k, out[True][k]["batched_cycles"]))
    assert np.array_equal(_march(lib, reqs[k], **opts), out[True][k]["state"])


def test_serve_matches_oracle(lib):
    stdg = lib.stdg
    rq = _small_stream(1, sizes=(4,), degrees=(2,), n_slabs=2)[0]
    m = rq["mesh"]
    d = oracle_disc(m)
    from oracle import fields
    s = fields.project(d, fields.mode_superposition(rq["init"].mnl, rq["init"].abc), 0.0)
    for _ in range(rq["n_slabs"]):
        s = d.level_state(d.solve_direct(s, rq["dt"]), 1)
    srv = stdg.stdg_serve_start(lib.ctx, hbm_budget=1 << 28, **OPTS)
    try:
        r = _wait(stdg, srv, [_submit(stdg, srv, rq)], [m.state_size()])[0]
    finally:
        stdg.stdg_serve_stop(srv)
    assert r["status"] == 0
    assert rel_err(r["state"], s) < 1e-10


def test_admission_waits_for_memory(lib):
    stdg = lib.stdg
    reqs = _small_stream(3, sizes=(6,), degrees=(3,), n_slabs=2)
    sizes = [r["mesh"].state_size() for r in reqs]
    srv = stdg.stdg_serve_start(lib.ctx, hbm_budget=1 << 30, **OPTS)
    try:
        one = _wait(stdg, srv, [_submit(stdg, srv, reqs[0])], sizes[:1])[0]
    finally:
        stdg.stdg_serve_stop(srv)
    # an arena that holds one of these requests but not two
    budget = int(one["device_bytes"] * 1.5)
    srv = stdg.stdg_serve_start(lib.ctx, hbm_budget=budget, **OPTS)
    try:
        res = _wait(stdg, srv, [_submit(stdg, srv, r) for r in reqs], sizes)
    finally:
        stdg.stdg_serve_stop(srv)
    for a, b in zip(res, res[1:]):
        assert b["t_admit"] >= a["t_done"] - 1e-3
    for r in res:
        assert r["status"] == 0
    assert np.array_equal(res[0]["state"], one["state"])


def test_errors_stay_per_request(lib):
    stdg = lib.stdg
    good = _small_stream(1, sizes=(4,), degrees=(2,), n_slabs=2)[0]
    srv = stdg.stdg_serve_start(lib.ctx, hbm_budget=1 << 26, **OPTS)
    try:
        # larger than the whole arena: refused at submit
        big = synth.serving_stream(n_requests=1, sizes=(16,), degrees=(6,), n_slabs=1)[0]
        with pytest.raises(stdg.StdgError) as ei:
            _submit(stdg, srv, big)
        assert ei.value.status == -7
        # invalid degree: refused at submit
        m = good["mesh"]
        with pytest.raises(stdg.StdgError):
            stdg.stdg_serve_submit(srv, m.vertices, m.hexes, np.full(m.n_elements, 12), m.q, m.eps, m.mu, 0.0,
                                   good["dt"], 1)
        # a face shared by three elements: the mesh analysis refuses it at submit
        bad_h = m.hexes.copy()
        bad_h[1] = bad_h[0]
        bad_h[2] = bad_h[0]
        with pytest.raises(stdg.StdgError) as ei:
            stdg.stdg_serve_submit(srv, m.vertices, bad_h, m.p, m.q, m.eps, m.mu, 0.0, good["dt"], 1)
        assert ei.value.status == -1
        # a request whose slab fails inside the server (non-finite initial state)
        t_bad = stdg.stdg_serve_submit(srv, m.vertices, m.hexes, m.p, m.q, m.eps, m.mu, 0.0, good["dt"], 2,
                                       init_state=np.full(m.state_size(), np.nan))
        t_good = _submit(stdg, srv, good)
        r_bad, r_good = _wait(stdg, srv, [t_bad, t_good], [m.state_size(), m.state_size()])
    finally:
        stdg.stdg_serve_stop(srv)
    assert r_bad["status"] == -1 and r_bad["slabs_done"] == 0
    assert r_good["status"] == 0 and r_good["slabs_done"] == 2


def test_not_converged_is_reported(lib):
    stdg = lib.stdg
    rq = _small_stream(1, sizes=(4,), degrees=(2,), n_slabs=2)[0]
    srv = stdg.stdg_serve_start(lib.ctx, hbm_budget=1 << 26, inner_prec=0, rtol=1e-14, max_iters=1)
    try:
        r = _wait(stdg, srv, [_submit(stdg, srv, rq)], [rq["mesh"].state_size()])[0]
    finally:
        stdg.stdg_serve_stop(srv)
    assert r["status"] == -5 and r["slabs_done"] == 2 and 0 < r["max_rel_res"] < 1


def test_stop_with_work_in_flight(lib):
    stdg = lib.stdg
    reqs = _small_stream(6, sizes=(6, 8), degrees=(3, 4), n_slabs=20)
    srv = stdg.stdg_serve_start(lib.ctx, hbm_budget=1 << 30, max_active=2, **OPTS)
    tickets = [_submit(stdg, srv, r) for r in reqs]
    time.sleep(0.05)
    t0 = time.time()
    stdg.stdg_serve_stop(srv)
    assert time.time() - t0 < 30
    assert len(tickets) == 6


def test_inexact_serving_within_eta(lib):
    """Requests solved inexactly (Section 5.3): each stops its slabs at a share
    of the iteration-error budget; the accumulated eta_it is within the budget,
    the true error against the oracle's exact march is below it, and the
    result is the same alone and in a mix."""
    stdg = lib.stdg
    from oracle import fields
    reqs = _small_stream(4, sizes=(2,), degrees=(2, 3), n_slabs=3)
    sizes = [r["mesh"].state_size() for r in reqs]
    eta_rel = 1e-3
    srv = stdg.stdg_serve_start(lib.ctx, hbm_budget=1 << 30, eta_rel=eta_rel, **OPTS)
    try:
        alone = _wait(stdg, srv, [_submit(stdg, srv, reqs[1])], [sizes[1]])[0]
        mix = _wait(stdg, srv, [_submit(stdg, srv, r) for r in reqs], sizes)
    finally:
        stdg.stdg_serve_stop(srv)
    assert np.array_equal(alone["state"], mix[1]["state"])
    rq = reqs[1]
    d = oracle_disc(rq["mesh"])
    s = fields.project(d, fields.mode_superposition(rq["init"].mnl, rq["init"].abc), 0.0)
    budget = eta_rel * np.sqrt(2 * d.energy(s))
    for n in range(rq["n_slabs"]):
        note("inexact serving: oracle slab %d" % n)
        s = d.level_state(d.solve_direct(s, rq["dt"]), 1)
    r = mix[1]
    err = np.sqrt(2 * d.energy(r["state"] - s))
    note("inexact serving: error %.3e, eta_it %.3e, budget %.3e, iters %d" % (err, r["eta_it"], budget, r["iters"]))
    assert r["status"] == 0
    assert r["eta_it"] <= budget * (1 + 1e-12)
    assert err <= r["eta_it"]


def test_serving_with_dissipation(lib):
    """Requests with the dissipative stabilisation D_h (remark closing
    Section 4), on an affine and on a trilinear mesh: bitwise the plain march
    with stdg_mesh_set_dissipation, and the energy drops."""
    stdg = lib.stdg
    rq = _small_stream(1, sizes=(4,), degrees=(3,), n_slabs=3)[0]
    m = rq["mesh"]
    c = 0.6
    v, h = synth.box_mesh((2, 2, 2))
    v = synth.perturb_interior(v, (2, 2, 2), 0.1, seed=3)
    tri = synth.Mesh(v, h, np.full(8, 2, np.int32), np.full(8, 1, np.int32), np.ones(8), np.ones(8))
    init = np.random.default_rng(3).standard_normal(tri.state_size())
    srv = stdg.stdg_serve_start(lib.ctx, hbm_budget=1 << 28, **OPTS)
    try:
        t = stdg.stdg_serve_submit(srv, m.vertices, m.hexes, m.p, m.q, m.eps, m.mu, 0.0, rq["dt"], rq["n_slabs"],
                                   mnl=rq["init"].mnl, abc=rq["init"].abc, c_diss=c)
        t2 = stdg.stdg_serve_submit(srv, tri.vertices, tri.hexes, tri.p, tri.q, tri.eps, tri.mu, 0.0, 0.05, 2,
                                    init_state=init, c_diss=c)
        r, r2 = _wait(stdg, srv, [t, t2], [m.state_size(), tri.state_size()])
    finally:
        stdg.stdg_serve_stop(srv)
    for x in (r, r2):
        assert x["status"] == 0
        assert x["energy_end"] < x["energy_start"]
    mh = lib.upload(m)
    try:
        stdg.stdg_mesh_set_dissipation(mh, c)
        st = lib.torch.zeros(m.state_size(), dtype=lib.torch.float64, device="cuda")
        stdg.stdg_project_modes(mh, rq["init"].mnl, rq["init"].abc, st)
        for n in range(rq["n_slabs"]):
            assert stdg.stdg_slab_solve(mh, n * rq["dt"], rq["dt"], None, st, **OPTS)["status"] == 0
        ref = st.cpu().numpy()
    finally:
        stdg.stdg_mesh_free(mh)
    assert np.array_equal(ref, r["state"])
    mh = lib.upload(tri)
    try:
        stdg.stdg_mesh_set_dissipation(mh, c)
        st = lib.dev(init, lib.torch.float64)
        for n in range(2):
            assert stdg.stdg_slab_solve(mh, n * 0.05, 0.05, None, st, **OPTS)["status"] == 0
        ref2 = st.cpu().numpy()
    finally:
        stdg.stdg_mesh_free(mh)
    assert np.array_equal(ref2, r2["state"])


def test_serving_trilinear_with_source(lib):
    """A request on a perturbed (trilinear) mesh with mixed degrees, driven
    by the Gaussian-pulse current from a zero field: its load is assembled
    per slab inside the server; bitwise the plain march."""
    stdg = lib.stdg
    v, h = synth.box_mesh((3, 3, 3))
    v = synth.perturb_interior(v, (3, 3, 3), 0.1, seed=21)
    rng = np.random.default_rng(21)
    p = rng.integers(1, 4, 27).astype(np.int32)
    q = rng.integers(1, 3, 27).astype(np.int32)
    m = synth.Mesh(v, h, p, q, rng.uniform(1, 3, 27), np.ones(27))
    src = synth.Source(kind=1, amp=1.0, center=(0.5, 0.5, 0.5), sigma_x=0.15, f0=4.0, t0=0.05, sigma_t=0.05)
    dt, n_slabs = 0.02, 3
    srv = stdg.stdg_serve_start(lib.ctx, hbm_budget=1 << 28, **OPTS)
    try:
        t = stdg.stdg_serve_submit(srv, m.vertices, m.hexes, m.p, m.q, m.eps, m.mu, 0.0, dt, n_slabs, source=src)
        r = _wait(stdg, srv, [t], [m.state_size()])[0]
    finally:
        stdg.stdg_serve_stop(srv)
    assert r["status"] == 0 and r["slabs_done"] == n_slabs
    mh = lib.upload(m)
    try:
        st = lib.torch.zeros(m.state_size(), dtype=lib.torch.float64, device="cuda")
        ld = lib.torch.zeros(stdg.stdg_mesh_info(mh)["unknown_size"], dtype=lib.torch.float64, device="cuda")
        for n in range(n_slabs):
            stdg.stdg_load_assemble(mh, src, n * dt, dt, ld)
            assert stdg.stdg_slab_solve(mh, n * dt, dt, ld, st, **OPTS)["status"] == 0
        ref = st.cpu().numpy()
    finally:
        stdg.stdg_mesh_free(mh)
    assert np.abs(ref).max() > 0
    assert np.array_equal(ref, r["state"])
