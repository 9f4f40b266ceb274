"""Serving engine on the GPU: continuous batching of mixed requests.

Checks that every request's result is the same served alone and served in
a mix (merged launches across requests do the same per-node arithmetic),
that results match the oracle, that admission waits for pool memory, and
that oversize requests are rejected."""
import numpy as np
import pytest

import tcgen
from oracle import statevector as sv
from paper_2205_10091_amd import _lib as L
from paper_2205_10091_amd import serve
from gpu_common import TOL_C64, assert_grad, rel_err

pytestmark = pytest.mark.gpu


def small_requests(n, rate=2000.0, seed=11):
    return tcgen.serving_requests(n, rate, seed=seed, max_width=14, max_chain_shallow=40,
                                  depth_range=(2, 4))


def serve_alone(rq):
    srv = serve.Server(pool_bytes=1 << 30, max_active=4)
    rep = serve.run(srv, [rq], realtime=False)
    srv.close()
    return rep.results[0]


def test_mix_matches_alone_and_oracle():
    reqs = small_requests(40)
    srv = serve.Server(pool_bytes=4 << 30, max_active=16)
    rep = serve.run(srv, reqs, realtime=False)
    srv.close()
    assert not rep.rejected
    assert len(rep.results) == len(reqs)
    for i, rq in enumerate(reqs):
        r = rep.results[i]
        assert r.status == 0
        if i % 4 == 0:
            a = serve_alone(rq)
            assert abs(a.value - r.value) <= 1e-12 * max(1.0, abs(a.value))
            if rq.want_grad:
                assert np.max(np.abs(a.grad - r.grad)) <= 1e-12 * max(1.0, np.max(np.abs(a.grad)))
        if rq.circuit.n_qubits <= 16:
            if rq.want_grad:
                e_ref, g_ref = sv.energy_grad(rq.circuit, rq.params, rq.observable)
                assert_grad(r.grad, g_ref, TOL_C64)
            else:
                e_ref = sv.energy(rq.circuit, rq.params, rq.observable).real
            assert rel_err(r.value, e_ref, 1.0) < TOL_C64


def _request(rid, shape, a, b, depth, grad, seed):
    if shape == "chain":
        circ, obs = tcgen.chain_ladder(a, depth), tcgen.tfim_zz_x(a, 0.7 + 0.1 * (seed % 7))
    else:
        circ, obs = tcgen.grid_ladder(a, b, depth), tcgen.tfim_zz_x_grid(a, b, 0.7 + 0.1 * (seed % 7))
    return tcgen.Request(rid, 0.0, circ, obs, tcgen.draw_angles(seed, (circ.n_params,)), grad,
                         shape, depth)


def test_serving_mix_shaped_like_the_workload():
    """Requests of the serving workload's extremes, submitted together
    under a 4 GiB per-request cap: a 600-qubit chain at depth 2, a 64-qubit
    chain at depth 6, a 6x6 grid at depth 2, and grids whose terms must run
    in groups to fit the cap (4x5 at depth 5 with gradient: 137 GB with
    every term live; 3x6 at depth 6 with gradient).  Each result equals the
    same request served alone; requests of at most 20 qubits also match
    the state-vector oracle."""
    reqs = [_request(0, "chain", 600, 0, 2, True, 1), _request(1, "chain", 64, 0, 6, False, 2),
            _request(2, "chain", 20, 0, 5, True, 3), _request(3, "grid", 4, 5, 5, False, 4),
            _request(4, "grid", 4, 5, 5, True, 5), _request(5, "grid", 6, 6, 2, False, 6),
            _request(6, "grid", 3, 6, 6, True, 7), _request(7, "chain", 12, 0, 10, True, 8)]
    srv = serve.Server(pool_bytes=48 << 30, max_request_bytes=4 << 30, max_active=16,
                       path_trials=1)
    rep = serve.run(srv, reqs, realtime=False)
    srv.close()
    assert not rep.rejected and len(rep.results) == len(reqs)
    for i, rq in enumerate(reqs):
        r = rep.results[i]
        assert r.status == 0
        alone = serve.Server(pool_bytes=8 << 30, max_request_bytes=4 << 30, max_active=2,
                             path_trials=1)
        a = serve.run(alone, [rq], realtime=False).results[0]
        alone.close()
        print(f"request {i} ({rq.shape}, {rq.circuit.n_qubits} qubits, depth {rq.depth}, "
              f"grad {int(rq.want_grad)}): E = {r.value:.8f}, alone {a.value:.8f}, "
              f"latency {r.latency_s * 1e3:.1f} ms")
        assert abs(a.value - r.value) <= 1e-12 * max(1.0, abs(a.value))
        if rq.want_grad:
            assert np.max(np.abs(a.grad - r.grad)) <= 1e-12 * max(1.0, np.max(np.abs(a.grad)))
        if rq.circuit.n_qubits <= 20:
            if rq.want_grad:
                e_ref, g_ref = sv.energy_grad(rq.circuit, rq.params, rq.observable)
                assert_grad(r.grad, g_ref, TOL_C64, what=f"request {i}")
            else:
                e_ref = sv.energy(rq.circuit, rq.params, rq.observable).real
            assert rel_err(r.value, e_ref, 1.0) < TOL_C64, i


def test_poisson_arrivals_complete_with_latency():
    reqs = small_requests(60, rate=500.0, seed=12)
    srv = serve.Server(pool_bytes=4 << 30, max_active=32)
    rep = serve.run(srv, reqs, realtime=True)
    srv.close()
    s = rep.summary()
    assert s["completed"] == len(reqs)
    assert s["p50_ms"] > 0 and s["p99_ms"] >= s["p50_ms"]
    for i in (0, 17, 59):
        a = serve_alone(reqs[i])
        assert abs(a.value - rep.results[i].value) <= 1e-12 * max(1.0, abs(a.value))


def test_admission_waits_for_pool_memory():
    reqs = small_requests(12, seed=13)
    # a pool that holds only a few request workspaces at a time
    from paper_2205_10091_amd import api
    sizes = []
    for rq in reqs:
        net = api.Network(rq.circuit, rq.observable)
        plan = api.Plan(net, api.Path(net, n_trials=4, seed=0x5eed), want_grad=rq.want_grad)
        sizes.append(plan.info().workspace_bytes)
    pool = int(max(sizes) * 2.5)
    srv = serve.Server(pool_bytes=pool, max_request_bytes=pool, max_active=16)
    rep = serve.run(srv, reqs, realtime=False)
    srv.close()
    assert len(rep.results) == len(reqs) and not rep.rejected
    for i, rq in enumerate(reqs):
        if rq.circuit.n_qubits <= 16:
            e_ref = sv.energy(rq.circuit, rq.params, rq.observable).real
            assert rel_err(rep.results[i].value, e_ref, 1.0) < TOL_C64


def test_oversize_request_is_rejected():
    circ = tcgen.grid_ladder(8, 8, 6)
    obs = tcgen.tfim_zz_x_grid(8, 8)
    p = tcgen.draw_angles(1, (circ.n_params,))
    srv = serve.Server(pool_bytes=1 << 30, max_request_bytes=64 << 20, max_active=4)
    with pytest.raises(L.TcxError) as e:
        srv.submit(circ, obs, p, False)
    assert e.value.status == L.TC_ERR_TOO_LARGE
    srv.close()
