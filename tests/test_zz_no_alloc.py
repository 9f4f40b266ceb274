"""The no-allocation contraction entry point against the bound-workspace one.

tc_contract_grad_device_noalloc runs a plan in the library's static per-GPU
scratch array; tc_contract_grad_device runs the same plan in its bound
workspace.  Both go through the C ABI.  Two calls in a row, the second on a
smaller plan (the array keeps the first call's contents), then the first
plan again; every result also against the complex128 oracle."""
import numpy as np
import pytest

import tcgen
from oracle import statevector as sv
from paper_2205_10091_amd import _lib as L
from paper_2205_10091_amd import api
from gpu_common import TOL_C64, device_params, grad_err, rel_err

pytestmark = pytest.mark.gpu


def _both(plan, P, B):
    import torch
    p = device_params(P, B)
    v_ref = torch.full((B,), float("nan"), dtype=torch.float64, device="cuda")
    g_ref = torch.full((B, plan.n_params), float("nan"), dtype=torch.float64, device="cuda")
    plan.contract_grad_device(p, v_ref, g_ref)
    torch.cuda.synchronize()
    v = torch.full((B,), float("nan"), dtype=torch.float64, device="cuda")
    g = torch.full((B, plan.n_params), float("nan"), dtype=torch.float64, device="cuda")
    plan.contract_grad_device_noalloc(p, v, g)
    torch.cuda.synchronize()
    return v.cpu().numpy(), g.cpu().numpy(), v_ref.cpu().numpy(), g_ref.cpu().numpy()


def _check(circ, P, obs, B, v, g, v_ref, g_ref):
    # same kernels on the same inputs: the same numbers as the bound plan
    assert np.array_equal(v, v_ref)
    assert np.array_equal(g, g_ref)
    for b in range(B):
        e_o, g_o = sv.energy_grad(circ, P[b], obs)
        assert rel_err(v[b], e_o, 1.0) < TOL_C64
        assert grad_err(g[b], g_o) < TOL_C64
        assert np.max(np.abs(g[b] - g_o)) < TOL_C64


def test_noalloc_matches_bound_workspace_twice_then_smaller():
    big = tcgen.workload_batched_vqe(batch=4, n=14, layers=5)
    small = tcgen.workload_batched_vqe(batch=2, n=8, layers=3)
    plans = []
    for (circ, P, obs), B in ((big, 4), (small, 2)):
        plan = api.compile(circ, obs, batch=B, want_grad=True)
        assert plan.info().workspace_bytes <= (64 << 20)
        plans.append(plan)
    assert plans[1].info().workspace_bytes < plans[0].info().workspace_bytes
    for (circ, P, obs), B, plan in ((big, 4, plans[0]), (small, 2, plans[1]),
                                    (big, 4, plans[0])):
        v, g, v_ref, g_ref = _both(plan, P, B)
        _check(circ, P, obs, B, v, g, v_ref, g_ref)


def test_noalloc_unbound_plan_and_errors():
    import torch
    circ, P, obs = tcgen.workload_batched_vqe(batch=3, n=10, layers=3)
    plan = api.compile(circ, obs, batch=3, want_grad=True, bind=False)
    v = torch.zeros(3, dtype=torch.float64, device="cuda")
    g = torch.zeros(3, plan.n_params, dtype=torch.float64, device="cuda")
    plan.contract_grad_device_noalloc(device_params(P, 3), v, g)
    torch.cuda.synchronize()
    for b in range(3):
        e_o, g_o = sv.energy_grad(circ, P[b], obs)
        assert rel_err(v[b].item(), e_o, 1.0) < TOL_C64
        assert np.max(np.abs(g[b].cpu().numpy() - g_o)) < TOL_C64
    # a plan without the reverse sweep
    fwd = api.compile(circ, obs, batch=3, bind=False)
    with pytest.raises(L.TcxError) as e:
        fwd.contract_grad_device_noalloc(device_params(P, 3), v, g)
    assert e.value.status == L.TC_ERR_STATE
    # a workspace beyond the static array: rejected before any device work
    cb, PB, ob = tcgen.workload_batched_vqe(batch=1024)
    huge = api.compile(cb, ob, batch=1024, want_grad=True, bind=False, n_trials=1)
    assert huge.info().workspace_bytes > (64 << 20)
    vb = torch.zeros(1024, dtype=torch.float64, device="cuda")
    gb = torch.zeros(1024, huge.n_params, dtype=torch.float64, device="cuda")
    with pytest.raises(L.TcxError) as e:
        huge.contract_grad_device_noalloc(device_params(PB, 1024), vb, gb)
    assert e.value.status == L.TC_ERR_TOO_LARGE
