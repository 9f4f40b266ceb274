"""GPU parity of sliced contractions (tc_slice: bonds fixed value by value,
the slices summed as terms; section "Outlook and concluding remarks")."""
import json
import os

import numpy as np
import pytest

import tcgen
from oracle import statevector as sv
from paper_2205_10091_amd import api
from paper_2205_10091_amd import serve
from gpu_common import TOL_C64, assert_grad, device_params, rel_err, true_rel_err

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_sliced_grid_amplitude_against_golden():
    path = os.path.join(GOLDEN, "grid6x6_d8_amplitude.json")
    if not os.path.exists(path):
        pytest.skip("reference amplitude not generated")
    ref = json.load(open(path))
    r = complex(ref["values"]["col2"]["re"], ref["values"]["col2"]["im"])
    circ, p, amp = tcgen.workload_grid_amplitude()
    net = api.Network(circ, amp)
    pth = api.Path(net, n_trials=32, seed=1)
    peak = int(round(pth.stats().log2_size))
    snet, spath, s = pth.sliced(peak - 4)
    assert s >= 2
    plan = api.Plan(snet, spath)
    plan.bind_torch()
    a = plan.contract(device_params(p))[0]
    print(f"6x6 depth 8 sliced into {2 ** s} networks of at most 2^{peak - 4}: "
          f"true relative error {true_rel_err(a, r):.2e}")
    assert true_rel_err(a, r) < TOL_C64


def test_sliced_energy_and_gradient_against_oracle():
    circ = tcgen.chain_ladder(12, 4)
    obs = tcgen.tfim_zz_x(12, 0.8)
    p = tcgen.draw_angles(6, (circ.n_params,))
    net = api.Network(circ, obs)
    pth = api.Path(net, n_trials=4, seed=1)
    peak = int(round(pth.stats().log2_size))
    snet, spath, s = pth.sliced(peak - 3)
    assert s >= 1
    plan = api.Plan(snet, spath, want_grad=True)
    plan.bind_torch()
    e, g = plan.contract_grad(device_params(p))
    e_ref, g_ref = sv.energy_grad(circ, p, obs)
    assert rel_err(e[0], e_ref, 1.0) < TOL_C64
    assert_grad(g[0], g_ref, TOL_C64)


def test_serving_slices_a_request_that_does_not_fit():
    """The 6x6 depth-8 grid amplitude (single-trial path: 2^25-element
    intermediates, 574 MB live) under a 256 MiB per-request cap: the engine
    slices it (8 slices in groups) and the result matches the oracle's
    amplitude; with a flops limit below its cost it is rejected instead."""
    path = os.path.join(GOLDEN, "grid6x6_d8_amplitude.json")
    if not os.path.exists(path):
        pytest.skip("reference amplitude not generated")
    ref = json.load(open(path))
    r = complex(ref["values"]["col2"]["re"], ref["values"]["col2"]["im"])
    circ, p, amp = tcgen.workload_grid_amplitude()
    rq = tcgen.Request(0, 0.0, circ, amp, p, False, "grid", 8)
    srv = serve.Server(pool_bytes=2 << 30, max_request_bytes=256 << 20, max_active=4,
                       path_trials=1)
    rep = serve.run(srv, [rq], realtime=False)
    srv.close()
    assert not rep.rejected, rep.reasons
    a = complex(rep.results[0].value, rep.results[0].value_im)
    print(f"served sliced amplitude: true relative error {true_rel_err(a, r):.2e}")
    assert true_rel_err(a, r) < TOL_C64
    srv = serve.Server(pool_bytes=2 << 30, max_request_bytes=256 << 20, max_active=4,
                       path_trials=1, max_request_flops=1e9)
    rep = serve.run(srv, [rq], realtime=False)
    srv.close()
    assert rep.rejected == [0] and "flops" in rep.reasons[0]
