"""C-ABI library: loads, exports every declared symbol, host-side calls work
and fail cleanly (no GPU needed; no compute call is made)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import tcgen
from paper_2205_10091_amd import _lib as L
from paper_2205_10091_amd import api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tcx.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tc_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = L.load()
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), f"libtcx.so does not export {n}"
    # the binding declares exactly the header's functions
    assert sorted(s[0] for s in L.SIGNATURES) == names


def test_status_strings_and_version():
    lib = L.load()
    assert lib.tc_status_string(0) == b"ok"
    assert lib.tc_status_string(4) == b"too large"
    assert lib.tc_version() >= 100


def test_invalid_circuits_are_rejected():
    c = tcgen.Circuit(3, 1)
    c.gates.append(tcgen.Gate("rzz", (0, 0), (0,), (0.0,)))
    with pytest.raises(L.TcxError) as e:
        api.Network(c, tcgen.pauli_string(3, z=(0,)))
    assert e.value.status == L.TC_ERR_INVALID_ARG
    c = tcgen.Circuit(3, 1)
    c.gates.append(tcgen.Gate("rx", (5,), (0,), (0.0,)))
    with pytest.raises(L.TcxError) as e:
        api.Network(c, tcgen.pauli_string(3, z=(0,)))
    assert "qubit out of range" in str(e.value)
    c = tcgen.Circuit(3, 1)
    c.gates.append(tcgen.Gate("rx", (1,), (3,), (0.0,)))
    with pytest.raises(L.TcxError):
        api.Network(c, tcgen.pauli_string(3, z=(0,)))
    obs = tcgen.Observable("pauli_sum", structures=np.array([[0, 4, 0]], np.uint8),
                           weights=np.array([1.0]))
    with pytest.raises(L.TcxError):
        api.Network(tcgen.chain_ladder(3, 1), obs)


def test_unknown_gate_kind_is_unsupported():
    lib = L.load()
    g = (L.Gate * 1)()
    g[0].kind = 99
    circ = L.Circuit(2, 0, 1, C.cast(g, C.POINTER(L.Gate)))
    obs = L.Observable(0, None, 0, None, None)
    h = C.c_void_p()
    assert lib.tc_build_network(C.byref(circ), C.byref(obs), None, C.byref(h)) == \
        L.TC_ERR_UNSUPPORTED
    assert b"unknown kind" in lib.tc_last_error()


def test_free_null_is_noop():
    lib = L.load()
    lib.tc_network_free(None)
    lib.tc_path_free(None)
    lib.tc_plan_free(None)
    lib.tc_serve_free(None)


def test_bad_path_is_rejected():
    circ, _, _, amp = tcgen.workload_forward_chain()
    net = api.Network(circ, amp)
    path = api.Path(net)
    pairs = path.pairs(0).copy()
    bad = pairs.copy()
    bad[3] = bad[2]
    with pytest.raises(L.TcxError):
        path.replace_term(0, bad)
    with pytest.raises(L.TcxError):
        path.replace_term(0, pairs[:-1])
    path.replace_term(0, pairs)  # the original is accepted


def test_checkpointing_shrinks_the_workspace_under_a_budget():
    circ, p, obs = tcgen.workload_vqe_chain()
    net = api.Network(circ, obs)
    path = api.Path(net, n_trials=8, seed=1)
    full = api.Plan(net, path, batch=256, want_grad=True, checkpoint_every=-1).info()
    forced = api.Plan(net, path, batch=256, want_grad=True, checkpoint_every=3).info()
    assert full.checkpoint_every == 0 and forced.checkpoint_every == 3
    assert forced.workspace_bytes < full.workspace_bytes
    assert forced.grad_flops > full.grad_flops          # recomputation
    assert forced.flops == full.flops
    budget = (full.workspace_bytes + forced.workspace_bytes) // 2
    auto = api.Plan(net, path, batch=256, want_grad=True, mem_budget_bytes=budget).info()
    # 39 terms: the planner first runs them in groups (no recomputation)
    assert auto.n_term_groups > 1 and auto.checkpoint_every == 0
    assert auto.workspace_bytes <= budget and auto.grad_flops == full.grad_flops
    # one term: only checkpointed segments can shrink the workspace
    one = tcgen.Observable("pauli_sum", structures=obs.structures[:1], weights=obs.weights[:1])
    net1 = api.Network(circ, one)
    path1 = api.Path(net1, n_trials=8, seed=1)
    full1 = api.Plan(net1, path1, batch=256, want_grad=True, checkpoint_every=-1).info()
    forced1 = api.Plan(net1, path1, batch=256, want_grad=True, checkpoint_every=3).info()
    assert forced1.workspace_bytes < full1.workspace_bytes
    budget1 = (full1.workspace_bytes + forced1.workspace_bytes) // 2
    auto1 = api.Plan(net1, path1, batch=256, want_grad=True, mem_budget_bytes=budget1).info()
    assert auto1.checkpoint_every >= 2 and auto1.n_term_groups == 1
    assert auto1.workspace_bytes <= budget1
    with pytest.raises(L.TcxError) as e:
        api.Plan(net, path, batch=256, want_grad=True, checkpoint_every=1)
    assert e.value.status == L.TC_ERR_INVALID_ARG


def test_plan_is_host_only_and_reports_sizes():
    circ, p, obs = tcgen.workload_vqe_chain()
    net = api.Network(circ, obs)
    path = api.Path(net, n_trials=4, seed=1)
    plan = api.Plan(net, path, batch=1, want_grad=True)
    info = plan.info()
    st = path.stats()
    assert info.n_terms == 39
    assert info.n_nodes == st.n_steps
    assert info.n_params == 240
    # forward flops of the plan equal the path's flops (8 per complex MAC)
    assert abs(info.flops - st.flops) <= 1e-9 * st.flops
    assert info.grad_flops > info.flops
    assert info.workspace_bytes > 0
    plan4 = api.Plan(net, path, batch=1024, want_grad=True)
    assert plan4.info().flops > 900 * info.flops
    with pytest.raises(L.TcxError) as e:
        api.Plan(net, path, batch=1024, want_grad=True, mem_budget_bytes=1 << 20)
    assert e.value.status == L.TC_ERR_TOO_LARGE


def test_tile_mode_wide_nodes_and_split_sums_on_host():
    # the 6x6 depth-12 grid's widest nodes take 128 x 128 tiles by default
    # (the planner stores their operands dense), none with tile_mode 1
    circ, p, amp = tcgen.workload_grid_amplitude(6, 6, 12)
    net = api.Network(circ, amp)
    path = api.Path(net, n_trials=32, seed=1)
    auto = api.Plan(net, path).info()
    assert auto.n_wide_nodes > 0
    assert api.Plan(net, path, tile_mode=1).info().n_wide_nodes == 0
    # the wide tiles read their operands as planes (8 bytes per element of
    # workspace, FP32 and split BF16 alike); under a budget that leaves no
    # room for them the wide nodes fall back to 64 x 64 tiles instead of
    # failing
    for prec in (0, 1):
        wide = api.Plan(net, path, precision=prec).info()
        ws64 = api.Plan(net, path, precision=prec, tile_mode=1).info().workspace_bytes
        assert wide.n_wide_nodes > 0 and wide.workspace_bytes > ws64
        budget = ws64 + (64 << 20)
        assert budget < wide.workspace_bytes
        tight = api.Plan(net, path, precision=prec, mem_budget_bytes=budget).info()
        assert tight.n_wide_nodes == 0 and tight.workspace_bytes <= budget
    for bad in (-1, 3):
        with pytest.raises(L.TcxError) as e:
            api.Plan(net, path, tile_mode=bad)
        assert e.value.status == L.TC_ERR_INVALID_ARG
    # the 4x6 depth-12 grid ends in a long inner product: split sums
    circ, p, amp = tcgen.workload_grid_amplitude(4, 6, 12)
    net = api.Network(circ, amp)
    path = api.Path(net, n_trials=32, seed=1)
    info = api.Plan(net, path).info()
    assert info.n_split_sums >= 1
    # forced wide tiles on a small tree (used by the GPU tests) are valid plans
    assert api.Plan(net, path, tile_mode=2).info().n_wide_nodes >= 0


def test_batched_plan_uses_masked_wave_tiles():
    # at 1024 rows, nodes with M, N, K >= 8 below the GEMM rule go to the
    # GEMM branch (masked wave tiles): many more GEMM nodes than at 1 row
    circ, P, obs = tcgen.workload_batched_vqe(batch=1024)
    net = api.Network(circ, obs)
    path = api.Path(net, n_trials=4, seed=1)
    many = api.Plan(net, path, batch=1024, want_grad=True).info().n_gemm_nodes
    few = api.Plan(net, path, batch=32, want_grad=True).info().n_gemm_nodes
    assert many > 2 * max(few, 1)
