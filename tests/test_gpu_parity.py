"""GPU parity: the HIP contraction path against the CPU oracle.

Every value is computed by libtcx.so through the C ABI (the Python binding
only marshals arguments) and compared with the oracle on the same seeded
inputs, at the tolerance of the plain complex64 form (1e-5 relative with the
amplitude floor 2^(-n/2), energies and expectations floored at 1)."""
import json
import math
import os

import numpy as np
import pytest

import tcgen
from oracle import statevector as sv
from paper_2205_10091_amd import _lib as L
from paper_2205_10091_amd import api
from gpu_common import TOL_C64, assert_grad, device_params, grad_err, rel_err, true_rel_err

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def one(circ, obs, params, **kw):
    plan = api.compile(circ, obs, **kw)
    return plan, plan.contract(device_params(params))[0]


def test_library_is_the_native_build():
    lib = L.load()
    assert os.path.basename(lib._name) == "libtcx.so"


# ------------------------------------------------------------ forward chain

def test_forward_chain_amplitude_and_zz():
    circ, p, zz, amp = tcgen.workload_forward_chain()
    n = circ.n_qubits
    _, a = one(circ, amp, p)
    assert rel_err(a, sv.amplitude(circ, p), 2 ** (-n / 2)) < TOL_C64
    _, z = one(circ, zz, p)
    ref = sv.energy(circ, p, zz)
    assert rel_err(z, ref, 1.0) < TOL_C64
    assert abs(z.imag) < TOL_C64


@pytest.mark.parametrize("split,lightcone", [(0, 0), (1, 0), (0, 1)])
def test_forward_chain_network_options(split, lightcone):
    circ, p, zz, amp = tcgen.workload_forward_chain()
    _, z = one(circ, zz, p, split_2q=split, lightcone=lightcone)
    assert rel_err(z, sv.energy(circ, p, zz), 1.0) < TOL_C64


def test_amplitudes_of_several_bitstrings():
    circ, p, _, _ = tcgen.workload_forward_chain()
    n = circ.n_qubits
    rng = np.random.default_rng(0)
    for _ in range(4):
        bits = tuple(int(b) for b in rng.integers(0, 2, n))
        _, a = one(circ, tcgen.amplitude(n, bits), p)
        assert rel_err(a, sv.amplitude(circ, p, bits), 2 ** (-n / 2)) < TOL_C64


# ------------------------------------------------------------ VQE energy + gradient

def test_vqe_chain_energy_and_gradient():
    circ, p, obs = tcgen.workload_vqe_chain()
    plan = api.compile(circ, obs, want_grad=True, n_trials=8, seed=1)
    e, g = plan.contract_grad(device_params(p))
    e_ref, g_ref = sv.energy_grad(circ, p, obs)
    assert rel_err(e[0], e_ref, 1.0) < TOL_C64
    assert_grad(g[0], g_ref, TOL_C64)
    # slots no gate reaches are exactly zero; the first RZZ layer has zero
    # gradient up to rounding
    gg = g[0].reshape(6, 2, 20)
    assert np.all(gg[:, 0, 19] == 0.0)
    assert np.max(np.abs(gg[0, 0, :])) < 1e-5
    # forward-only call of the same plan agrees with the gradient call
    v = plan.contract(device_params(p))[0]
    assert abs(v.real - e[0]) < 1e-6 and abs(v.imag) < TOL_C64


def test_vqe_chain_in_the_benchmark_configuration():
    """The plan the benchmark times: 1024 path trials and the depth cap of
    the path finder's time model, device-resident outputs."""
    import torch
    circ, p, obs = tcgen.workload_vqe_chain()
    plan = api.compile(circ, obs, want_grad=True, n_trials=1024, seed=1, max_depth=-1)
    info = plan.info()
    assert info.n_levels <= 18
    e_dev = torch.empty(1, dtype=torch.float64, device="cuda")
    g_dev = torch.empty(circ.n_params, dtype=torch.float64, device="cuda")
    plan.contract_grad_device(device_params(p), e_dev, g_dev)
    e_ref, g_ref = sv.energy_grad(circ, p, obs)
    print(f"benchmark plan: {info.n_levels} levels, |dE| {abs(e_dev.item() - e_ref):.2e}")
    assert rel_err(e_dev.item(), e_ref, 1.0) < TOL_C64
    assert_grad(g_dev.cpu().numpy(), g_ref, TOL_C64, "benchmark plan")


def test_device_outputs_in_place_match_staged_outputs():
    """tc_contract_grad_device reads the parameters and writes E and the
    gradient in place through a graph captured for those three buffers:
    the same kernels as the staged path (host outputs), so the results are
    bit-identical, on a second call with the same buffers holding new
    parameters, and after a switch to other output buffers (a new capture)."""
    import torch
    B = 8
    circ, P, obs = tcgen.workload_batched_vqe(batch=B, n=12, layers=4)
    plan = api.compile(circ, obs, batch=B, want_grad=True, n_trials=4, seed=1)
    npar = circ.n_params
    rng = np.random.default_rng(5)
    P2 = (P + rng.normal(0, 0.3, P.shape)).astype(np.float32)
    pd = device_params(P, B)
    e_dev = torch.empty(B, dtype=torch.float64, device="cuda")
    g_dev = torch.empty(B * npar, dtype=torch.float64, device="cuda")
    for params in (P, P2):
        pd.copy_(device_params(params, B))
        e_h, g_h = plan.contract_grad(device_params(params, B))
        plan.contract_grad_device(pd, e_dev, g_dev)
        assert np.array_equal(e_dev.cpu().numpy(), e_h)
        assert np.array_equal(g_dev.cpu().numpy().reshape(B, npar), g_h.reshape(B, npar))
    e2 = torch.empty(B, dtype=torch.float64, device="cuda")
    g2 = torch.empty(B * npar, dtype=torch.float64, device="cuda")
    plan.contract_grad_device(pd, e2, g2)
    assert np.array_equal(e2.cpu().numpy(), e_dev.cpu().numpy())
    assert np.array_equal(g2.cpu().numpy(), g_dev.cpu().numpy())
    e_ref, g_ref = sv.energy_grad(circ, P2[3], obs)
    assert rel_err(e2[3].item(), e_ref, 1.0) < TOL_C64
    assert_grad(g2.cpu().numpy().reshape(B, npar)[3], g_ref, TOL_C64)


def test_vqe_gradient_vs_parameter_shift_and_fd_on_gpu():
    """The GPU gradient against the GPU's own energies at shifted angles:
    the exact two-point shift rule and central differences (h = 1e-3)."""
    n, Ld = 8, 3
    circ = tcgen.chain_ladder(n, Ld)
    obs = tcgen.tfim_zz_x(n, 1.0)
    p = tcgen.draw_angles(31, (Ld, 2, n)).reshape(-1)
    gplan = api.compile(circ, obs, want_grad=True)
    _, g = gplan.contract_grad(device_params(p))
    P = len(p)
    shifts = []
    for s in range(P):
        for d in (math.pi / 2, -math.pi / 2, 1e-3, -1e-3):
            q = p.astype(np.float64).copy()
            q[s] += d
            shifts.append(q)
    B = len(shifts)
    fplan = api.compile(circ, obs, batch=B)
    vals = fplan.contract(device_params(np.array(shifts, np.float32), B)).real.reshape(P, 4)
    ps = 0.5 * (vals[:, 0] - vals[:, 1])
    fd = (vals[:, 2] - vals[:, 3]) / 2e-3
    assert grad_err(g[0], ps) < 1e-5
    # fp32 energies limit central differences to ~1e-7/1e-3 per slot
    assert grad_err(g[0], fd) < 2e-3
    # and both against the oracle
    _, g_ref = sv.energy_grad(circ, p, obs)
    assert grad_err(ps, g_ref) < 1e-5


# ------------------------------------------------------------ batched sweep

def test_batched_sweep_matches_oracle_and_single_calls():
    B = 64
    circ, P, obs = tcgen.workload_batched_vqe(batch=B, n=12, layers=4)
    plan = api.compile(circ, obs, batch=B, want_grad=True, n_trials=4, seed=1)
    e, g = plan.contract_grad(device_params(P, B))
    single = api.compile(circ, obs, want_grad=True, n_trials=4, seed=1)
    for b in (0, 17, 63):
        e_ref, g_ref = sv.energy_grad(circ, P[b], obs)
        assert rel_err(e[b], e_ref, 1.0) < TOL_C64
        assert_grad(g[b], g_ref, TOL_C64)
        e1, g1 = single.contract_grad(device_params(P[b]))
        assert abs(e1[0] - e[b]) < 1e-6
        assert np.max(np.abs(g1[0] - g[b])) < 1e-6


@pytest.mark.parametrize("B", [100, 200])
def test_batched_sweep_ragged_rows(B):
    """Batch sizes that are not a multiple of the 64 rows a row-tile
    workgroup stages (100 = 64 + 36, 200 = 3 x 64 + 8), so the last row
    tile of every small batched node is partial and the masked wave tiles
    run over a ragged row count: every row against a batch-1 plan called
    row by row, sampled rows (first, last, the first of the partial tile)
    against the oracle.  As in the full-size test below, the differences
    between the two plans are divided by sum_j |a_j| (|dE| <= sum_j |a_j|
    |dT_j| for E summed in FP64 from complex64 terms T_j)."""
    circ, P, obs = tcgen.workload_batched_vqe(batch=B, n=12, layers=4)
    plan = api.compile(circ, obs, batch=B, want_grad=True, n_trials=4, seed=1)
    e, g = plan.contract_grad(device_params(P, B))
    assert np.all(np.isfinite(e)) and np.all(np.isfinite(g))
    for b in (0, 64, B - 1):
        e_ref, g_ref = sv.energy_grad(circ, P[b], obs)
        assert rel_err(e[b], e_ref, 1.0) < TOL_C64
        assert_grad(g[b], g_ref, TOL_C64)
    single = api.compile(circ, obs, want_grad=True, n_trials=4, seed=1)
    pd = device_params(P, B)
    scale = float(np.sum(np.abs(obs.weights)))
    for b in range(B):
        e1, g1 = single.contract_grad(pd[b].contiguous())
        assert abs(e1[0] - e[b]) / scale < 1e-6, b
        assert np.max(np.abs(g1[0] - g[b])) / scale < 1e-6, b


def test_batched_sweep_full_size_every_row():
    """1024 parameter vectors in one launch: every row's energy and every
    gradient component against a batch-1 plan of the same network called
    row by row, and sampled rows against the oracle.  E = sum_j a_j T_j is
    summed in FP64 from complex64 terms, so |dE| <= sum_j |a_j| |dT_j|: the
    differences are divided by sum_j |a_j| (39 here), which leaves the
    per-term contraction difference, required below 1e-6."""
    B = 1024
    circ, P, obs = tcgen.workload_batched_vqe(batch=B)
    plan = api.compile(circ, obs, batch=B, want_grad=True, n_trials=8, seed=1)
    e, g = plan.contract_grad(device_params(P, B))
    assert np.all(np.isfinite(e)) and np.all(np.isfinite(g))
    for b in (0, 511, 1023):
        e_ref, g_ref = sv.energy_grad(circ, P[b], obs)
        assert rel_err(e[b], e_ref, 1.0) < TOL_C64
        assert_grad(g[b], g_ref, TOL_C64)
    del plan
    single = api.compile(circ, obs, want_grad=True, n_trials=8, seed=1)
    pd = device_params(P, B)
    scale = float(np.sum(np.abs(obs.weights)))
    worst_e = worst_g = worst_rel = 0.0
    for b in range(B):
        e1, g1 = single.contract_grad(pd[b].contiguous())
        worst_e = max(worst_e, abs(e1[0] - e[b]))
        worst_rel = max(worst_rel, abs(e1[0] - e[b]) / max(1.0, abs(e1[0])))
        worst_g = max(worst_g, float(np.max(np.abs(g1[0] - g[b]))))
    print(f"batch 1024 vs batch 1 over {B} rows: max |dE| {worst_e:.2e} "
          f"(relative to |E|: {worst_rel:.2e}), max gradient component diff {worst_g:.2e}; "
          f"sum |a_j| = {scale}")
    assert worst_e / scale < 1e-6 and worst_g / scale < 1e-6


# ------------------------------------------------------------ grid amplitudes

@pytest.mark.parametrize("rows,cols", [(2, 4), (3, 3), (4, 4)])
def test_grid_amplitude_small(rows, cols):
    circ, p, amp = tcgen.workload_grid_amplitude(rows, cols, 8)
    n = circ.n_qubits
    for seed in (0, 1):
        _, a = one(circ, amp, p, n_trials=8, seed=seed)
        assert rel_err(a, sv.amplitude(circ, p), 2 ** (-n / 2)) < TOL_C64


def test_grid_amplitude_full_size_against_golden():
    path = os.path.join(GOLDEN, "grid6x6_d8_amplitude.json")
    if not os.path.exists(path):
        pytest.skip("reference amplitude not generated")
    ref = json.load(open(path))
    vals = [complex(v["re"], v["im"]) for v in ref["values"].values()]
    assert abs(vals[0] - vals[1]) <= 1e-12 * abs(vals[0])
    circ, p, amp = tcgen.workload_grid_amplitude()
    _, a = one(circ, amp, p, n_trials=32, seed=1)
    # the amplitude (|ref| = 3.8e-7) is far below the 2^-18 floor, so the
    # unfloored relative error is checked as well
    print(f"6x6 depth 8, c64: rel_err {rel_err(a, vals[0], 2 ** (-18)):.2e}, "
          f"true relative error {true_rel_err(a, vals[0]):.2e}")
    assert rel_err(a, vals[0], 2 ** (-18)) < TOL_C64
    assert true_rel_err(a, vals[0]) < TOL_C64


def test_split_k_wide_nodes_fp32_and_bf16x3():
    """The 6x6 grid's widest nodes have few output tiles and deep K, so
    their K is cut into slices; a reduction kernel adds the slices' partial
    tiles in slice order.  Both precisions against the oracle's amplitude,
    and repeated calls bit-identical."""
    from gpu_common import TOL_BF16X3
    path = os.path.join(GOLDEN, "grid6x6_d8_amplitude.json")
    if not os.path.exists(path):
        pytest.skip("reference amplitude not generated")
    ref = json.load(open(path))
    r = complex(ref["values"]["col2"]["re"], ref["values"]["col2"]["im"])
    circ, p, amp = tcgen.workload_grid_amplitude()
    for prec, tol in ((0, TOL_C64), (1, TOL_BF16X3)):
        plan = api.compile(circ, amp, n_trials=32, seed=1, precision=prec)
        assert plan.info().n_split_nodes > 0
        a1 = plan.contract(device_params(p))[0]
        a2 = plan.contract(device_params(p))[0]
        assert a1 == a2, prec
        print(f"6x6 depth 8, precision {prec}: rel_err {rel_err(a1, r, 2 ** (-18)):.2e}, "
              f"true relative error {true_rel_err(a1, r):.2e}")
        assert rel_err(a1, r, 2 ** (-18)) < tol, prec
        assert true_rel_err(a1, r) < tol, prec


def test_split_sums_deep_grid_fp32_and_bf16x3():
    """The 4x6 depth-12 grid ends in a long sum with few outputs; its K is
    cut into slices summed by the split gather kernel and added in slice
    order by the reduction.  Both precisions against the oracle's amplitude
    (state vector and time-order sweep, stored), repeats bit-identical."""
    from gpu_common import TOL_BF16X3
    path = os.path.join(GOLDEN, "grid4x6_d12_amplitude.json")
    if not os.path.exists(path):
        pytest.skip("reference amplitude not generated")
    ref = json.load(open(path))
    r = complex(ref["values"]["statevector"]["re"], ref["values"]["statevector"]["im"])
    circ, p, amp = tcgen.workload_grid_amplitude(4, 6, 12)
    for prec, tol in ((0, TOL_C64), (1, TOL_BF16X3)):
        plan = api.compile(circ, amp, n_trials=32, seed=1, precision=prec)
        assert plan.info().n_split_sums > 0
        a1 = plan.contract(device_params(p))[0]
        a2 = plan.contract(device_params(p))[0]
        assert a1 == a2, prec
        print(f"4x6 depth 12, precision {prec}: rel_err {rel_err(a1, r, 2 ** (-12)):.2e}, "
              f"true relative error {true_rel_err(a1, r):.2e}")
        assert rel_err(a1, r, 2 ** (-12)) < tol, prec
        assert true_rel_err(a1, r) < tol, prec


def test_wide_tiles_against_golden_and_64_tiles():
    """128 x 128 tiles (dense operands, FP32 and split BF16) on the 6x6
    depth-8 and 4x6 depth-12 grids, forced onto every node whose operands
    allow them, against the oracle's amplitudes; repeats bit-identical."""
    from gpu_common import TOL_BF16X3
    cases = []
    for (rows, cols, depth, key) in ((6, 6, 8, "col2"), (4, 6, 12, "statevector")):
        path = os.path.join(GOLDEN, f"grid{rows}x{cols}_d{depth}_amplitude.json")
        if not os.path.exists(path):
            pytest.skip("reference amplitude not generated")
        ref = json.load(open(path))
        cases.append((rows, cols, depth, complex(ref["values"][key]["re"], ref["values"][key]["im"])))
    for rows, cols, depth, r in cases:
        circ, p, amp = tcgen.workload_grid_amplitude(rows, cols, depth)
        floor = 2 ** (-rows * cols / 2)
        for prec, tol in ((0, TOL_C64), (1, TOL_BF16X3)):
            plan = api.compile(circ, amp, n_trials=32, seed=1, precision=prec, tile_mode=2)
            assert plan.info().n_wide_nodes > 0
            a1 = plan.contract(device_params(p))[0]
            a2 = plan.contract(device_params(p))[0]
            assert a1 == a2, (rows, cols, prec)
            print(f"{rows}x{cols} depth {depth}, forced 128x128 tiles, precision {prec}: "
                  f"rel_err {rel_err(a1, r, floor):.2e}, true relative error {true_rel_err(a1, r):.2e}")
            assert rel_err(a1, r, floor) < tol, (rows, cols, prec)
            assert true_rel_err(a1, r) < tol, (rows, cols, prec)
            ref64 = api.compile(circ, amp, n_trials=32, seed=1, precision=prec, tile_mode=1)
            assert ref64.info().n_wide_nodes == 0
            assert rel_err(a1, ref64.contract(device_params(p))[0], floor) < tol


@pytest.mark.parametrize("rows,cols", [(5, 5), (4, 7)])
def test_wide_tiles_default_plan_against_golden(rows, cols):
    """Depth-16 grids whose default plan (no tile forcing, 32 greedy trials)
    puts its widest nodes on 128 x 128 tiles: launches of 256 to 65536
    tiles, both tile orders (XCD-striped where the tile grid allows it,
    row-major otherwise), K from 32 to 16384.  FP32 and split BF16 against
    the stored oracle amplitude (state vector and time-order sweep, which
    agree to ~1e-15); repeats bit-identical."""
    from gpu_common import TOL_BF16X3
    path = os.path.join(GOLDEN, f"grid{rows}x{cols}_d16_amplitude.json")
    if not os.path.exists(path):
        pytest.skip("reference amplitude not generated")
    ref = json.load(open(path))
    r = complex(ref["values"]["statevector"]["re"], ref["values"]["statevector"]["im"])
    r2 = complex(ref["values"]["time"]["re"], ref["values"]["time"]["im"])
    assert abs(r - r2) <= 1e-12 * abs(r)
    circ, p, amp = tcgen.workload_grid_amplitude(rows, cols, 16)
    floor = 2 ** (-rows * cols / 2)
    for prec, tol in ((0, TOL_C64), (1, TOL_BF16X3)):
        plan = api.compile(circ, amp, n_trials=32, seed=1, precision=prec)
        assert plan.info().n_wide_nodes > 0
        a1 = plan.contract(device_params(p))[0]
        a2 = plan.contract(device_params(p))[0]
        del plan
        assert a1 == a2, prec
        print(f"{rows}x{cols} depth 16, default plan, precision {prec}: "
              f"rel_err {rel_err(a1, r, floor):.2e}, true relative error {true_rel_err(a1, r):.2e}")
        assert rel_err(a1, r, floor) < tol, prec
        assert true_rel_err(a1, r) < tol, prec


def test_reconfigured_paths_against_golden():
    """Subtree-reconfigured trees (frontiers of 8 inputs) of the 6x6 depth-8
    and 5x5 depth-16 grids, both precisions, against the stored oracle
    amplitudes."""
    from gpu_common import TOL_BF16X3
    for rows, cols, depth, key in ((6, 6, 8, "col2"), (5, 5, 16, "statevector")):
        path = os.path.join(GOLDEN, f"grid{rows}x{cols}_d{depth}_amplitude.json")
        if not os.path.exists(path):
            pytest.skip("reference amplitude not generated")
        ref = json.load(open(path))
        r = complex(ref["values"][key]["re"], ref["values"][key]["im"])
        circ, p, amp = tcgen.workload_grid_amplitude(rows, cols, depth)
        for prec, tol in ((0, TOL_C64), (1, TOL_BF16X3)):
            plan = api.compile(circ, amp, n_trials=32, seed=1, precision=prec, reconf_k=8)
            a = plan.contract(device_params(p))[0]
            del plan
            print(f"{rows}x{cols} depth {depth}, reconfigured, precision {prec}: "
                  f"true relative error {true_rel_err(a, r):.2e}")
            assert true_rel_err(a, r) < tol


def test_wide_tiles_full_size_deep_grid():
    """The 6x6 depth-12 grid's 16384 x 65536 x 4096 node runs 128 x 128
    tiles by default: FP32 against the 64 x 64 tiles of the same tree, and
    split BF16 against FP32 (no oracle amplitude at this depth: 2^36
    entries)."""
    from gpu_common import TOL_BF16X3
    circ, p, amp = tcgen.workload_grid_amplitude(6, 6, 12)
    floor = 2 ** -18
    wide = api.compile(circ, amp, n_trials=32, seed=1)
    assert wide.info().n_wide_nodes > 0
    a = wide.contract(device_params(p))[0]
    del wide
    narrow = api.compile(circ, amp, n_trials=32, seed=1, tile_mode=1)
    assert narrow.info().n_wide_nodes == 0
    b = narrow.contract(device_params(p))[0]
    del narrow
    assert rel_err(a, b, floor) < TOL_C64
    w16 = api.compile(circ, amp, n_trials=32, seed=1, precision=1)
    c = w16.contract(device_params(p))[0]
    del w16
    assert rel_err(c, a, floor) < TOL_BF16X3


# ------------------------------------------------------------ term groups

@pytest.mark.parametrize("rows,cols,depth,grad,budget_mb", [
    (4, 5, 5, False, 512), (4, 5, 5, True, 4096), (3, 6, 6, True, 4096)])
def test_term_groups_match_oracle(rows, cols, depth, grad, budget_mb):
    """Plans whose terms run in groups under a memory budget (each group's
    forward pass and reverse sweep before the next group's; with the 4x5
    gradient also checkpointed segments) against the state-vector oracle."""
    circ = tcgen.grid_ladder(rows, cols, depth)
    obs = tcgen.tfim_zz_x_grid(rows, cols, 0.8)
    p = tcgen.draw_angles(21, (circ.n_params,))
    plan = api.compile(circ, obs, want_grad=grad, n_trials=1, mem_budget_bytes=budget_mb << 20)
    info = plan.info()
    assert info.n_term_groups > 1 and info.workspace_bytes <= budget_mb << 20
    if grad:
        e, g = plan.contract_grad(device_params(p))
        e_ref, g_ref = sv.energy_grad(circ, p, obs)
        assert rel_err(e[0], e_ref, 1.0) < TOL_C64
        assert_grad(g[0], g_ref, TOL_C64)
        # the forward sequence alone of the same plan
        v = plan.contract(device_params(p))[0]
        assert abs(v.real - e[0]) < 1e-6
    else:
        v = plan.contract(device_params(p))[0]
        assert rel_err(v, sv.energy(circ, p, obs), 1.0) < TOL_C64


# ------------------------------------------------------------ edge cases

def test_all_gate_kinds_random_circuits():
    for seed in range(3):
        n = 6
        circ = tcgen.random_circuit(n, 50, seed)
        p = np.random.default_rng(seed).uniform(-3, 3, circ.n_params).astype(np.float32)
        rng = np.random.default_rng(10 + seed)
        s = rng.integers(0, 4, size=(4, n)).astype(np.uint8)
        obs = tcgen.Observable("pauli_sum", structures=s, weights=rng.normal(size=4))
        _, e = one(circ, obs, p)
        ref = sv.energy(circ, p.astype(np.float64), obs)
        scale = max(1.0, float(np.sum(np.abs(obs.weights))))
        assert abs(e - ref) / scale < 1e-5


def test_identity_and_norm():
    circ, p, obs = tcgen.workload_vqe_chain(n=10, layers=3)
    ident = tcgen.Observable("pauli_sum", structures=np.zeros((1, 10), np.uint8),
                             weights=np.array([2.5]))
    _, e = one(circ, ident, p)          # empty network after the light cone
    assert e == 2.5
    _, e = one(circ, ident, p, lightcone=False)   # <psi|psi> contracted
    assert abs(e - 2.5) < 2.5e-5


def test_single_qubit_and_unparameterised_terms():
    c = tcgen.Circuit(1, 1).add("rx", (0,), (0,))
    p = np.array([0.7], np.float32)
    _, z = one(c, tcgen.pauli_string(1, z=(0,)), p)
    assert abs(z - math.cos(0.7)) < 1e-6
    # a term that sees no parameter is shared by every batch row
    c = tcgen.Circuit(3, 1).add("h", (0,)).add("cnot", (0, 1)).add("rx", (2,), (0,))
    obs = tcgen.Observable("pauli_sum", structures=np.array([[3, 3, 0], [0, 0, 3]], np.uint8),
                           weights=np.array([1.0, 1.0]))
    B = 5
    P = np.linspace(0, 3, B).astype(np.float32).reshape(B, 1)
    plan = api.compile(c, obs, batch=B, want_grad=True)
    e, g = plan.contract_grad(device_params(P, B))
    np.testing.assert_allclose(e, 1 + np.cos(P[:, 0].astype(np.float64)), atol=1e-6)
    np.testing.assert_allclose(g[:, 0], -np.sin(P[:, 0].astype(np.float64)), atol=1e-6)


def test_determinism_and_caller_workspace():
    import torch
    circ, p, obs = tcgen.workload_vqe_chain(n=12, layers=4)
    plan = api.compile(circ, obs, want_grad=True, bind=False)
    ws = torch.empty(int(plan.info().workspace_bytes), dtype=torch.uint8, device="cuda")
    plan.bind(ws)
    e1, g1 = plan.contract_grad(device_params(p))
    e2, g2 = plan.contract_grad(device_params(p))
    assert e1[0] == e2[0] and np.array_equal(g1, g2)
    own = api.compile(circ, obs, want_grad=True, bind=False)
    own.bind(None)      # library-allocated workspace
    e3, g3 = own.contract_grad(device_params(p))
    assert e3[0] == e1[0] and np.array_equal(g3, g1)


def test_gemm_path_matches_gather_path():
    """Same trees, once with wide nodes on the MFMA GEMM and once with every
    node on the gather kernels; both against the oracle."""
    circ, p, obs = tcgen.workload_vqe_chain()
    gm = api.compile(circ, obs, want_grad=True, n_trials=8, seed=1, gemm_min_k=4,
                     gemm_min_macs=1)
    gc = api.compile(circ, obs, want_grad=True, n_trials=8, seed=1, gemm_min_k=1 << 30)
    assert gm.info().n_gemm_nodes > 0 and gc.info().n_gemm_nodes == 0
    e1, g1 = gm.contract_grad(device_params(p))
    e2, g2 = gc.contract_grad(device_params(p))
    e_ref, g_ref = sv.energy_grad(circ, p, obs)
    for e, g in ((e1, g1), (e2, g2)):
        assert rel_err(e[0], e_ref, 1.0) < TOL_C64
        assert_grad(g[0], g_ref, TOL_C64)
    # batched rows through the GEMM tiles
    B = 16
    circ, P, obs = tcgen.workload_batched_vqe(batch=B, n=14, layers=5)
    gm = api.compile(circ, obs, batch=B, want_grad=True, gemm_min_k=4, gemm_min_macs=1)
    e, g = gm.contract_grad(device_params(P, B))
    for b in (0, 9):
        e_ref, g_ref = sv.energy_grad(circ, P[b], obs)
        assert rel_err(e[b], e_ref, 1.0) < TOL_C64
        assert_grad(g[b], g_ref, TOL_C64)


def test_grid_gemm_nodes_fp32_and_bf16x3():
    from gpu_common import TOL_BF16X3
    circ, p, amp = tcgen.workload_grid_amplitude(4, 5, 8)
    n = circ.n_qubits
    ref = sv.amplitude(circ, p)
    # one greedy trial leaves wide nodes in the tree
    for prec, tol in ((0, TOL_C64), (1, TOL_BF16X3)):
        plan = api.compile(circ, amp, n_trials=1, precision=prec, gemm_min_k=4,
                           gemm_min_macs=1)
        assert plan.info().n_gemm_nodes > 0
        a = plan.contract(device_params(p))[0]
        assert rel_err(a, ref, 2 ** (-n / 2)) < tol, prec


@pytest.mark.parametrize("ckpt", [2, 3, 5])
def test_checkpointed_gradient_matches(ckpt):
    B = 8
    circ, P, obs = tcgen.workload_batched_vqe(batch=B, n=14, layers=5)
    full = api.compile(circ, obs, batch=B, want_grad=True, checkpoint_every=-1)
    ck = api.compile(circ, obs, batch=B, want_grad=True, checkpoint_every=ckpt)
    assert ck.info().checkpoint_every == ckpt
    assert ck.info().workspace_bytes < full.info().workspace_bytes
    e1, g1 = full.contract_grad(device_params(P, B))
    e2, g2 = ck.contract_grad(device_params(P, B))
    assert np.max(np.abs(e1 - e2)) < 1e-6
    assert np.max(np.abs(g1 - g2)) < 1e-6
    e_ref, g_ref = sv.energy_grad(circ, P[3], obs)
    assert_grad(g2[3], g_ref, TOL_C64)


def test_term_mode_matches_level_mode_and_oracle():
    """One workgroup per term (leaves and every level behind workgroup
    barriers) against level-synchronous launches of the same trees and
    against the oracle: the VQE chain with gradient, the same with
    checkpointed segments, batch rows inside a term, and a forward-only
    amplitude."""
    circ, p, obs = tcgen.workload_vqe_chain()
    tm = api.compile(circ, obs, want_grad=True, n_trials=8, seed=1, exec_mode=2)
    lev = api.compile(circ, obs, want_grad=True, n_trials=8, seed=1, exec_mode=1)
    ck = api.compile(circ, obs, want_grad=True, n_trials=8, seed=1, exec_mode=2,
                     checkpoint_every=3)
    assert lev.info().exec_mode == 1 and ck.info().exec_mode == 2
    assert tm.info().n_launches + tm.info().n_grad_launches == 4
    e_ref, g_ref = sv.energy_grad(circ, p, obs)
    results = [pl.contract_grad(device_params(p)) for pl in (tm, lev, ck)]
    for e, g in results:
        assert rel_err(e[0], e_ref, 1.0) < TOL_C64
        assert_grad(g[0], g_ref, TOL_C64)
    # repeated calls reuse the same per-term regions
    e2, g2 = tm.contract_grad(device_params(p))
    assert e2[0] == results[0][0][0] and np.array_equal(g2, results[0][1])
    # batch rows inside each term's workgroup
    B = 6
    circ, P, obs = tcgen.workload_batched_vqe(batch=B, n=12, layers=4)
    tm = api.compile(circ, obs, batch=B, want_grad=True, exec_mode=2)
    assert tm.info().exec_mode == 2
    e, g = tm.contract_grad(device_params(P, B))
    for b in (0, 5):
        e_ref, g_ref = sv.energy_grad(circ, P[b], obs)
        assert rel_err(e[b], e_ref, 1.0) < TOL_C64
        assert_grad(g[b], g_ref, TOL_C64)
    # forward only, amplitude: a light tree, term mode chosen automatically
    circ, p, zz, amp = tcgen.workload_forward_chain()
    pa, a = one(circ, amp, p)
    assert pa.info().exec_mode == 2
    assert rel_err(a, sv.amplitude(circ, p), 2 ** (-circ.n_qubits / 2)) < TOL_C64


def test_autograd_function_matches_oracle():
    import torch
    B = 4
    circ, P, obs = tcgen.workload_batched_vqe(batch=B, n=10, layers=3)
    plan = api.compile(circ, obs, batch=B, want_grad=True)
    x = torch.from_numpy(P.copy()).cuda().requires_grad_(True)
    e = api.tc_contract(x, plan)
    w = torch.tensor([1.0, -2.0, 0.5, 3.0], dtype=torch.float64, device="cuda")
    loss = (w * e).sum()
    (gx,) = torch.autograd.grad(loss, x)
    for b in range(B):
        e_ref, g_ref = sv.energy_grad(circ, P[b], obs)
        assert abs(e[b].item() - e_ref) < TOL_C64
        assert_grad(gx[b].cpu().numpy() / w[b].item(), g_ref, TOL_C64)


def test_state_errors():
    circ, p, obs = tcgen.workload_vqe_chain(n=6, layers=2)
    plan = api.compile(circ, obs)
    with pytest.raises(L.TcxError) as e:
        plan.contract_grad(device_params(p))
    assert e.value.status == L.TC_ERR_STATE
    with pytest.raises(ValueError):
        plan.contract(device_params(p[:-1]))
