"""Benchmark of the tensor-network contraction path on one MI355X.

Default workload (--workload vqe): TFIM VQE energy + gradient on a 20-qubit
open chain, 6 layers of [RZZ ladder, RX layer] (240 parameter slots),
E = sum_i Z_i Z_{i+1} + g sum_i X_i with g = 1 (39 Pauli terms, each its own
tensor network).  One step = one evaluation of E and its gradient through
the whole path: leaf materialisation from the parameters, the level-ordered
contraction of all 39 trees, the FP64 root sum, the reverse sweep and the
FP64 gradient sum.  Parameters are resident in HBM before the timed region;
the plan (network, greedy path, tables, HIP graph) is built once beforehand,
as the paper excludes JIT staging from its timings.

Other workloads: --workload batched (the same chain, 1024 parameter vectors
per launch), forward (10-qubit brickwork: amplitude and <Z0 Z1>), grid (6x6
fSim grid amplitude, depth 8, FP32 and split BF16 against the stored oracle
amplitude), wide (the 4x7 grid at depth 16, whose default tree holds six
GEMM nodes in 128 x 128 tiles, up to 1024 x 65536 x 16384, against its stored
oracle amplitude; --wide-grid 6x6x12 takes the 6x6 grid at depth 12, which
has no oracle value), serve (the serving mix).  The default run also
reports the batched sweep, the forward chain's latency, the 6x6 depth-8 grid
and the 4x7 depth-16 grid beside the main line.

Prints one JSON line.  --copy-calibration BYTES also runs one plain device
copy of that many bytes (used to scale HBM byte counters).
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3   # dense FP32 MFMA
PEAK_BF16_TFLOPS = 2500.0  # dense BF16 MFMA
KIND_NAMES = {0: "k_leaf", 2: "k_gemm", 3: "k_gather", 4: "k_root", 5: "k_grad", 6: "k_term",
              7: "k_gemm_wide", 8: "k_rowtile", 9: "k_gather_split"}
KERNEL_SOURCES = ["paper_2205_10091_amd/csrc/exec.hip", "paper_2205_10091_amd/csrc/gemm_tile.h",
                  "paper_2205_10091_amd/csrc/gates.h", "paper_2205_10091_amd/csrc/ops.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed counter runs, or
    None if they are missing or the kernels changed since they were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    e = t.get(workload, {}).get(kernel)
    if not e or t.get("kernel_source_hash") != kernel_source_hash():
        return None
    return e["hbm_bytes_per_launch"]


def roofline(profile, workload, precision=0):
    """Dominant kernel (most time over a step) with its algorithmic bytes /
    flops per launch over its mean launch duration.  Split-BF16 GEMM tiles
    (precision 1) are priced against the BF16 MFMA peak with the flops the
    matrix cores execute: three BF16 products per real product."""
    kinds, ms, flops, by = profile
    agg = {}
    for k, t, f, b in zip(kinds, ms, flops, by):
        a = agg.setdefault(int(k), [0.0, 0.0, 0.0, 0])
        a[0] += t
        a[1] += f
        a[2] += b
        a[3] += 1
    k, (t, f, b, n) = max(agg.items(), key=lambda kv: kv[1][0])
    secs = t / 1e3
    ai = f / b if b else 0.0
    name = KIND_NAMES[k]
    if ai > PEAK_FP32_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9):
        # above the ridge: FP32 MFMA for the GEMM tiles, FP32 vector ALU else
        gemm = name in ("k_gemm", "k_gemm_wide")
        rl = {"bound": "mfma" if gemm else "alu",
              "achieved": f / secs / 1e12, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s"}
        if gemm and precision == 1:
            rl.update({"achieved": 3 * f / secs / 1e12, "peak": PEAK_BF16_TFLOPS,
                       "dtype": "bf16 (hi/lo split, 3 products per real product)",
                       "algorithmic_tflops": f / secs / 1e12})
    else:
        rl = {"bound": "hbm", "achieved": b / secs / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    rl["frac"] = rl["achieved"] / rl["peak"]
    rl["traffic"] = measured_traffic(workload, name + ("_bf16x3" if precision == 1 and
                                                       name.startswith("k_gemm") else ""))
    rl.update({"kernel": name, "launches_per_step": n, "mean_launch_us": t / n * 1e3,
               "alg_bytes_per_launch": b / n, "alg_flops_per_launch": f / n})
    tot = sum(x[0] for x in agg.values())
    share = {KIND_NAMES[kk]: round(v[0] / tot, 4) for kk, v in agg.items()}
    return rl, share


def cpu_baseline(circ, p, obs, budget_s=12.0):
    """The oracle's energy + gradient rate on this host: once with one BLAS
    thread, once with the BLAS pool as configured (its thread count is
    reported; os.cpu_count() beside it)."""
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import statevector as sv

    def run(limit):
        with threadpool_limits(limits=limit):
            threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
            t0 = time.perf_counter()
            n = 0
            while True:
                sv.energy_grad(circ, p, obs)
                n += 1
                if time.perf_counter() - t0 > budget_s or n >= 50:
                    break
            return n, time.perf_counter() - t0, int(threads)

    n, dt, threads = run(None)
    n1, dt1, _ = run(1)
    return {"value": n / dt, "unit": "evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} energy+gradient evaluations of the 20-qubit chain by the "
                      f"complex128 state-vector oracle with the adjoint method "
                      f"({dt:.1f} s, {threads} BLAS threads)",
            "single_thread": {"value": n1 / dt1, "unit": "evals/s", "cores": 1,
                              "sample": f"{n1} evaluations ({dt1:.1f} s)"},
            "host_cpu_count": os.cpu_count()}


def serving_leg(n_req=60, fracs=(0.8,), n_plain=30, path_trials=4):
    """Serving mix (seed 6): chains and grids of 8-64 qubits (chains up to
    600 at depth 2), depth 2-10, TFIM energy (g ~ U[0.5, 1.5]) with gradient
    for half of them, Poisson arrivals, 4 GiB per request.  The plain
    per-circuit form (plan + contract each request alone, one after
    another, same per-request cap) sets the saturated rate; the engine is
    driven at the given fractions of it, and once with every request
    submitted at t = 0 (its capacity)."""
    import torch
    import tcgen
    from paper_2205_10091_amd import _lib as L
    from paper_2205_10091_amd import api, serve
    reqs = tcgen.serving_requests(n_req, 1.0, seed=6)
    t0 = time.perf_counter()
    done = rejected = 0
    for k, rq in enumerate(reqs[:n_plain]):
        if k % 10 == 0:
            print(f"[serve] plain per-circuit {k}/{n_plain} t={time.perf_counter() - t0:.1f}s",
                  file=sys.stderr, flush=True)
        try:
            plan = api.compile(rq.circuit, rq.observable, want_grad=rq.want_grad,
                               n_trials=path_trials, seed=0x5eed, mem_budget_bytes=4 << 30)
        except L.TcxError as e:
            if e.status != L.TC_ERR_TOO_LARGE:
                raise
            rejected += 1
            continue
        par = torch.from_numpy(rq.params).cuda()
        if rq.want_grad:
            plan.contract_grad(par)
        else:
            plan.contract(par)
        del plan
        done += 1
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    lam = (done + rejected) / plain_s
    res = {"workload": "serving_mix_chain_grid_8_64_depth_2_10", "requests": n_req,
           "max_request_bytes": 4 << 30, "path_trials": path_trials,
           "plain_per_circuit": {"requests": done + rejected, "rejected": rejected,
                                 "requests_per_s": lam}}

    def engine(rate, realtime):
        srv = serve.Server(pool_bytes=64 << 30, max_request_bytes=4 << 30, max_active=64,
                           path_trials=path_trials)
        rep = serve.run(srv, tcgen.serving_requests(n_req, rate, seed=6), realtime=realtime,
                        progress=lambda t, d, r, p: print(
                            f"[serve]   t={t:.1f}s done={d} rejected={r} pending={p}",
                            file=sys.stderr, flush=True))
        srv.close()
        x = rep.summary()
        x["rejected_frac"] = len(rep.rejected) / n_req
        return x

    runs = []
    for frac in fracs:
        print(f"[serve] engine at {frac:.2f} of the plain rate ({frac * lam:.2f} req/s)",
              file=sys.stderr, flush=True)
        x = engine(frac * lam, True)
        x.update({"rate_per_s": frac * lam, "rate_frac_of_plain": frac})
        runs.append(x)
    print("[serve] engine saturated (all requests at t = 0)", file=sys.stderr, flush=True)
    res["poisson"] = runs
    res["saturated"] = engine(1.0, False)
    res["saturated"]["vs_plain_per_circuit"] = res["saturated"]["evals_per_s"] / lam if lam else None
    return res


def serve_workload(args, out):
    """--workload serve: the serving leg at 0.5, 0.8 and 0.95 of the plain
    rate; value = evaluations/s at 0.95."""
    res = serving_leg(n_req=max(args.steps, 20), fracs=(0.5, 0.8, 0.95))
    best = res["poisson"][-1]
    out.update({"metric": "circuit evals/s under Poisson arrivals (serving mix), p50/p99 latency",
                "value": best["evals_per_s"], "unit": "evals/s",
                "ms_per_step": 1e3 / best["evals_per_s"] if best["evals_per_s"] else None,
                "dtype": "c64 (fp32) + fp64 sums",
                "config": {"workload": res["workload"], "requests": res["requests"],
                           "max_active": 64, "path_trials": res["path_trials"]},
                "serving": res})


def mpo_leg(trials, steps=20):
    """TFIM energy + gradient with the operator as one MPO network (bond 3)
    against the same operator as a sum of light-coned Pauli-term networks,
    both planned under the time score: the 20-qubit chain at depth 6 (39
    terms) and 10, and a 600-qubit chain at depth 2 (1199 terms)."""
    import torch
    import tcgen
    from oracle import statevector as sv
    from paper_2205_10091_amd import api
    res = {}
    for n, layers, label in ((20, 6, "vqe_chain_n20_L6"), (20, 10, "chain_n20_L10"),
                             (600, 2, "chain_n600_L2")):
        circ = tcgen.chain_ladder(n, layers)
        p = tcgen.draw_angles(2, (circ.n_params,))
        params = torch.from_numpy(p).to("cuda:0")
        r = {}
        vals = {}
        for form, obs in (("mpo", tcgen.tfim_mpo(n, 1.0)), ("pauli_sum", tcgen.tfim_zz_x(n, 1.0))):
            t0 = time.perf_counter()
            plan = api.compile(circ, obs, want_grad=True, n_trials=trials, seed=1, score=4)
            plan_s = time.perf_counter() - t0
            info = plan.info()
            e_dev = torch.empty(1, dtype=torch.float64, device="cuda:0")
            g_dev = torch.empty(info.n_params, dtype=torch.float64, device="cuda:0")
            dt, _ = timed(lambda: plan.contract_grad_device(params, e_dev, g_dev), steps, 2)
            vals[form] = (e_dev.item(), g_dev.cpu().numpy())
            r[form] = {"evals_per_s": steps / dt, "ms_per_step": dt / steps * 1e3,
                       "networks": info.n_terms, "flops": info.flops + info.grad_flops,
                       "launches_per_step": info.n_launches + info.n_grad_launches,
                       "workspace_bytes": int(info.workspace_bytes), "plan_seconds": plan_s}
            del plan
        r["mpo_vs_pauli_sum"] = r["mpo"]["evals_per_s"] / r["pauli_sum"]["evals_per_s"]
        r["energy_diff_mpo_vs_pauli"] = abs(vals["mpo"][0] - vals["pauli_sum"][0])
        if n <= 20:
            e_ref, g_ref = sv.energy_grad(circ, p, tcgen.tfim_mpo(n, 1.0))
            r["mpo"]["rel_err_energy"] = abs(vals["mpo"][0] - e_ref) / max(abs(e_ref), 1.0)
            r["mpo"]["max_abs_err_grad"] = float(np.max(np.abs(vals["mpo"][1] - g_ref)))
        res[label] = r
    return res


def qgt_leg(trials=8, steps=20):
    """The geometric tensor (QFI = 4 Re G) of the paper's gradient-benchmark
    circuit: 12 qubits, 4 blocks of [CNOT ladder, RX, RZ, RX], 144 slots;
    the oracle (state Jacobian in complex128, numpy) timed beside it."""
    import torch
    import tcgen
    from oracle import statevector as sv
    from paper_2205_10091_amd import api
    circ = tcgen.qfi_blocks(12, 4)
    p = tcgen.draw_angles(3, (circ.n_params,))
    params = torch.from_numpy(p).to("cuda:0")
    plan = api.compile(circ, tcgen.Observable("state"), qgt=True, n_trials=trials, seed=1)
    info = plan.info()
    dt, g = timed(lambda: plan.geometric_tensor(params), steps, 2)
    t0 = time.perf_counter()
    ref = sv.geometric_tensor(circ, p.astype(np.float64))
    oracle_s = time.perf_counter() - t0
    return {"workload": "qfi_blocks_n12_b4", "n_params": circ.n_params,
            "rows": info.n_qgt_rows, "evals_per_s": steps / dt, "ms_per_eval": dt / steps * 1e3,
            "flops": info.flops + info.grad_flops,
            "launches": info.n_launches + info.n_grad_launches,
            "max_abs_err": float(np.max(np.abs(g - ref))),
            "oracle_seconds": oracle_s}


def structures_leg(trials=8, steps=20):
    """Batched circuit structures (section "Demonstration of barren
    plateaus", table "bpbench": 10 qubits, 10 layers, 100 circuits, each
    gate of a layer RX/RY/RZ by a status): the energy <Z0 Z1> and its
    gradient for all 100 circuits in one launch, and the gradient variance
    the benchmark is about; the oracle timed on the same 100 rows."""
    import torch
    import tcgen
    from oracle import statevector as sv
    from paper_2205_10091_amd import api
    B = 100
    circ, P, obs = tcgen.workload_barren_plateau(batch=B)
    plan = api.compile(circ, obs, batch=B, want_grad=True, n_trials=trials, seed=1)
    info = plan.info()
    par = torch.from_numpy(P.reshape(-1)).to("cuda:0")
    e_dev = torch.empty(B, dtype=torch.float64, device="cuda:0")
    g_dev = torch.empty(B * info.n_params, dtype=torch.float64, device="cuda:0")
    dt, _ = timed(lambda: plan.contract_grad_device(par, e_dev, g_dev), steps, 3)
    g = g_dev.cpu().numpy().reshape(B, -1)
    t0 = time.perf_counter()
    refs = [sv.energy_grad(circ, P[b], obs)[1] for b in range(B)]
    oracle_s = time.perf_counter() - t0
    return {"workload": "barren_plateau_n10_L10_100_structures", "batch": B,
            "seconds_per_launch": dt / steps, "circuits_per_s": B * steps / dt,
            "grad_variance_theta0": float(np.var(g[:, 0])),
            "max_abs_err_grad": float(np.max(np.abs(g - np.array(refs)))),
            "oracle_seconds_100_circuits": oracle_s,
            "launches": info.n_launches + info.n_grad_launches,
            "flops": info.flops + info.grad_flops}


def golden_amplitude(rows, cols, depth):
    """The stored oracle amplitude of a seeded fSim grid (two independent
    oracle methods, tests/golden/), its methods' seconds, or None."""
    path = os.path.join(ROOT, "tests", "golden", f"grid{rows}x{cols}_d{depth}_amplitude.json")
    if not os.path.exists(path):
        return None, {}
    ref = json.load(open(path))
    key = "statevector" if "statevector" in ref["values"] else sorted(ref["values"])[0]
    v = ref["values"][key]
    return complex(v["re"], v["im"]), {k: x.get("seconds") for k, x in ref["values"].items()}


def grid_leg(rows, cols, depth, trials, steps, warmup, workload, reconf_k=0):
    """A seeded fSim grid amplitude in FP32 and in split BF16 (wide nodes):
    evaluations/s, achieved TFLOP/s, the dominant kernel's roofline and the
    error against the stored oracle amplitude, floored at 2^(-n/2) (the RMS
    amplitude) and unfloored."""
    import torch
    import tcgen
    from paper_2205_10091_amd import api
    circ, p, amp = tcgen.workload_grid_amplitude(rows, cols, depth)
    n = rows * cols
    ref, oracle_s = golden_amplitude(rows, cols, depth)
    params = torch.from_numpy(p).to("cuda:0")
    res, vals = {"workload": f"grid{rows}x{cols}_d{depth}_amplitude", "n_qubits": n,
                 "reconf_k": reconf_k}, {}
    for prec, key in ((0, "fp32"), (1, "bf16x3")):
        t0 = time.perf_counter()
        plan = api.compile(circ, amp, n_trials=trials, seed=1, precision=prec, reconf_k=reconf_k)
        plan_s = time.perf_counter() - t0
        info = plan.info()
        out = torch.empty(2, dtype=torch.float64, device="cuda:0")
        dt, _ = timed(lambda: plan.contract_device(params, out), steps, warmup)
        vals[key] = complex(*out.cpu().numpy())
        rl, share = roofline(plan.profile(params, which=0, reps=2 if info.flops > 1e12 else 10),
                             workload, precision=prec)
        r = {"evals_per_s": steps / dt, "ms_per_step": dt / steps * 1e3,
             "achieved_tflops": info.flops / (dt / steps) / 1e12,
             "roofline": rl, "time_share_by_kernel": share,
             "wide_nodes": info.n_wide_nodes, "gemm_nodes": info.n_gemm_nodes,
             "flops": info.flops, "workspace_bytes": int(info.workspace_bytes),
             "largest_intermediate_bytes": int(info.peak_tensor_bytes), "plan_seconds": plan_s}
        if ref is not None:
            r["rel_err"] = abs(vals[key] - ref) / max(abs(ref), 2 ** (-n / 2))
            r["true_rel_err"] = abs(vals[key] - ref) / abs(ref)
        res[key] = r
        del plan
        torch.cuda.empty_cache()
    res["oracle_amplitude"] = None if ref is None else [ref.real, ref.imag]
    res["oracle_seconds"] = oracle_s
    res["rel_diff_bf16x3_vs_fp32"] = abs(vals["bf16x3"] - vals["fp32"]) / max(abs(vals["fp32"]), 2 ** (-n / 2))
    return res


def timed(step, steps, warmup):
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = step()
    torch.cuda.synchronize()
    return time.perf_counter() - t0, r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--workload", default="vqe",
                    choices=["vqe", "batched", "forward", "grid", "wide", "serve", "mpo"])
    ap.add_argument("--trials", type=int, default=0,
                    help="greedy path trials (default: 1024 for the chain workloads, whose "
                         "launches are latency bound and gain from the fewest flops; 32 for "
                         "the grids)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES")
    ap.add_argument("--wide-grid", default="4x7x16", metavar="RxCxD",
                    help="grid of --workload wide (4x7x16: oracle-pinned; 6x6x12: larger, "
                         "no oracle value)")
    args = ap.parse_args()
    chain_trials = args.trials or 1024
    grid_trials = args.trials or 32
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the contraction path is built and "
              "measured per GPU; multi-GPU sharding is a design note, not a run.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import tcgen
    from oracle import statevector as sv
    from paper_2205_10091_amd import api

    dev = torch.device("cuda:0")
    out = {"n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "data": "synthetic (seeded angles)"}

    if args.workload in ("vqe", "batched"):
        B = 1 if args.workload == "vqe" else 1024
        if B == 1:
            circ, p, obs = tcgen.workload_vqe_chain()
            P = p
        else:
            circ, P, obs = tcgen.workload_batched_vqe(batch=B)
        t0 = time.perf_counter()
        # batch 1 is launch bound: the depth cap that the path finder's time
        # model prefers trades a few flops of the deepest terms for fewer
        # dependent launches; a batched sweep is flop bound and keeps the
        # cheapest trees
        depth = -1 if B == 1 else 0
        plan = api.compile(circ, obs, batch=B, want_grad=True, n_trials=chain_trials, seed=1,
                           max_depth=depth)
        plan_s = time.perf_counter() - t0
        params = torch.from_numpy(np.ascontiguousarray(P.reshape(-1))).to(dev)
        info = plan.info()
        # the timed step leaves E and dE/dtheta in HBM, where a device-side
        # optimiser step would read them; steps are still ordered on the
        # plan's stream, each evaluation after the previous one
        e_dev = torch.empty(B, dtype=torch.float64, device=dev)
        g_dev = torch.empty(B * info.n_params, dtype=torch.float64, device=dev)
        dt, _ = timed(lambda: plan.contract_grad_device(params, e_dev, g_dev), args.steps,
                      args.warmup)
        e = e_dev.cpu().numpy()
        g = g_dev.cpu().numpy().reshape(B, -1)
        # the same evaluation with both results copied to host memory and
        # waited for on every call
        n_host = max(1, min(args.steps, 100))
        dt_h, _ = timed(lambda: plan.contract_grad(params), n_host, min(args.warmup, 5))
        out["host_roundtrip"] = {"evals_per_s": B * n_host / dt_h,
                                 "ms_per_step": dt_h / n_host * 1e3}
        out.update({
            "metric": "circuit evals/s (TFIM energy + 240-entry gradient, 20-qubit chain, "
                      "39 Pauli-term networks)",
            "value": B * args.steps / dt, "unit": "evals/s", "ms_per_step": dt / args.steps * 1e3,
            "dtype": "c64 (fp32) + fp64 sums",
            "config": {"workload": f"vqe_chain_n20_L6_tfim_energy_grad_batch{B}",
                       "n_qubits": 20, "layers": 6, "n_params": 240, "n_terms": 39,
                       "batch": B, "path_trials": chain_trials,
                       "path_depth_cap": "auto (time model)" if depth < 0 else "none"},
            "achieved_tflops": (info.flops + info.grad_flops) / (dt / args.steps) / 1e12,
            "outputs": "E and dE/dtheta left in HBM (device-side optimiser form)"})
        prof = plan.profile(params, which=1, reps=20 if B == 1 else 2)
        rl, share = roofline(prof, args.workload)
        b0 = 7 if B > 1 else 0
        e_ref, g_ref = sv.energy_grad(circ, P.reshape(B, -1)[b0], obs)
        out["rel_err_energy"] = abs(e[b0] - e_ref) / max(abs(e_ref), 1.0)
        out["rel_err_grad"] = float(np.linalg.norm(g[b0] - g_ref) /
                                    max(np.linalg.norm(g_ref), 1.0))
        out["max_abs_err_grad"] = float(np.max(np.abs(g[b0] - g_ref)))
    elif args.workload == "forward":
        circ, p, zz, amp = tcgen.workload_forward_chain()
        t0 = time.perf_counter()
        pa = api.compile(circ, amp, n_trials=chain_trials, seed=1)
        pz = api.compile(circ, zz, n_trials=chain_trials, seed=1)
        plan_s = time.perf_counter() - t0
        params = torch.from_numpy(p).to(dev)
        dt, _ = timed(lambda: (pa.contract(params), pz.contract(params)), args.steps,
                      args.warmup)
        a, z = pa.contract(params)[0], pz.contract(params)[0]
        info = pz.info()
        out.update({"metric": "circuit evals/s (10-qubit brickwork: amplitude and <Z0 Z1>)",
                    "value": args.steps / dt, "unit": "evals/s",
                    "ms_per_step": dt / args.steps * 1e3, "dtype": "c64 (fp32)",
                    "config": {"workload": "brickwork_n10_L4_amp_zz", "batch": 1}})
        prof = pz.profile(params, which=0, reps=20)
        rl, share = roofline(prof, args.workload)
        out["rel_err_amplitude"] = abs(a - sv.amplitude(circ, p)) / max(abs(sv.amplitude(circ, p)), 2 ** -5)
        out["rel_err_zz"] = abs(z - sv.energy(circ, p, zz))
    elif args.workload == "serve":
        pass  # handled below
    elif args.workload == "mpo":
        # the TFIM energy + gradient as one MPO network vs the Pauli sum;
        # value = MPO evaluations/s on the 20-qubit chain at depth 10
        res = mpo_leg(chain_trials if args.trials else 16, steps=min(args.steps, 20))
        r = res["chain_n20_L10"]["mpo"]
        out.update({"metric": "circuit evals/s (TFIM energy + gradient, operator as one MPO "
                              "network, 20-qubit chain at depth 10)",
                    "value": r["evals_per_s"], "unit": "evals/s", "ms_per_step": r["ms_per_step"],
                    "dtype": "c64 (fp32) + fp64 sums",
                    "config": {"workload": "chain_n20_L10_tfim_mpo_energy_grad", "batch": 1},
                    "mpo": res, "roofline": None})
    elif args.workload == "wide":
        # 4x7 grid at depth 16 (oracle-pinned; 1.8e13 flops) or, with
        # --wide-grid 6x6x12, the 6x6 grid at depth 12 (no oracle value)
        rows, cols, depth = (int(x) for x in args.wide_grid.split("x"))
        out["steps"], out["warmup"] = min(args.steps, 10), 1
        w = grid_leg(rows, cols, depth, grid_trials, out["steps"], 1, "wide")
        f = w["fp32"]
        out.update({"metric": f"circuit evals/s ({rows}x{cols} fSim grid amplitude, depth {depth})",
                    "value": f["evals_per_s"], "unit": "evals/s",
                    "ms_per_step": f["ms_per_step"], "dtype": "c64 (fp32)",
                    "config": {"workload": w["workload"], "batch": 1},
                    "achieved_tflops": f["achieved_tflops"], "roofline": f["roofline"],
                    "time_share_by_kernel": f["time_share_by_kernel"],
                    "rel_err": f.get("rel_err"), "true_rel_err": f.get("true_rel_err"),
                    "bf16x3": w["bf16x3"],
                    "rel_diff_bf16x3_vs_fp32": w["rel_diff_bf16x3_vs_fp32"]})
    else:
        # 6x6 grid, depth 8: FP32 and split BF16 against the oracle amplitude
        g = grid_leg(6, 6, 8, grid_trials, args.steps, args.warmup, "grid")
        f = g["fp32"]
        out.update({"metric": "circuit evals/s (6x6 fSim grid amplitude, depth 8)",
                    "value": f["evals_per_s"], "unit": "evals/s",
                    "ms_per_step": f["ms_per_step"], "dtype": "c64 (fp32)",
                    "config": {"workload": "grid6x6_d8_amplitude", "batch": 1},
                    "achieved_tflops": f["achieved_tflops"], "roofline": f["roofline"],
                    "time_share_by_kernel": f["time_share_by_kernel"],
                    "rel_err": f.get("rel_err"), "true_rel_err": f.get("true_rel_err"),
                    "bf16x3": g["bf16x3"], "oracle_seconds": g["oracle_seconds"]})

    if args.workload == "serve":
        serve_workload(args, out)
        out["roofline"] = None   # a mix of plans: see the per-workload runs
    elif args.workload in ("vqe", "batched", "forward"):
        out["plan"] = {"flops": info.flops, "grad_flops": info.grad_flops,
                       "alg_bytes": info.alg_bytes + info.grad_alg_bytes,
                       "workspace_bytes": int(info.workspace_bytes), "nodes": info.n_nodes,
                       "gemm_nodes": info.n_gemm_nodes, "levels": info.n_levels,
                       "launches_per_step": info.n_launches + info.n_grad_launches,
                       "checkpoint_every": info.checkpoint_every, "plan_seconds": plan_s}
        out["roofline"] = rl
        out["time_share_by_kernel"] = share
    out["kernel_source_hash"] = kernel_source_hash()

    if args.workload == "vqe" and not args.no_extras:
        # batched sweep: 1024 parameter vectors per launch vs the plain form
        B = 1024
        circ4, P4, obs4 = tcgen.workload_batched_vqe(batch=B)
        plan4 = api.compile(circ4, obs4, batch=B, want_grad=True, n_trials=chain_trials, seed=1)
        par4 = torch.from_numpy(P4.reshape(-1)).to(dev)
        i4 = plan4.info()
        # results left in HBM, as for the main line; then with the 1024
        # energies and gradients copied to host memory on every call
        e4d = torch.empty(B, dtype=torch.float64, device=dev)
        g4d = torch.empty(B * i4.n_params, dtype=torch.float64, device=dev)
        d4, _ = timed(lambda: plan4.contract_grad_device(par4, e4d, g4d), 5, 1)
        e4 = e4d.cpu().numpy()
        d4h, _ = timed(lambda: plan4.contract_grad(par4), 3, 1)
        rl4, share4 = roofline(plan4.profile(par4, which=1, reps=1), "batched")
        e4_ref, _ = sv.energy_grad(circ4, P4[7], obs4)
        out["batched"] = {
            "workload": "vqe_chain_n20_L6_batch1024", "evals_per_s": 5 * B / d4,
            "ms_per_launch": d4 / 5 * 1e3, "vs_plain_per_circuit": (5 * B / d4) / out["value"],
            "host_roundtrip_evals_per_s": 3 * B / d4h,
            "achieved_tflops": (i4.flops + i4.grad_flops) / (d4 / 5) / 1e12,
            "roofline": rl4, "time_share_by_kernel": share4,
            "rel_err_row7": abs(e4[7] - e4_ref) / max(abs(e4_ref), 1.0)}
        del plan4
        # forward latency of the 10-qubit brickwork (amplitude + <Z0 Z1>)
        circ1, p1, zz, amp = tcgen.workload_forward_chain()
        pa = api.compile(circ1, amp)
        pz = api.compile(circ1, zz)
        par1 = torch.from_numpy(p1).to(dev)
        lat = []
        for i in range(2200):
            t1 = time.perf_counter()
            pa.contract(par1)
            pz.contract(par1)
            if i >= 200:
                lat.append(time.perf_counter() - t1)
        lat = np.array(lat) * 1e6
        out["forward_chain_latency_us"] = {"p50": float(np.percentile(lat, 50)),
                                           "p99": float(np.percentile(lat, 99)),
                                           "evals_per_s": 1e6 / float(np.mean(lat))}

    if args.workload == "vqe" and not args.no_extras:
        # the 36-qubit precision-stress grid (depth 8) and the oracle-pinned
        # wide-node grid (4x7, depth 16), each in FP32 and split BF16
        print("[bench] grid 6x6 depth 8", file=sys.stderr, flush=True)
        out["grid_amplitude"] = grid_leg(6, 6, 8, grid_trials, 50, 5, "grid")
        print("[bench] grid 4x7 depth 16 (wide nodes)", file=sys.stderr, flush=True)
        out["wide_nodes"] = grid_leg(4, 7, 16, grid_trials, 5, 1, "wide")
        # the same grid on a subtree-reconfigured tree (10x fewer flops)
        print("[bench] grid 4x7 depth 16, reconfigured tree", file=sys.stderr, flush=True)
        # (no counter run covers the reconfigured tree's launches)
        out["wide_nodes_reconfigured"] = grid_leg(4, 7, 16, grid_trials, 10, 1, "wide_reconfigured",
                                                  reconf_k=8)
        print("[bench] batched circuit structures", file=sys.stderr, flush=True)
        out["structures"] = structures_leg()
        print("[bench] geometric tensor", file=sys.stderr, flush=True)
        out["qgt"] = qgt_leg()
        print("[bench] MPO vs Pauli-sum energy", file=sys.stderr, flush=True)
        out["mpo"] = mpo_leg(16)
        # the first 20 requests of the serving stream (the full 60-request
        # run at three rates is --workload serve, about ten minutes)
        print("[bench] serving mix", file=sys.stderr, flush=True)
        out["serving"] = serving_leg(n_req=20, n_plain=20)

    if args.copy_calibration:
        n = args.copy_calibration // 4
        x = torch.ones(n, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = 4 * n

    if args.workload == "vqe" and not args.no_cpu_baseline:
        circ, p, obs = tcgen.workload_vqe_chain()
        out["cpu_baseline"] = cpu_baseline(circ, p, obs)
    order = ["metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
             "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
             "roofline", "cpu_baseline"]
    line = {k: out[k] for k in order if k in out}
    line.update({k: v for k, v in out.items() if k not in line})
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
