"""Python binding of the C ABI (include/tcx.h): argument marshalling only.

Every step of the contraction path runs in the HIP library; this module
converts circuit and observable descriptions (``tcgen.Circuit`` /
``tcgen.Observable``, or anything with the same attributes) to the ABI's
structs, owns the returned handles, and moves torch device pointers in and
out.  PyTorch provides device memory and the stream only.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np

from . import _lib as L


def lib():
    return L.load()


class _CCircuit:
    """Keeps the ctypes arrays of a circuit alive while the ABI reads them."""

    def __init__(self, circ):
        n = len(circ.gates)
        self.gates = (L.Gate * max(n, 1))()
        self.mats = []
        for i, g in enumerate(circ.gates):
            cg = self.gates[i]
            cg.kind = L.GATE_KIND[g.kind]
            for k, q in enumerate(g.qubits):
                cg.q[k] = q
            params = tuple(g.params) + (-1, -1)
            fixed = tuple(g.fixed) + (0.0, 0.0)
            cg.param[0], cg.param[1] = params[0], params[1]
            cg.fixed[0], cg.fixed[1] = fixed[0], fixed[1]
            if g.matrix is not None:
                flat = np.array(g.matrix, dtype=np.float64).reshape(-1)
                arr = (C.c_double * len(flat))(*flat)
                self.mats.append(arr)
                cg.matrix = C.cast(arr, C.POINTER(C.c_double))
            else:
                cg.matrix = None
        self.c = L.Circuit(circ.n_qubits, circ.n_params, n,
                           C.cast(self.gates, C.POINTER(L.Gate)))


class _CObservable:
    def __init__(self, obs, n_qubits):
        self.keep = []
        if obs.kind == "amplitude":
            bits = obs.bits if obs.bits is not None else (0,) * n_qubits
            b = (C.c_uint8 * n_qubits)(*bits)
            self.keep.append(b)
            self.o = L.Observable(0, C.cast(b, C.POINTER(C.c_uint8)), 0, None, None, None, None)
        elif obs.kind == "state":
            self.o = L.Observable(3, None, 0, None, None, None, None)
        elif obs.kind == "mpo":
            ts = [np.asarray(t, np.complex128) for t in obs.mpo]
            bonds = np.ascontiguousarray([t.shape[1] for t in ts[:-1]], dtype=np.int32)
            flat = np.ascontiguousarray(
                np.concatenate([t.reshape(-1) for t in ts]).view(np.float64))
            self.keep += [bonds, flat]
            self.o = L.Observable(2, None, 0, None, None, bonds.ctypes.data_as(L.I32P),
                                  flat.ctypes.data_as(L.F64P))
        else:
            s = np.ascontiguousarray(obs.structures, dtype=np.uint8)
            w = np.ascontiguousarray(obs.weights, dtype=np.float64)
            self.keep += [s, w]
            self.o = L.Observable(
                1, None, int(s.shape[0]),
                s.ctypes.data_as(C.POINTER(C.c_uint8)),
                w.ctypes.data_as(C.POINTER(C.c_double)), None, None)


class Network:
    """Owns a tc_network*."""

    def __init__(self, circ, obs, split_2q=True, lightcone=True, absorb_1q=True):
        self.circ = circ
        cc = _CCircuit(circ)
        co = _CObservable(obs, circ.n_qubits)
        opts = L.BuildOpts(int(split_2q), int(lightcone), int(absorb_1q))
        h = C.c_void_p()
        L.check(lib().tc_build_network(C.byref(cc.c), C.byref(co.o),
                                       C.byref(opts), C.byref(h)))
        self.h = h

    def __del__(self):
        try:
            if getattr(self, "h", None) and L._lib is not None:
                L._lib.tc_network_free(self.h)
                self.h = None
        except (AttributeError, TypeError):  # interpreter shutdown
            pass

    def info(self) -> L.NetworkInfo:
        out = L.NetworkInfo()
        L.check(lib().tc_network_info_get(self.h, C.byref(out)))
        return out

    def term_leaves(self, term: int):
        info = self.info()
        m = max(info.max_leaves, 1)
        arrs = [np.zeros(m, np.int32) for _ in range(5)]
        legs = np.zeros(8 * m, np.int32)
        n = C.c_int32()
        ptr = lambda a: a.ctypes.data_as(L.I32P)  # noqa: E731
        L.check(lib().tc_network_term_leaves(self.h, term, C.byref(n),
                                             *[ptr(a) for a in arrs], ptr(legs)))
        k = n.value
        kind, gate, part, conj, rank = (a[:k] for a in arrs)
        return dict(kind=kind, gate=gate, part=part, conj=conj, rank=rank,
                    legs=legs[:8 * k].reshape(k, 8))


class Path:
    """Owns a tc_path*."""

    def __init__(self, net: Network, seed=0, n_trials=1, score=3, temperature=0.1, reconf_k=0,
                 max_depth=0):
        self.net = net
        opts = L.PathOpts(seed, n_trials, score, temperature, reconf_k, max_depth)
        h = C.c_void_p()
        L.check(lib().tc_greedy_path(net.h, C.byref(opts), C.byref(h)))
        self.h = h

    def __del__(self):
        try:
            if getattr(self, "h", None) and L._lib is not None:
                L._lib.tc_path_free(self.h)
                self.h = None
        except (AttributeError, TypeError):  # interpreter shutdown
            pass

    def stats(self, term: int = -1) -> L.PathStats:
        out = L.PathStats()
        L.check(lib().tc_path_stats_get(self.h, term, C.byref(out)))
        return out

    def pairs(self, term: int) -> np.ndarray:
        n = C.c_int32()
        L.check(lib().tc_path_term_pairs(self.h, term, None, C.byref(n)))
        out = np.zeros(2 * max(n.value, 1), np.int32)
        L.check(lib().tc_path_term_pairs(self.h, term, out.ctypes.data_as(L.I32P),
                                         C.byref(n)))
        return out[:2 * n.value].reshape(-1, 2)

    def sliced(self, max_log2_size: int, max_labels: int = 16):
        """tc_slice: (network, path, s) for the sum over slices whose
        intermediates fit 2^max_log2_size elements."""
        hn, hp = C.c_void_p(), C.c_void_p()
        s = C.c_int32()
        L.check(lib().tc_slice(self.net.h, self.h, int(max_log2_size), int(max_labels),
                               C.byref(hn), C.byref(hp), C.byref(s)))
        net = Network.__new__(Network)
        net.circ, net.h = self.net.circ, hn
        path = Path.__new__(Path)
        path.net, path.h = net, hp
        return net, path, s.value

    def replace_term(self, term: int, pairs):
        p = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1)
        L.check(lib().tc_path_replace_term(self.h, term, p.ctypes.data_as(L.I32P),
                                           len(p) // 2))


class Plan:
    """Owns a tc_plan*; contraction calls take torch tensors on the GPU."""

    def __init__(self, net: Network, path: Path, batch=1, want_grad=False,
                 precision=0, device=0, mem_budget_bytes=0, stream=None, gemm_min_k=0,
                 checkpoint_every=0, gemm_min_macs=0, exec_mode=0, tile_mode=0, qgt=False):
        self.net, self.path = net, path
        self.batch = batch
        self.want_grad = want_grad
        self.qgt = bool(qgt)
        opts = L.PlanOpts(precision, batch, int(want_grad), device,
                          mem_budget_bytes, stream, gemm_min_k, checkpoint_every,
                          gemm_min_macs, exec_mode, tile_mode, int(qgt))
        h = C.c_void_p()
        L.check(lib().tc_plan_create(net.h, path.h, C.byref(opts), C.byref(h)))
        self.h = h
        self.workspace = None
        self.torch_stream = None
        self.n_params = net.circ.n_params

    def __del__(self):
        try:
            if getattr(self, "h", None) and L._lib is not None:
                L._lib.tc_plan_free(self.h)
                self.h = None
        except (AttributeError, TypeError):  # interpreter shutdown
            pass

    def info(self) -> L.PlanInfo:
        out = L.PlanInfo()
        L.check(lib().tc_plan_info_get(self.h, C.byref(out)))
        return out

    def bind(self, workspace=None):
        """Bind a caller device buffer (a torch uint8 tensor on the GPU) or
        let the library allocate when workspace is None."""
        if workspace is None:
            L.check(lib().tc_plan_bind(self.h, None, 0))
        else:
            self.workspace = workspace
            L.check(lib().tc_plan_bind(self.h, C.c_void_p(workspace.data_ptr()),
                                       workspace.numel() * workspace.element_size()))

    def bind_torch(self, device="cuda"):
        import torch
        nbytes = int(self.info().workspace_bytes)
        ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        self.bind(ws)
        return ws

    def _params_ptr(self, params):
        import torch
        if not (isinstance(params, torch.Tensor) and params.is_cuda):
            raise TypeError("params must be a CUDA (HIP) float32 tensor")
        if params.dtype != torch.float32 or not params.is_contiguous():
            raise TypeError("params must be contiguous float32")
        if params.numel() != self.batch * self.n_params:
            raise ValueError(f"params must hold batch*n_params = "
                             f"{self.batch * self.n_params} floats")
        if self.torch_stream is not None:
            # parameters written on torch's current stream are visible to the plan
            self.torch_stream.wait_stream(torch.cuda.current_stream(params.device))
        return C.c_void_p(params.data_ptr())

    def geometric_tensor(self, params) -> np.ndarray:
        """G[i, j] = <d_i psi|d_j psi> - <d_i psi|psi><psi|d_j psi> as a
        complex128 (n_params, n_params) array (plans made with qgt=True)."""
        n = self.n_params
        out = np.zeros(2 * max(n * n, 1), np.float64)
        L.check(lib().tc_contract_qgt(self.h, self._params_ptr(params),
                                      out.ctypes.data_as(L.F64P)))
        return (out[0::2] + 1j * out[1::2])[:n * n].reshape(n, n)

    def contract(self, params) -> np.ndarray:
        """Complex values (numpy complex128, shape [batch])."""
        out = np.zeros(2 * self.batch, np.float64)
        L.check(lib().tc_contract(self.h, self._params_ptr(params),
                                  out.ctypes.data_as(L.F64P)))
        return out[0::2] + 1j * out[1::2]

    def contract_grad(self, params):
        """(Re E [batch], dE/dparams [batch, n_params]) as numpy float64."""
        val = np.zeros(self.batch, np.float64)
        grad = np.zeros(self.batch * self.n_params, np.float64)
        L.check(lib().tc_contract_grad(self.h, self._params_ptr(params),
                                       val.ctypes.data_as(L.F64P),
                                       grad.ctypes.data_as(L.F64P)))
        return val, grad.reshape(self.batch, self.n_params)

    def profile(self, params, which=0, reps=10):
        """Per-kernel (kind, mean ms, algorithmic flops, bytes) arrays from an
        eager replay with HIP events around each kernel (a level has a GEMM
        and a gather kernel)."""
        info = self.info()
        cap = 3 * (info.n_launches + info.n_grad_launches) + 8
        kinds = np.zeros(cap, np.int32)
        ms, fl, by = (np.zeros(cap, np.float64) for _ in range(3))
        n = C.c_int32()
        L.check(lib().tc_plan_profile(self.h, self._params_ptr(params), which, reps, cap,
                                      C.byref(n), kinds.ctypes.data_as(L.I32P),
                                      ms.ctypes.data_as(L.F64P), fl.ctypes.data_as(L.F64P),
                                      by.ctypes.data_as(L.F64P)))
        if n.value > cap:
            raise RuntimeError(f"profile reported {n.value} kernels, more than {cap}")
        k = n.value
        return kinds[:k], ms[:k], fl[:k], by[:k]

    def contract_device(self, params, out_dev):
        L.check(lib().tc_contract_device(self.h, self._params_ptr(params),
                                         C.c_void_p(out_dev.data_ptr())))

    def contract_grad_device(self, params, value_dev, grad_dev):
        L.check(lib().tc_contract_grad_device(
            self.h, self._params_ptr(params), C.c_void_p(value_dev.data_ptr()),
            C.c_void_p(grad_dev.data_ptr())))

    def contract_grad_device_noalloc(self, params, value_dev, grad_dev):
        """tc_contract_grad_device_noalloc: the same outputs, computed in the
        library's static per-GPU scratch array (no device allocation)."""
        L.check(lib().tc_contract_grad_device_noalloc(
            self.h, self._params_ptr(params), C.c_void_p(value_dev.data_ptr()),
            C.c_void_p(grad_dev.data_ptr())))


def compile(circ, obs, batch=1, want_grad=False, precision=0, split_2q=True,
            lightcone=True, absorb_1q=True, seed=0, n_trials=8,
            mem_budget_bytes=0, device=0, bind=True, gemm_min_k=0, stream=None,
            checkpoint_every=0, gemm_min_macs=0, exec_mode=0, tile_mode=0,
            score=3, qgt=False, reconf_k=0, max_depth=0) -> Plan:
    """Network + greedy path + plan (+ bind with a torch workspace).
    score: the path score of tc_greedy_path (3 combo, 4 time estimate);
    max_depth: cap on each term's tree levels (0 = none)."""
    net = Network(circ, obs, split_2q, lightcone, absorb_1q)
    path = Path(net, seed=seed, n_trials=n_trials, score=score, reconf_k=reconf_k,
                max_depth=max_depth)
    torch_stream = None
    if stream is None and bind:
        # a dedicated torch stream (default priority): torch work orders
        # around the plan with wait_stream, and the plan's HIP graph is
        # captured on a real stream rather than the null stream
        import torch
        torch_stream = torch.cuda.Stream(device=f"cuda:{device}")
        stream = torch_stream.cuda_stream
    plan = Plan(net, path, batch, want_grad, precision, device, mem_budget_bytes,
                stream, gemm_min_k, checkpoint_every, gemm_min_macs, exec_mode, tile_mode,
                qgt)
    plan.torch_stream = torch_stream
    if bind:
        plan.bind_torch(f"cuda:{device}")
    return plan


def _make_function():
    import torch

    class TCContract(torch.autograd.Function):
        """E(params) = Re sum_j alpha_j <P_j> through the HIP plan.

        forward runs the plan's forward sweep and reverse sweep in one call
        (tc_contract_grad_device: values and dE/dparams land in device
        buffers on the plan's stream); backward scales the stored gradient by
        the incoming gradient.  params: [batch, n_params] float32 on the GPU;
        returns [batch] float64.  The plan must be compiled with
        want_grad=True and bound to the current stream's device."""

        @staticmethod
        def forward(ctx, params, plan):
            p = params.detach().contiguous()
            if p.dtype != torch.float32:
                p = p.float()
            value = torch.empty(plan.batch, dtype=torch.float64, device=p.device)
            grad = torch.empty(plan.batch, plan.n_params, dtype=torch.float64, device=p.device)
            cur = torch.cuda.current_stream(p.device)
            ps = getattr(plan, "torch_stream", None)
            if ps is None:
                raise ValueError("compile the plan with api.compile(..., bind=True) so that it "
                                 "runs on a torch stream")
            ps.wait_stream(cur)           # params ready before the plan reads them
            plan.contract_grad_device(p, value, grad)
            cur.wait_stream(ps)           # results ready before torch reads them
            ctx.save_for_backward(grad)
            ctx.in_dtype = params.dtype
            return value

        @staticmethod
        def backward(ctx, g_out):
            (grad,) = ctx.saved_tensors
            return (g_out.to(grad.dtype)[:, None] * grad).to(ctx.in_dtype), None

    return TCContract


_TCContract = None


def tc_contract(params, plan):
    """Differentiable energy: torch.autograd.Function over the reverse sweep."""
    global _TCContract
    if _TCContract is None:
        _TCContract = _make_function()
    return _TCContract.apply(params, plan)
