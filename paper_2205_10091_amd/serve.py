"""Python driver of the serving engine (tc_serve_* in include/tcx.h).

The engine itself (admission by HBM footprint, plan cache, merged launches
across live requests) is native; this module marshals requests, runs the
Poisson arrival clock in a submitter thread and the engine loop in the
caller's thread, and collects per-request latencies.
"""
from __future__ import annotations

import ctypes as C
import threading
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from . import _lib as L
from .api import _CCircuit, _CObservable, lib


@dataclass
class Result:
    rid: int
    value: float
    value_im: float
    latency_s: float
    grad: Optional[np.ndarray]
    status: int
    plan_s: float = 0.0           # host planning inside latency_s
    device_s: float = 0.0         # admission to result inside latency_s


class Server:
    def __init__(self, pool_bytes=16 << 30, max_request_bytes=4 << 30, max_active=64,
                 path_trials=4, device=0, max_request_flops=0.0):
        opts = L.ServeOpts(device, pool_bytes, max_request_bytes, max_active, path_trials, None,
                           float(max_request_flops))
        h = C.c_void_p()
        L.check(lib().tc_serve_create(C.byref(opts), C.byref(h)))
        self.h = h
        self.n_params: Dict[int, int] = {}

    def close(self):
        if getattr(self, "h", None):
            lib().tc_serve_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except (AttributeError, TypeError):  # interpreter shutdown
            pass

    def submit(self, circ, obs, params, want_grad: bool) -> int:
        """Returns the engine's request id; raises TcxError (TOO_LARGE for
        requests over the per-request memory cap)."""
        cc = _CCircuit(circ)
        co = _CObservable(obs, circ.n_qubits)
        p = np.ascontiguousarray(np.asarray(params, np.float32).reshape(-1))
        rid = C.c_int64()
        L.check(lib().tc_serve_submit(self.h, C.byref(cc.c), C.byref(co.o),
                                      p.ctypes.data_as(L.F32P), int(want_grad), C.byref(rid)))
        self.n_params[rid.value] = circ.n_params
        return rid.value

    def step(self) -> int:
        n = C.c_int32()
        L.check(lib().tc_serve_step(self.h, C.byref(n)))
        return n.value

    def result(self, rid: int) -> Optional[Result]:
        out = L.ServeResult()
        g = np.zeros(max(self.n_params.get(rid, 0), 1), np.float64)
        st = lib().tc_serve_result_get(self.h, rid, C.byref(out), g.ctypes.data_as(L.F64P))
        if st == L.TC_ERR_BUSY:
            return None
        L.check(st)
        npar = self.n_params.pop(rid, 0)
        return Result(rid, out.value, out.value_im, out.submit_to_done_s,
                      g[:npar].copy() if out.want_grad else None, out.status,
                      out.plan_s, out.admit_to_done_s)


@dataclass
class ServeReport:
    results: Dict[int, Result] = field(default_factory=dict)   # keyed by request index
    rejected: List[int] = field(default_factory=list)
    reasons: Dict[int, str] = field(default_factory=dict)      # request index -> why rejected
    wall_s: float = 0.0

    def latencies(self):
        return np.array([r.latency_s for r in self.results.values()])

    def summary(self):
        lat = self.latencies()
        n = len(lat)
        pct = lambda a, q: float(np.percentile(a, q) * 1e3) if len(a) else None  # noqa: E731
        plan = np.array([r.plan_s for r in self.results.values()])
        dev = np.array([r.device_s for r in self.results.values()])
        why = {}
        for msg in self.reasons.values():
            if "flops" in msg:
                k = "flops above the per-request limit"
            elif "sliced labels" in msg:
                k = "more than 12 sliced bonds needed"
            elif "rank > 31" in msg:
                k = "an intermediate above 2^31 elements"
            elif "one term at a time" in msg:
                k = "one term's intermediates above the per-request cap"
            else:
                k = "workspace above the per-request cap"
            why[k] = why.get(k, 0) + 1
        return {"completed": n, "rejected": len(self.rejected), "wall_s": self.wall_s,
                "evals_per_s": n / self.wall_s if self.wall_s else 0.0,
                "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
                "plan_p50_ms": pct(plan, 50), "plan_p99_ms": pct(plan, 99),
                "admitted_to_done_p50_ms": pct(dev, 50), "admitted_to_done_p99_ms": pct(dev, 99),
                "rejected_reasons": why}


def run(server: Server, requests, realtime: bool = True, poll_sleep: float = 0.0,
        progress=None, progress_every_s: float = 10.0, planners: int = 8) -> ServeReport:
    """Submit `requests` (objects with circuit, observable, params,
    want_grad, arrival_s) at their arrival times (realtime) or all at once,
    and step the engine until every accepted request finished.  Each
    submission (which plans the request on the host, or finds its plan in
    the engine's cache) runs on one of `planners` threads, so that host
    planning of one request overlaps others' planning and the device work.
    If given, `progress(elapsed_s, n_done, n_rejected, n_pending)` is called
    about every `progress_every_s` seconds."""
    from concurrent.futures import ThreadPoolExecutor
    rep = ServeReport()
    ids: Dict[int, int] = {}
    lock = threading.Lock()
    done_submitting = threading.Event()
    errors = []

    def submit_one(i, rq):
        try:
            rid = server.submit(rq.circuit, rq.observable, rq.params, rq.want_grad)
            with lock:
                ids[rid] = i
        except L.TcxError as e:
            if e.status == L.TC_ERR_TOO_LARGE:
                with lock:
                    rep.rejected.append(i)
                    rep.reasons[i] = str(e)
            else:
                errors.append(e)
        except Exception as e:  # surfaced in the engine thread
            errors.append(e)

    def submitter():
        t0 = time.perf_counter()
        try:
            with ThreadPoolExecutor(max_workers=max(1, planners)) as pool:
                for i, rq in enumerate(requests):
                    if realtime:
                        dt = rq.arrival_s - (time.perf_counter() - t0)
                        if dt > 0:
                            time.sleep(dt)
                    pool.submit(submit_one, i, rq)
        except Exception as e:  # surfaced in the engine thread
            errors.append(e)
        finally:
            done_submitting.set()

    t0 = time.perf_counter()
    last_report = t0
    th = threading.Thread(target=submitter, daemon=True)
    th.start()
    while True:
        live = server.step()
        with lock:
            pending = list(ids.items())
        for rid, i in pending:
            r = server.result(rid)
            if r is not None:
                rep.results[i] = r
                with lock:
                    del ids[rid]
        if errors:
            raise errors[0]
        if done_submitting.is_set() and live == 0:
            with lock:
                if not ids:
                    break
        if progress is not None and time.perf_counter() - last_report >= progress_every_s:
            last_report = time.perf_counter()
            with lock:
                progress(last_report - t0, len(rep.results), len(rep.rejected), len(ids))
        if poll_sleep:
            time.sleep(poll_sleep)
    th.join()
    rep.wall_s = time.perf_counter() - t0
    return rep
