"""Continuous-batching server for many independent 2-D advection problems.

A thin wrapper of the sl_server_* C calls (admission by arena budget, one tick
= one step of every resident request in batched launches, completion polling)
plus a driver that replays a stream of requests with Poisson arrivals and
reports latency percentiles.
"""
from __future__ import annotations

import ctypes as C
import time
from collections import deque

import numpy as np

from . import binding as B
from . import workloads as W

_VP = C.c_void_p


def _lib():
    return B.load()


def request_desc(req: W.Request):
    return B.make_desc(req.shape, req.nfields, value_prec="f32", order_max=2, limiter=True,
                       vel_kind=W.VEL_FOURIER, vel_params=[1.0], modes=req.modes)


class Server:
    """Server over a device arena of `budget_bytes` (the HBM budget)."""

    def __init__(self, budget_bytes: int, max_requests: int = 256, max_inflight: int = 2,
                 device="cuda", stream=None, mode: str = "batched", window: int = 1):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.arena = torch.empty(int(budget_bytes), dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = _VP()
        B.check(_lib().sl_server_create(C.c_void_p(self.arena.data_ptr()), int(budget_bytes),
                                        int(max_requests), int(max_inflight),
                                        C.c_void_p(self.stream.cuda_stream), C.byref(h)),
                "sl_server_create")
        self._h = h
        self._inputs = {}
        self.set_mode(mode, window)

    def set_mode(self, mode: str = "batched", window: int = 1):
        """"batched": one launch per (precision, field count) and tick, one
        step per request; "queued": one launch per (precision, field count)
        running `window` steps of every request from device-side tile queues
        (sl_server_set_mode)."""
        if mode not in ("batched", "queued"):
            raise ValueError("mode must be 'batched' or 'queued'")
        m = B.SL_SERVE_QUEUED if mode == "queued" else B.SL_SERVE_BATCHED
        B.check(_lib().sl_server_set_mode(self._h, m, int(window)), "sl_server_set_mode")

    def close(self):
        if getattr(self, "_h", None):
            _lib().sl_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def request_bytes(desc) -> int:
        return int(_lib().sl_server_request_bytes(C.byref(desc)))

    @staticmethod
    def arena_overhead(max_requests: int) -> int:
        """Arena bytes a server with max_requests slots keeps for itself."""
        return int(_lib().sl_server_arena_overhead(int(max_requests)))

    def admit(self, desc, fields, dt: float, nsteps: int, t0: float = 0.0):
        """Admit one request (fields: device tensors); returns its id, or None
        when the arena or the request slots are full."""
        ptrs = (_VP * len(fields))(*[f.data_ptr() for f in fields])
        rid = C.c_int64(0)
        rc = _lib().sl_server_admit(self._h, C.byref(desc), ptrs, float(t0), float(dt),
                                    int(nsteps), C.byref(rid))
        if rc == B.SL_EBUSY:
            return None
        B.check(rc, "sl_server_admit")
        self._inputs[rid.value] = fields  # keep the sources alive until done
        return rid.value

    def tick(self) -> int:
        active = C.c_int(0)
        B.check(_lib().sl_server_tick(self._h, C.byref(active)), "sl_server_tick")
        return active.value

    def poll(self, max_ids: int = 1024) -> list:
        ids = (C.c_int64 * max_ids)()
        n = C.c_int(0)
        B.check(_lib().sl_server_poll(self._h, ids, max_ids, C.byref(n)), "sl_server_poll")
        return [ids[i] for i in range(n.value)]

    def fetch(self, rid: int, out_fields):
        ptrs = (_VP * len(out_fields))(*[f.data_ptr() for f in out_fields])
        B.check(_lib().sl_server_fetch(self._h, int(rid), ptrs), "sl_server_fetch")
        self._inputs.pop(rid, None)

    def sync(self):
        st = B.SlStats()
        rc = _lib().sl_server_sync(self._h, C.byref(st))
        return rc, st.as_dict()

    def info(self) -> dict:
        st = B.SlServerStatus()
        B.check(_lib().sl_server_info(self._h, C.byref(st)), "sl_server_info")
        return {k: getattr(st, k) for k, _ in B.SlServerStatus._fields_}


def run_stream(requests, budget_bytes: int, max_requests: int = 256, max_inflight: int = 2,
               keep_results: bool = False, device="cuda", time_scale: float = 1.0,
               mode: str = "batched", window: int = 1):
    """Replay `requests` (workloads.Request, with arrival times in seconds)
    against a fresh server.  Requests wait in a FIFO queue until the arena has
    room; every loop iteration admits what fits, runs one tick and collects
    completions.  Returns a report with per-request latency (arrival to
    completion seen by the host) and throughput."""
    import torch
    srv = Server(budget_bytes, max_requests=max_requests, max_inflight=max_inflight,
                 device=device, mode=mode, window=window)
    dev = srv.device
    # Inputs are prepared before the clock starts (they are the clients'
    # data, already on the device when a request arrives).
    prepared = {}
    for r in requests:
        prepared[r.rid] = (request_desc(r), r.fields_torch(dev, torch.float32))
    torch.cuda.synchronize(dev)
    pending = deque(sorted(requests, key=lambda q: q.arrival))
    queue = deque()
    by_id = {}
    arrival, admitted, done = {}, {}, {}
    results = {}
    ticks = 0
    t_start = time.perf_counter()
    while pending or queue or by_id:
        now = time.perf_counter() - t_start
        while pending and pending[0].arrival * time_scale <= now:
            r = pending.popleft()
            arrival[r.rid] = r.arrival * time_scale
            queue.append(r)
        while queue:
            r = queue[0]
            (desc, keep), fields = prepared[r.rid]
            sid = srv.admit(desc, fields, r.dt, r.nsteps)
            if sid is None:
                break
            queue.popleft()
            by_id[sid] = r
            admitted[r.rid] = time.perf_counter() - t_start
        if by_id:
            srv.tick()
            ticks += 1
        for sid in srv.poll():
            r = by_id.pop(sid)
            out = [torch.empty(r.shape, dtype=torch.float32, device=dev)
                   for _ in range(r.nfields)]
            srv.fetch(sid, out)
            done[r.rid] = time.perf_counter() - t_start
            if keep_results:
                results[r.rid] = out
        if not by_id and not queue and pending:
            wait = pending[0].arrival * time_scale - (time.perf_counter() - t_start)
            if wait > 0:
                time.sleep(min(wait, 0.01))
        elif by_id and not srv.info()["active"]:
            # Everything resident has finished stepping; wait for the device.
            time.sleep(0.0002)
    rc, stats = srv.sync()
    makespan = time.perf_counter() - t_start
    lat = np.array([done[r.rid] - arrival[r.rid] for r in requests])
    qwait = np.array([admitted[r.rid] - arrival[r.rid] for r in requests])
    node_updates = sum(r.nodes * r.nsteps for r in requests)
    report = {
        "requests": len(requests), "ticks": ticks, "makespan_s": makespan,
        "node_updates": node_updates, "node_updates_per_s": node_updates / makespan,
        "latency_p50_ms": float(np.percentile(lat, 50) * 1e3),
        "latency_p99_ms": float(np.percentile(lat, 99) * 1e3),
        "latency_mean_ms": float(lat.mean() * 1e3),
        "queue_wait_p50_ms": float(np.percentile(qwait, 50) * 1e3),
        "queue_wait_p99_ms": float(np.percentile(qwait, 99) * 1e3),
        "status": rc, "stats": stats,
    }
    srv.close()
    if keep_results:
        return report, results
    return report
