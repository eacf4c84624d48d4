"""Open-loop load generator for the request server.

Requests mix resident mechanisms, point counts n = round(10^U(3, 6)), ops
(production rates alone or with transport, 50/50) and precision (FP64 or
mixed, 50/50).  Arrivals are Poisson; every latency is measured from the
request's *scheduled* arrival time to its completion on the device, so a
client that falls behind does not hide queueing (no coordinated omission).
Inputs are device-resident before the clock starts: each mechanism gets a
pool of input sets whose sizes are drawn from the same log-uniform law, and
each request uses one of them.
"""
from __future__ import annotations

import threading
import time

import numpy as np
import torch

from . import kx


def make_pool(mech_dev, ns: int, sizes, seed: int, device: int = 0):
    """Device input sets (T, p, Y) for the given point counts: T ~ U[300, 2800] K,
    p ~ U[1, 40] atm, Y ~ Dirichlet(0.3) over the species."""
    g = torch.Generator(device=f"cuda:{device}")
    g.manual_seed(seed)
    kw = dict(dtype=torch.float64, device=f"cuda:{device}")
    pool = []
    for n in sizes:
        n = int(n)
        T = 300.0 + 2500.0 * torch.rand(n, generator=g, **kw)
        p = 1013250.0 * (1.0 + 39.0 * torch.rand(n, generator=g, **kw))
        # Dirichlet(0.3): normalised Gamma(0.3) draws per point
        gam = torch._standard_gamma(torch.full((ns, n), 0.3, **kw), generator=g)
        Y = (gam / gam.sum(0, keepdim=True)).contiguous()
        pool.append((n, T, p, Y))
    torch.cuda.synchronize(device)
    return pool


def make_stream(n_req: int, pools: dict, seed: int):
    """Per request: (mechanism name, pool index, transport?, precision)."""
    rng = np.random.default_rng(seed)
    names = sorted(pools)
    out = []
    for _ in range(n_req):
        name = names[rng.integers(len(names))]
        out.append((name, int(rng.integers(len(pools[name]))), bool(rng.integers(2)),
                    "mixed" if rng.integers(2) else "fp64"))
    return out


def make_host_pool(pool, ns: int):
    """Pinned host copies of device input sets, with pinned output buffers:
    per entry (n, (T, p, Y), (wdot, mu, lambda, Dmix))."""
    out = []
    for n, T, p, Y in pool:
        hin = tuple(torch.empty(t.shape, dtype=t.dtype, pin_memory=True).copy_(t)
                    for t in (T, p, Y))
        kw = dict(dtype=torch.float64, pin_memory=True)
        hout = (torch.empty((ns, n), **kw), torch.empty(n, **kw), torch.empty(n, **kw),
                torch.empty((ns, n), **kw))
        out.append((n, hin, hout))
    return out


class _Collector(threading.Thread):
    """Waits for tickets in submission order, records timings, releases.
    `finish(ticket, meta, result)`, if given, runs before the release (the
    host-staged client copies the outputs out there)."""

    def __init__(self, srv: kx.Server, finish=None):
        super().__init__(daemon=True)
        self.finish = finish
        self.srv = srv
        self.q = []
        self.cv = threading.Condition()
        self.closed = False
        self.records = []
        self.error = None

    def push(self, item):
        with self.cv:
            self.q.append(item)
            self.cv.notify()

    def close(self):
        with self.cv:
            self.closed = True
            self.cv.notify()

    def run(self):
        try:
            while True:
                with self.cv:
                    while not self.q and not self.closed:
                        self.cv.wait()
                    if not self.q and self.closed:
                        return
                    ticket, meta = self.q.pop(0)
                r = self.srv.wait(ticket, 120.0)
                if r["state"] != "done":
                    raise RuntimeError(f"request {ticket} ended {r['state']}")
                if self.finish is not None:
                    self.finish(ticket, meta, r)
                self.records.append((meta, r))
                self.srv.release(ticket)
        except Exception as e:  # surfaced by the caller
            self.error = e


def run_stream(srv: kx.Server, mechs: dict, pools: dict, stream, qps: float | None,
               seed: int):
    """Submit `stream`; qps=None submits everything at once (back-to-back).
    Returns per-request records (meta, result dict)."""
    rng = np.random.default_rng(seed)
    col = _Collector(srv)
    col.start()
    t0 = kx.clock() + 0.01
    gaps = rng.exponential(1.0 / qps, len(stream)) if qps else np.zeros(len(stream))
    sched = t0 + np.cumsum(gaps)
    for (name, idx, tr, prec), ts in zip(stream, sched):
        if qps:
            while True:
                d = ts - kx.clock()
                if d <= 0:
                    break
                time.sleep(d if d > 2e-4 else 0)
        n, T, p, Y = pools[name][idx]
        t = srv.submit(mechs[name], T, p, Y, transport=tr, precision=prec,
                       arrival=float(ts) if qps else None)
        col.push((t, (name, n, tr, prec)))
        if col.error:
            break
    col.close()
    col.join()
    if col.error:
        raise col.error
    return col.records


def run_stream_staged(srv: kx.Server, mechs: dict, hpools: dict, stream, qps: float | None,
                      seed: int):
    """As run_stream, for a client whose data live in pinned host memory: at
    its scheduled arrival a request's inputs are copied into fresh device
    buffers (on a client stream, waited for) and it is submitted; once it is
    done its outputs are copied back into pinned host buffers.  The request's
    "t_host" is when that copy has completed (the server's clock)."""
    rng = np.random.default_rng(seed)
    dev = torch.device(f"cuda:{srv.device}")
    cin = torch.cuda.Stream(dev)
    cout = torch.cuda.Stream(dev)

    def finish(ticket, meta, r):
        _, _, tr, _, idx = meta
        _, _, (w, mu, lam, Dm) = hpools[meta[0]][idx]
        srv.copy_outputs(ticket, w, mu if tr else None, lam if tr else None,
                         Dm if tr else None, stream=cout)
        r["t_host"] = kx.clock()

    col = _Collector(srv, finish)
    col.start()
    t0 = kx.clock() + 0.01
    gaps = rng.exponential(1.0 / qps, len(stream)) if qps else np.zeros(len(stream))
    sched = t0 + np.cumsum(gaps)
    for (name, idx, tr, prec), ts in zip(stream, sched):
        if qps:
            while True:
                d = ts - kx.clock()
                if d <= 0:
                    break
                time.sleep(d if d > 2e-4 else 0)
        n, (hT, hp, hY), _ = hpools[name][idx]
        with torch.cuda.stream(cin):
            T, p, Y = (h.to(dev, non_blocking=True) for h in (hT, hp, hY))
        cin.synchronize()
        t = srv.submit(mechs[name], T, p, Y, transport=tr, precision=prec,
                       arrival=float(ts) if qps else None)
        col.push((t, (name, n, tr, prec, idx)))
        if col.error:
            break
    col.close()
    col.join()
    if col.error:
        raise col.error
    return col.records


def summarize(records, skip: int = 0, end: str = "t_done"):
    """Latency percentiles from the scheduled arrival to `end` ("t_done":
    outputs ready on the device; "t_host": copied to the host)."""
    recs = records[skip:]
    lat = np.array([r[end] - r["t_arrival"] for _, r in recs])
    queue = np.array([r["t_launch"] - r["t_arrival"] for _, r in recs])
    service = np.array([r["t_done"] - r["t_launch"] for _, r in recs])
    pts = sum(m[1] for m, _ in recs)
    t_first = min(r["t_arrival"] for _, r in recs)
    t_last = max(r[end] for _, r in recs)
    span = max(t_last - t_first, 1e-9)
    return {"requests": len(recs), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3),
            "queue_p50_ms": float(np.percentile(queue, 50) * 1e3),
            "service_p50_ms": float(np.percentile(service, 50) * 1e3),
            "achieved_rps": len(recs) / span, "achieved_Mpoints_s": pts / span / 1e6}


def direct_sequential(mechs: dict, pools: dict, stream):
    """The same requests as plain synchronous calls one after another (no
    batching, one stream): seconds."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for name, idx, tr, prec in stream:
        n, T, p, Y = pools[name][idx]
        kx.production_rates(mechs[name], T, p, Y, precision=prec)
        if tr:
            kx.transport(mechs[name], T, p, Y, precision=prec)
        torch.cuda.synchronize()
    return time.perf_counter() - t0
