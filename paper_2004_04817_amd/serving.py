"""Client side of the request loop: replay a timed stream of deformation
requests against a :class:`Server` and collect per-request latencies.

A request is (arrival time, mesh key, boundary size, field seed).  The first
request of a key brings its mesh (boundary and base displacement field); a
later request of the same key brings the same boundary with a new field.
Each request deforms ``nv_per_nb * nb`` volume points taken from a shared
device point cloud of the mesh's kind.  Arrival times are measured on the
server's clock, so a request submitted late (the host was busy in
``progress``) still counts from its true arrival.
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np

from . import Server, clock


@dataclasses.dataclass
class StreamRequest:
    t: float            # arrival, seconds after the stream starts
    key: int            # mesh identity
    nb: int             # boundary nodes (target size)
    field_seed: int     # seed of the displacement field (repeats only)


@dataclasses.dataclass
class Served:
    ticket: int
    req: StreamRequest
    xyz: np.ndarray
    disp: np.ndarray
    radius: float
    m: int
    tol_abs: float
    seed: int
    vol: object          # device tensor (nv, 3)
    out: object          # device tensor (nv, 3)
    result: dict | None = None


def materialise(stream, meshes_cache=None):
    """Boundary, field and parameters of every request (CPU, deterministic)."""
    import synth
    meshes = {} if meshes_cache is None else meshes_cache
    out = []
    for t, key, nbt, fseed in stream:
        first = key not in meshes
        if first:
            meshes[key] = synth.request_mesh(key, nbt)
        base = meshes[key]
        disp = base.disp if first else synth.request_field(base, fseed)
        tol = 1e-5 * float(np.sqrt((disp * disp).sum(axis=1)).max())
        out.append((StreamRequest(t, key, base.nb, fseed), base, np.ascontiguousarray(disp), tol))
    return out


def volume_pool(max_nv: int, device, dtype=None):
    """One graded wing cloud and one ellipsoid-exterior cloud of max_nv points on the device."""
    import torch
    import synth
    dtype = torch.float64 if dtype is None else dtype
    ell = synth.ellipsoid_volume(max_nv, gen=synth.rng(5_000_001, 2))
    wing = synth.wing_volume(max_nv, 3, 3, gen=synth.rng(5_000_002, 2))
    return {0: torch.from_numpy(ell).to(device=device, dtype=dtype).contiguous(),
            1: torch.from_numpy(wing).to(device=device, dtype=dtype).contiguous()}


def replay(server: Server, items, pool, nv_per_nb: int = 25, iterations: int = 16, time_limit: float = 600.0,
           out_dtype=None, record: bool = False):
    """Submit each request at its arrival time, drive the server until every
    request is done, and return the Served records (with results).
    record=True asks the server for each selection's support set, weights and
    log (verification: the copies synchronise the stream)."""
    import torch
    served = []
    start = clock() + 0.05
    pending = list(items)
    nxt = 0
    in_flight = 0
    deadline = time.monotonic() + time_limit
    while nxt < len(pending) or in_flight > 0:
        if time.monotonic() > deadline:
            raise RuntimeError("request stream did not finish within the time limit")
        now = clock()
        while nxt < len(pending) and start + pending[nxt][0].t <= now:
            req, base, disp, tol = pending[nxt]
            cloud = pool[req.key % 2]
            nv = min(nv_per_nb * base.nb, cloud.shape[0])
            vol = cloud[:nv]
            out = torch.empty((nv, 3), dtype=out_dtype or cloud.dtype, device=cloud.device)
            tk = server.submit(base.xyz, disp, base.radius, base.m, tol, seed=base.seed, mesh_key=req.key,
                               vol=vol, out=out, t_arrival=start + req.t, record=record)
            served.append(Served(tk, req, base.xyz, disp, base.radius, base.m, tol, base.seed, vol, out))
            nxt += 1
            in_flight += 1
        if nxt < len(pending) and in_flight == 0:
            wait = start + pending[nxt][0].t - clock()
            if wait > 0:
                time.sleep(min(wait, 0.002))
                continue
        in_flight = server.progress(iterations)
    torch.cuda.synchronize()
    for s in served:
        s.result = server.result(s.ticket)
        server.forget(s.ticket)   # the server keeps no record of finished requests
    return served


def latency_summary(served, skip: int = 0) -> dict:
    """p50 / p99 / mean latency (arrival -> output complete) in ms, and throughput."""
    done = [s for s in served[skip:] if s.result["state"] == 3]
    lat = np.array([1e3 * (s.result["t_done"] - s.result["t_arrival"]) for s in done])
    if len(lat) == 0:
        return {"requests": 0}
    t0 = min(s.result["t_arrival"] for s in done)
    t1 = max(s.result["t_done"] for s in done)
    pairs = sum(s.result["pairs_group"] + s.result["pairs_append"] + s.vol.shape[0] * s.result["nc"] for s in done)
    return {"requests": len(done), "failed": sum(1 for s in served[skip:] if s.result["state"] < 0),
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "max_ms": float(lat.max()),
            "requests_per_s": len(done) / (t1 - t0), "pair_evals_per_s": pairs / (t1 - t0),
            "warm": sum(1 for s in done if s.result["warm"])}
