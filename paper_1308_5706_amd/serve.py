"""Serving form: continuous batching of wavelet-analysis requests of mixed (L, N) on one GPU.

Requests arrive over time.  The scheduler keeps them in arrival order; whenever one of
its HIP streams is free it forms a batch from the oldest pending request and the pending
requests with the same (L, N) (up to ``max_batch``), admits it if its HBM footprint fits
(the batch's W and W^Phi plus the stream workspace the library will hold for it, on top
of what is in flight and what the library caches), and launches it with the batched C
entry point on that stream.  Batches of different sizes therefore overlap on the device,
and requests that arrive while others run join the next batch of their size.  Results
(W, W^Phi) stay in HBM on the request until the caller drops them.

Each result is bitwise the one of a single-map call with the same parameters: the batched
kernels compute every map exactly as the single-map ones.

Benchmark (one JSON line per precision)::

    python -m paper_1308_5706_amd.serve --requests 10000 --load 0.7

draws the configuration's request mix (L from {64, 128, 256, 512, 1024} with weights
.4/.25/.2/.1/.05, N from {1, 4, 8}, lambda = 2, J_min = 1) from seeded generators, measures
the saturated throughput with every request queued at once, then replays Poisson arrivals
at ``load`` times that rate and reports throughput and p50/p99 latency (arrival to the
host seeing the batch's completion event).  Input maps come from a pool of seeded f_lm per
L (drawn as in the benchmark: complex Gaussian, C_l = 1/(l+1)^2, real-signal symmetry).
"""
from __future__ import annotations

import argparse
import gc
import json
import math
import sys
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import s2dw
from .inputs import random_flm


@dataclass
class Request:
    rid: int
    L: int
    N: int
    flm: torch.Tensor                  # complex128 [L*L] on the device
    t_arrival: float = 0.0
    t_launch: float = 0.0
    t_done: float = 0.0
    W: torch.Tensor | None = None      # [S][2N-1][L][2L-1] once done
    Wphi: torch.Tensor | None = None
    error: Exception | None = None     # set when its batch failed to launch
    cancelled: bool = False            # set by Server.cancel; no results are kept


@dataclass
class _Batch:
    reqs: list
    event: object                      # completion marker with .query()
    bytes: int
    W: torch.Tensor = None
    Wp: torch.Tensor = None


class CudaBackend:
    """The device side of the server: HIP streams, memory queries and the batched C entry
    point.  The scheduler only uses these methods, so that its logic runs with any backend."""

    def __init__(self, device: str, streams: int):
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(streams)]

    def total_memory(self) -> int:
        return torch.cuda.get_device_properties(self.device).total_memory

    def held_bytes(self) -> int:
        """The library's plans and workspaces plus torch's live tensors (results in flight or
        kept by the caller)."""
        return s2dw.cache_bytes() + torch.cuda.memory_allocated(self.device)

    def cache_bytes(self) -> int:
        return s2dw.cache_bytes()

    def workspace_bytes(self, L, N, lam, J_min, n, precision) -> int:
        return s2dw.workspace_bytes(L, N, lam, J_min, count=n, precision=precision)

    def warm(self, L, N, lam, J_min, n, precision):
        f = torch.zeros((n, L * L), dtype=torch.complex128, device=self.device)
        for st in self.streams:
            with torch.cuda.stream(st):
                s2dw.analysis_batched(f, L, N, lam, J_min, precision=precision)
            torch.cuda.synchronize()
        torch.cuda.empty_cache()

    def launch(self, i, reqs, L, N, lam, J_min, precision):
        """Analysis of the batch on stream i: (W, W^Phi, completion event)."""
        st = self.streams[i]
        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st):
            F = torch.stack([r.flm for r in reqs])
            W, Wp = s2dw.analysis_batched(F, L, N, lam, J_min, precision=precision)
            ev = torch.cuda.Event()
            ev.record(st)
        return W, Wp, ev


@dataclass
class Server:
    lam: float = 2.0
    J_min: int = 1
    precision: str = "fp64"
    streams: int = 4
    max_batch: int = 16
    max_batch_bytes: int = 2 << 30     # cap on the W + W^Phi bytes of one batch
    max_bytes: int | None = None
    device: str = "cuda:0"
    backend: object = None             # CudaBackend(device, streams) unless given
    on_launch: object = None           # called with a batch's requests before it launches; an
                                       # exception it raises fails that batch only
    _pending: deque = field(default_factory=deque)
    _busy: list = field(default_factory=list)
    _inflight_bytes: int = 0
    _finished: list = field(default_factory=list)

    def __post_init__(self):
        if self.backend is None:
            self.backend = CudaBackend(self.device, self.streams)
        if self.max_bytes is None:
            self.max_bytes = int(0.7 * self.backend.total_memory())
        self._busy = [None] * self.streams
        self._wel = 4 if self.precision == "mixed" else 8

    # -- footprint of a batch: W + W^Phi of its maps and the stream workspace it needs
    def _w_bytes(self, L, N):
        S = s2dw.num_scales(L, self.lam, self.J_min)
        return S * (2 * N - 1) * L * (2 * L - 1) * self._wel + 16 * L * L

    def _batch_cap(self, L, N):
        return max(1, min(self.max_batch, self.max_batch_bytes // self._w_bytes(L, N)))

    def _footprint(self, L, N, n):
        return n * self._w_bytes(L, N) + self.backend.workspace_bytes(L, N, self.lam, self.J_min, n, self.precision)

    def submit(self, req: Request):
        if self.backend.cache_bytes() + self._footprint(req.L, req.N, 1) > self.max_bytes:
            raise MemoryError(f"a request with L={req.L}, N={req.N} does not fit the HBM budget "
                              f"({self.max_bytes} bytes)")
        self._pending.append(req)

    def cancel(self, rid: int) -> bool:
        """Cancels a request: a pending one leaves the queue, one in flight keeps running but
        its results are dropped.  Either way it is returned by the next step() with
        cancelled set.  Returns False if the server does not hold the request."""
        for r in self._pending:
            if r.rid == rid:
                self._pending.remove(r)
                r.cancelled = True
                self._finished.append(r)
                return True
        for b in self._busy:
            if b is not None:
                for r in b.reqs:
                    if r.rid == rid:
                        r.cancelled = True
                        return True
        return False

    def idle(self) -> bool:
        return not self._pending and not self._finished and all(b is None for b in self._busy)

    def warm(self, shapes, per_stream=True):
        """Builds the plans of the (L, N) shapes and, per stream, their workspaces (the first
        call on a stream allocates), so that serving itself allocates only result buffers."""
        for (L, N) in shapes:
            self.backend.warm(L, N, self.lam, self.J_min, self._batch_cap(L, N), self.precision)

    def step(self) -> list:
        """Collects finished batches, then launches new ones on free streams.  Returns the
        requests completed since the last call: with results, or with error or cancelled set."""
        done = self._finished
        self._finished = []
        now = None
        for i, b in enumerate(self._busy):
            if b is not None and b.event.query():
                now = now or time.perf_counter()
                for k, r in enumerate(b.reqs):
                    r.t_done = now
                    if not r.cancelled:
                        r.W = b.W[k]
                        r.Wphi = b.Wp[k]
                    done.append(r)
                self._inflight_bytes -= b.bytes
                self._busy[i] = None
        for i in range(self.streams):
            if self._busy[i] is None and self._pending:
                if not self._launch(i):
                    break
        done.extend(self._finished)
        self._finished = []
        return done

    def _launch(self, i) -> bool:
        head = self._pending[0]
        key = (head.L, head.N)
        picked = [r for r in self._pending if (r.L, r.N) == key][: self._batch_cap(*key)]
        held = self.backend.held_bytes()
        while picked:
            need = self._footprint(key[0], key[1], len(picked))
            if held + need <= self.max_bytes:
                break
            picked = picked[: len(picked) // 2]
        if not picked:
            return False  # wait for batches to finish or for the caller to drop results
        ids = {id(r) for r in picked}
        self._pending = deque(r for r in self._pending if id(r) not in ids)
        L, N = key
        t = time.perf_counter()
        try:
            if self.on_launch is not None:
                self.on_launch(picked)
            W, Wp, ev = self.backend.launch(i, picked, L, N, self.lam, self.J_min, self.precision)
        except Exception as e:  # this batch fails; the others go on
            for r in picked:
                r.error = e
                r.t_done = time.perf_counter()
                self._finished.append(r)
            return True
        for r in picked:
            r.t_launch = t
        self._busy[i] = _Batch(picked, ev, need, W, Wp)
        self._inflight_bytes += need
        return True


# ------------------------------------------------------------------------------ benchmark

L_CHOICES = [64, 128, 256, 512, 1024]
L_WEIGHTS = [0.4, 0.25, 0.2, 0.1, 0.05]
N_CHOICES = [1, 4, 8]


def draw_mix(n, seed=4):
    rng = np.random.Generator(np.random.PCG64(seed))
    Ls = rng.choice(L_CHOICES, size=n, p=L_WEIGHTS)
    Ns = rng.choice(N_CHOICES, size=n)
    return [int(x) for x in Ls], [int(x) for x in Ns], rng


def run(server: Server, Ls, Ns, pool, arrivals):
    """Feeds requests at the given arrival offsets (seconds, non-decreasing; zeros = all at
    once) and returns the completed requests and the wall time."""
    n = len(Ls)
    reqs = [Request(i, Ls[i], Ns[i], pool[Ls[i]][i % len(pool[Ls[i]])]) for i in range(n)]
    done = []
    # Python's cyclic collector is paused for the timed loop, so that a full collection over
    # the request objects cannot stall the queue mid-stream (reference counting still frees
    # every result as soon as it is dropped); it runs once before and resumes after.
    gc.collect()
    gc.disable()
    try:
        t0 = time.perf_counter()
        nxt = 0
        while len(done) < n:
            now = time.perf_counter() - t0
            while nxt < n and arrivals[nxt] <= now:
                reqs[nxt].t_arrival = t0 + arrivals[nxt]
                server.submit(reqs[nxt])
                nxt += 1
            fin = server.step()
            for r in fin:
                r.W = None  # results are not kept by the benchmark
                r.Wphi = None
            done.extend(fin)
        T = time.perf_counter() - t0
    finally:
        gc.enable()
    return done, T


def coeffs_of(L, N, lam, J_min):
    return s2dw.num_scales(L, lam, J_min) * (2 * N - 1) * L * (2 * L - 1)


def benchmark(requests: int = 10000, load: float = 0.7, precisions=("fp64", "mixed"), streams: int = 4,
              max_batch: int = 16, lam: float = 2.0, J_min: int = 1) -> list:
    """The serving benchmark of the request mix: per precision, the plain path (each request
    alone, one after the other), the saturated rate (every request queued at once) and a
    Poisson stream at `load` times that rate with its p50/p99 latency.  Returns one dict per
    precision."""
    Ls, Ns, rng = draw_mix(requests)
    pool = {L: [torch.as_tensor(random_flm(L, 4_000_000 + 10 * L + k)).to("cuda") for k in range(4)]
            for L in L_CHOICES}
    gaps = rng.exponential(1.0, size=requests)  # unit-rate Poisson gaps, scaled below
    total_coeffs = sum(coeffs_of(L, N, lam, J_min) for L, N in zip(Ls, Ns))
    results = []
    for prec in precisions:
        # the plain GPU path at equal accuracy: each request alone, one after the other
        for (L, N) in sorted(set(zip(Ls, Ns))):
            s2dw.analysis(pool[L][0], L, N, lam, J_min, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i, (L, N) in enumerate(zip(Ls, Ns)):
            W, Wp = s2dw.analysis(pool[L][i % len(pool[L])], L, N, lam, J_min, precision=prec)
            del W, Wp
        torch.cuda.synchronize()
        plain = requests / (time.perf_counter() - t0)
        print(f"# {prec}: plain path {plain:.1f} requests/s", file=sys.stderr, flush=True)
        srv = Server(lam=lam, J_min=J_min, precision=prec, streams=streams, max_batch=max_batch)
        print(f"# {prec}: warming plans and stream workspaces", file=sys.stderr, flush=True)
        srv.warm(sorted(set(zip(Ls, Ns))))
        done, T = run(srv, Ls, Ns, pool, np.zeros(requests))
        r_max = requests / T
        print(f"# {prec}: saturated {r_max:.1f} requests/s", file=sys.stderr, flush=True)
        rate = load * r_max
        arrivals = np.cumsum(gaps) / rate
        done, T = run(srv, Ls, Ns, pool, arrivals)
        lat = np.array([r.t_done - r.t_arrival for r in done]) * 1e3
        print(f"# {prec}: {requests} Poisson requests at {rate:.0f}/s: p50 {np.percentile(lat, 50):.2f} ms, "
              f"p99 {np.percentile(lat, 99):.2f} ms", file=sys.stderr, flush=True)
        results.append({"metric": "SO(3) wavelet coeffs/s (analysis) served, mixed-L request stream",
                        "value": total_coeffs / T, "unit": "SO(3) coeffs/s", "precision": prec,
                        "requests": requests, "requests_per_s": requests / T,
                        "saturated_requests_per_s": r_max, "offered_requests_per_s": rate, "load": load,
                        "plain_path_requests_per_s": plain,
                        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                        "mean_ms": float(np.mean(lat)),
                        "streams": streams, "max_batch": max_batch, "data": "synthetic",
                        "mix": {"L": dict(zip(map(str, L_CHOICES), L_WEIGHTS)), "N": N_CHOICES, "lambda": lam,
                                "J_min": J_min}})
        del srv
    return results


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=10000)
    ap.add_argument("--load", type=float, default=0.7, help="offered rate as a fraction of the saturated rate")
    ap.add_argument("--precision", choices=["fp64", "mixed", "both"], default="both")
    ap.add_argument("--streams", type=int, default=4)
    ap.add_argument("--max-batch", type=int, default=16)
    args = ap.parse_args()
    precisions = ["fp64", "mixed"] if args.precision == "both" else [args.precision]
    for out in benchmark(args.requests, args.load, precisions, args.streams, args.max_batch):
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
