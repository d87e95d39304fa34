"""The serving scheduler's host logic on the CPU, with a stand-in for the device side: a small
HBM budget, a per-batch error forced from the host, and cancellation of a pending and of an
in-flight request.  Every other request must still complete, no launch may exceed the budget,
and every request is returned exactly once."""
import torch

from paper_1308_5706_amd.serve import Request, Server


class FakeEvent:
    def __init__(self, polls):
        self.left = polls

    def query(self):
        self.left -= 1
        return self.left < 0


class FakeBackend:
    """Streams that finish a batch after a few polls; memory held = a fixed base plus the
    footprints of the batches in flight."""

    def __init__(self, streams, total, base, ws_per_map, polls=2):
        self.streams = [None] * streams
        self.total, self.base, self.ws = total, base, ws_per_map
        self.polls = polls
        self.inflight = []          # (event, bytes) of launched batches
        self.launched = []          # (stream, rids) in launch order
        self.peak = 0

    def total_memory(self):
        return self.total

    def _live(self):
        self.inflight = [(e, b) for e, b in self.inflight if e.left >= 0]
        return sum(b for _, b in self.inflight)

    def held_bytes(self):
        return self.base + self._live()

    def cache_bytes(self):
        return self.base

    def workspace_bytes(self, L, N, lam, J_min, n, precision):
        return self.ws * n

    def warm(self, *args):
        pass

    def launch(self, i, reqs, L, N, lam, J_min, precision):
        n = len(reqs)
        ev = FakeEvent(self.polls)
        self.launched.append((i, [r.rid for r in reqs]))
        W = torch.full((n, 1), float(L))
        Wp = torch.full((n, 1), float(N))
        self.inflight.append((ev, self.owner._footprint(L, N, n)))
        self.peak = max(self.peak, self.held_bytes())
        return W, Wp, ev


def test_budget_errors_and_cancellation():
    shapes = [(32, 4), (16, 2)]
    reqs = [Request(i, *shapes[i % 3 == 2], flm=None) for i in range(24)]
    be = FakeBackend(streams=2, total=1 << 40, base=1000, ws_per_map=5000)

    refused = []

    def hook(batch):
        if any(r.rid == 5 for r in batch):
            refused.extend(r.rid for r in batch)
            raise RuntimeError("forced launch failure")

    srv = Server(lam=2.0, J_min=1, streams=2, max_batch=3, backend=be, on_launch=hook)
    be.owner = srv
    one = srv._footprint(32, 4, 1)
    srv.max_bytes = be.base + 3 * one  # at most three maps of the larger shape in flight
    for r in reqs[:12]:
        srv.submit(r)
    done = srv.step()
    assert srv.cancel(9) or any(r.rid == 9 for r in done)  # still pending: leaves the queue
    inflight0 = any(0 in rids for _, rids in be.launched)
    assert inflight0 and srv.cancel(0)  # in flight: results dropped
    for r in reqs[12:]:
        srv.submit(r)
    for _ in range(1000):
        if srv.idle():
            break
        done += srv.step()
    assert srv.idle()
    assert sorted(r.rid for r in done) == list(range(24))  # each once
    assert be.peak <= srv.max_bytes
    failed = {r.rid for r in done if r.error is not None}
    assert 5 in failed and failed == set(refused)  # exactly the batch the hook refused
    assert {r.rid for r in done if r.cancelled} == {0, 9}
    for r in done:
        if r.error is None and not r.cancelled:
            assert r.W is not None and float(r.W[0]) == r.L  # each got its own batch row
        else:
            assert r.W is None
    assert all(5 not in rids for _, rids in be.launched)  # the failed batch never launched
    assert max(len(rids) for _, rids in be.launched) > 1  # requests were batched
    # the requests of one launch share (L, N) and go oldest first
    for _, rids in be.launched:
        assert len({(reqs[k].L, reqs[k].N) for k in rids}) == 1 and rids == sorted(rids)


def test_request_too_large_is_refused_at_submission():
    be = FakeBackend(streams=1, total=1 << 40, base=0, ws_per_map=10)
    srv = Server(lam=2.0, J_min=1, streams=1, backend=be)
    be.owner = srv
    srv.max_bytes = srv._footprint(16, 2, 1) - 1
    try:
        srv.submit(Request(0, 16, 2, flm=None))
    except MemoryError:
        pass
    else:
        raise AssertionError("an oversized request was admitted")
    assert srv.idle()
