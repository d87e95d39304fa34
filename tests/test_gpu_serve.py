"""Serving form: requests of mixed (L, N) arriving while others run are batched and
overlapped on several streams; every result is bitwise the one of the request run alone."""
import time

import numpy as np
import pytest
import torch

from paper_1308_5706_amd import s2dw
from paper_1308_5706_amd.inputs import random_flm
from paper_1308_5706_amd.serve import Request, Server

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_results_alone_and_in_the_mix_agree(precision):
    print(f"serving mix {precision}", flush=True)
    rng = np.random.Generator(np.random.PCG64(7))
    shapes = [(16, 1), (32, 4), (48, 4), (32, 8)]
    n = 40
    picks = rng.integers(0, len(shapes), size=n)
    reqs = []
    for i, k in enumerate(picks):
        L, N = shapes[k]
        reqs.append(Request(i, L, N, torch.as_tensor(random_flm(L, 500 + i)).to("cuda")))
    srv = Server(lam=2.0, J_min=1, precision=precision, streams=3, max_batch=6)
    srv.warm(shapes)
    # staggered arrivals: half at once, the rest while the first batches run
    done = []
    for r in reqs[: n // 2]:
        r.t_arrival = time.perf_counter()
        srv.submit(r)
    done += srv.step()
    for r in reqs[n // 2:]:
        r.t_arrival = time.perf_counter()
        srv.submit(r)
        done += srv.step()
    while not srv.idle():
        done += srv.step()
    assert sorted(r.rid for r in done) == list(range(n))
    for r in done:
        W, Wp = s2dw.analysis(r.flm, r.L, r.N, 2.0, 1, precision=precision)
        torch.cuda.synchronize()
        assert torch.equal(r.W, W), r.rid
        assert torch.equal(r.Wphi, Wp), r.rid
        assert r.t_done >= r.t_arrival


def test_admission_waits_for_memory():
    # a budget that holds one batch of one map at a time: requests still all complete
    L, N = 32, 4
    srv = Server(lam=2.0, J_min=1, streams=2, max_batch=4)
    srv.warm([(L, N)])
    reqs = [Request(i, L, N, torch.as_tensor(random_flm(L, 600 + i)).to("cuda")) for i in range(5)]
    torch.cuda.synchronize()
    one = srv._footprint(L, N, 1)
    srv.max_bytes = s2dw.cache_bytes() + torch.cuda.memory_allocated() + one + 1
    for r in reqs:
        srv.submit(r)
    done = 0
    while not srv.idle():
        fin = srv.step()
        assert sum(b is not None for b in srv._busy) <= 1  # one batch of one map fits at a time
        for r in fin:  # the caller takes its results and drops them
            r.W = r.Wphi = None
        done += len(fin)
    assert done == 5
