"""GPU tests of the labelling server: requests submitted while others run are
batched together with them, and every result is bit-identical to the same
lattice labelled alone with hk_label (and to the oracle)."""
from __future__ import annotations

import time

import numpy as np
import pytest

import oracle
from paper_1405_1931_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def hk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1405_1931_amd as hk

    hk.set_brick(0, 0)
    return hk


def _items(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for j in range(n):
        shape = tuple(int(v) for v in rng.integers(2, 96, size=3))
        if j % 2:
            phi = W.droplets(shape, max(1, int(np.prod(shape)) // 15000), 3.0, 9.0, seed=seed + j,
                             periodic=(j & 1, j & 2, j & 4))
        else:
            phi = W.percolation(shape, float(rng.uniform(0.15, 0.6)), seed=seed + j)
        out.append((torch.from_numpy(phi).cuda(), int(rng.integers(0, 8))))
    return out


def _alone(hk, phi, mask):
    lab, k, sz = hk.label(phi, mask)
    return lab, k, sz


def test_served_mix_equals_alone_and_oracle(hk):
    from paper_1405_1931_amd.serve import Server

    items = _items(40, seed=100)
    print(f"[server] mix of {len(items)} requests, 3 slots", flush=True)
    with Server(2 << 30, slots=3, max_batch=16) as s:
        tickets = []
        for j, (phi, m) in enumerate(items):
            tickets.append(s.submit(phi, m))
            if j % 7 == 6:
                time.sleep(0.002)  # let batches start while more requests arrive
        s.drain(60)
        st = s.stats()
        assert st["completed"] == len(items) and st["failed"] == 0
        assert st["batches"] < len(items)
        for j, ((phi, m), t) in enumerate(zip(items, tickets)):
            lab, k, sz, lat = s.result(t)
            el, ek, es = _alone(hk, phi, m)
            assert k == ek, f"request {j}: K {k} != {ek} alone"
            assert torch.equal(lab, el), f"request {j}: labels differ from the lattice labelled alone"
            assert torch.equal(sz, es), f"request {j}: sizes differ"
            if j < 8:
                ol, ok, osz = oracle.label(phi.cpu().numpy(), m)
                assert k == ok and np.array_equal(lab.cpu().numpy(), ol) and np.array_equal(sz.cpu().numpy(), osz)
            s.release(t)
        assert s.stats()["arena_in_use"] == 0
    assert hk.device_error() == 0


def test_served_poisson_stream_and_tight_arena(hk):
    """Poisson arrivals into a server whose arena holds only a few requests
    at a time: admission waits for memory, results stay exact."""
    from paper_1405_1931_amd.serve import Server

    items = _items(24, seed=300)
    with Server(1 << 20, simulate=(0, 0.0)) as probe:
        fp = max(probe.footprint(p.shape) for p, _ in items)
    arena = 3 * fp
    arrivals = W.poisson_arrivals(len(items), rate=4000.0, seed=7)
    print(f"[server] {len(items)} Poisson arrivals, arena {arena} B", flush=True)
    with Server(arena, slots=2, max_batch=8) as s:
        t0 = s.now_ns()
        tickets = []
        for (phi, m), a in zip(items, arrivals):
            at = t0 + int(a * 1e9)
            while s.now_ns() < at:
                pass
            tickets.append(s.submit(phi, m, arrival_ns=at))
        results = []
        for t in tickets:
            s.wait(t, 60)
            results.append(s.result(t))
            s.release(t)
        st = s.stats()
        assert st["completed"] == len(items) and st["arena_peak"] <= arena
        assert st["latency_samples"] == len(items) and st["latency_p99_ns"] >= st["latency_p50_ns"] > 0
        for j, ((phi, m), (lab, k, sz, lat)) in enumerate(zip(items, results)):
            el, ek, es = _alone(hk, phi, m)
            assert k == ek and torch.equal(lab, el) and torch.equal(sz, es), f"request {j} differs from alone"
    assert hk.device_error() == 0
