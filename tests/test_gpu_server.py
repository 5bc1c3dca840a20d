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
            ol, ok, osz = oracle.label(phi.cpu().numpy(), m)
            assert k == ok and np.array_equal(lab.cpu().numpy(), ol) and np.array_equal(sz.cpu().numpy(), osz), \
                f"request {j} differs from the oracle"
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
            ol, ok, osz = oracle.label(phi.cpu().numpy(), m)
            assert k == ok and np.array_equal(lab.cpu().numpy(), ol) and np.array_equal(sz.cpu().numpy(), osz), \
                f"request {j} differs from the oracle"
    assert hk.device_error() == 0


def test_served_stream_of_256_poisson_replay_equals_oracle(hk):
    """The 256-lattice stream (uneven shapes, percolation and droplets, random
    masks) replayed as Poisson arrivals through the server: every one of the
    256 results equals the oracle's, labels, K and sizes."""
    import concurrent.futures as cf

    from paper_1405_1931_amd.serve import Server

    jobs = W.stream()
    items = [(torch.from_numpy(j.phi).cuda(), j.mask) for j in jobs]
    with Server(1 << 20, simulate=(0, 0.0)) as probe:
        arena = int(1.25 * sum(probe.footprint(p.shape) for p, _ in items)) + (64 << 20)
    arrivals = W.poisson_arrivals(len(items), 100000.0, seed=5)
    print(f"[server] 256-lattice stream, Poisson replay, arena {arena} B", flush=True)
    with Server(arena, slots=3, max_batch=64) as s:
        t0 = s.now_ns() + 2_000_000
        tickets = [s.submit(phi, m, arrival_ns=t0 + int(a * 1e9)) for (phi, m), a in zip(items, arrivals)]
        s.drain(120)
        st = s.stats()
        assert st["completed"] == len(items) and st["failed"] == 0
        got = []
        for t in tickets:
            lab, k, sz, _ = s.result(t)
            got.append((lab.cpu().numpy(), k, sz.cpu().numpy()))
            s.release(t)
    lib = oracle.load()
    with cf.ThreadPoolExecutor(16) as ex:
        exp = list(ex.map(lambda j: oracle.label(j.phi, j.mask, lib=lib), jobs))
    for j, ((lab, k, sz), (el, ek, es)) in enumerate(zip(got, exp)):
        assert k == ek, f"job {j}: K {k} != {ek}"
        assert np.array_equal(lab, el), f"job {j}: labels differ from the oracle"
        assert np.array_equal(sz, es), f"job {j}: sizes differ from the oracle"
    assert hk.device_error() == 0


def test_submit_orders_after_the_producer_stream(hk):
    """phi still in the making on a side stream when it is submitted: the
    batch waits for that stream's work on the device, so the result is the
    labelling of the finished field."""
    from paper_1405_1931_amd.serve import Server

    side = torch.cuda.Stream()
    gen = torch.Generator(device="cuda").manual_seed(17)
    shapes = [(96, 80, 112), (64, 96, 128), (120, 72, 88)]
    with Server(2 << 30, slots=2, max_batch=8) as s:
        outs = []
        with torch.cuda.stream(side):
            a = torch.randn(2048, 2048, device="cuda")
            for shape in shapes:
                for _ in range(6):  # keep the side stream busy before phi is written
                    a = torch.tanh(a @ a * 1e-3)
                phi = (torch.rand(shape, device="cuda", generator=gen) - (1.0 - W.P_SITE)).contiguous()
                outs.append((phi, s.submit(phi, 7)))  # default: torch's current stream, the side stream
        s.drain(60)
        side.synchronize()
        for phi, t in outs:
            lab, k, sz, _ = s.result(t)
            el, ek, es = oracle.label(phi.cpu().numpy(), 7)
            assert k == ek and np.array_equal(lab.cpu().numpy(), el) and np.array_equal(sz.cpu().numpy(), es)
            s.release(t)
    assert hk.device_error() == 0
