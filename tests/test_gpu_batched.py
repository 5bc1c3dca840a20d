"""GPU parity of the batched launches: every job of a mix equals the
same job labelled alone and the oracle, bit for bit; hipGraph replays of a
captured batched call equal the eager call."""
from __future__ import annotations

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


def _mix(n, seed, lo=1, hi=120):
    rng = np.random.default_rng(seed)
    items = []
    for j in range(n):
        shape = tuple(int(v) for v in rng.integers(lo, hi, size=3))
        if j % 3 == 2:
            phi = W.droplets(shape, max(1, int(np.prod(shape)) // 20000), 3.0, 9.0, seed=j,
                             periodic=(j & 1, j & 2, j & 4))
        else:
            phi = W.percolation(shape, float(rng.uniform(0.1, 0.7)), seed=j)
        items.append((phi, int(rng.integers(0, 8))))
    return items


def _check_batch(hk, items, what):
    print(f"[batched] {what}: {len(items)} jobs", flush=True)
    dev = [(torch.from_numpy(p).cuda(), m) for p, m in items]
    out = hk.label_batched(dev)
    torch.cuda.synchronize()
    assert hk.device_error() == 0
    for j, ((phi, m), (lab, k, sz)) in enumerate(zip(items, out)):
        exp = oracle.label(phi, m)
        assert k == exp[1], f"{what} job {j}: K {k} != {exp[1]}"
        assert np.array_equal(lab.cpu().numpy(), exp[0]), f"{what} job {j}: labels differ"
        assert np.array_equal(sz.cpu().numpy(), exp[2]), f"{what} job {j}: sizes differ"
    return dev, out


def test_batched_mix_equals_oracle_and_alone(hk):
    items = _mix(40, seed=1)
    dev, out = _check_batch(hk, items, "mix40")
    for (phi, m), (lab, k, sz) in zip(dev[:10], out[:10]):
        l1, k1, s1 = hk.label(phi, m)
        assert k1 == k and torch.equal(l1, lab) and torch.equal(s1, sz)


def test_batched_single_and_tiny(hk):
    _check_batch(hk, [(W.percolation((1, 1, 1), 0.9, seed=1), 7)], "one site")
    _check_batch(hk, [(W.constant((3, 3, 3), -1.0), 0), (W.constant((2, 5, 70), 1.0), 7)], "empty+full")
    _check_batch(hk, _mix(12, seed=5, lo=1, hi=6), "tiny")


def test_batched_repeat_and_order(hk):
    items = _mix(24, seed=9)
    dev = [(torch.from_numpy(p).cuda(), m) for p, m in items]
    a = hk.label_batched(dev)
    b = hk.label_batched(dev[::-1])[::-1]
    torch.cuda.synchronize()
    for (la, ka, sa), (lb, kb, sb) in zip(a, b):
        assert ka == kb and torch.equal(la, lb) and torch.equal(sa, sb)


def test_config5_stream(hk):
    jobs = W.stream()
    _check_batch(hk, [(j.phi, j.mask) for j in jobs], "config5")


def test_graph_capture_replay(hk):
    """Capture one batched call in a hipGraph and replay it; the eager result
    equals the oracle and every replay equals the eager result."""
    items = _mix(16, seed=21)
    jobs = []
    for phi_np, m in items:
        phi = torch.from_numpy(phi_np).cuda()
        nz, ny, nx = phi.shape
        jobs.append((phi, m, torch.empty_like(phi, dtype=torch.int32), torch.zeros(1, dtype=torch.int64, device="cuda"),
                     torch.empty(max(1, hk.max_clusters(nx, ny, nz)), dtype=torch.int64, device="cuda")))
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        hk.reserve(hk.batched_workspace_bytes([j[0] for j in jobs]))
        hk.label_batched_into(jobs)
    s.synchronize()
    eager = [(j[2].clone(), int(j[3].item()), j[4][: int(j[3].item())].clone()) for j in jobs]
    for (phi_np, m), (el, ek, es) in zip(items, eager):
        ol, ok, osz = oracle.label(phi_np, m)
        assert ek == ok and np.array_equal(el.cpu().numpy(), ol) and np.array_equal(es.cpu().numpy(), osz)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        hk.label_batched_into(jobs)
    for rep in range(4):
        for j in jobs:
            j[2].fill_(-1)
            j[3].fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for j, (el, ek, es) in zip(jobs, eager):
            assert int(j[3].item()) == ek, rep
            assert torch.equal(j[2], el), rep
            assert torch.equal(j[4][:ek], es), rep
    assert hk.device_error(stream=s) == 0


def test_autotune_installs_a_shape_and_keeps_results_exact(hk, tmp_path):
    """The tuner times every candidate brick shape, installs the fastest for
    the lattice's bucket, and the labelling stays bit-exact under it."""
    phi_np = W.percolation((70, 90, 130), 0.3116, seed=41)
    phi = torch.from_numpy(phi_np).cuda()
    print("[autotune] single lattice 130x90x70", flush=True)
    by, bz, ms = hk.autotune(phi, 7, reps=2)
    assert by * bz <= 256 and ms > 0
    assert hk.get_brick(130, 90, 70) == (by, bz)
    lab, k, sz = hk.label(phi, 7)
    exp = oracle.label(phi_np, 7)
    assert k == exp[1] and np.array_equal(lab.cpu().numpy(), exp[0]) and np.array_equal(sz.cpu().numpy(), exp[2])
    path = tmp_path / "bricks.txt"
    hk.tune_save(path)
    hk.set_brick_for_shape(130, 90, 70, 0, 0)
    hk.tune_load(path)
    assert hk.get_brick(130, 90, 70) == (by, bz)
    hk.set_brick_for_shape(130, 90, 70, 0, 0)

    items = _mix(12, seed=77, lo=8, hi=100)
    jobs = []
    for phi_np, m in items:
        p = torch.from_numpy(phi_np).cuda()
        nz, ny, nx = p.shape
        jobs.append((p, m, torch.empty_like(p, dtype=torch.int32), torch.zeros(1, dtype=torch.int64, device="cuda"),
                     torch.empty(max(1, hk.max_clusters(nx, ny, nz)), dtype=torch.int64, device="cuda")))
    print("[autotune] batch of 12", flush=True)
    by, bz, ms = hk.autotune_batched(jobs, reps=2)
    assert by * bz <= 256 and ms > 0
    torch.cuda.synchronize()
    for j, ((phi_np, m), job) in enumerate(zip(items, jobs)):
        exp = oracle.label(phi_np, m)
        k = int(job[3].item())
        assert k == exp[1] and np.array_equal(job[2].cpu().numpy(), exp[0]), f"job {j}"
        assert np.array_equal(job[4][:k].cpu().numpy(), exp[2]), f"job {j}"
    for phi_np, _ in items:
        nz, ny, nx = phi_np.shape
        hk.set_brick_for_shape(nx, ny, nz, 0, 0)
    assert hk.device_error() == 0


def test_single_lattice_graph_capture_replay(hk):
    """hk_label enqueues kernels only: captured in a hipGraph once the stream's
    workspace exists, every replay (into cleared outputs, with the stream's
    own eager work between replays) equals the eager call, which equals the
    oracle; two lattices of different shapes and masks, each its own graph."""
    cases = ((W.percolation((45, 61, 77), 0.3116, seed=51), 5), (W.percolation((64, 64, 64), 0.45, seed=52), 7))
    s = torch.cuda.Stream()
    for phi_np, m in cases:
        print(f"[graph] hk_label capture, shape {phi_np.shape} mask {m}", flush=True)
        phi = torch.from_numpy(phi_np).cuda()
        nz, ny, nx = phi.shape
        labels = torch.empty_like(phi, dtype=torch.int32)
        k = torch.zeros(1, dtype=torch.int64, device="cuda")
        sizes = torch.empty(hk.max_clusters(nx, ny, nz), dtype=torch.int64, device="cuda")
        with torch.cuda.stream(s):
            hk.label_into(phi, m, labels, k, sizes, stream=s)
        s.synchronize()
        ek = int(k.item())
        el, es = labels.clone(), sizes[:ek].clone()
        ol, ok, osz = oracle.label(phi_np, m)
        assert ek == ok and np.array_equal(el.cpu().numpy(), ol) and np.array_equal(es.cpu().numpy(), osz)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            hk.label_into(phi, m, labels, k, sizes, stream=s)
        for rep in range(4):
            labels.fill_(-1)
            k.fill_(-1)
            sizes.fill_(-1)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert int(k.item()) == ek, rep
            assert torch.equal(labels, el), rep
            assert torch.equal(sizes[:ek], es), rep
            # eager work of the same stream between replays
            with torch.cuda.stream(s):
                hk.label_into(phi, m, labels, k, sizes, stream=s)
            s.synchronize()
            assert int(k.item()) == ek and torch.equal(labels, el), rep
        del g
    assert hk.device_error(stream=s) == 0
