"""The degenerate cases of the method at the largest lattice of the
workloads (1024^3), checked element by element against closed forms
computed on the GPU with torch (the oracle would need ~12 GiB of host memory
here; it covers the same patterns at smaller sizes in test_gpu_parity.py):

* site checkerboard -- every occupied site its own cluster, K = N/2 (the
  Sec. 3 bound V/2), every size 1, label = 1 + #occupied sites before it;
* block checkerboards with b^3 blocks, b = 2, 4, 8, 64 (the Sec. 3
  benchmark lattice, whose cluster count it varies) -- K = (1024/b)^3 / 2,
  every size b^3, labels in closed form;
* full and empty lattices -- K = 1 with size N, and K = 0.
Both with and without periodic wrap (even lengths: the wraps join nothing
in the checkerboards)."""
from __future__ import annotations

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N1 = 1024


@pytest.fixture(scope="module")
def hk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1405_1931_amd as hk

    hk.set_brick(0, 0)
    return hk


def axes(n):
    a = torch.arange(n, device="cuda", dtype=torch.int32)
    return a.view(n, 1, 1), a.view(1, n, 1), a.view(1, 1, n)  # z, y, x


@pytest.mark.parametrize("mask", [0, 7])
def test_site_checkerboard_1024(hk, mask):
    print(f"[maxsize] site checkerboard 1024^3 mask {mask}", flush=True)
    n = N1
    z, y, x = axes(n)
    occ = ((x + y + z) & 1) == 0
    phi = torch.where(occ, 1.0, -1.0).to(torch.float32)
    labels, k, sizes = hk.label(phi, mask)
    assert k == n ** 3 // 2
    assert bool((sizes == 1).all())
    q = (y + z) & 1
    expect = (y + n * z) * (n // 2) + torch.div(x + 1 - q, 2, rounding_mode="floor") + 1
    assert torch.equal(labels, torch.where(occ, expect, 0).to(torch.int32))
    assert hk.device_error() == 0


@pytest.mark.parametrize("mask", [0, 7])
@pytest.mark.parametrize("b", [2, 4, 8, 64])
def test_block_checkerboard_1024(hk, mask, b):
    print(f"[maxsize] block checkerboard {b}^3 blocks, 1024^3 mask {mask}", flush=True)
    n = N1
    nb = n // b
    z, y, x = axes(n)
    bi, bj, bk = torch.div(x, b, rounding_mode="floor"), torch.div(y, b, rounding_mode="floor"), \
        torch.div(z, b, rounding_mode="floor")
    occ = ((bi + bj + bk) & 1) == 0
    phi = torch.where(occ, 1.0, -1.0).to(torch.float32)
    labels, k, sizes = hk.label(phi, mask)
    assert k == nb ** 3 // 2
    assert bool((sizes == b ** 3).all())
    expect = (bk * nb + bj) * (nb // 2) + torch.div(bi, 2, rounding_mode="floor") + 1
    assert torch.equal(labels, torch.where(occ, expect, 0).to(torch.int32))
    assert hk.device_error() == 0


@pytest.mark.parametrize("mask", [0, 7])
def test_full_and_empty_1024(hk, mask):
    print(f"[maxsize] full and empty 1024^3 mask {mask}", flush=True)
    n = N1
    phi = torch.ones((n, n, n), dtype=torch.float32, device="cuda")
    labels, k, sizes = hk.label(phi, mask)
    assert k == 1 and sizes.tolist() == [n ** 3]
    assert bool((labels == 1).all())
    phi.fill_(-1.0)
    labels, k, sizes = hk.label(phi, mask)
    assert k == 0 and sizes.numel() == 0
    assert bool((labels == 0).all())
    assert hk.device_error() == 0
