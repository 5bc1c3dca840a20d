"""Lattices above 2^30 sites, where the 32-bit site indices of the path are
closest to their limit (N <= INT32_MAX): 1024 x 1024 x 2047 sites
(2,146,435,072), checked against closed forms computed on the GPU with
torch, one z-slab at a time (the oracle would need ~25 GiB of host memory):

* full lattice: K = 1, size N, every label 1;
* empty lattice: K = 0;
* planes of even x: K = 1024 planes of ny * nz sites, plane x numbered
  x / 2 + 1; with x periodic (nx = 2047 odd) the planes x = 0 and 2046 are
  wrap neighbours and merge: K = 1023, cluster 1 twice the size;
* the site checkerboard without wraps: K = N / 2, every size 1, label = 1 +
  the number of occupied sites before the site in linear order."""
from __future__ import annotations

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

NX, NY, NZ = 2047, 1024, 1024
SLAB = 64  # z-planes compared at once


@pytest.fixture(scope="module")
def hk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1405_1931_amd as hk

    hk.set_brick(0, 0)
    return hk


@pytest.fixture(scope="module")
def bufs():
    phi = torch.empty((NZ, NY, NX), dtype=torch.float32, device="cuda")
    yield phi
    del phi
    torch.cuda.empty_cache()


def label(hk, phi, mask):
    print(f"[huge] {NX}x{NY}x{NZ} mask {mask}", flush=True)
    lab, k, sz = hk.label(phi, mask)
    assert hk.device_error() == 0
    return lab, k, sz


def test_full_and_empty(hk, bufs):
    assert NX * NY * NZ > 2 ** 30
    bufs.fill_(1.0)
    lab, k, sz = label(hk, bufs, 7)
    assert k == 1 and sz.tolist() == [NX * NY * NZ]
    assert bool((lab == 1).all())
    del lab, sz
    bufs.fill_(-1.0)
    lab, k, sz = label(hk, bufs, 0)
    assert k == 0 and bool((lab == 0).all())


@pytest.mark.parametrize("mask", [0, 1, 7])
def test_even_x_planes(hk, bufs, mask):
    x = torch.arange(NX, device="cuda", dtype=torch.int32).view(1, 1, NX)
    occ = (x % 2) == 0
    bufs.copy_(torch.where(occ, 1.0, -1.0).to(torch.float32).expand(NZ, NY, NX))
    lab, k, sz = label(hk, bufs, mask)
    plane = NY * NZ
    expect = torch.where(occ, torch.div(x, 2, rounding_mode="floor") + 1, 0).to(torch.int32)
    if mask & 1:
        assert k == NX // 2  # 1024 planes, the last joins the first
        expect = torch.where(x == NX - 1, 1, expect).to(torch.int32)
        assert sz[0].item() == 2 * plane and bool((sz[1:] == plane).all())
    else:
        assert k == NX // 2 + 1
        assert bool((sz == plane).all())
    for z0 in range(0, NZ, SLAB):
        assert torch.equal(lab[z0:z0 + SLAB], expect.expand(min(SLAB, NZ - z0), NY, NX)), z0


def test_site_checkerboard(hk, bufs):
    z = torch.arange(NZ, device="cuda", dtype=torch.int64).view(NZ, 1, 1)
    y = torch.arange(NY, device="cuda", dtype=torch.int64).view(1, NY, 1)
    x = torch.arange(NX, device="cuda", dtype=torch.int64).view(1, 1, NX)
    for z0 in range(0, NZ, SLAB):
        zz = z[z0:z0 + SLAB]
        bufs[z0:z0 + SLAB] = torch.where(((x + y + zz) % 2) == 0, 1.0, -1.0).to(torch.float32)
    lab, k, sz = label(hk, bufs, 0)
    n = NX * NY * NZ
    assert k == n // 2
    assert bool((sz == 1).all())
    # A row (y, z) is even when y + z is even: it holds (NX + 1) / 2 occupied
    # sites (even x), an odd row (NX - 1) / 2.  Before row (y, z) lie z whole
    # planes (NY / 2 even rows each, NY being even) and the rows y' < y of
    # plane z, of which ceil(y / 2) are even when z is even, floor(y / 2)
    # when z is odd.  Before x in its row: ceil(x / 2) occupied sites in an
    # even row, floor(x / 2) in an odd one.
    for z0 in range(0, NZ, SLAB):
        zz = z[z0:z0 + SLAB]
        r = y + NY * zz
        even_rows = zz * (NY // 2) + torch.where(zz % 2 == 0, (y + 1) // 2, y // 2)
        q = (y + zz) % 2
        before_rows = even_rows * ((NX + 1) // 2) + (r - even_rows) * ((NX - 1) // 2)
        in_row = torch.where(q == 0, (x + 1) // 2, x // 2)
        occ = ((x + y + zz) % 2) == 0
        expect = torch.where(occ, before_rows + in_row + 1, 0).to(torch.int32)
        assert torch.equal(lab[z0:z0 + SLAB], expect), z0
