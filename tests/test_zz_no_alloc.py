"""hk_label_noalloc (labelling with the workspace in the library's fixed
device array, no allocation): through the C-ABI, two calls in a row, the
second on a smaller lattice, each equal to hk_label on the same field and
to the oracle, bit for bit; a lattice whose workspace does not fit the
array is refused before any write."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

import oracle
from paper_1405_1931_amd import _lib
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


def noalloc(phi, mask):
    nz, ny, nx = phi.shape
    labels = torch.full(phi.shape, -7, dtype=torch.int32, device="cuda")
    k = torch.full((1,), -7, dtype=torch.int64, device="cuda")
    sizes = torch.full(((nx * ny * nz + 1) // 2,), -7, dtype=torch.int64, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    rc = _lib.load().hk_label_noalloc(phi.data_ptr(), nx, ny, nz, mask, labels.data_ptr(), k.data_ptr(),
                                      sizes.data_ptr(), ctypes.c_void_p(st))
    torch.cuda.synchronize()
    return rc, labels, int(k.item()), sizes


def test_noalloc_equals_hk_label_twice_second_smaller(hk):
    cases = [(W.percolation((150, 140, 160), W.P_SITE, seed=71), 7),
             (W.droplets((45, 70, 130), 20, 4.0, 10.0, seed=72, periodic=(1, 0, 1)), 5)]
    for phi_np, mask in cases:
        print(f"[noalloc] {phi_np.shape} mask {mask}", flush=True)
        phi = torch.from_numpy(phi_np).cuda()
        rc, lab, k, sz = noalloc(phi, mask)
        assert rc == _lib.HK_OK
        el, ek, es = hk.label(phi, mask)
        torch.cuda.synchronize()
        assert k == ek
        assert torch.equal(lab, el)
        assert torch.equal(sz[:k], es)
        ol, ok, osz = oracle.label(phi_np, mask)
        assert k == ok and np.array_equal(lab.cpu().numpy(), ol) and np.array_equal(sz[:k].cpu().numpy(), osz)
    assert hk.device_error() == 0


def test_noalloc_refuses_a_lattice_beyond_its_array(hk):
    phi = torch.ones((200, 200, 200), dtype=torch.float32, device="cuda")
    rc, lab, k, sz = noalloc(phi, 0)
    assert rc == _lib.HK_ERR_TOO_LARGE
    assert k == -7 and bool((lab == -7).all())  # nothing written
