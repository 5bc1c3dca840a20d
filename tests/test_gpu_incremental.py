"""GPU parity of incremental relabelling (hk_incr_*): over sequences of
fields that change a little from call to call, every call's labels, K and
sizes equal the oracle's for that field, exactly; and the number of bricks
labelled anew is the number whose occupancy changed."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1405_1931_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def hk():
    """64x16x16 bricks for every lattice of this module, so that the bricks a
    change touches are known; the default shape is restored afterwards."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1405_1931_amd as hk

    hk.set_brick(16, 16)
    yield hk
    hk.set_brick(0, 0)


def check(hk, st, phi_np, mask, what, expect_relabelled=None):
    print(f"[incr] {what} {phi_np.shape} mask {mask}", flush=True)
    phi = torch.from_numpy(np.ascontiguousarray(phi_np)).cuda()
    labels, k, sizes, rel = st.label(phi)
    el, ek, es = oracle.label(phi_np, mask)
    assert k == ek, what
    assert np.array_equal(labels.cpu().numpy(), el), what
    assert np.array_equal(sizes.cpu().numpy(), es[:ek]), what
    if expect_relabelled is not None:
        lo, hi = expect_relabelled
        assert lo <= rel <= hi, (what, rel)
    assert st.device_error() == 0
    return rel


def flip_box(phi, z0, y0, x0, d=3):
    out = phi.copy()
    out[z0:z0 + d, y0:y0 + d, x0:x0 + d] *= -1.0
    return out


@pytest.mark.parametrize("shape,mask", [((70, 45, 130), 0), ((70, 45, 130), 7), ((33, 64, 64), 5)])
def test_sequence_of_small_changes(hk, shape, mask):
    f0 = W.percolation(shape, W.P_SITE, seed=sum(shape) + mask)
    nz, ny, nx = shape
    nb = -(-nx // 64) * -(-ny // 16) * -(-nz // 16)
    with hk.Incremental(shape, mask) as st:
        first = check(hk, st, f0, mask, "first call", (nb, nb))
        check(hk, st, f0, mask, "same field again", (0, 0))
        f1 = flip_box(f0, 5, 5, 5)        # inside one brick
        check(hk, st, f1, mask, "one box flipped", (1, 1))
        f2 = flip_box(f1, 0, 0, 0, 2)     # a corner: on the wrap faces when periodic
        check(hk, st, f2, mask, "corner flipped", (1, 1))
        f3 = W.percolation(shape, 0.45, seed=99)
        check(hk, st, f3, mask, "a new field", (1, first))
        f4 = flip_box(f3, shape[0] - 1, shape[1] - 1, shape[2] - 1, 1)  # the last site only
        check(hk, st, f4, mask, "last site", (1, 1))
        check(hk, st, f4, mask, "unchanged", (0, 0))


def test_moving_droplet_field(hk):
    phi, mask = W.config(2, 4)  # 128^3 droplets, periodic
    shape = phi.shape
    with hk.Incremental(shape, mask) as st:
        total = check(hk, st, phi, mask, "droplets")
        rng = np.random.default_rng(1)
        for step in range(3):
            # a new ball of radius 4 somewhere: the bricks it touches change
            c = rng.integers(8, 120, 3)
            z, y, x = np.ogrid[:shape[0], :shape[1], :shape[2]]
            ball = (z - c[0]) ** 2 + (y - c[1]) ** 2 + (x - c[2]) ** 2 <= 16
            phi = np.where(ball, np.float32(1.0), phi).astype(np.float32)
            check(hk, st, phi, mask, f"droplet step {step}", (0, 8))
        check(hk, st, phi, mask, "no change", (0, 0))
        assert total > 8


def test_interleaved_with_other_calls(hk):
    """Other labellings on the same stream (the shared workspace) leave the
    state's tables alone."""
    shape, mask = (40, 50, 70), 3
    f0 = W.percolation(shape, W.P_SITE, seed=4)
    other = torch.from_numpy(W.percolation((40, 50, 70), 0.5, seed=5)).cuda()
    with hk.Incremental(shape, mask) as st:
        check(hk, st, f0, mask, "first")
        hk.label(other, 7)
        check(hk, st, f0, mask, "after another lattice", (0, 0))
        hk.label(other, 0)
        check(hk, st, flip_box(f0, 10, 10, 10), mask, "after another lattice, one box", (1, 1))


def test_outputs_optional_and_errors(hk):
    shape, mask = (20, 30, 40), 0
    f0 = torch.from_numpy(W.percolation(shape, W.P_SITE, seed=8)).cuda()
    with hk.Incremental(shape, mask) as st:
        labels = torch.empty(shape, dtype=torch.int32, device="cuda")
        k = torch.zeros(1, dtype=torch.int64, device="cuda")
        st.label_into(f0, labels, k)  # no sizes, no count
        el, ek, _ = oracle.label(f0.cpu().numpy(), mask)
        assert int(k.item()) == ek and np.array_equal(labels.cpu().numpy(), el)
        with pytest.raises(ValueError):
            st.label(torch.zeros((20, 30, 41), dtype=torch.float32, device="cuda"))
    with pytest.raises(RuntimeError):
        st.label(f0)
