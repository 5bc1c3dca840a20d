"""GPU parity of hk_label_pred (occupancy by another predicate: field > t,
field == v, byte mask) against the predicate oracle, exactly: labels, K and
sizes; and the Sec. 6 pipeline, labelling the sites of the capsule workload
that kept the far-field proximity value, then classifying them."""
from __future__ import annotations

import struct

import numpy as np
import pytest

import oracle
from oracle import classify as C
from oracle import predicates as P
from paper_1405_1931_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DEN = struct.unpack("<f", struct.pack("<I", 1))[0]


@pytest.fixture(scope="module")
def hk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1405_1931_amd as hk

    hk.set_brick(0, 0)
    return hk


def special_field(rng, shape):
    vals = np.array([0.0, -0.0, DEN, -DEN, 1e-38, -1e-38, 0.25, -0.25, 0.5, -1.0, -1.0, -1.0, np.inf, -np.inf,
                     np.nan, 2.0], dtype=np.float32)
    return rng.choice(vals, size=shape).astype(np.float32)


def check(hk, field_np, pred, t, mask, what):
    print(f"[pred] {what} {field_np.shape} {pred} {t} mask {mask}", flush=True)
    f = torch.from_numpy(np.ascontiguousarray(field_np)).cuda()
    labels, k, sizes = hk.label_pred(f, pred, t, mask)
    el, ek, es = P.label(field_np, pred, t, mask)
    assert k == ek, what
    assert np.array_equal(labels.cpu().numpy(), el), what
    assert np.array_equal(sizes.cpu().numpy(), es[:ek]), what
    return labels, k


@pytest.mark.parametrize("shape", [(1, 1, 7), (3, 5, 70), (9, 33, 65), (17, 20, 130), (40, 41, 42)])
def test_float_predicates_all_masks(hk, shape):
    rng = np.random.default_rng(sum(shape) + 7)
    field = special_field(rng, shape)
    for mask in range(8):
        for pred, t in (("gt", 0.3), ("gt", -0.3), ("gt", DEN), ("gt", -np.inf), ("eq", -1.0), ("eq", 0.0),
                        ("eq", -0.0)):
            check(hk, field, pred, t, mask, "special values")


@pytest.mark.parametrize("shape", [(1, 1, 7), (5, 6, 64), (17, 20, 130), (33, 40, 129)])
def test_byte_mask_all_masks(hk, shape):
    rng = np.random.default_rng(sum(shape) + 8)
    u8 = (rng.random(shape) < 0.31).astype(np.uint8) * rng.integers(1, 256, size=shape).astype(np.uint8)
    for mask in range(8):
        check(hk, u8, "u8", 0.0, mask, "byte mask")


def test_gt_zero_is_hk_label(hk):
    phi_np, mask = W.config(1)
    phi = torch.from_numpy(phi_np).cuda()
    l0, k0, s0 = hk.label(phi, mask)
    for t in (0.0, -0.0):
        l1, k1, s1 = hk.label_pred(phi, "gt", t, mask)
        assert k1 == k0 and torch.equal(l1, l0) and torch.equal(s1, s0)


def test_threshold_on_percolation_field(hk):
    """phi > t on a percolation field is percolation at another p."""
    phi_np, _ = W.config(1, 1)
    for t in (0.1, -0.2):
        check(hk, phi_np, "gt", t, 7, "percolation threshold")


def test_capsule_pipeline_from_proximity(hk):
    """Sec. 6: label the sites with I == I0, then classify the clusters."""
    for scale in (2, 1):
        phi_np, I_np, mask = W.capsule_config(scale)
        I = torch.from_numpy(I_np).cuda()
        labels, k, sizes = hk.label_pred(I, "eq", W.I0, mask)
        l0, k0, s0 = hk.label(torch.from_numpy(phi_np).cuda(), mask)
        assert k == k0 and torch.equal(labels, l0) and torch.equal(sizes, s0)
        if scale == 2:
            el, ek, es = oracle.label(phi_np, mask)
            assert ek == k and np.array_equal(labels.cpu().numpy(), el)
        kt = torch.tensor([k], dtype=torch.int64, device="cuda")
        neg, pos, inside = hk.classify(I, labels, kt, mask)
        en, ep, ei = C.classify(I_np, labels.cpu().numpy(), k, mask)
        assert np.array_equal(inside.cpu().numpy(), ei)
        assert ei[0] == 0 and np.all(ei[1:] == 1)
    assert hk.device_error() == 0


def test_invalid_arguments(hk):
    from paper_1405_1931_amd import _lib

    f = torch.zeros((4, 4, 4), dtype=torch.float32, device="cuda")
    for pred in ("gt", "eq"):
        with pytest.raises(_lib.HkError):
            hk.label_pred(f, pred, float("nan"))
    with pytest.raises(TypeError):
        hk.label_pred(f, "u8")
    with pytest.raises(TypeError):
        hk.label_pred(f.to(torch.uint8), "gt", 0.5)
