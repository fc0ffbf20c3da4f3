"""GPU parity of cell keys, the (key, id) sort and the CIC paint against the oracle."""
import numpy as np
import pytest
import torch

import synth
from oracle import mesh as M
from paper_1805_02247_amd import api
from _gpu import DEV, rel_l2, require_gpu, say

pytestmark = pytest.mark.gpu


def _clustered(seed, B, npart, box):
    """Positions with heavy-tailed cell occupancy: half uniform, half in tight blobs, plus
    particles exactly on nodes, on cell faces and at the box edge."""
    P = npart ** 3
    r = np.random.default_rng(seed)
    x = r.uniform(0, box, (B, 3, P))
    nb = max(P // 2, 1)
    centers = r.uniform(0, box, (B, 3, 16))
    which = r.integers(0, 16, (B, nb))
    for b in range(B):
        x[b, :, :nb] = (centers[b][:, which[b]] + r.normal(0, box / 200, (3, nb))) % box
    x[:, :, nb] = 0.0
    x[:, :, nb + 1] = box / 4
    x[:, :, nb + 2] = np.nextafter(box, 0)
    return x


def _oracle_order(x, n_mesh, box):
    B, _, P = x.shape
    keys = np.concatenate([b * n_mesh ** 3 + M.cell_keys(x[b], n_mesh, box) for b in range(B)])
    order = M.sort_order(keys)
    return keys[order], order


@pytest.mark.parametrize("B,npart,nm", [(1, 16, 16), (2, 16, 32), (3, 32, 64), (1, 128, 128),
                                       (4, 32, 128), (2, 64, 256)])
def test_keys_and_order_bit_exact(B, npart, nm):
    require_gpu()
    box = 100.0
    say(f"sort B={B} np={npart} nm={nm}")
    x = _clustered(B * 100 + npart, B, npart, box)
    keys, ids, rows = api.cic_sort(torch.from_numpy(x).to(DEV), nm, box)
    k_ref, o_ref = _oracle_order(x, nm, box)
    assert np.array_equal(keys.cpu().numpy().view(np.uint32), k_ref.astype(np.uint32))
    assert np.array_equal(ids.cpu().numpy().view(np.uint32), o_ref.astype(np.uint32))
    row_ref = np.searchsorted(k_ref // nm, np.arange(B * nm * nm + 1), side="left")
    assert np.array_equal(rows.cpu().numpy().view(np.uint32), row_ref.astype(np.uint32))


@pytest.mark.parametrize("B,npart,nm", [(1, 16, 16), (2, 16, 32), (2, 32, 32), (1, 64, 128)])
def test_paint_matches_oracle_and_is_reproducible(B, npart, nm):
    require_gpu()
    box = 64.0
    say(f"paint B={B} np={npart} nm={nm}")
    x = _clustered(B * 7 + nm, B, npart, box)
    xt = torch.from_numpy(x).to(DEV)
    keys, ids, rows = api.cic_sort(xt, nm, box)
    mass = (nm / npart) ** 3
    d1 = api.cic_paint(xt, keys, ids, rows, nm, box, mass, 1.0)
    d2 = api.cic_paint(xt, keys, ids, rows, nm, box, mass, 1.0)
    assert torch.equal(d1, d2)
    got = d1.cpu().numpy()
    for b in range(B):
        ref = M.cic_paint(x[b], nm, box, np.full(npart ** 3, mass)).ravel() - 1.0
        e = rel_l2(got[b] + 1.0, ref + 1.0)
        say(f"  item {b}: rel-L2 of rho {e:.2e}, mass {got[b].sum() + nm ** 3:.3f}")
        assert e < 1e-6
        assert abs((got[b].astype(np.float64) + 1).sum() - npart ** 3 * mass) < 1e-4 * npart ** 3 * mass


def test_paint_empty_rows_and_single_particle():
    """All particles in one cell: every other row is empty; the four target rows get the
    exact CIC weights."""
    require_gpu()
    box, npart, nm = 16.0, 16, 16
    x = np.full((1, 3, npart ** 3), 5.25)
    x[0, 2] = 7.5
    xt = torch.from_numpy(x).to(DEV)
    keys, ids, rows = api.cic_sort(xt, nm, box)
    d = api.cic_paint(xt, keys, ids, rows, nm, box, 1.0, 0.0).cpu().numpy()[0].reshape(nm, nm, nm)
    ref = M.cic_paint(x[0], nm, box, np.ones(npart ** 3))
    np.testing.assert_allclose(d, ref, rtol=1e-6)
    assert np.count_nonzero(d) == 8


@pytest.mark.parametrize("layout", ["one_cell", "lattice"])
def test_degenerate_layouts_at_full_size(layout):
    """The two extremes of cell occupancy at 128^3 particles on a 128^3 mesh, batch 4 (the
    benchmark's launch size), cell size 1 so that the CIC weights are exact dyadics:
    * one_cell: all 2^21 particles of item b in one cell (a different cell per item, with
      fractions 1/4, 1/2, 3/4): every key of an item is equal, so the stable sort keeps the
      ids in order, one row holds the whole item, and the paint puts N * w_corner into 8
      cells (sums of equal dyadic terms: exact in FP32);
    * lattice: one particle on every node: every key is distinct, each row holds 128
      particles, and the density contrast is 0 everywhere."""
    require_gpu()
    B, npart, nm = 4, 128, 128
    box = float(nm)
    P = npart ** 3
    say(f"degenerate layout {layout}: B={B} np={npart} nm={nm}")
    if layout == "one_cell":
        cells = [(5, 7, 100), (127, 0, 3), (64, 64, 127), (0, 127, 0)]
        frac = (0.25, 0.5, 0.75)
        x = np.empty((B, 3, P))
        for b, c in enumerate(cells):
            for a in range(3):
                x[b, a] = c[a] + frac[a]
    else:
        q = np.arange(P)
        lat = np.stack([q // (npart * npart), (q // npart) % npart, q % npart]).astype(np.float64)
        x = np.broadcast_to(lat, (B, 3, P)).copy()
    xt = torch.from_numpy(x).to(DEV)
    keys, ids, rows = api.cic_sort(xt, nm, box)
    k_ref, o_ref = _oracle_order(x, nm, box)
    assert np.array_equal(keys.cpu().numpy().view(np.uint32), k_ref.astype(np.uint32))
    assert np.array_equal(ids.cpu().numpy().view(np.uint32), o_ref.astype(np.uint32))
    row_ref = np.searchsorted(k_ref // nm, np.arange(B * nm * nm + 1), side="left")
    assert np.array_equal(rows.cpu().numpy().view(np.uint32), row_ref.astype(np.uint32))
    if layout == "one_cell":
        # stable: equal keys keep id order
        assert np.array_equal(o_ref, np.arange(B * P))
    d = api.cic_paint(xt, keys, ids, rows, nm, box, 1.0, 0.0).cpu().numpy()
    want = np.zeros((B, nm, nm, nm), dtype=np.float64)
    if layout == "one_cell":
        for b, c in enumerate(cells):
            for ox in (0, 1):
                for oy in (0, 1):
                    for oz in (0, 1):
                        w = ((frac[0] if ox else 1 - frac[0]) * (frac[1] if oy else 1 - frac[1])
                             * (frac[2] if oz else 1 - frac[2]))
                        want[b, (c[0] + ox) % nm, (c[1] + oy) % nm, (c[2] + oz) % nm] = P * w
    else:
        want[:] = 1.0
    assert np.array_equal(d.astype(np.float64), want.reshape(B, -1))
