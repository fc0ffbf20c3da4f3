"""Oracle pins: cloud-in-cell paint/readout, cell keys and the (key, id) sort order."""
import numpy as np

import synth
from oracle import mesh as M


def test_mass_conservation_and_node_deposit():
    n, box = 8, 20.0
    x = synth.random_positions(1, 500, box)
    rho = M.cic_paint(x, n, box, np.full(500, 0.7))
    assert abs(rho.sum() - 350.0) < 1e-11
    # a particle exactly on a node puts all its mass there
    node = np.array([[3 * box / n], [5 * box / n], [7 * box / n]])
    r1 = M.cic_paint(node, n, box, np.array([2.0]))
    assert r1[3, 5, 7] == 2.0 and r1.sum() == 2.0


def test_perfect_lattice_is_uniform():
    """The unperturbed lattice (half a mesh cell off the nodes) paints a uniform density,
    with the particle mesh equal to or half as fine as the force mesh."""
    for npart, nm in ((8, 8), (8, 16)):
        box = 30.0
        q = M.lattice_positions(npart, box, nm)
        rho = M.cic_paint(q, nm, box, np.full(q.shape[1], (nm / npart) ** 3))
        np.testing.assert_allclose(rho, 1.0, atol=1e-13)


def test_lattice_on_the_nodes_is_uniform():
    npart = nm = 8
    box = 16.0
    q = M.wrap(M.lattice_positions(npart, box, nm) - 0.5 * box / nm, box)
    rho = M.cic_paint(q, nm, box, np.ones(q.shape[1]))
    np.testing.assert_allclose(rho, 1.0, atol=1e-14)


def test_paint_readout_are_transposes():
    n, box = 8, 10.0
    x = synth.random_positions(2, 300, box)
    v = synth.unit_normal(3, 300)
    m = synth.unit_normal(4, (n, n, n))
    lhs = np.sum(M.cic_paint(x, n, box, v) * m)
    rhs = np.sum(v * M.cic_readout(x, n, box, m))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_readout_grad_matches_finite_difference():
    n, box = 8, 10.0
    x = synth.random_positions(5, 40, box)
    m = synth.unit_normal(6, (2, n, n, n))
    g = M.cic_readout_grad(x, n, box, m)
    h = 1e-7
    for a in range(3):
        xp, xm = x.copy(), x.copy()
        xp[a] += h
        xm[a] -= h
        fd = (M.cic_readout(xp, n, box, m) - M.cic_readout(xm, n, box, m)) / (2 * h)
        np.testing.assert_allclose(g[:, a], fd, rtol=1e-6, atol=1e-6)


def test_keys_brute_force():
    n, box = 8, 13.0
    x = synth.random_positions(7, 200, box)
    x[:, 0] = [0.0, 0.0, 0.0]
    x[:, 1] = [box * (1 - 1e-17), box / n, 2 * box / n]  # rounds to the box edge / nodes
    keys = M.cell_keys(x, n, box)
    for p in range(x.shape[1]):
        c = []
        for a in range(3):
            u = x[a, p] * (n / box)
            c.append(int(np.floor(u)) % n)
        assert keys[p] == (c[0] * n + c[1]) * n + c[2]


def test_sort_order_is_key_then_id():
    keys = np.array([5, 3, 5, 0, 3, 3, 9, 0])
    order = M.sort_order(keys)
    expect = sorted(range(len(keys)), key=lambda i: (keys[i], i))
    assert list(order) == expect


def test_wrap_range():
    box = 7.0
    x = np.array([-1e-300, -3.5, 7.0, 14.25, 6.999999999])
    w = M.wrap(x, box)
    assert np.all(w >= 0) and np.all(w <= box)
    np.testing.assert_allclose(w[1:], [3.5, 0.0, 0.25, 6.999999999])
