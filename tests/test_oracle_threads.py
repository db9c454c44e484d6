"""The oracle's optional thread count (used to time it on all host cores and
to check the 1.1M-particle system in minutes): the close-pair list and the
product M x must be bitwise those of the serial loops, and Algorithm 1 must
reach the same point (only its sums over contacts are added in a different
order), for any thread count."""
import numpy as np
import pytest

import oracle as O
import workloads as W


@pytest.fixture(scope="module")
def system():
    s = W.rods_and_spheres(3000, 600, seed=W.SEED_BASE + 61)
    c, u, q = O.setup(s)
    return s, c, u, q


@pytest.mark.parametrize("nt", [2, 3, 8])
def test_threaded_contacts_and_product_are_the_serial_ones(system, nt):
    s, c, u, q = system
    assert O.get_threads() == 1
    x = np.random.default_rng(3).standard_normal(c.nc)
    y1 = O.mvop(s, c, x)
    with O.threads(nt):
        assert O.get_threads() == nt
        ct = O.find_contacts(s)
        yt = O.mvop(s, c, x)
    assert O.get_threads() == 1
    for name in ("i", "j", "phi", "nrm", "tau_i", "tau_j", "st"):
        assert np.array_equal(getattr(ct, name), getattr(c, name)), name
    assert (ct.n_parallel, ct.n_zero) == (c.n_parallel, c.n_zero)
    assert np.array_equal(yt, y1)


def test_threaded_bbpgd_reaches_the_serial_point(system):
    s, c, u, q = system
    g1, gg1, st1 = O.bbpgd(s, c, q, tol=1e-10)
    with O.threads(4):
        g4, gg4, st4 = O.bbpgd(s, c, q, tol=1e-10)
    assert st1.status == 0 and st4.status == 0
    assert st4.residual < 1e-10
    assert np.linalg.norm(g4 - g1) <= 1e-8 * np.linalg.norm(g1)
    # one thread again: the serial iterates, bit for bit
    g1b, _, st1b = O.bbpgd(s, c, q, tol=1e-10)
    assert np.array_equal(g1b, g1) and st1b.iters == st1.iters


def test_threaded_walls_and_tiny_systems():
    """Walls (each particle's wall contacts come first) and fewer particles
    than threads give the serial lists too."""
    rng = np.random.default_rng(9)
    n = 5
    pos = rng.uniform(0.3, 2.7, (n, 3))
    rad = np.full(n, 0.5)
    s = W.Suspension("tiny", pos, np.tile([0.0, 0.0, 1.0], (n, 1)), rad, np.zeros(n),
                     W.sphere_mobility(rad), rng.standard_normal((n, 6)), np.full(3, 3.0), 0.1,
                     1e-3, 1e-6, periodic=0)
    s.walls = 63
    c1 = O.find_contacts(s)
    with O.threads(8):
        c8 = O.find_contacts(s)
    assert c1.nc > 0 and np.any(c1.j < 0)
    assert np.array_equal(c1.keys(), c8.keys()) and np.array_equal(c1.phi, c8.phi)
