"""Pins of the oracle's Eq. (3D) (gamma_3d: the direct sum over sorted
l-triples with h^2 from the Wigner symbol) and of the Gosper form of the
symbol that Eq. (3D) prints."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1503_08809_amd import synth


def _inp(kind, n1, lmax, nr=5):
    return synth.make_inputs(synth.small_config(lmax=lmax, nk=60, nr=nr, n1=n1, kind=kind, seed_index=95))


def _nw(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("kind,n1,lmax", [("ordered", 3, 20), ("symmetric", 4, 24), ("symmetric", 3, 64)])
def test_3d_equals_separable(kind, n1, lmax):
    """The exact-3j direct sum equals the separable mu-quadrature form
    (Eq. (2D), exact Gauss-Legendre rule): two routes to the same Gamma',
    one with no Legendre polynomials, one with no Wigner symbols."""
    inp = _inp(kind, n1, lmax)
    assert _nw(O.gamma_3d(inp), O.gamma_full(inp)) <= 1e-12


def test_3d_equals_ordered_brute_force():
    """Ordered lists: the sum over sorted triples and their orderings equals
    the plain sum over the whole cube."""
    inp = _inp("ordered", 3, 18)
    assert _nw(O.gamma_3d(inp), O.brute_force_gamma_ordered(inp)) <= 1e-13


def test_gosper_symbol_error():
    """For l >= 2 the Gosper form is off by up to ~2.3 % where a triangle is
    nearly degenerate (some L_i small) and converges where every L_i is
    large."""
    worst = 0.0
    for l1 in range(2, 41):
        for l2 in range(l1, 41):
            for l3 in range(l2 + l1 % 2, l1 + l2 + 1, 2):
                e = O.threej000_sq(l1, l2, l3)
                worst = max(worst, abs(O.threej000_sq_gosper(l1, l2, l3) / e - 1.0))
    assert 0.015 < worst < 0.025, worst
    assert O.threej000_sq_gosper(2, 3, 4) == 0.0 and O.threej000_sq_gosper(1, 1, 3) == 0.0
    for t, bar in [((100, 100, 100), 2e-5), ((500, 700, 1000), 2e-6)]:
        assert abs(O.threej000_sq_gosper(*t) / O.threej000_sq(*t) - 1.0) < bar


def test_gosper_gamma_close_to_exact():
    """With the Gosper symbol Gamma' moves by the approximation's weighted
    error (about 1e-3 here), not by a dropped factor."""
    inp = _inp("symmetric", 3, 40)
    d = _nw(O.gamma_3d(inp, "gosper"), O.gamma_3d(inp))
    assert 1e-4 < d < 5e-3, d
