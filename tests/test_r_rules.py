"""r rules (Modal3D algorithmic change, Eq. (hermite)): the oracle's
interval-by-interval integrals pinned by closed forms, and the library's
host-side weights (modal_r_weights) against the oracle.  No GPU needed."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1503_08809_amd import synth


def _grid(n, seed=0):
    return np.sort(np.random.default_rng(seed).uniform(1.0, 5.0, n))


@pytest.mark.parametrize("rule", ["trapezoid", "hermite"])
def test_oracle_exact_for_linear(rule):
    """Both rules integrate a line exactly on an uneven grid.  For the
    Hermite rule this fails if the derivative terms lose their interval
    width or a basis cubic its sign."""
    r = _grid(13)
    y = 3.0 * r - 2.0
    exact = 1.5 * (r[-1] ** 2 - r[0] ** 2) - 2.0 * (r[-1] - r[0])
    assert abs(O.r_rule_integral(rule, r, y) - exact) <= 1e-13 * abs(exact)


def test_oracle_hermite_uniform_is_end_corrected_trapezium():
    """On an even grid of width h the Hermite corrections telescope: the
    rule is the trapezium plus (h / 12)(dy_0 - dy_{n-2}), dy_k = y_{k+1} - y_k."""
    r = np.linspace(2.0, 3.0, 17)
    h = r[1] - r[0]
    y = np.random.default_rng(1).standard_normal(r.size)
    dy = np.diff(y)
    want = O.r_rule_integral("trapezoid", r, y) + h / 12.0 * (dy[0] - dy[-1])
    assert abs(O.r_rule_integral("hermite", r, y) - want) <= 1e-14 * np.abs(y).sum()


@pytest.mark.parametrize("graded", [False, True])
def test_oracle_convergence_orders(graded):
    """Against the closed-form integral of sin(3r) + r^3: each halving of
    the intervals divides the trapezium's error by about 4 (second order) and
    the Hermite rule's by about 8 (third order: the chord slopes make its
    correction cancel the trapezium's leading error term)."""
    F = lambda r: -np.cos(3 * r) / 3 + r ** 4 / 4
    errs = {"trapezoid": [], "hermite": []}
    for n in (20, 40, 80, 160):
        t = np.linspace(0.0, 1.0, n)
        r = 1.0 + (0.5 * t * t + 0.5 * t if graded else t)
        y = np.sin(3 * r) + r ** 3
        for rule in errs:
            errs[rule].append(abs(O.r_rule_integral(rule, r, y) - (F(r[-1]) - F(r[0]))))
    rt = np.array(errs["trapezoid"][:-1]) / np.array(errs["trapezoid"][1:])
    rh = np.array(errs["hermite"][:-1]) / np.array(errs["hermite"][1:])
    assert np.all((rt > 3.6) & (rt < 4.6)), rt
    assert np.all(rh > 7.0), rh


@pytest.fixture(scope="module")
def mp():
    from paper_1503_08809_amd import modalproj
    return modalproj


@pytest.mark.parametrize("rule", ["trapezoid", "hermite"])
@pytest.mark.parametrize("which", ["uneven", "clustered", "two"])
def test_library_weights_vs_oracle(mp, rule, which):
    """sum_j w_j y_j with the library's weights against the oracle's
    interval integrals, for random y (and each unit vector on a short grid)."""
    if which == "uneven":
        r = _grid(40, seed=2)
    elif which == "clustered":
        r = synth.r_grid(synth.workload("lmax2500_symmetric_n30"))
    else:
        r = np.array([1.0, 1.5])
    w = mp.r_weights(rule, r)
    rng = np.random.default_rng(3)
    for _ in range(3):
        y = rng.standard_normal(r.size)
        ref = O.r_rule_integral(rule, r, y)
        assert abs(w @ y - ref) <= 1e-13 * (np.abs(w) @ np.abs(y))
    if r.size <= 40:
        for j in range(r.size):
            e = np.zeros(r.size)
            e[j] = 1.0
            assert abs(w[j] - O.r_rule_integral(rule, r, e)) <= 1e-13 * (r[-1] - r[0])


def test_library_weights_rejects(mp):
    with pytest.raises(mp.ModalError) as e:
        mp.r_weights("hermite", np.array([1.0]))
    assert e.value.status == 2
    with pytest.raises(mp.ModalError) as e:
        mp.r_weights("trapezoid", np.array([1.0, 3.0, 2.0]))
    assert e.value.status == 2 and "ascending" in str(e.value)
    with pytest.raises(mp.ModalError) as e:
        mp.r_weights("hermite", np.array([1.0, np.nan, 2.0]))
    assert e.value.status == 5
    with pytest.raises(mp.ModalError) as e:
        mp.r_weights(7, np.array([1.0, 2.0]))
    assert e.value.status == 1
