"""Pins of the test oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: every check is against a
closed form, an exact rational value, an independent library routine
(mpmath, scipy, numpy, sympy), a brute-force direct sum of the paper's
non-separable definition, or an invariant of the method.
"""
import math
import dataclasses
import os

import numpy as np
import pytest

from paper_1503_08809_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------- Gauss-Legendre
@pytest.mark.parametrize("n", [1, 2, 5, 97, 752])
def test_gl_moments_and_symmetry(oracle, n):
    x, w = oracle.gauss_legendre(n)
    assert np.all(np.diff(x) > 0)
    assert abs(w.sum() - 2.0) < 1e-14
    np.testing.assert_array_equal(x, -x[::-1])
    np.testing.assert_allclose(w, w[::-1], rtol=1e-14)
    # exact for monomials of degree <= 2n-1: Int x^(2j) = 2/(2j+1)
    for j in range(0, min(n, 40)):
        assert abs(np.sum(w * x ** (2 * j)) - 2.0 / (2 * j + 1)) < 1e-13


@pytest.mark.parametrize("n", [3, 50, 200])
def test_gl_vs_numpy(oracle, n):
    x, w = oracle.gauss_legendre(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    np.testing.assert_allclose(x, xr, atol=1e-14)
    # numpy's companion-matrix weights carry ~1e-11 relative error at n = 200
    # (the paper's Sec. 2.2 remark on library GL accuracy); mpmath below is the tight pin
    np.testing.assert_allclose(w, wr, rtol=1e-10, atol=1e-16)


def test_gl_vs_mpmath_roots(oracle):
    mpmath = pytest.importorskip("mpmath")
    n = 97
    x, w = oracle.gauss_legendre(n)
    mpmath.mp.dps = 40
    for i in [0, 7, 30, 48, 60, 96]:
        root = mpmath.findroot(lambda t: mpmath.legendre(n, t), x[i])
        dp = mpmath.diff(lambda t: mpmath.legendre(n, t), root)
        wt = 2 / ((1 - root ** 2) * dp ** 2)
        assert abs(float(root) - x[i]) < 1e-15
        assert abs(float(wt) - w[i]) < 1e-15 * float(wt) * 10


# --------------------------------------------------------------- Legendre
def test_legendre_endpoints_parity_scipy(oracle):
    from scipy.special import eval_legendre
    lmax = 300
    mu = np.array([-1.0, -0.7, -0.1, 0.0, 0.3, 0.999, 1.0])
    P = oracle.legendre_table(lmax, mu)
    np.testing.assert_allclose(P[-1], 1.0, rtol=1e-13)
    np.testing.assert_allclose(P[0], (-1.0) ** np.arange(lmax + 1), rtol=1e-13)
    ref = eval_legendre(np.arange(lmax + 1)[None, :], mu[:, None])
    np.testing.assert_allclose(P, ref, atol=1e-12)
    Pm = oracle.legendre_table(lmax, -mu)
    np.testing.assert_allclose(Pm, P * (-1.0) ** np.arange(lmax + 1)[None, :], atol=1e-14)


def test_legendre_vs_mpmath_high_l(oracle):
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 30
    mu = np.array([0.01234, 0.5, 0.95])
    P = oracle.legendre_table(4000, mu)
    for j, m in enumerate(mu):
        for l in [1000, 2500, 4000]:
            ref = float(mpmath.legendre(l, mpmath.mpf(m)))
            assert abs(P[j, l] - ref) < 1e-12


def test_legendre_discrete_orthogonality(oracle):
    n = 61
    x, w = oracle.gauss_legendre(n)
    P = oracle.legendre_table(60, x)          # l + l' <= 120 <= 2n - 1
    G = (P * w[:, None]).T @ P
    np.testing.assert_allclose(G, np.diag(2.0 / (2 * np.arange(61) + 1)), atol=1e-13)


# --------------------------------------------------------------- Wigner 3j / Gaunt
def _golden_3j():
    rows = []
    with open(os.path.join(GOLDEN, "threej000_sq.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                l1, l2, l3, num, den = map(int, line.split())
                rows.append((l1, l2, l3, num / den))
    return rows


def test_threej_golden_and_sympy(oracle):
    from sympy.physics.wigner import wigner_3j
    for l1, l2, l3, val in _golden_3j():
        assert oracle.threej000_sq(l1, l2, l3) == pytest.approx(val, rel=1e-15, abs=0)
        assert float(wigner_3j(l1, l2, l3, 0, 0, 0) ** 2) == pytest.approx(val, rel=1e-14, abs=0)
    rng = np.random.default_rng(5)
    for _ in range(40):
        l1, l2, l3 = (int(v) for v in rng.integers(0, 40, 3))
        ref = float(wigner_3j(l1, l2, l3, 0, 0, 0) ** 2)
        assert oracle.threej000_sq(l1, l2, l3) == pytest.approx(ref, rel=1e-13, abs=0)


def test_gaunt_identity_small(oracle):
    """Sec. 2.2: Int P_l1 P_l2 P_l3 dmu = 2 (l1 l2 l3; 000)^2, exactly by
    Gauss-Legendre when 2 N - 1 >= l1 + l2 + l3."""
    lmax = 64
    x, w = oracle.gauss_legendre(97)
    P = oracle.legendre_table(lmax, x)
    rng = np.random.default_rng(7)
    trip = rng.integers(2, lmax + 1, size=(400, 3))
    trip = np.vstack([trip, [[2, 2, 2], [64, 64, 64], [2, 30, 31], [10, 20, 40], [64, 64, 2]]])
    for l1, l2, l3 in trip:
        lhs = np.sum(w * P[:, l1] * P[:, l2] * P[:, l3])
        rhs = 2.0 * oracle.threej000_sq(int(l1), int(l2), int(l3))
        assert abs(lhs - rhs) < 2e-15, (l1, l2, l3, lhs, rhs)


def test_gaunt_identity_large_l(oracle):
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 40
    lmax = 2500
    n = (3 * lmax + 2) // 2 + 1
    x, w = oracle.gauss_legendre(n)
    P = oracle.legendre_table(lmax, x)

    def tj2(l1, l2, l3):
        L = l1 + l2 + l3
        if L % 2 or l3 > l1 + l2 or l1 > l2 + l3 or l2 > l1 + l3:
            return 0.0
        g = L // 2
        f = mpmath.factorial
        return float(f(L - 2 * l1) * f(L - 2 * l2) * f(L - 2 * l3) / f(L + 1)
                     * (f(g) / (f(g - l1) * f(g - l2) * f(g - l3))) ** 2)

    for l1, l2, l3 in [(2500, 2500, 2), (1000, 1500, 2498), (2000, 2100, 2200), (7, 2493, 2500),
                       (2500, 2499, 2499), (1200, 1300, 2501 - 1)]:
        lhs = np.sum(w * P[:, l1] * P[:, l2] * P[:, l3])
        rhs = 2.0 * tj2(l1, l2, l3)
        # P_l from the upward recurrence carries ~l * eps relative rounding
        assert abs(lhs - rhs) < 1e-11 * abs(rhs) + 1e-15, (l1, l2, l3, lhs, rhs)


# --------------------------------------------------------------- spherical Bessel
def test_sph_bessel_closed_forms(oracle):
    x = np.array([1e-3, 0.135, 0.9, 1.0, 2.5, 7.0, 31.4, 100.0, 725.0])
    J = oracle.sph_bessel_table(2, x)
    j0 = np.sin(x) / x
    j1 = np.sin(x) / x ** 2 - np.cos(x) / x
    j2 = (3 / x ** 2 - 1) * np.sin(x) / x - 3 * np.cos(x) / x ** 2
    np.testing.assert_allclose(J[:, 0], j0, rtol=1e-14, atol=1e-17)
    np.testing.assert_allclose(J[:, 1][2:], j1[2:], rtol=1e-12, atol=1e-16)
    np.testing.assert_allclose(J[:, 2][3:], j2[3:], rtol=1e-11, atol=1e-16)
    # small-x series j_l ~ x^l / (2l+1)!!
    Js = oracle.sph_bessel_table(6, np.array([1e-3]))
    for l in range(7):
        dfact = np.prod(np.arange(1, 2 * l + 2, 2, dtype=np.float64))
        assert Js[0, l] == pytest.approx(1e-3 ** l / dfact, rel=1e-6)


def test_sph_bessel_sum_rule(oracle):
    """Sum_l (2l+1) j_l(x)^2 = 1 (all terms kept: lmax >> x)."""
    x = np.array([0.2, 3.0, 50.0, 400.0, 1500.0])
    J = oracle.sph_bessel_table(2200, x)
    s = (J ** 2 * (2 * np.arange(2201) + 1)[None, :]).sum(axis=1)
    np.testing.assert_allclose(s, 1.0, rtol=1e-12)


def test_sph_bessel_vs_mpmath(oracle):
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 50
    cases = []
    for l, x in [(2, 0.135), (40, 3.0), (64, 700.0), (500, 100.0), (500, 499.0), (500, 510.0),
                 (500, 1400.0), (2500, 2400.0), (2500, 2500.0), (2500, 2560.0), (2500, 4500.0),
                 (4000, 3950.0), (4000, 4030.0), (3000, 60.0), (1000, 980.0), (100, 101.5)]:
        cases.append((l, x))
    xs = np.array(sorted({x for _, x in cases}))
    J = oracle.sph_bessel_table(4000, xs)
    for l, x in cases:
        i = int(np.searchsorted(xs, x))
        ref = mpmath.besselj(l + 0.5, x) * mpmath.sqrt(mpmath.pi / (2 * x))
        peak = 1.0 / x if x > 1 else 1.0
        assert abs(J[i, l] - float(ref)) < 1e-13 * peak, (l, x, J[i, l], float(ref))


def test_sph_bessel_vs_scipy_grid(oracle):
    from scipy.special import spherical_jn
    x = np.geomspace(0.1, 3000, 200)
    J = oracle.sph_bessel_table(1500, x)
    ref = spherical_jn(np.arange(1501)[None, :], x[:, None])
    peak = np.maximum(np.abs(ref).max(axis=1), 1e-300)
    err = (np.abs(J - ref).max(axis=1)) / peak
    assert err.max() < 1e-11


# --------------------------------------------------------------- beta
def test_beta_single_k_node(oracle):
    """q_p Delta_l nonzero at one k node: beta = (2/pi) wk k^2 q Delta j_l(k r)."""
    from scipy.special import spherical_jn
    cfg = synth.small_config(lmax=30, nk=50, nr=6, n1=3)
    inp = synth.make_inputs(cfg)
    i0 = 31
    inp.delta[:, :] = 0.0
    inp.delta[:, i0] = np.linspace(0.5, 1.5, cfg.L)
    b = oracle.beta(inp)
    ells = inp.ells
    for p in range(3):
        ref = (2 / np.pi * inp.wk[i0] * inp.k[i0] ** 2 * inp.qk[p, i0]
               * inp.delta[:, i0][:, None] * spherical_jn(ells[:, None], inp.k[i0] * inp.r[None, :]))
        np.testing.assert_allclose(b[p], ref, rtol=1e-11, atol=1e-14 * np.abs(ref).max())


def test_beta_linear(oracle):
    cfg = synth.small_config(lmax=25, nk=40, nr=5, n1=2)
    inp = synth.make_inputs(cfg)
    b1 = oracle.beta(inp)
    inp2 = synth.make_inputs(cfg)
    inp2.delta[:] = 3.0 * inp.delta
    b2 = oracle.beta(inp2)
    np.testing.assert_allclose(b2, 3.0 * b1, rtol=1e-13, atol=1e-14 * np.abs(b1).max())


# --------------------------------------------------------------- S
def test_S_single_l_basis(oracle):
    """qbar_a = delta_{l,l0}: S_ap(r,mu) = w_l0 P_l0(mu) beta_p(l0, r)."""
    from scipy.special import eval_legendre
    cfg = synth.small_config(lmax=30, nk=40, nr=5, n1=2)
    inp = synth.make_inputs(cfg)
    l0 = 17
    inp.ql[:] = 0.0
    inp.ql[0, l0 - cfg.lmin] = 1.0
    inp.ql[1, l0 - cfg.lmin] = -2.0
    mu, wmu = oracle.gauss_legendre(cfg.nmu)
    b = oracle.beta(inp)
    S = oracle.S_pairs(inp, mu, b, [(0, 0), (1, 1)])
    wl = (2 * l0 + 1) ** (5.0 / 6.0) / np.sqrt(inp.cl[l0 - cfg.lmin])
    ref0 = wl * eval_legendre(l0, mu)[None, :] * b[0, l0 - cfg.lmin][:, None]
    ref1 = -2.0 * wl * eval_legendre(l0, mu)[None, :] * b[1, l0 - cfg.lmin][:, None]
    np.testing.assert_allclose(S[0], ref0, rtol=1e-12, atol=1e-14 * np.abs(ref0).max())
    np.testing.assert_allclose(S[1], ref1, rtol=1e-12, atol=1e-14 * np.abs(ref1).max())


def test_S_mu_parity(oracle):
    """Even-l (odd-l) bases give S even (odd) in mu."""
    cfg = synth.small_config(lmax=30, nk=40, nr=4, n1=2)
    inp = synth.make_inputs(cfg)
    ells = inp.ells
    inp.ql[0] = np.where(ells % 2 == 0, 1.0 + 0.01 * ells, 0.0)
    inp.ql[1] = np.where(ells % 2 == 1, 1.0 - 0.01 * ells, 0.0)
    mu, _ = oracle.gauss_legendre(cfg.nmu)
    b = oracle.beta(inp)
    S = oracle.S_pairs(inp, mu, b, [(0, 0), (1, 0)])
    sc = np.abs(S).max()
    np.testing.assert_allclose(S[0][:, ::-1], S[0], atol=1e-13 * sc)
    np.testing.assert_allclose(S[1][:, ::-1], -S[1], atol=1e-13 * sc)


# --------------------------------------------------------------- Gamma
def test_gamma_vs_bruteforce_lmax64(oracle):
    """Config lmax=64: the separable mu-quadrature form equals the paper's
    non-separable inner product with exact Wigner symbols (Eq. (3D) with
    exact h^2) to 1e-12 normwise."""
    inp = synth.make_inputs(synth.workload("lmax64_ordered_n8"))
    g = oracle.gamma_full(inp)
    bf = oracle.brute_force_gamma_ordered(inp)
    err = np.abs(g - bf).max() / np.abs(bf).max()
    assert err < 1e-12, err


def test_gamma_vs_bruteforce_unequal_sizes(oracle):
    cfg = synth.small_config(lmax=23, nk=70, nr=7, n1=4, kind="ordered", v_power=0.0)
    inp = synth.make_inputs(cfg)
    g = oracle.gamma_full(inp)
    bf = oracle.brute_force_gamma_ordered(inp)
    assert np.abs(g - bf).max() / np.abs(bf).max() < 1e-12


def test_gamma_bruteforce_catches_too_few_nodes(oracle):
    """With fewer mu nodes than exactness needs, the separable form departs
    from the exact-3j sum (the pin has teeth)."""
    cfg = synth.small_config(lmax=23, nk=70, nr=7, n1=3, kind="ordered")
    inp = synth.make_inputs(cfg)
    mu, w = oracle.gauss_legendre(20)          # 2*20-1 = 39 < 3*23
    g = oracle.gamma_full(inp, mu, w)
    bf = oracle.brute_force_gamma_ordered(inp)
    assert np.abs(g - bf).max() / np.abs(bf).max() > 1e-6


def _ordered_to_sym(n1, G_ord):
    """(1/6) Sum_sigma Gamma_ord[a, sigma p] over sorted triples."""
    import itertools
    st = synth.sym_triples(n1)
    out = np.zeros((st.shape[0], st.shape[0]))
    idx = lambda t: t[0] * n1 * n1 + t[1] * n1 + t[2]
    for i, a in enumerate(st):
        for j, p in enumerate(st):
            out[i, j] = sum(G_ord[idx(a), idx(tuple(p[list(s)]))]
                            for s in itertools.permutations(range(3))) / 6.0
    return out


def test_symmetric_equals_symmetrised_ordered(oracle):
    """Eq. (2D)'s permanent with 1/(48 pi) equals (1/6) Sum over the six
    p-permutations of the ordered Gamma with 1/(8 pi) (Appendix: Q_n and
    Q-tilde_n each carry 1/6 over six terms)."""
    cfg_o = synth.small_config(lmax=20, nk=50, nr=5, n1=4, kind="ordered")
    cfg_s = synth.small_config(lmax=20, nk=50, nr=5, n1=4, kind="symmetric")
    go = oracle.gamma_full(synth.make_inputs(cfg_o))
    gs = oracle.gamma_full(synth.make_inputs(cfg_s))
    ref = _ordered_to_sym(4, go)
    assert np.abs(gs - ref).max() / np.abs(ref).max() < 1e-13


def test_ordered_simultaneous_permutation_symmetry(oracle):
    import itertools
    n1 = 4
    cfg = synth.small_config(lmax=20, nk=50, nr=5, n1=n1, kind="ordered")
    g = oracle.gamma_full(synth.make_inputs(cfg))
    tri = synth.ordered_triples(n1)
    idx = {tuple(t): i for i, t in enumerate(tri)}
    sc = np.abs(g).max()
    for s in itertools.permutations(range(3)):
        perm = np.array([idx[tuple(t[list(s)])] for t in tri])
        np.testing.assert_allclose(g[np.ix_(perm, perm)], g, atol=1e-14 * sc)


def test_gamma_scalings(oracle):
    """C -> lam C gives lam^(-3/2); Delta -> lam Delta gives lam^3;
    qbar_a -> lam qbar_a scales a row by lam^(multiplicity of a)."""
    cfg = synth.small_config(lmax=18, nk=40, nr=4, n1=3, kind="symmetric")
    base = synth.make_inputs(cfg)
    g0 = oracle.gamma_full(base)
    sc = np.abs(g0).max()
    i1 = synth.make_inputs(cfg)
    i1.cl[:] = 4.0 * base.cl
    np.testing.assert_allclose(oracle.gamma_full(i1), g0 / 8.0, atol=1e-13 * sc)
    i2 = synth.make_inputs(cfg)
    i2.delta[:] = 2.0 * base.delta
    np.testing.assert_allclose(oracle.gamma_full(i2), 8.0 * g0, atol=1e-12 * sc)
    i3 = synth.make_inputs(cfg)
    i3.ql[1] = 3.0 * base.ql[1]
    mult = (base.tri_a == 1).sum(axis=1)
    np.testing.assert_allclose(oracle.gamma_full(i3), g0 * (3.0 ** mult)[:, None],
                               atol=1e-12 * sc * 27)


def test_gamma_single_l_closed_form(oracle):
    """Delta-in-l late-time bases at l1, l2, l3 (ordered): Gamma =
    (1/8pi) w1 w2 w3 * 2 (3j)^2 * Sum_r wr r^2 beta_p1 beta_p2 beta_p3."""
    cfg = synth.small_config(lmax=30, nk=60, nr=6, n1=3, kind="ordered")
    inp = synth.make_inputs(cfg)
    ls = [8, 11, 13]          # sum even, triangle holds
    inp.ql[:] = 0.0
    for a, l in enumerate(ls):
        inp.ql[a, l - cfg.lmin] = 1.0
    g = oracle.gamma_full(inp)
    b = oracle.beta(inp)
    w = oracle.weights_l(inp)
    tri = inp.tri_a
    n1 = 3
    row = 0 * 9 + 1 * 3 + 2        # a = (0, 1, 2)
    tj = oracle.threej000_sq(*ls)
    wr2 = inp.wr * inp.r ** 2
    for col, p in enumerate(inp.tri_p):
        ref = (1 / (8 * np.pi) * w[ls[0] - 2] * w[ls[1] - 2] * w[ls[2] - 2] * 2 * tj
               * np.sum(wr2 * b[p[0], ls[0] - 2] * b[p[1], ls[1] - 2] * b[p[2], ls[2] - 2]))
        assert g[row, col] == pytest.approx(ref, rel=1e-11, abs=1e-13 * abs(g).max())
    # a row whose l's break parity is exactly zero
    row_bad = 0 * 9 + 0 * 3 + 1        # (l1, l1, l2) = (8, 8, 11): odd sum
    assert np.abs(g[row_bad]).max() < 1e-13 * np.abs(g).max()


def test_mode_list_example_order():
    """The symmetric triple order reproduces the Appendix's example list."""
    rows = np.loadtxt(os.path.join(GOLDEN, "mode_list_example.txt"), dtype=int)
    st = synth.sym_triples(3)
    for n, i, j, k in rows:
        assert tuple(st[n]) == (i, j, k)
    assert st.shape[0] == 10
    assert synth.sym_triples(30).shape[0] == 4960
    assert synth.sym_triples(20).shape[0] == 1540
    assert synth.sym_triples(40).shape[0] == 11480


def test_sampled_entries_match_full(oracle):
    cfg = synth.small_config(lmax=20, nk=40, nr=5, n1=4, kind="symmetric")
    inp = synth.make_inputs(cfg)
    g = oracle.gamma_full(inp)
    rows = [0, 3, 7, 19, 19]
    cols = [5, 0, 19, 2, 11]
    ge = oracle.gamma_entries(inp, rows, cols)
    np.testing.assert_allclose(ge, g[rows, cols], rtol=1e-14, atol=0)


def test_inputs_deterministic():
    cfg = synth.small_config()
    a = synth.make_inputs(cfg)
    b = synth.make_inputs(cfg)
    for f in ("k", "wk", "r", "wr", "cl", "delta", "qk", "ql"):
        np.testing.assert_array_equal(getattr(a, f), getattr(b, f))
    assert np.all(np.isfinite(a.delta))
    assert abs(a.wk.sum() - (a.k[-1] - a.k[0])) < 1e-14


def test_stored_rows_come_from_the_oracle(oracle):
    """The stored oracle rows of the lmax = 1000 workload (GPU parity at large
    sizes reads them) agree with the oracle as it stands: three entries,
    values and magnitude scales, recomputed (the whole file takes the oracle
    too long)."""
    import stored_rows
    cfg = synth.workload("lmax1000_symmetric_n20")
    rows, cols, ref, scale = stored_rows.load(cfg.name)
    assert np.unique(rows).size == 6 and rows.size == 6 * 1540
    pick = [0, rows.size // 2 + 17, rows.size - 1]
    inp = synth.make_inputs(cfg)
    v, sc = oracle.gamma_entries(inp, rows[pick], cols[pick], return_scale=True)
    np.testing.assert_allclose(v, ref[pick], rtol=1e-15, atol=0)
    np.testing.assert_allclose(sc, scale[pick], rtol=1e-15, atol=0)


def test_entry_scale_bounds_the_entry(oracle):
    """The magnitude scale is the same sum over absolute values: it bounds
    |Gamma| and equals it when every product term has one sign (ordered
    Gamma with S > 0), and it is linear in each S row's magnitude."""
    inp = synth.make_inputs(synth.small_config(lmax=24, nk=60, nr=5, n1=4, kind="symmetric"))
    mu, wmu = oracle.gauss_legendre(inp.cfg.nmu)
    S, _ = oracle.full_S(inp, mu)
    S = S.reshape(-1, inp.cfg.nr, mu.size)
    n = 40
    rng = np.random.default_rng(5)
    sidx = rng.integers(0, S.shape[0], size=(n, 9)).astype(np.int32)
    g, sc = oracle.gamma_from_S(inp, wmu, S, sidx, return_scale=True)
    assert np.all(sc >= np.abs(g)) and np.all(sc > 0)
    # all terms positive: the scale is the value itself
    cfg_o = dataclasses.replace(inp.cfg, kind="ordered")
    inp_o = dataclasses.replace(inp, cfg=cfg_o)
    g2, sc2 = oracle.gamma_from_S(inp_o, wmu, np.abs(S), sidx, return_scale=True)
    np.testing.assert_allclose(sc2, g2, rtol=1e-14)
    # flipping the sign of S leaves the scale unchanged and negates Gamma
    g3, sc3 = oracle.gamma_from_S(inp, wmu, -S, sidx, return_scale=True)
    np.testing.assert_allclose(g3, -g, rtol=1e-14)
    np.testing.assert_allclose(sc3, sc, rtol=1e-14)


def test_stored_rows_detect_a_perturbed_S_row(oracle):
    """The elementwise check against stored rows catches a wrong S row: at
    lmax = 500 (ordered), 64 stored entries of the row a = (2, 1, 0) that use
    the pair (a = 1, p = 3) are recomputed by the oracle with that S row
    unchanged (equal to the stored values), zeroed, scaled by 1 + 1e-3
    (both fail the mixed bar) and scaled by 1 + 1e-7 (fails the FP64 bar).
    The perturbation is planted in the oracle's S, on the CPU."""
    import stored_rows
    cfg = synth.workload("lmax500_ordered_n16")
    rows, cols, ref, scale = stored_rows.load(cfg.name)
    inp = synth.make_inputs(cfg)
    r210 = 2 * 256 + 1 * 16 + 0
    sel = np.nonzero((rows == r210) & (inp.tri_p[cols][:, 1] == 3))[0][:64]
    assert sel.size == 64
    mu, wmu = oracle.gauss_legendre(cfg.nmu)
    g, S, need = oracle.gamma_entries(inp, rows[sel], cols[sel], mu, wmu, return_S=True)
    assert stored_rows.worst(g, ref[sel], scale[sel]) <= 1e-14
    # the 3x3 index blocks of these entries, as gamma_entries forms them
    ta, tp = inp.tri_a[rows[sel]], inp.tri_p[cols[sel]]
    pos = {p: i for i, p in enumerate(np.unique(tp))}
    sidx = np.array([[need[(int(ta[e, s]), pos[int(tp[e, t])])] for s in range(3) for t in range(3)]
                     for e in range(sel.size)], dtype=np.int32)
    k = need[(1, pos[3])]
    for factor, bar in ((0.0, stored_rows.MIXED_TOL), (1 + 1e-3, stored_rows.MIXED_TOL),
                        (1 + 1e-7, stored_rows.FP64_TOL)):
        Sp = S.copy()
        Sp[k] *= factor
        gp = oracle.gamma_from_S(inp, wmu, Sp, sidx)
        assert stored_rows.worst(gp, ref[sel], scale[sel]) > bar, factor


def test_stored_gradient_satisfies_euler_identity():
    """The stored oracle gradient at lmax = 1000 (GPU parity of the adjoint
    reads it): Gamma is cubic in q (beta is linear in q), so
    L = Sum (Gamma * W)^2 is homogeneous of degree 6 in q and
    <dL/dq, q> = 6 L exactly; L is the oracle's, stored with the gradient."""
    import stored_rows
    cfg = synth.workload("lmax1000_symmetric_n20")
    dq, rows, L = stored_rows.load_grad(cfg.name)
    inp = synth.make_inputs(cfg, with_delta=False)
    assert dq.shape == inp.qk.shape and len(rows) == 18 and L > 0
    e = float((dq * inp.qk).sum()) / (6.0 * L) - 1.0
    assert abs(e) <= 1e-11, e
