"""Parity of the HIP path with the oracle, stage by stage and end to end.

Every case feeds the same seeded inputs to the HIP library (through the C
ABI) and to the oracle, and compares element by element.  Tolerances:

* tables and single stages (j_l, P_l, Gauss-Legendre, beta, S): FP64
  rounding of the recurrences and of sums of ~10^3-10^4 terms, written per
  test (1e-13 .. 1e-11 relative to the largest value);
* Gamma from the FP64 path: normwise error max|G - G_ref| / max|G_ref| at
  most 1e-6 (the FP64 bar), and elementwise within 1e-9 of max|G_ref|;
* Gamma from the mixed path: normwise at most 1e-4 (the mixed bar);
* at the large workloads (lmax = 500, 1000, 2500, 4000), every entry of six
  whole stored oracle rows (tests/golden, written by the oracle alone)
  elementwise, |G - ref| <= tol * scale with the oracle's per-entry magnitude
  scale: tol = 1e-9 for the FP64 path, 1e-4 for the mixed path.
"""
import numpy as np
import pytest

import stored_rows
from paper_1503_08809_amd import synth

pytestmark = pytest.mark.gpu

FP64_BAR = 1e-6
MIXED_BAR = 1e-4


@pytest.fixture(scope="module")
def mp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1503_08809_amd import modalproj
    return modalproj


@pytest.fixture(scope="module")
def ctx(mp):
    c = mp.Context(0)
    yield c
    c.close()


def _np(t):
    return t.detach().cpu().numpy()


def normwise(a, ref):
    return float(np.abs(a - ref).max() / np.abs(ref).max())


# ------------------------------------------------------------------ step a
@pytest.mark.parametrize("n", [1, 2, 5, 97, 752, 3752, 6002])
def test_gauss_legendre(mp, ctx, oracle, n):
    x, w = (_np(v) for v in mp.gauss_legendre(ctx, n))
    xr, wr = oracle.gauss_legendre(n)
    # both sides refine the roots beyond FP64 and round once
    assert np.abs(x - xr).max() <= 2.3e-16
    # The oracle carries its nodes in 64-bit long double; near +-1 its weight
    # 2 / ((1 - x^2) P_n'^2) inherits the relative error ~1e-19 / (1 - x^2)
    # of 1 - x^2 (2.5e-12 at n = 6002).  The HIP rule refines in
    # double-double; the mpmath test below pins it to 1e-15 at the ends.
    rel = np.abs(w - wr) / wr
    one_minus = (1 - np.abs(xr)) * (1 + np.abs(xr))
    assert np.all(rel <= 1e-15 + 2e-19 / one_minus)
    np.testing.assert_array_equal(x, -x[::-1])


@pytest.mark.parametrize("n", [97, 752, 3752, 6002])
def test_gauss_legendre_host_equals_device(mp, ctx, n):
    """The host rule (modal_gauss_legendre without a context) and the device
    kernel run the same double-double refinement from slightly different
    starting guesses (host and device cos): the same values to within one
    unit in the last place (in practice the same bits)."""
    x, w = (_np(v) for v in mp.gauss_legendre(ctx, n))
    xh, wh = np.empty(n), np.empty(n)
    assert mp.lib().modal_gauss_legendre(None, n, xh.ctypes.data, wh.ctypes.data) == 0
    same = int((xh == x).sum() + (wh == w).sum())
    print(f"GL n={n}: host and device rules agree bit for bit on {same} of {2 * n} values")
    assert np.all(np.abs(xh - x) <= np.spacing(np.abs(x)))
    assert np.all(np.abs(wh - w) <= np.spacing(w))


def test_gauss_legendre_end_nodes_vs_mpmath(mp, ctx):
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 40
    n = 752
    x, w = (_np(v) for v in mp.gauss_legendre(ctx, n))
    def dP(t):
        return n * (t * mpmath.legendre(n, t) - mpmath.legendre(n - 1, t)) / (t * t - 1)

    for i in [n - 1, n - 2, n - 5, n // 2 + 3]:
        root = mpmath.mpf(x[i])
        for _ in range(4):                       # Newton at 40 digits
            root -= mpmath.legendre(n, root) / dP(root)
        wt = 2 / ((1 - root ** 2) * dP(root) ** 2)
        assert abs(float(root) - x[i]) <= 1.2e-16
        assert abs(float(wt) - w[i]) <= 2e-16 * float(wt)


def test_legendre_table(mp, ctx, oracle):
    mu, _ = oracle.gauss_legendre(97)
    mu = np.concatenate([mu, [-1.0, 1.0, 0.0, 0.3333]])
    P = _np(mp.legendre_table(ctx, 300, mu))
    ref = oracle.legendre_table(300, mu).T
    assert P.shape == ref.shape
    assert np.abs(P - ref).max() <= 1e-13


def test_legendre_table_high_l(mp, ctx, oracle):
    mu, _ = oracle.gauss_legendre(3752)
    P = _np(mp.legendre_table(ctx, 2500, mu))
    ref = oracle.legendre_table(2500, mu).T
    # the upward recurrence carries ~l eps of rounding on each side (different
    # contraction of the products): 5e-12 at l = 2500
    assert np.abs(P - ref).max() <= 5e-12


def test_legendre_table_lmax4000(mp, ctx, oracle):
    """l up to 4000 on the 6002 Gauss-Legendre nodes of the lmax = 4000
    workload.  The oracle's own table is within 6.5e-12 of a long-double
    evaluation of the same recurrence there (checked on the CPU); the two
    sides round independently, so they may differ by twice that."""
    mu, _ = oracle.gauss_legendre(6002)
    P = _np(mp.legendre_table(ctx, 4000, mu))
    ref = oracle.legendre_table(4000, mu).T
    assert P.shape == ref.shape
    err = np.abs(P - ref).max()
    print(f"P_l, l <= 4000, 6002 nodes: max |P - P_ref| = {err:.2e}")
    assert err <= 1.5e-11


def test_sph_bessel_table(mp, ctx, oracle):
    x = np.concatenate([[0.0, 1e-25, 1e-6, 1e-3, 0.135, 0.5, 1.0, 2.0],
                        np.geomspace(3.0, 4500.0, 300), [2499.5, 2500.0, 2500.5]])
    lmax = 2500
    J = _np(mp.sph_bessel_table(ctx, lmax, x))
    ref = oracle.sph_bessel_table(lmax, x).T
    peak = np.maximum(np.abs(ref).max(axis=0), 1e-300)
    err = (np.abs(J - ref).max(axis=0)) / peak
    assert err.max() <= 1e-11, (x[err.argmax()], err.max())


def test_sph_bessel_table_lmax4000(mp, ctx, oracle):
    """j_l for l <= 4000 over the x = k r range of the lmax = 4000 workload
    (k <= 0.3, r up to about 14900: x up to about 4.5e3), with points at the
    turning point x ~ l for the highest l."""
    x = np.concatenate([[0.0, 1e-6, 0.5, 2.0], np.geomspace(3.0, 4500.0, 400),
                        [2999.5, 3500.0, 3999.0, 3999.5, 4000.0, 4000.5, 4001.0, 4040.0, 4470.0]])
    lmax = 4000
    J = _np(mp.sph_bessel_table(ctx, lmax, x))
    ref = oracle.sph_bessel_table(lmax, x).T
    peak = np.maximum(np.abs(ref).max(axis=0), 1e-300)
    err = (np.abs(J - ref).max(axis=0)) / peak
    print(f"j_l, l <= 4000, x <= 4500: max error relative to the peak over l {err.max():.2e}")
    assert err.max() <= 1e-11, (x[err.argmax()], err.max())


def test_sph_bessel_ragged_count(mp, ctx, oracle):
    x = np.linspace(0.0, 70.0, 129)[1:]             # 128 + ragged handled by the grid
    J = _np(mp.sph_bessel_table(ctx, 90, x[:77]))
    ref = oracle.sph_bessel_table(90, x[:77]).T
    assert np.abs(J - ref).max() <= 1e-13


# ------------------------------------------------------------------ step b, c
def _small(kind="ordered", **kw):
    base = dict(lmax=40, nk=150, nr=21, n1=5, kind=kind)
    base.update(kw)
    return synth.make_inputs(synth.small_config(**base))


def test_beta(mp, ctx, oracle):
    inp = _small()
    pr = mp.projection_from_inputs(ctx, inp)
    b = _np(pr.beta())
    ref = oracle.beta(inp)
    assert normwise(b, ref) <= 1e-12


def test_beta_single_chunk_edges(mp, ctx, oracle):
    inp = _small(lmax=12, nk=33, nr=3, n1=1)
    pr = mp.projection_from_inputs(ctx, inp)
    assert normwise(_np(pr.beta()), oracle.beta(inp)) <= 1e-12


def test_S_from_oracle_beta(mp, ctx, oracle):
    inp = _small()
    mu, _ = oracle.gauss_legendre(inp.cfg.nmu)
    S_ref, bet = oracle.full_S(inp, mu)
    pr = mp.projection_from_inputs(ctx, inp)
    S = _np(pr.S(bet))
    assert normwise(S, S_ref) <= 1e-12


# ------------------------------------------------------------------ step d
@pytest.mark.parametrize("kind", ["ordered", "symmetric"])
def test_gamma_from_oracle_S(mp, ctx, oracle, kind):
    inp = _small(kind=kind)
    mu, wmu = oracle.gauss_legendre(inp.cfg.nmu)
    S_ref, bet = oracle.full_S(inp, mu)
    ref = oracle.gamma_full(inp, mu, wmu)
    pr = mp.projection_from_inputs(ctx, inp, mu=mu, wmu=wmu)
    g = _np(pr.gamma_from_S(S_ref.reshape(inp.ql.shape[0], inp.qk.shape[0], inp.cfg.nr, -1)))
    assert normwise(g, ref) <= 1e-12


@pytest.mark.parametrize("kind,n1,lmax,nr,nk", [
    ("ordered", 5, 40, 21, 150),
    ("symmetric", 5, 40, 21, 150),
    ("symmetric", 7, 33, 9, 70),      # U = 49: ragged row blocks and tiles
    ("ordered", 1, 20, 4, 40),        # U = 1
    ("symmetric", 12, 24, 5, 60),     # U = 144: two row super-blocks
])
def test_gamma_end_to_end_small(mp, ctx, oracle, kind, n1, lmax, nr, nk):
    """Normwise, and every entry against its own magnitude scale (as at the
    large workloads)."""
    inp = _small(kind=kind, n1=n1, lmax=lmax, nr=nr, nk=nk)
    pr = mp.projection_from_inputs(ctx, inp)
    g = _np(pr.gamma())
    ta, tp = g.shape
    rows, cols = np.meshgrid(np.arange(ta), np.arange(tp), indexing="ij")
    ref, scale = oracle.gamma_entries(inp, rows.ravel(), cols.ravel(), return_scale=True)
    ref, scale = ref.reshape(ta, tp), scale.reshape(ta, tp)
    assert np.all(scale > 0)
    err = normwise(g, ref)
    worst = float((np.abs(g - ref) / scale).max())
    print(f"FP64 normwise error {err:.3e}, worst |G - ref| / scale {worst:.2e} over {g.size} entries")
    assert err <= FP64_BAR
    assert np.abs(g - ref).max() <= 1e-9 * np.abs(ref).max()
    assert worst <= stored_rows.FP64_TOL


def test_gamma_lmax64_full(mp, ctx, oracle):
    """lmax = 64, 512 x 512 ordered Gamma: the whole matrix."""
    inp = synth.make_inputs(synth.workload("lmax64_ordered_n8"))
    pr = mp.projection_from_inputs(ctx, inp)
    g = _np(pr.gamma())
    ref = oracle.gamma_full(inp)
    assert g.shape == (512, 512)
    assert normwise(g, ref) <= FP64_BAR
    assert np.abs(g - ref).max() <= 1e-9 * np.abs(ref).max()


def test_gamma_lmax500_rows(mp, ctx):
    """lmax = 500, 4096 x 4096 ordered Gamma: every entry of the stored oracle
    rows, FP64 and mixed; simultaneous permutation symmetry of the whole
    FP64 matrix."""
    cfg = synth.workload("lmax500_ordered_n16")
    inp = synth.make_inputs(cfg)
    pr = mp.projection_from_inputs(ctx, inp)
    g = _np(pr.gamma())
    assert g.shape == (4096, 4096)
    assert np.all(np.isfinite(g))
    stored_rows.check(g, cfg.name, stored_rows.FP64_TOL, "lmax=500 FP64")
    gm = _np(pr.gamma("mixed"))
    stored_rows.check(gm, cfg.name, stored_rows.MIXED_TOL, "lmax=500 mixed")
    err = normwise(gm, g)
    print(f"mixed vs fp64 normwise error at lmax=500: {err:.3e}")
    assert err <= MIXED_BAR
    # simultaneous permutation of a and p leaves the ordered Gamma unchanged
    n1 = cfg.n1
    tri = inp.tri_a
    perm = (tri[:, 1] * n1 + tri[:, 2]) * n1 + tri[:, 0]
    np.testing.assert_array_equal(g[np.ix_(perm, perm)], g)


# ------------------------------------------------------------------ properties
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_deterministic(mp, ctx, prec):
    """Run to run, bit for bit: no atomics and fixed summation orders in
    every kernel, forward and adjoint (U = 289: several row blocks, tasks
    and workgroups per CU)."""
    inp = _small(kind="symmetric", n1=17, lmax=24, nr=5, nk=60)
    pr = mp.projection_from_inputs(ctx, inp)
    a = _np(pr.gamma(prec))
    b = _np(pr.gamma(prec))
    np.testing.assert_array_equal(a, b)
    g = ctx.to_dev(np.cos(np.arange(a.size, dtype=np.float64)).reshape(a.shape))
    dq1, dd1 = (_np(x) for x in pr.gamma_backward(g, prec))
    dq2, dd2 = (_np(x) for x in pr.gamma_backward(g, prec))
    np.testing.assert_array_equal(dq1, dq2)
    np.testing.assert_array_equal(dd1, dd2)


def test_host_pointers_match_device(mp, ctx):
    """The ABI accepts host arrays as well as device arrays."""
    import ctypes
    inp = _small(kind="ordered", n1=3)
    pr = mp.projection_from_inputs(ctx, inp)
    g_dev = _np(pr.gamma())
    c = inp.cfg
    keep = [np.ascontiguousarray(a) for a in (inp.k, inp.wk, inp.r, inp.wr, inp.delta, inp.cl,
                                              inp.qk, inp.ql)]
    tri = np.ascontiguousarray(inp.tri_a, dtype=np.int32)
    g = mp.ModalGrid(c.lmin, c.lmax, c.nk, keep[0].ctypes.data, keep[1].ctypes.data, c.nr,
                     keep[2].ctypes.data, keep[3].ctypes.data, c.nmu, None, None, 0)
    p = mp.ModalProblem(keep[4].ctypes.data, keep[5].ctypes.data, inp.qk.shape[0],
                        keep[6].ctypes.data, inp.ql.shape[0], keep[7].ctypes.data, c.v_power, 0,
                        tri.shape[0], tri.ctypes.data, tri.shape[0], tri.ctypes.data)
    out = np.zeros((tri.shape[0], tri.shape[0]))
    ctx.check(mp.lib().modal_gamma(ctx.handle, ctypes.byref(g), ctypes.byref(p), 0,
                                   out.ctypes.data))
    np.testing.assert_array_equal(out, g_dev)


def test_empty_outputs(mp, ctx):
    inp = _small(kind="symmetric", n1=3)
    pr = mp.projection_from_inputs(ctx, inp, tri_a=inp.tri_a[:0])
    g = pr.gamma()
    assert tuple(g.shape) == (0, inp.tri_p.shape[0])


def test_errors(mp, ctx):
    inp = _small(kind="symmetric", n1=3)
    bad_mu = mp.projection_from_inputs(ctx, inp, nmu=inp.cfg.nmu // 2)
    with pytest.raises(mp.ModalError) as e:
        bad_mu.gamma()
    assert e.value.status == 2
    cl = inp.cl.copy()
    cl[3] = 0.0
    with pytest.raises(mp.ModalError) as e:
        mp.projection_from_inputs(ctx, inp, cl=cl).gamma()
    assert e.value.status == 5
    tri = inp.tri_p.copy()
    tri[1, 2] = 3
    with pytest.raises(mp.ModalError) as e:
        mp.projection_from_inputs(ctx, inp, tri_p=tri).gamma()
    assert e.value.status == 2
    with pytest.raises(mp.ModalError) as e:
        ctx.check(mp.lib().modal_gamma(ctx.handle, None, None, 0, None))
    assert e.value.status == 1
    # the context still works after errors
    g = mp.projection_from_inputs(ctx, inp).gamma()
    assert np.all(np.isfinite(_np(g)))


def test_non_finite_inputs_rejected(mp, ctx):
    """A NaN or an infinity in Delta, q or qbar (device or host arrays) is
    refused with MODAL_ERR_NUMERIC before any stage runs; the context keeps
    working."""
    import ctypes
    inp = _small(kind="symmetric", n1=3)
    for field, val in (("delta", np.nan), ("qk", np.inf), ("ql", -np.inf)):
        arr = getattr(inp, field).copy()
        arr.flat[arr.size // 2] = val
        with pytest.raises(mp.ModalError) as e:
            mp.projection_from_inputs(ctx, inp, **{field: arr}).gamma()
        assert e.value.status == 5 and "finite" in str(e.value), field
    # host arrays take the host-side scan
    c = inp.cfg
    delta = inp.delta.copy()
    delta[2, 3] = np.nan
    keep = [np.ascontiguousarray(a) for a in (inp.k, inp.wk, inp.r, inp.wr, delta, inp.cl, inp.qk, inp.ql)]
    tri = np.ascontiguousarray(inp.tri_a, dtype=np.int32)
    g = mp.ModalGrid(c.lmin, c.lmax, c.nk, keep[0].ctypes.data, keep[1].ctypes.data, c.nr,
                     keep[2].ctypes.data, keep[3].ctypes.data, c.nmu, None, None, 0)
    p = mp.ModalProblem(keep[4].ctypes.data, keep[5].ctypes.data, inp.qk.shape[0],
                        keep[6].ctypes.data, inp.ql.shape[0], keep[7].ctypes.data, c.v_power, 1,
                        tri.shape[0], tri.ctypes.data, tri.shape[0], tri.ctypes.data)
    out = np.zeros((tri.shape[0], tri.shape[0]))
    assert mp.lib().modal_gamma(ctx.handle, ctypes.byref(g), ctypes.byref(p), 0, out.ctypes.data) == 5
    assert np.all(np.isfinite(_np(mp.projection_from_inputs(ctx, inp).gamma())))


def test_follows_torch_current_stream(mp, ctx):
    """A context made without a stream runs each call on torch's current
    stream: results computed on a side stream (forward, and the adjoint
    reusing the forward's tables) equal those on the default stream."""
    import torch
    inp = _small(kind="symmetric", n1=4)
    c2 = mp.Context(0)
    try:
        c2.set_forward_reuse(True)
        pr = mp.projection_from_inputs(c2, inp)
        g0 = pr.gamma("fp64")
        dG = c2.to_dev(np.random.default_rng(3).standard_normal(tuple(g0.shape)))
        dq0, dd0 = pr.gamma_backward(dG, "fp64")
        side = torch.cuda.Stream()
        with torch.cuda.stream(side):
            g1 = pr.gamma("fp64")
            dq1, dd1 = pr.gamma_backward(dG, "fp64")
            assert c2.stream.cuda_stream == side.cuda_stream
        torch.cuda.synchronize()
        np.testing.assert_array_equal(_np(g1), _np(g0))
        np.testing.assert_array_equal(_np(dq1), _np(dq0))
        np.testing.assert_array_equal(_np(dd1), _np(dd0))
        g2 = pr.gamma("fp64")                  # back on the default stream
        assert c2.stream.cuda_stream == torch.cuda.current_stream().cuda_stream
        np.testing.assert_array_equal(_np(g2), _np(g0))
    finally:
        c2.close()


def test_workspace_limit(mp, ctx):
    inp = _small(kind="symmetric", n1=3)
    c2 = mp.Context(0)
    c2.set_workspace_limit(1 << 12)
    with pytest.raises(mp.ModalError) as e:
        mp.projection_from_inputs(c2, inp).gamma()
    assert e.value.status == 3
    c2.close()


# ------------------------------------------------------------------ mixed path
@pytest.mark.parametrize("kind,n1,lmax,nr,nk", [
    ("ordered", 5, 40, 21, 150),
    ("symmetric", 5, 40, 21, 150),
    ("symmetric", 7, 33, 9, 70),
    ("ordered", 1, 20, 4, 40),
    ("symmetric", 17, 24, 5, 60),     # U = 289: two 256-row super-blocks
])
def test_gamma_mixed_small(mp, ctx, oracle, kind, n1, lmax, nr, nk):
    """Normwise, and every entry against its own magnitude scale (the oracle's
    c Sum_r wr r^2 Sum_mu wmu Sum_terms |S S S|), as at the large workloads:
    U = 49 and 289 leave ragged row blocks and tiles, and the row blocks that
    hold some i <= j take every count the forward kernel distinguishes."""
    inp = _small(kind=kind, n1=n1, lmax=lmax, nr=nr, nk=nk)
    pr = mp.projection_from_inputs(ctx, inp)
    g = _np(pr.gamma("mixed"))
    ta, tp = g.shape
    rows, cols = np.meshgrid(np.arange(ta), np.arange(tp), indexing="ij")
    ref, scale = oracle.gamma_entries(inp, rows.ravel(), cols.ravel(), return_scale=True)
    ref, scale = ref.reshape(ta, tp), scale.reshape(ta, tp)
    assert np.all(scale > 0)
    err = normwise(g, ref)
    worst = float((np.abs(g - ref) / scale).max())
    print(f"mixed normwise error {err:.3e}, worst |G - ref| / scale {worst:.2e} over {g.size} entries")
    assert err <= MIXED_BAR
    assert worst <= stored_rows.MIXED_TOL


def test_gamma_mixed_lmax64_full(mp, ctx, oracle):
    inp = synth.make_inputs(synth.workload("lmax64_ordered_n8"))
    pr = mp.projection_from_inputs(ctx, inp)
    g = _np(pr.gamma("mixed"))
    ref = oracle.gamma_full(inp)
    err = normwise(g, ref)
    print(f"mixed normwise error at lmax=64: {err:.3e}")
    assert err <= MIXED_BAR


# ------------------------------------------------------------------ large workloads
def _rows_fp64_and_mixed(mp, ctx, name, shape):
    cfg = synth.workload(name)
    inp = synth.make_inputs(cfg)
    pr = mp.projection_from_inputs(ctx, inp)
    g64 = _np(pr.gamma("fp64"))
    gm = _np(pr.gamma("mixed"))
    assert g64.shape == shape and np.all(np.isfinite(g64)) and np.all(np.isfinite(gm))
    stored_rows.check(g64, name, stored_rows.FP64_TOL, f"{name} FP64")
    stored_rows.check(gm, name, stored_rows.MIXED_TOL, f"{name} mixed")
    ew = normwise(gm, g64)
    print(f"{name}: mixed vs FP64 normwise {ew:.2e}")
    assert ew <= MIXED_BAR


def test_gamma_lmax1000_rows(mp, ctx):
    """lmax = 1000, 1540 x 1540 symmetric Gamma: both paths against every
    stored oracle entry, and the mixed path against the FP64 path."""
    _rows_fp64_and_mixed(mp, ctx, "lmax1000_symmetric_n20", (1540, 1540))


def test_gamma_lmax2500_rows(mp, ctx):
    """lmax = 2500, 4960 x 4960 symmetric Gamma: both paths against every
    stored oracle entry, and the mixed path against the FP64 path."""
    _rows_fp64_and_mixed(mp, ctx, "lmax2500_symmetric_n30", (4960, 4960))


@pytest.fixture(scope="module")
def lmax4000(mp, ctx):
    cfg = synth.workload("lmax4000_symmetric_n40")
    inp = synth.make_inputs(cfg)
    return cfg, inp, mp.projection_from_inputs(ctx, inp)


def test_gamma_lmax4000_mixed_rows(mp, ctx, lmax4000):
    """lmax = 4000, 11480 x 11480 symmetric Gamma (the stress workload):
    the mixed path against every stored oracle entry."""
    cfg, inp, pr = lmax4000
    gm = _np(pr.gamma("mixed"))
    assert gm.shape == (11480, 11480) and np.all(np.isfinite(gm))
    stored_rows.check(gm, cfg.name, stored_rows.MIXED_TOL, "lmax=4000 mixed")


@pytest.mark.timeout(400)
def test_gamma_lmax4000_fp64_rows(mp, ctx, lmax4000):
    """lmax = 4000: the FP64 path (about 95 s) against every stored oracle
    entry."""
    cfg, inp, pr = lmax4000
    g = _np(pr.gamma("fp64"))
    assert g.shape == (11480, 11480) and np.all(np.isfinite(g))
    stored_rows.check(g, cfg.name, stored_rows.FP64_TOL, "lmax=4000 FP64")
