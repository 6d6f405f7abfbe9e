"""The late-time Gram matrix <Q_n, Q_m> (modal_gram) and the full Gamma =
<Q, Q>^-1 Gamma' (modal_gamma_modal) against the oracle.

Tolerances: the Gram matrix is the same FP64 arithmetic as Gamma' at one
radial point: normwise 1e-10 (FP64), 1e-4 (mixed).  The full Gamma adds a
solve whose rounding grows with the condition number of <Q, Q>: FP64
normwise 1e-8 against the oracle's solve at small sizes; the mixed path by
its backward error, max|<Q,Q> X - Gamma'| / max|Gamma'| <= 1e-4 with the
oracle's <Q, Q> and Gamma'.  At lmax = 2500 the 4960-mode Gram matrix is
checked on sampled entries, and the full Gamma with 4 and 6 modes per
dimension (a positive definite <Q, Q>; more modes of this basis make it
numerically singular at this lmax).
"""
import numpy as np
import pytest

from paper_1503_08809_amd import synth

pytestmark = pytest.mark.gpu


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


CASES = [("ordered", 3, 20, 6, 60), ("symmetric", 4, 26, 5, 60), ("symmetric", 5, 21, 4, 50)]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("kind,n1,lmax,nr,nk", CASES)
def test_gram_vs_oracle(mp, ctx, oracle, prec, kind, n1, lmax, nr, nk):
    inp = synth.make_inputs(synth.small_config(lmax=lmax, nk=nk, nr=nr, n1=n1, kind=kind, seed_index=91))
    pr = mp.projection_from_inputs(ctx, inp)
    g = _np(pr.gram(prec))
    ref = oracle.gram_full(inp)
    err = normwise(g, ref)
    print(f"Gram {kind} n1={n1} {prec}: {err:.2e}")
    assert err <= (1e-10 if prec == "fp64" else 1e-4)


@pytest.mark.parametrize("kind,n1,lmax,nr,nk", CASES)
def test_gamma_modal_vs_oracle(mp, ctx, oracle, kind, n1, lmax, nr, nk):
    inp = synth.make_inputs(synth.small_config(lmax=lmax, nk=nk, nr=nr, n1=n1, kind=kind, seed_index=92))
    pr = mp.projection_from_inputs(ctx, inp)
    gram, gp = oracle.gram_full(inp), oracle.gamma_full(inp)
    ref = np.linalg.solve(gram, gp)
    x64 = _np(pr.gamma_modal("fp64"))
    xm = _np(pr.gamma_modal("mixed"))
    e64 = normwise(x64, ref)
    bm = float(np.abs(gram @ xm - gp).max() / np.abs(gp).max())
    print(f"full Gamma {kind} n1={n1}: FP64 {e64:.2e}, mixed backward error {bm:.2e}")
    assert e64 <= 1e-8 and bm <= 1e-4


@pytest.mark.parametrize("n1,lmax", [(5, 40), (6, 60)])
def test_gamma_modal_blocked_solve(mp, ctx, oracle, n1, lmax):
    """Ordered lists of 125 and 216 modes: the blocked Cholesky runs over
    two and four 64-wide diagonal blocks (the last ragged) with GEMM updates
    between them.  <Q, Q> is positive definite here (condition number 5.7e6
    and 8.6e8).  FP64: backward error with the oracle's <Q, Q> and Gamma'
    <= 1e-12, forward error against numpy's solve <= 1e-13 cond(<Q, Q>)."""
    inp = synth.make_inputs(synth.small_config(lmax=lmax, nk=40, nr=3, n1=n1, kind="ordered", seed_index=94))
    pr = mp.projection_from_inputs(ctx, inp)
    gram, gp = oracle.gram_full(inp), oracle.gamma_full(inp)
    ref = np.linalg.solve(gram, gp)
    cond = float(np.linalg.cond(gram))
    x64 = _np(pr.gamma_modal("fp64"))
    b64 = float(np.abs(gram @ x64 - gp).max() / np.abs(gp).max())
    e64 = normwise(x64, ref)
    print(f"full Gamma ordered n1={n1} ({gram.shape[0]} modes, cond {cond:.1e}): backward {b64:.2e}, "
          f"forward {e64:.2e}")
    assert gram.shape[0] > 64
    assert b64 <= 1e-12 and e64 <= 1e-13 * cond


def test_gram_lmax2500_sampled(mp, ctx, oracle):
    """lmax = 2500, 4960 x 4960: sampled <Q, Q> entries (the lowest modes
    among them) against the oracle, FP64 and mixed, and the symmetry of the
    whole matrix."""
    cfg = synth.workload("lmax2500_symmetric_n30")
    inp = synth.make_inputs(cfg)
    pr = mp.projection_from_inputs(ctx, inp)
    rows = np.array([0, 0, 1, 2, 100, 1234, 4000, 4959])
    cols = np.array([0, 1, 1, 2, 3000, 77, 4000, 4959])
    ref = oracle.gram_entries(inp, rows, cols)
    g = _np(pr.gram("fp64"))
    gm = _np(pr.gram("mixed"))
    scale = np.abs(g).max()
    sym = float(np.abs(g - g.T).max() / scale)
    err = float(np.abs(g[rows, cols] - ref).max() / scale)
    errm = float(np.abs(gm[rows, cols] - ref).max() / scale)
    big = np.abs(ref) >= 1e-3 * scale
    rel = float((np.abs(g[rows, cols] - ref)[big] / np.abs(ref[big])).max())
    print(f"lmax=2500 Gram: FP64 vs oracle {err:.2e} ({int(big.sum())} large entries, "
          f"elementwise {rel:.2e}), mixed {errm:.2e}, symmetry {sym:.2e}")
    assert err <= 1e-10 and big.sum() >= 1 and rel <= 1e-9 and errm <= 1e-4 and sym <= 1e-14


@pytest.mark.parametrize("n1", [4, 6])
def test_gamma_modal_lmax2500_vs_oracle(mp, ctx, oracle, n1):
    """The full Gamma at lmax = 2500 with few enough modes that <Q, Q> is
    positive definite in FP64 (condition number 4e5 at n1 = 4, 6e9 at
    n1 = 6; the Legendre-in-l basis at n1 >= 10 is numerically singular at
    this lmax, and the call then fails with MODAL_ERR_NUMERIC).  FP64:
    backward error with the oracle's <Q, Q> and Gamma' <= 1e-9, forward
    error <= 1e-13 cond(<Q, Q>); mixed: backward error <= 1e-4."""
    c3 = synth.workload("lmax2500_symmetric_n30")
    cfg = synth.small_config(lmax=2500, nk=200, nr=4, n1=n1, kind="symmetric",
                             kmin=c3.kmin, kmax=c3.kmax, seed_index=93)
    inp = synth.make_inputs(cfg)
    pr = mp.projection_from_inputs(ctx, inp)
    gram, gp = oracle.gram_full(inp), oracle.gamma_full(inp)
    ref = np.linalg.solve(gram, gp)
    cond = float(np.linalg.cond(gram))
    x64 = _np(pr.gamma_modal("fp64"))
    xm = _np(pr.gamma_modal("mixed"))
    b64 = float(np.abs(gram @ x64 - gp).max() / np.abs(gp).max())
    bm = float(np.abs(gram @ xm - gp).max() / np.abs(gp).max())
    e64 = normwise(x64, ref)
    print(f"lmax=2500 full Gamma n1={n1} (cond {cond:.1e}): FP64 backward {b64:.2e}, "
          f"forward {e64:.2e}; mixed backward {bm:.2e}")
    assert b64 <= 1e-9 and e64 <= 1e-13 * cond and bm <= 1e-4


def test_gamma_modal_rejects_singular_gram(mp, ctx):
    """A late-time mode that is zero makes <Q, Q> singular: the call fails
    with MODAL_ERR_NUMERIC instead of returning a solve of it."""
    inp = synth.make_inputs(synth.small_config(lmax=20, nk=40, nr=4, n1=3, kind="symmetric"))
    inp.ql[0] = 0.0
    pr = mp.projection_from_inputs(ctx, inp)
    with pytest.raises(mp.ModalError) as e:
        pr.gamma_modal("fp64")
    assert "positive definite" in str(e.value)


def test_gram_v_power_zero(mp, ctx, oracle):
    """v_power = 0: the Gram weights become (2l+1) (no v_l), against the oracle."""
    inp = synth.make_inputs(synth.small_config(lmax=22, nk=30, nr=3, n1=4, kind="symmetric", seed_index=101,
                                               v_power=0.0))
    pr = mp.projection_from_inputs(ctx, inp)
    assert normwise(_np(pr.gram("fp64")), oracle.gram_full(inp)) <= 1e-10


def test_gram_rejects_too_many_modes(mp, ctx):
    """na^2 above 8192 late-time pairs is refused before any device work."""
    inp = synth.make_inputs(synth.small_config(lmax=20, nk=20, nr=2, n1=91, kind="symmetric"), with_delta=False)
    inp.qk = inp.qk[:2].copy()                      # np = 2: only the Gram's own limit applies
    inp.tri_a = inp.tri_a[:4].copy()
    inp.tri_p = np.zeros((1, 3), dtype=np.int32)
    pr = mp.projection_from_inputs(ctx, inp)
    with pytest.raises(mp.ModalError) as e:
        pr.gram("fp64")
    assert e.value.status == 2 and "na * na" in str(e.value)
