"""Parity of the HIP adjoint (modal_gamma_backward) with the oracle's
adjoint, its torch.autograd wrapper, and central finite differences at the
lmax = 1000 workload.

Tolerances: against the oracle the adjoint is FP64 arithmetic of sums of up
to ~10^8 terms: normwise 1e-10.  Finite differences (absolute step 1e-6 in
q or Delta, FP64 forward): |g_fd - g| <= 1e-6 max|g| + 1e-5 |g|.  Mixed
forward + adjoint against the FP64 gradient: normwise 1e-4.
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


def large_rel(a, ref, frac=1e-3):
    """Largest relative error over the entries of ref above frac of its
    largest: an entry-wise check that a wrong subset of entries cannot hide
    behind the largest ones."""
    big = np.abs(ref) >= frac * np.abs(ref).max()
    return float((np.abs(a - ref)[big] / np.abs(ref[big])).max())


@pytest.mark.parametrize("kind,n1,lmax,nr,nk", [
    ("ordered", 3, 30, 7, 80),
    ("symmetric", 4, 30, 7, 80),
    ("symmetric", 5, 21, 5, 50),
    ("ordered", 1, 16, 3, 30),
])
def test_backward_vs_oracle(mp, ctx, oracle, kind, n1, lmax, nr, nk):
    cfg = synth.small_config(lmax=lmax, nk=nk, nr=nr, n1=n1, kind=kind, seed_index=71)
    inp = synth.make_inputs(cfg)
    dG = np.random.default_rng(9).standard_normal((inp.tri_a.shape[0], inp.tri_p.shape[0]))
    pr = mp.projection_from_inputs(ctx, inp)
    dq, dd = pr.gamma_backward(ctx.to_dev(dG))
    rq, rd = oracle.gamma_full_backward(inp, dG)
    assert normwise(_np(dq), rq) <= 1e-10
    assert normwise(_np(dd), rd) <= 1e-10
    assert large_rel(_np(dq), rq) <= 1e-8 and large_rel(_np(dd), rd) <= 1e-8


@pytest.mark.parametrize("kind,n1,lmax,nr,nk", [
    ("ordered", 3, 30, 7, 80),
    ("symmetric", 5, 21, 5, 50),
    ("symmetric", 6, 26, 4, 40),      # U = 36: three 16-row blocks, ragged
    ("ordered", 1, 16, 3, 30),
])
def test_backward_mixed_vs_oracle(mp, ctx, oracle, kind, n1, lmax, nr, nk):
    """Mixed adjoint of step d (split-BF16 products, FP32 partial sums,
    FP64 output) against the FP64 oracle: normwise 1e-4."""
    cfg = synth.small_config(lmax=lmax, nk=nk, nr=nr, n1=n1, kind=kind, seed_index=72)
    inp = synth.make_inputs(cfg)
    dG = np.random.default_rng(12).standard_normal((inp.tri_a.shape[0], inp.tri_p.shape[0]))
    pr = mp.projection_from_inputs(ctx, inp)
    dq, dd = pr.gamma_backward(ctx.to_dev(dG), "mixed")
    rq, rd = oracle.gamma_full_backward(inp, dG)
    eq, ed = normwise(_np(dq), rq), normwise(_np(dd), rd)
    # mixed: entries above 1e-2 of the largest (an entry far below it can be
    # a deep cancellation, whose error follows the size of its terms)
    lq, ld = large_rel(_np(dq), rq, 1e-2), large_rel(_np(dd), rd, 1e-2)
    print(f"mixed adjoint {kind} n1={n1}: dq {eq:.2e}, ddelta {ed:.2e}; large entries {lq:.2e}, {ld:.2e}")
    assert eq <= 1e-4 and ed <= 1e-4
    assert lq <= 1e-3 and ld <= 1e-3


# U = n1^2 rows against the adjoint kernels' row blocks (FP64: 128 rows,
# mixed: 256), with 16-row tiles: U below one block (81: six live tiles),
# exact multiples (256), a last block of one (144, 900 - 7 * 128 = 4 rows
# likewise), seven (225), eight (121: handled as a full block) and nine (400,
# mixed) live tiles; nr = 10 gives several z tiles and a ragged last one.
@pytest.mark.parametrize("prec,n1", [
    ("fp64", 9), ("fp64", 11), ("fp64", 12), ("fp64", 15), ("fp64", 16),
    ("mixed", 12), ("mixed", 17), ("mixed", 20),
])
def test_backward_row_tails_vs_oracle(mp, ctx, oracle, prec, n1):
    cfg = synth.small_config(lmax=14, nk=30, nr=10, n1=n1, kind="symmetric", seed_index=80 + n1)
    inp = synth.make_inputs(cfg)
    dG = np.random.default_rng(n1).standard_normal((inp.tri_a.shape[0], inp.tri_p.shape[0]))
    pr = mp.projection_from_inputs(ctx, inp)
    dq, dd = pr.gamma_backward(ctx.to_dev(dG), prec)
    rq, rd = oracle.gamma_full_backward(inp, dG)
    eq, ed = normwise(_np(dq), rq), normwise(_np(dd), rd)
    frac, tol, ltol = (1e-3, 1e-10, 1e-8) if prec == "fp64" else (1e-2, 1e-4, 1e-3)
    lq, ld = large_rel(_np(dq), rq, frac), large_rel(_np(dd), rd, frac)
    print(f"{prec} adjoint U={n1 * n1}: dq {eq:.2e}, ddelta {ed:.2e}; large entries {lq:.2e}, {ld:.2e}")
    assert eq <= tol and ed <= tol
    assert lq <= ltol and ld <= ltol


def test_backward_mixed_lmax500_vs_fp64(mp, ctx):
    """lmax = 500, U = 256 ordered: the mixed adjoint against the FP64 one."""
    inp = synth.make_inputs(synth.workload("lmax500_ordered_n16"))
    dG = np.random.default_rng(13).standard_normal((inp.tri_a.shape[0], inp.tri_p.shape[0]))
    pr = mp.projection_from_inputs(ctx, inp)
    G = ctx.to_dev(dG)
    fq, fd = pr.gamma_backward(G, "fp64")
    mq, md = pr.gamma_backward(G, "mixed")
    eq, ed = normwise(_np(mq), _np(fq)), normwise(_np(md), _np(fd))
    print(f"mixed vs FP64 adjoint at lmax=500: dq {eq:.2e}, ddelta {ed:.2e}")
    assert eq <= 1e-4 and ed <= 1e-4


def test_backward_lmax64_vs_oracle(mp, ctx, oracle):
    inp = synth.make_inputs(synth.workload("lmax64_ordered_n8"))
    dG = np.random.default_rng(10).standard_normal((512, 512))
    pr = mp.projection_from_inputs(ctx, inp)
    dq, dd = pr.gamma_backward(ctx.to_dev(dG))
    rq, rd = oracle.gamma_full_backward(inp, dG)
    assert normwise(_np(dq), rq) <= 1e-10
    assert normwise(_np(dd), rd) <= 1e-10
    assert large_rel(_np(dq), rq) <= 1e-8 and large_rel(_np(dd), rd) <= 1e-8


def test_backward_host_outputs_and_null(mp, ctx):
    import ctypes
    inp = synth.make_inputs(synth.small_config(lmax=20, nk=40, nr=4, n1=3, kind="symmetric"))
    pr = mp.projection_from_inputs(ctx, inp)
    dG = np.random.default_rng(1).standard_normal((inp.tri_a.shape[0], inp.tri_p.shape[0]))
    dq_dev, dd_dev = pr.gamma_backward(ctx.to_dev(dG))
    g, p = pr.structs()
    dq = np.zeros(inp.qk.shape)
    ctx.check(mp.lib().modal_gamma_backward(ctx.handle, ctypes.byref(g), ctypes.byref(p), 0,
                                            dG.ctypes.data, dq.ctypes.data, None))
    np.testing.assert_array_equal(dq, _np(dq_dev))
    with pytest.raises(mp.ModalError):
        ctx.check(mp.lib().modal_gamma_backward(ctx.handle, ctypes.byref(g), ctypes.byref(p), 0,
                                                dG.ctypes.data, None, None))


def test_backward_rejects_repeated_triples(mp, ctx):
    inp = synth.make_inputs(synth.small_config(lmax=20, nk=40, nr=4, n1=3, kind="symmetric"))
    tri = inp.tri_a.copy()
    tri[1] = tri[0][::-1]                       # same sorted triple twice
    pr = mp.projection_from_inputs(ctx, inp, tri_a=tri)
    dG = np.ones((tri.shape[0], inp.tri_p.shape[0]))
    with pytest.raises(mp.ModalError) as e:
        pr.gamma_backward(ctx.to_dev(dG))
    assert e.value.status == 2


def test_autograd_function(mp, ctx):
    import torch
    inp = synth.make_inputs(synth.small_config(lmax=24, nk=50, nr=5, n1=3, kind="symmetric"))
    pr = mp.projection_from_inputs(ctx, inp)
    W = ctx.to_dev(np.random.default_rng(2).standard_normal((inp.tri_a.shape[0], inp.tri_p.shape[0])))
    qk = pr.qk.clone().requires_grad_(True)
    de = pr.delta.clone().requires_grad_(True)
    G = mp.ModalProjectionFunction.apply(qk, de, pr, "fp64")
    L = ((G * W) ** 2).sum()
    L.backward()
    dq, dd = pr.gamma_backward(2 * G.detach() * W * W)
    np.testing.assert_allclose(_np(qk.grad), _np(dq), rtol=0, atol=0)
    np.testing.assert_allclose(_np(de.grad), _np(dd), rtol=0, atol=0)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_forward_reuse(mp, ctx, prec):
    """modal_set_forward_reuse: a backward after a forward on the same inputs
    takes the forward's tables and gives the recomputed gradient bit for bit;
    after a forward on other inputs, or another entry point in between, it
    recomputes (same result again)."""
    cfg = synth.small_config(lmax=26, nk=60, nr=6, n1=4, kind="symmetric", seed_index=75)
    inp = synth.make_inputs(cfg)
    pr = mp.projection_from_inputs(ctx, inp)
    other = mp.projection_from_inputs(ctx, synth.make_inputs(
        synth.small_config(lmax=26, nk=60, nr=6, n1=4, kind="symmetric", seed_index=76)))
    dG = ctx.to_dev(np.random.default_rng(5).standard_normal((inp.tri_a.shape[0], inp.tri_p.shape[0])))
    try:
        ctx.set_forward_reuse(False)
        pr.gamma(prec)
        ref = [_np(t) for t in pr.gamma_backward(dG, prec)]
        ctx.set_forward_reuse(True)
        cases = {
            "after its forward": lambda: pr.gamma(prec),
            "after a forward on other inputs": lambda: (pr.gamma(prec), other.gamma(prec)),
            "after another entry point": lambda: (pr.gamma(prec), other.beta()),
            "after a backward": lambda: pr.gamma_backward(dG, prec),
        }
        for name, before in cases.items():
            before()
            got = [_np(t) for t in pr.gamma_backward(dG, prec)]
            for g, r in zip(got, ref):
                np.testing.assert_array_equal(g, r, err_msg=name)
    finally:
        ctx.set_forward_reuse(False)


def test_forward_reuse_host_inputs(mp, ctx):
    """Reuse with every input in host memory: the forward's staged copies of
    the inputs stay in place while the backward stages dL/dGamma after them
    (the result equals the device-input backward bit for bit)."""
    import ctypes
    cfg = synth.small_config(lmax=22, nk=48, nr=5, n1=3, kind="ordered", seed_index=77)
    inp = synth.make_inputs(cfg)
    pr = mp.projection_from_inputs(ctx, inp)
    dG = np.random.default_rng(6).standard_normal((inp.tri_a.shape[0], inp.tri_p.shape[0]))
    ref = [_np(t) for t in pr.gamma_backward(ctx.to_dev(dG))]
    host = {name: np.ascontiguousarray(_np(getattr(pr, name))) for name in
            ("k", "wk", "r", "wr", "delta", "cl", "qk", "ql", "tri_a", "tri_p")}
    hp = lambda a: a.ctypes.data
    g = mp.ModalGrid(pr.lmin, pr.lmax, host["k"].size, hp(host["k"]), hp(host["wk"]), host["r"].size,
                     hp(host["r"]), hp(host["wr"]), pr.nmu, None, None, 0)
    p = mp.ModalProblem(hp(host["delta"]), hp(host["cl"]), pr.np_, hp(host["qk"]), pr.na, hp(host["ql"]),
                        pr.v_power, 0, host["tri_a"].shape[0], hp(host["tri_a"]), host["tri_p"].shape[0],
                        hp(host["tri_p"]))
    gamma = np.zeros((host["tri_a"].shape[0], host["tri_p"].shape[0]))
    dq = np.zeros(host["qk"].shape)
    dd = np.zeros(host["delta"].shape)
    try:
        ctx.set_forward_reuse(True)
        ctx.check(mp.lib().modal_gamma(ctx.handle, ctypes.byref(g), ctypes.byref(p), 0, gamma.ctypes.data))
        ctx.check(mp.lib().modal_gamma_backward(ctx.handle, ctypes.byref(g), ctypes.byref(p), 0,
                                                dG.ctypes.data, dq.ctypes.data, dd.ctypes.data))
    finally:
        ctx.set_forward_reuse(False)
    np.testing.assert_array_equal(dq, ref[0])
    np.testing.assert_array_equal(dd, ref[1])


def test_autograd_reuse_follows_inplace_changes(mp, ctx):
    """The autograd wrapper lets the library reuse the forward's tables only
    while no input has been modified in place: after q is scaled in place the
    gradient is that of the scaled q (recomputed), not the stale one."""
    import torch
    inp = synth.make_inputs(synth.small_config(lmax=24, nk=50, nr=5, n1=3, kind="symmetric"))
    pr = mp.projection_from_inputs(ctx, inp)
    W = ctx.to_dev(np.random.default_rng(3).standard_normal((inp.tri_a.shape[0], inp.tri_p.shape[0])))
    qk = pr.qk.clone().requires_grad_(True)
    de = pr.delta.clone().requires_grad_(True)
    G = mp.ModalProjectionFunction.apply(qk, de, pr, "fp64")
    with torch.no_grad():
        qk.mul_(1.5)
    ((G * W) ** 2).sum().backward()
    import dataclasses
    p2 = dataclasses.replace(pr, qk=qk.detach().clone(), delta=de.detach().clone())
    dq, dd = p2.gamma_backward(2 * G.detach() * W * W)
    np.testing.assert_array_equal(_np(qk.grad), _np(dq))
    np.testing.assert_array_equal(_np(de.grad), _np(dd))
    assert ctx.forward_reuse is False


def test_lmax1000_finite_differences_and_mixed(mp, ctx):
    """lmax = 1000, 1540 x 1540 symmetric Gamma, L = Sum (Gamma * W)^2 with W
    a seeded N(0,1) matrix: 32 seeded entries of each gradient against
    central differences with step 1e-6, and the mixed path's gradient
    against the FP64 one."""
    import torch
    cfg = synth.workload("lmax1000_symmetric_n20")
    inp = synth.make_inputs(cfg)
    pr = mp.projection_from_inputs(ctx, inp)
    W = ctx.to_dev(synth.loss_weights(cfg, inp.tri_a.shape[0], inp.tri_p.shape[0]))

    def loss(prj, prec="fp64"):
        G = prj.gamma(prec)
        return float(((G * W) ** 2).sum()), G

    L0, G = loss(pr)
    dq, dd = pr.gamma_backward(2 * G * W * W)
    dq, dd = _np(dq), _np(dd)
    h = 1e-6
    for name, grad, off in (("qk", dq, 0), ("delta", dd, 1)):
        base = getattr(pr, name)
        picks = synth.pick_entries(cfg, grad.shape, 32, seed_offset=off)
        for flat in picks:
            idx = np.unravel_index(int(flat), grad.shape)
            vals = []
            for sgn in (1.0, -1.0):
                t = base.clone()
                t[idx] += sgn * h
                prj = mp.projection_from_inputs(ctx, inp, **{name: t})
                vals.append(loss(prj)[0])
            fd = (vals[0] - vals[1]) / (2 * h)
            tol = 1e-6 * np.abs(grad).max() + 1e-5 * abs(grad[idx])
            assert abs(fd - grad[idx]) <= tol, (name, idx, fd, grad[idx])
    # mixed forward + adjoint against the FP64 gradient
    Lm, Gm = loss(pr, "mixed")
    mq, md = pr.gamma_backward(2 * Gm * W * W, "mixed")
    eq, ed = normwise(_np(mq), dq), normwise(_np(md), dd)
    print(f"mixed gradient normwise error: dq {eq:.3e}, ddelta {ed:.3e}")
    assert eq <= 1e-4 and ed <= 1e-4


def test_lmax1000_gradient_vs_stored_oracle(mp, ctx):
    """lmax = 1000, L = Sum (Gamma * W)^2: the gradient against the oracle's
    (stored: all of dL/dq, and dL/dDelta_l(k) at 18 values of l, every k),
    elementwise.  FP64: within 1e-10 of the largest stored value of each
    gradient, and 1e-8 relative on the entries above 1e-3 of it; mixed: the
    1e-4 bar."""
    import stored_rows
    cfg = synth.workload("lmax1000_symmetric_n20")
    rq, rows, _ = stored_rows.load_grad(cfg.name)
    ls = sorted(rows)
    rd = np.stack([rows[l] for l in ls])
    inp = synth.make_inputs(cfg)
    pr = mp.projection_from_inputs(ctx, inp)
    W = ctx.to_dev(synth.loss_weights(cfg, inp.tri_a.shape[0], inp.tri_p.shape[0]))
    for prec, tol in (("fp64", 1e-10), ("mixed", 1e-4)):
        G = pr.gamma(prec)
        dq, dd = pr.gamma_backward(2 * G * W * W, prec)
        dq, dd = _np(dq), _np(dd)[[l - cfg.lmin for l in ls]]
        eq, ed = normwise(dq, rq), normwise(dd, rd)
        big_q, big_d = np.abs(rq) >= 1e-3 * np.abs(rq).max(), np.abs(rd) >= 1e-3 * np.abs(rd).max()
        rel_q = float((np.abs(dq - rq)[big_q] / np.abs(rq[big_q])).max())
        rel_d = float((np.abs(dd - rd)[big_d] / np.abs(rd[big_d])).max())
        print(f"{prec} gradient vs stored oracle at lmax=1000: dq {eq:.2e} ({rq.size} entries, large "
              f"ones {rel_q:.2e} relative), ddelta {ed:.2e} ({rd.size} entries, {rel_d:.2e})")
        assert eq <= tol and ed <= tol
        if prec == "fp64":
            assert rel_q <= 1e-8 and rel_d <= 1e-8


def test_lmax2500_gradient_full_size(mp, ctx):
    """lmax = 2500, 4960 x 4960 symmetric Gamma, L = Sum (Gamma * W)^2.

    Gamma is cubic in q and cubic in Delta (beta is linear in each), so L is
    homogeneous of degree 6 in each: <dL/dq, q> = 6 L and <dL/dDelta, Delta>
    = 6 L exactly (Euler).  Also a central difference of the FP64 forward
    along a seeded direction (relative step 1e-4 in every q and Delta entry;
    truncation ~1e-7 relative), and the mixed gradient against the FP64 one."""
    cfg = synth.workload("lmax2500_symmetric_n30")
    inp = synth.make_inputs(cfg)
    pr = mp.projection_from_inputs(ctx, inp)
    W = ctx.to_dev(synth.loss_weights(cfg, inp.tri_a.shape[0], inp.tri_p.shape[0]))

    def loss(prj, prec="fp64"):
        G = prj.gamma(prec)
        return float(((G * W) ** 2).sum()), G

    L0, G = loss(pr)
    dq, dd = pr.gamma_backward(2 * G * W * W)
    e_q = float((dq * pr.qk).sum()) / (6 * L0) - 1
    e_d = float((dd * pr.delta).sum()) / (6 * L0) - 1
    print(f"FP64 Euler identities at lmax=2500: {e_q:.2e}, {e_d:.2e}")
    assert abs(e_q) <= 1e-9 and abs(e_d) <= 1e-9
    rng = np.random.default_rng(2500)
    xq = ctx.to_dev(rng.standard_normal(tuple(pr.qk.shape))) * pr.qk * 1e-4
    xd = ctx.to_dev(rng.standard_normal(tuple(pr.delta.shape))) * pr.delta * 1e-4
    Lp = loss(mp.projection_from_inputs(ctx, inp, qk=pr.qk + xq, delta=pr.delta + xd))[0]
    Lm = loss(mp.projection_from_inputs(ctx, inp, qk=pr.qk - xq, delta=pr.delta - xd))[0]
    lin_q, lin_d = float((dq * xq).sum()), float((dd * xd).sum())
    fd = (Lp - Lm) / 2
    print(f"directional derivative: fd {fd:.6e}, adjoint {lin_q + lin_d:.6e} (q {lin_q:.3e}, Delta {lin_d:.3e})")
    assert abs(fd - (lin_q + lin_d)) <= 1e-6 * (abs(lin_q) + abs(lin_d))
    Lm_, Gm = loss(pr, "mixed")
    mq, md = pr.gamma_backward(2 * Gm * W * W, "mixed")
    eq, ed = normwise(_np(mq), _np(dq)), normwise(_np(md), _np(dd))
    em_q = float((mq * pr.qk).sum()) / (6 * Lm_) - 1
    print(f"mixed vs FP64 gradient at lmax=2500: dq {eq:.2e}, ddelta {ed:.2e}; mixed Euler {em_q:.2e}")
    assert eq <= 1e-4 and ed <= 1e-4 and abs(em_q) <= 1e-5


def test_lmax4000_mixed_gradient_euler(mp, ctx):
    """lmax = 4000 stress workload, mixed forward + adjoint with the j_l
    tables regenerated: L = Sum (Gamma * W)^2 is homogeneous of degree 6 in q
    and in Delta, so <dL/dq, q> = <dL/dDelta, Delta> = 6 L."""
    cfg = synth.workload("lmax4000_symmetric_n40")
    inp = synth.make_inputs(cfg)
    pr = mp.projection_from_inputs(ctx, inp)
    W = ctx.to_dev(synth.loss_weights(cfg, inp.tri_a.shape[0], inp.tri_p.shape[0]))
    G = pr.gamma("mixed")
    L = float(((G * W) ** 2).sum())
    dq, dd = pr.gamma_backward(2 * G * W * W, "mixed")
    e_q = float((dq * pr.qk).sum()) / (6 * L) - 1
    e_d = float((dd * pr.delta).sum()) / (6 * L) - 1
    print(f"lmax=4000 mixed Euler identities: {e_q:.2e}, {e_d:.2e}")
    assert np.all(np.isfinite(_np(dq))) and np.all(np.isfinite(_np(dd)))
    assert abs(e_q) <= 1e-4 and abs(e_d) <= 1e-4
