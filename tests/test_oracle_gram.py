"""Pins of the oracle's late-time Gram matrix <Q_n, Q_m> and of the full
Gamma = <Q, Q>^-1 Gamma' (Appendix; the inner product of Sec. 2.1).

* the separable form (mu quadrature, Sec. 2.2) against the inner product
  written out with the exact Wigner symbol on tiny lmax (Gauss-Legendre is
  exact there, so the two agree to rounding);
* symmetric lists: the Gram matrix is the mean over the six orderings of
  one side of the ordered one (the permanent);
* symmetric and positive definite (a Gram matrix of independent modes);
* the full Gamma solves <Q, Q> Gamma = Gamma'.
"""
import dataclasses
import itertools

import numpy as np

from paper_1503_08809_amd import synth


def test_gram_matches_exact_3j(oracle):
    inp = synth.make_inputs(synth.small_config(lmax=14, nk=30, nr=3, n1=3, kind="ordered"))
    g = oracle.gram_full(inp)
    b = oracle.brute_force_gram_ordered(inp)
    assert np.abs(g - b).max() <= 1e-12 * np.abs(b).max()


def test_gram_symmetric_is_mean_of_ordered(oracle):
    cfg = synth.small_config(lmax=12, nk=30, nr=3, n1=3, kind="symmetric")
    inp = synth.make_inputs(cfg)
    gs = oracle.gram_full(inp)
    ordered = np.array(list(itertools.product(range(3), repeat=3)), dtype=np.int32)
    io = dataclasses.replace(inp, cfg=dataclasses.replace(cfg, kind="ordered"), tri_a=ordered,
                             tri_p=ordered)
    go = oracle.gram_full(io)
    index = {tuple(t): i for i, t in enumerate(ordered.tolist())}
    ta = inp.tri_a
    ref = np.empty_like(gs)
    for n in range(ta.shape[0]):
        for m in range(ta.shape[0]):
            perms = [index[tuple(ta[m][list(s)])] for s in itertools.permutations(range(3))]
            ref[n, m] = np.mean(go[index[tuple(ta[n])], perms])
    assert np.abs(gs - ref).max() <= 1e-13 * np.abs(ref).max()


def test_gram_symmetric_positive_definite(oracle):
    for kind in ("ordered", "symmetric"):
        inp = synth.make_inputs(synth.small_config(lmax=20, nk=30, nr=3, n1=4, kind=kind))
        g = oracle.gram_full(inp)
        assert np.abs(g - g.T).max() <= 1e-14 * np.abs(g).max()
        assert np.linalg.eigvalsh(g).min() > 0.0


def test_gamma_modal_solves_the_gram_system(oracle):
    inp = synth.make_inputs(synth.small_config(lmax=20, nk=40, nr=4, n1=3, kind="symmetric"))
    gp = oracle.gamma_full(inp)
    x = oracle.gamma_modal(inp)
    r = oracle.gram_full(inp) @ x - gp
    assert np.abs(r).max() <= 1e-10 * np.abs(gp).max()
