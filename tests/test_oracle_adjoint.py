"""Pins of the oracle's adjoint (gradient of a scalar loss of Gamma with
respect to q_p(k) and Delta_l(k)).

Checked against: central finite differences of the oracle's own forward
projection, float64 torch autograd of an independent dense formulation
(scipy j_l and P_l, numpy Gauss-Legendre), and the adjoint identity
<J v, u> = <v, J^T u> of each linear stage.
"""
import math

import numpy as np
import pytest

from paper_1503_08809_amd import synth


def _tiny(kind, n1=2, lmax=12, nk=24, nr=4, seed_index=70):
    cfg = synth.small_config(lmax=lmax, nk=nk, nr=nr, n1=n1, kind=kind, seed_index=seed_index)
    return synth.make_inputs(cfg)


def _loss_weights(inp, seed=3):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((inp.tri_a.shape[0], inp.tri_p.shape[0]))


@pytest.mark.parametrize("kind", ["ordered", "symmetric"])
def test_adjoint_vs_central_differences(oracle, kind):
    inp = _tiny(kind)
    Wt = _loss_weights(inp)
    dq, dd = oracle.gamma_full_backward(inp, Wt)

    def loss(i2):
        return float(np.sum(oracle.gamma_full(i2) * Wt))

    rng = np.random.default_rng(11)
    for name, arr, grad in (("qk", inp.qk, dq), ("delta", inp.delta, dd)):
        picks = rng.choice(arr.size, size=6, replace=False)
        for flat in picks:
            idx = np.unravel_index(flat, arr.shape)
            h = 1e-4 * max(abs(arr[idx]), 1e-3)
            ip = synth.make_inputs(inp.cfg)
            im = synth.make_inputs(inp.cfg)
            getattr(ip, name)[idx] += h
            getattr(im, name)[idx] -= h
            fd = (loss(ip) - loss(im)) / (2 * h)
            scale = np.abs(grad).max()
            assert abs(fd - grad[idx]) <= 1e-6 * scale + 1e-6 * abs(fd), (name, idx, fd, grad[idx])


def _torch_forward(inp, qk, delta):
    """Dense float64 torch version of the projection, built from library
    routines (scipy j_l and P_l, numpy Gauss-Legendre) and written from the
    definitions, for autograd."""
    import torch
    from scipy.special import eval_legendre, spherical_jn
    c = inp.cfg
    ells = inp.ells
    mu, wmu = np.polynomial.legendre.leggauss(c.nmu)
    J = spherical_jn(ells[:, None, None], inp.k[None, :, None] * inp.r[None, None, :])   # [l][k][r]
    P = eval_legendre(ells[:, None], mu[None, :])                                      # [l][mu]
    wl = (2 * ells + 1.0) ** (1.0 - c.v_power) / np.sqrt(inp.cl)
    t = lambda a: torch.as_tensor(a, dtype=torch.float64)
    kw = t(2 / np.pi * inp.wk * inp.k ** 2)
    beta = torch.einsum("pk,lk,lkr,k->plr", qk, delta, t(J), kw)
    S = torch.einsum("al,l,plr,lm->aprm", t(inp.ql), t(wl), beta, t(P))
    W = t(inp.wr * inp.r ** 2)[:, None] * t(wmu)[None, :]
    ta, tp = inp.tri_a, inp.tri_p
    G = torch.zeros(ta.shape[0], tp.shape[0], dtype=torch.float64)
    import itertools
    for n in range(ta.shape[0]):
        for m in range(tp.shape[0]):
            a, p = ta[n], tp[m]
            if c.kind == "ordered":
                F = S[a[0], p[0]] * S[a[1], p[1]] * S[a[2], p[2]]
                G[n, m] = (W * F).sum() / (8 * math.pi)
            else:
                F = 0
                for s in itertools.permutations(range(3)):
                    F = F + S[a[0], p[s[0]]] * S[a[1], p[s[1]]] * S[a[2], p[s[2]]]
                G[n, m] = (W * F).sum() / (48 * math.pi)
    return G


@pytest.mark.parametrize("kind", ["ordered", "symmetric"])
def test_adjoint_vs_torch_autograd(oracle, kind):
    import torch
    inp = _tiny(kind, n1=2, lmax=10, nk=18, nr=3)
    Wt = _loss_weights(inp, seed=5)
    qk = torch.tensor(inp.qk, dtype=torch.float64, requires_grad=True)
    de = torch.tensor(inp.delta, dtype=torch.float64, requires_grad=True)
    G = _torch_forward(inp, qk, de)
    # the forward itself agrees with the oracle
    g_or = oracle.gamma_full(inp)
    assert np.abs(G.detach().numpy() - g_or).max() <= 1e-10 * np.abs(g_or).max()
    (G * torch.as_tensor(Wt)).sum().backward()
    dq, dd = oracle.gamma_full_backward(inp, Wt)
    np.testing.assert_allclose(dq, qk.grad.numpy(), rtol=1e-8, atol=1e-10 * np.abs(dq).max())
    np.testing.assert_allclose(dd, de.grad.numpy(), rtol=1e-8, atol=1e-10 * np.abs(dd).max())


def test_S_stage_adjoint_identity(oracle):
    """<S(beta'), Shat> = <beta', S^T Shat> (Eq. (legendre) is linear in beta)."""
    inp = _tiny("ordered", n1=3, lmax=14, nk=20, nr=5)
    c = inp.cfg
    mu, _ = oracle.gauss_legendre(c.nmu)
    rng = np.random.default_rng(2)
    bet = rng.standard_normal((3, c.L, c.nr))
    pairs = [(a, p) for a in range(3) for p in range(3)]
    S = oracle.S_pairs(inp, mu, bet, pairs)
    Shat = rng.standard_normal(S.shape)
    bhat = oracle.S_adjoint(inp, mu, Shat, pairs, 3)
    lhs = float(np.sum(S * Shat))
    rhs = float(np.sum(bet * bhat))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_beta_stage_adjoint_identity(oracle):
    """beta is linear in q for fixed Delta and in Delta for fixed q."""
    inp = _tiny("ordered", n1=3, lmax=14, nk=20, nr=5)
    rng = np.random.default_rng(4)
    bhat = rng.standard_normal((3, inp.cfg.L, inp.cfg.nr))
    dq, dd = oracle.beta_adjoint(inp, bhat)
    b0 = oracle.beta(inp)
    # <d beta / dq . v, bhat> = <v, dq> with v = q (beta is linear in q)
    assert abs(float(np.sum(b0 * bhat)) - float(np.sum(inp.qk * dq))) <= 1e-12 * abs(float(np.sum(b0 * bhat)))
    assert abs(float(np.sum(b0 * bhat)) - float(np.sum(inp.delta * dd))) <= 1e-12 * abs(float(np.sum(b0 * bhat)))


def test_gamma_stage_adjoint_is_derivative(oracle):
    """dL/dS from the Gamma adjoint matches the derivative of the cubic
    form: for Gamma cubic in S, <dGamma/dS . S, g> = 3 <Gamma, g>."""
    for kind in ("ordered", "symmetric"):
        inp = _tiny(kind, n1=2, lmax=10, nk=18, nr=3)
        c = inp.cfg
        mu, wmu = oracle.gauss_legendre(c.nmu)
        S, bet = oracle.full_S(inp, mu)
        S = S.reshape(-1, c.nr, c.nmu)
        ta, tp = inp.tri_a, inp.tri_p
        sidx = (ta[:, None, :, None] * 2 + tp[None, :, None, :]).reshape(-1, 9)
        g = np.random.default_rng(8).standard_normal(sidx.shape[0])
        G = oracle.gamma_from_S(inp, wmu, S, sidx)
        Shat = oracle.gamma_adjoint_S(inp, wmu, S, sidx, g)
        assert abs(float(np.sum(Shat * S)) - 3 * float(np.sum(G * g))) <= 1e-12 * abs(3 * float(np.sum(G * g)))
