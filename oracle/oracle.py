"""Python face of the test oracle for the separable bispectrum projection.

TEST INFRASTRUCTURE ONLY: the product path never imports this module.
Only tests, the smoke check and the CPU-baseline leg of the benchmark use
it.  It shares no code with the HIP library (the seeded inputs it is fed
come from their own module, which holds none of the method's arithmetic).

The numerical work is in ``modal_oracle.c`` (plain FP64 loops); this file
marshals arrays, selects what a sampled entry needs, and holds the
brute-force exact-3j form of the inner product used to pin the separable
oracle (Sec. 2.1, Eq. (weight-function) and Eq. (3D) with the exact
Wigner symbol in place of the Gosper approximation).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "modal_oracle.c")
_LIB = os.path.join(_HERE, "libmodal_oracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        L.or_gauss_legendre.argtypes = [ctypes.c_int, _dp, _dp]
        L.or_legendre_table.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp]
        L.or_sph_bessel_table.argtypes = [ctypes.c_int, ctypes.c_int64, _dp, _dp]
        L.or_beta.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_int, _dp,
                              ctypes.c_int, _dp, _dp, ctypes.c_int, _ip, _dp]
        L.or_S.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_double, ctypes.c_int, _dp,
                           ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, _dp, ctypes.c_int, _ip, _dp]
        L.or_gamma_entries.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_int, _dp,
                                       ctypes.c_int, _dp, ctypes.c_int64, _ip, _dp, _dp]
        L.or_gamma_adjoint.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_int, _dp,
                                       ctypes.c_int, _dp, ctypes.c_int64, _ip, _dp, _dp]
        L.or_S_adjoint.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_double, ctypes.c_int,
                                   _dp, ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int,
                                   _ip, _dp, _dp]
        L.or_beta_adjoint.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp,
                                      ctypes.c_int, _dp, ctypes.c_int, _dp, _dp, _dp, _dp, _dp]
        L.or_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_ip)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def num_threads() -> int:
    return int(lib().or_num_threads())


# ---------------------------------------------------------------- stages
def gauss_legendre(n: int):
    """Gauss-Legendre nodes (ascending) and weights on [-1, 1] (Sec. 2.2)."""
    x = np.empty(n)
    w = np.empty(n)
    _check(lib().or_gauss_legendre(n, x.ctypes.data_as(_dp), w.ctypes.data_as(_dp)), "gl")
    return x, w


def legendre_table(lmax: int, mu) -> np.ndarray:
    """P[j][l] = P_l(mu_j), l = 0..lmax."""
    mu, pm = _d(mu)
    P = np.empty((mu.size, lmax + 1))
    lib().or_legendre_table(lmax, mu.size, pm, P.ctypes.data_as(_dp))
    return P


def sph_bessel_table(lmax: int, x) -> np.ndarray:
    """J[i][l] = j_l(x_i), l = 0..lmax (Appendix: projection kernel)."""
    x, px = _d(x)
    J = np.empty((x.size, lmax + 1))
    _check(lib().or_sph_bessel_table(lmax, x.size, px, J.ctypes.data_as(_dp)), "sph_bessel")
    return J


def beta(inp, psel=None) -> np.ndarray:
    """beta[s][l - lmin][r] for p = psel[s] (Appendix, projected modes, x 2/pi)."""
    c = inp.cfg
    if psel is None:
        psel = np.arange(inp.qk.shape[0])
    psel, pp = _i(psel)
    k, kp = _d(inp.k)
    wk, wkp = _d(inp.wk)
    r, rp = _d(inp.r)
    qk, qp = _d(inp.qk)
    de, dp = _d(inp.delta)
    out = np.empty((psel.size, c.L, r.size))
    _check(lib().or_beta(c.lmin, c.lmax, k.size, kp, wkp, r.size, rp, qk.shape[0], qp, dp,
                         psel.size, pp, out.ctypes.data_as(_dp)), "beta")
    return out


def weights_l(inp) -> np.ndarray:
    """w_l = (2l+1)^(1 - v_power) / sqrt(C_l) (Sec. 2.2, Eq. (legendre))."""
    l = inp.ells.astype(np.float64)
    return (2 * l + 1) ** (1.0 - inp.cfg.v_power) / np.sqrt(inp.cl)


def S_pairs(inp, mu, beta_arr, pairs) -> np.ndarray:
    """S[s][r][mu] = S_{a p}(r, mu) for (a, b) = pairs[s], b indexing beta_arr."""
    c = inp.cfg
    P = legendre_table(c.lmax, mu)
    pairs, pr = _i(np.asarray(pairs).reshape(-1, 2))
    cl, clp = _d(inp.cl)
    ql, qlp = _d(inp.ql)
    b, bp = _d(beta_arr)
    Pm, Pp = _d(P)
    out = np.empty((pairs.shape[0], c.nr, len(mu)))
    _check(lib().or_S(c.lmin, c.lmax, clp, c.v_power, ql.shape[0], qlp, c.nr, len(mu), Pp,
                      b.shape[0], bp, pairs.shape[0], pr, out.ctypes.data_as(_dp)), "S")
    return out


def _kind_code(kind: str) -> int:
    return 0 if kind == "ordered" else 1


def gamma_from_S(inp, wmu, S_arr, sidx, return_scale=False):
    """Gamma entries from an S stack and per-entry 3x3 index blocks (Eq. (2D)).

    With return_scale, also the per-entry magnitude scale
    c Sum_r wr r^2 Sum_mu wmu Sum_terms |S S S| (the same sums over absolute
    values of every product term): the yardstick of an elementwise check."""
    c = inp.cfg
    S_arr, sp_ = _d(S_arr)
    sidx, sip = _i(np.asarray(sidx).reshape(-1, 9))
    r, rp = _d(inp.r)
    wr, wrp = _d(inp.wr)
    wmu, wmp = _d(wmu)
    out = np.empty(sidx.shape[0])
    scale = np.empty(sidx.shape[0]) if return_scale else None
    _check(lib().or_gamma_entries(_kind_code(c.kind), c.nr, rp, wrp, wmu.size, wmp,
                                  S_arr.shape[0], sp_, sidx.shape[0], sip,
                                  out.ctypes.data_as(_dp),
                                  scale.ctypes.data_as(_dp) if return_scale else None), "gamma")
    return (out, scale) if return_scale else out


def gamma_entries(inp, rows, cols, mu=None, wmu=None, return_S=False, return_scale=False):
    """Gamma[tri_a[rows[e]], tri_p[cols[e]]] computed one entry at a time.

    Only the beta rows and S pairs the requested entries touch are formed.
    With return_scale the result is (values, scales), scales as in
    gamma_from_S; with return_S, (result, S stack, {(a, p): stack index}).
    """
    c = inp.cfg
    if mu is None:
        mu, wmu = gauss_legendre(c.nmu)
    rows = np.asarray(rows, dtype=np.int64).ravel()
    cols = np.asarray(cols, dtype=np.int64).ravel()
    ta = inp.tri_a[rows]
    tp = inp.tri_p[cols]
    pset = np.unique(tp)
    bet = beta(inp, pset)
    ppos = {int(p): i for i, p in enumerate(pset)}
    need = {}
    for e in range(rows.size):
        for s in range(3):
            for t in range(3):
                need.setdefault((int(ta[e, s]), int(tp[e, t])), len(need))
    pairs = np.array([(a, ppos[p]) for (a, p) in need], dtype=np.int32)
    S_arr = S_pairs(inp, mu, bet, pairs)
    sidx = np.empty((rows.size, 9), dtype=np.int32)
    for e in range(rows.size):
        for s in range(3):
            for t in range(3):
                sidx[e, 3 * s + t] = need[(int(ta[e, s]), int(tp[e, t]))]
    g = gamma_from_S(inp, wmu, S_arr, sidx, return_scale=return_scale)
    if return_S:
        return g, S_arr, need
    return g


def gamma_full(inp, mu=None, wmu=None) -> np.ndarray:
    """The whole Gamma[tri_a][tri_p] (small workloads only)."""
    c = inp.cfg
    if mu is None:
        mu, wmu = gauss_legendre(c.nmu)
    na, npm = inp.ql.shape[0], inp.qk.shape[0]
    bet = beta(inp)
    pairs = np.array([(a, p) for a in range(na) for p in range(npm)], dtype=np.int32)
    S_arr = S_pairs(inp, mu, bet, pairs)
    ta, tp = inp.tri_a, inp.tri_p
    A = ta[:, None, :, None] * npm                    # [ta][1][3][1]
    P = tp[None, :, None, :]                          # [1][tp][1][3]
    sidx = (A + P).reshape(-1, 9)
    return gamma_from_S(inp, wmu, S_arr, sidx).reshape(ta.shape[0], tp.shape[0])


def full_S(inp, mu):
    """S[a][p][r][mu] for all pairs (small workloads only)."""
    na, npm = inp.ql.shape[0], inp.qk.shape[0]
    bet = beta(inp)
    pairs = np.array([(a, p) for a in range(na) for p in range(npm)], dtype=np.int32)
    return S_pairs(inp, mu, bet, pairs).reshape(na, npm, inp.cfg.nr, len(mu)), bet


# ------------------------------------------------- adjoint (gradient of a scalar loss)
def gamma_adjoint_S(inp, wmu, S_arr, sidx, g) -> np.ndarray:
    """dL/dS for the S stack S_arr given dL/dGamma_e = g[e] of the entries
    described by sidx (as in gamma_from_S)."""
    c = inp.cfg
    S_arr, sp_ = _d(S_arr)
    sidx, sip = _i(np.asarray(sidx).reshape(-1, 9))
    g, gp = _d(np.asarray(g, dtype=np.float64).ravel())
    r, rp = _d(inp.r)
    wr, wrp = _d(inp.wr)
    wmu, wmp = _d(wmu)
    out = np.empty_like(S_arr)
    _check(lib().or_gamma_adjoint(_kind_code(c.kind), c.nr, rp, wrp, wmu.size, wmp,
                                  S_arr.shape[0], sp_, sidx.shape[0], sip, gp,
                                  out.ctypes.data_as(_dp)), "gamma adjoint")
    return out


def S_adjoint(inp, mu, Shat, pairs, nb) -> np.ndarray:
    """dL/dbeta[b][l][r] from dL/dS of the given (a, b) pairs."""
    c = inp.cfg
    P = legendre_table(c.lmax, mu)
    pairs, pr = _i(np.asarray(pairs).reshape(-1, 2))
    cl, clp = _d(inp.cl)
    ql, qlp = _d(inp.ql)
    Sh, shp = _d(Shat)
    Pm, Pp = _d(P)
    out = np.empty((nb, c.L, c.nr))
    _check(lib().or_S_adjoint(c.lmin, c.lmax, clp, c.v_power, ql.shape[0], qlp, c.nr, len(mu),
                              Pp, nb, pairs.shape[0], pr, shp, out.ctypes.data_as(_dp)),
           "S adjoint")
    return out


def beta_adjoint(inp, bhat):
    """(dL/dq [np][nk], dL/dDelta [L][nk]) from dL/dbeta [np][L][nr]."""
    c = inp.cfg
    k, kp = _d(inp.k)
    wk, wkp = _d(inp.wk)
    r, rp = _d(inp.r)
    qk, qp = _d(inp.qk)
    de, dp = _d(inp.delta)
    bh, bhp = _d(bhat)
    dq = np.empty_like(qk)
    dd = np.empty_like(de)
    _check(lib().or_beta_adjoint(c.lmin, c.lmax, k.size, kp, wkp, r.size, rp, qk.shape[0], qp, dp,
                                 bhp, dq.ctypes.data_as(_dp), dd.ctypes.data_as(_dp)),
           "beta adjoint")
    return dq, dd


def gamma_full_backward(inp, dG, mu=None, wmu=None):
    """Gradient of L with dL/dGamma = dG (shape [ta][tp]) with respect to
    q_p(k) and Delta_l(k): the stage adjoints applied in reverse order."""
    c = inp.cfg
    if mu is None:
        mu, wmu = gauss_legendre(c.nmu)
    na, npm = inp.ql.shape[0], inp.qk.shape[0]
    bet = beta(inp)
    pairs = np.array([(a, p) for a in range(na) for p in range(npm)], dtype=np.int32)
    S_arr = S_pairs(inp, mu, bet, pairs)
    ta, tp = inp.tri_a, inp.tri_p
    sidx = (ta[:, None, :, None] * npm + tp[None, :, None, :]).reshape(-1, 9)
    Shat = gamma_adjoint_S(inp, wmu, S_arr, sidx, np.asarray(dG).ravel())
    bhat = S_adjoint(inp, mu, Shat, pairs, npm)
    return beta_adjoint(inp, bhat)


# ------------------------------------------------- exact 3j and brute force
def threej000_sq(l1: int, l2: int, l3: int) -> float:
    """(l1 l2 l3; 0 0 0)^2 from its closed form in factorials, in exact
    integer arithmetic, rounded once to double.  Zero unless the triangle
    and parity conditions hold (Sec. 2.1)."""
    L = l1 + l2 + l3
    if L % 2 or l3 > l1 + l2 or l1 > l2 + l3 or l2 > l1 + l3:
        return 0.0
    g = L // 2
    f = math.factorial
    num = f(L - 2 * l1) * f(L - 2 * l2) * f(L - 2 * l3) * f(g) ** 2
    den = f(L + 1) * (f(g - l1) * f(g - l2) * f(g - l3)) ** 2
    return num / den


def brute_force_gamma_ordered(inp, beta_arr=None) -> np.ndarray:
    """Ordered Gamma from the inner product of Sec. 2.1 with the exact
    Wigner symbol: a direct sum over every ordered (l1, l2, l3) in
    [lmin, lmax]^3 of

        C(l1,l2,l3) * prod_s qbar_{a_s}(l_s) * Sum_r wr r^2 prod_s beta_{p_s}(l_s, r),
        C = 2 (l1 l2 l3; 000)^2 / (8 pi) * w_l1 w_l2 w_l3

    (h^2 / (v1 v2 v3)^2 * v1 v2 v3 / sqrt(C1 C2 C3) with
    h^2 = prod(2l+1)/(4 pi) (3j)^2 gives the 2/(8 pi) and w_l).  No
    Legendre polynomials and no mu quadrature appear.  The triple sum is
    evaluated, for each r, as three successive tensordot contractions of
    the dense coefficient tensor C with U_r[l, (a, p)] = qbar_a(l) beta_p(l, r).
    Only the ordered-triple lists of an ordered workload are supported.
    """
    c = inp.cfg
    if beta_arr is None:
        beta_arr = beta(inp)
    L = c.L
    C = np.zeros((L, L, L))
    cache = {}
    for i1 in range(L):
        for i2 in range(L):
            for i3 in range(L):
                key = tuple(sorted((i1 + c.lmin, i2 + c.lmin, i3 + c.lmin)))
                if key not in cache:
                    cache[key] = threej000_sq(*key)
                C[i1, i2, i3] = cache[key]
    w = weights_l(inp)
    C *= 2.0 / (8.0 * math.pi) * w[:, None, None] * w[None, :, None] * w[None, None, :]
    na, npm = inp.ql.shape[0], beta_arr.shape[0]
    G = np.zeros((na, npm, na, npm, na, npm))
    for q in range(c.nr):
        U = inp.ql.T[:, :, None] * beta_arr[:, :, q].T[:, None, :]     # [l][a][p]
        T1 = np.tensordot(C, U, axes=([2], [0]))                        # [l1][l2][a3][p3]
        T2 = np.tensordot(T1, U, axes=([1], [0]))                       # [l1][a3][p3][a2][p2]
        T3 = np.tensordot(U, T2, axes=([0], [0]))                       # [a1][p1][a3][p3][a2][p2]
        G += inp.wr[q] * inp.r[q] ** 2 * T3.transpose(0, 1, 4, 5, 2, 3)
    G = G.reshape(na, npm, na, npm, na, npm)
    ta, tp = inp.tri_a, inp.tri_p
    return G[ta[:, 0][:, None], tp[:, 0][None, :], ta[:, 1][:, None], tp[:, 1][None, :],
             ta[:, 2][:, None], tp[:, 2][None, :]]


# ---------------------------------------------------------------- the full Gamma
# Gamma = <Q, Q>^-1 <Q, Q~> (Appendix): the late-time Gram matrix <Q_n, Q_m>
# is the inner product of Sec. 2.1 between two late-time modes.  With h^2 as
# the Gauss-Legendre mu integral (Sec. 2.2) it separates like Eq. (2D), with
# G_ab(mu) = Sum_l (2l+1) / v_l^2 qbar_a(l) qbar_b(l) P_l(mu) in place of
# P_ii'(r, mu) and no r integral.


def gram_G(inp, mu) -> np.ndarray:
    """G[a][b][j] = Sum_l (2l+1)^(1 - 2 v_power) qbar_a(l) qbar_b(l) P_l(mu_j)."""
    c = inp.cfg
    P = legendre_table(c.lmax, mu)[:, c.lmin:]                      # [mu][l - lmin]
    l = inp.ells.astype(np.float64)
    W = (2 * l + 1) ** (1.0 - 2.0 * c.v_power)
    # for each a, a product over l of the rows W qbar_a qbar_b with the P table
    return np.stack([(inp.ql * (W * inp.ql[a])) @ P.T for a in range(inp.ql.shape[0])])


def gram_entries(inp, rows, cols, mu=None, wmu=None) -> np.ndarray:
    """<Q_n, Q_m> for n = tri_a[rows[e]], m = tri_a[cols[e]]: the mu sum of
    the product (ordered lists, constant 1/(8 pi)) or of the permanent of the
    3x3 block G[n_s][m_t] (symmetric lists, 1/(48 pi))."""
    c = inp.cfg
    if mu is None:
        mu, wmu = gauss_legendre(c.nmu)
    G = gram_G(inp, mu)
    ta = inp.tri_a
    out = np.empty(len(rows))
    for e, (n, m) in enumerate(zip(rows, cols)):
        a, b = ta[n], ta[m]
        M = [[G[a[s], b[t]] for t in range(3)] for s in range(3)]
        if c.kind == "ordered":
            f = M[0][0] * M[1][1] * M[2][2]
            out[e] = (wmu * f).sum() / (8.0 * math.pi)
        else:
            f = np.zeros_like(wmu)
            for sg in ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)):
                f = f + M[0][sg[0]] * M[1][sg[1]] * M[2][sg[2]]
            out[e] = (wmu * f).sum() / (48.0 * math.pi)
    return out


def gram_full(inp, mu=None, wmu=None) -> np.ndarray:
    """The whole Gram matrix [ta][ta] (small workloads only)."""
    n = inp.tri_a.shape[0]
    rows, cols = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return gram_entries(inp, rows.ravel(), cols.ravel(), mu, wmu).reshape(n, n)


def gamma_modal(inp) -> np.ndarray:
    """Gamma = <Q, Q>^-1 Gamma' (Gamma' = gamma_full), a dense linear solve."""
    return np.linalg.solve(gram_full(inp), gamma_full(inp))


def brute_force_gram_ordered(inp) -> np.ndarray:
    """Ordered Gram matrix straight from the inner product of Sec. 2.1 with
    the exact Wigner symbol: Sum over every ordered (l1, l2, l3) of

        2 (l1 l2 l3; 000)^2 / (8 pi) * prod_s (2 l_s + 1)^(1 - 2 v_power)
            * prod_s qbar_{a_s}(l_s) qbar_{b_s}(l_s)

    (h^2 / (v1 v2 v3)^2 with h^2 = prod(2l+1)/(4 pi) (3j)^2).  No Legendre
    polynomials and no mu quadrature appear."""
    c = inp.cfg
    L = c.L
    C = np.zeros((L, L, L))
    cache = {}
    for i1 in range(L):
        for i2 in range(L):
            for i3 in range(L):
                key = tuple(sorted((i1 + c.lmin, i2 + c.lmin, i3 + c.lmin)))
                if key not in cache:
                    cache[key] = threej000_sq(*key)
                C[i1, i2, i3] = cache[key]
    l = inp.ells.astype(np.float64)
    W = (2 * l + 1) ** (1.0 - 2.0 * c.v_power)
    C *= 2.0 / (8.0 * math.pi) * W[:, None, None] * W[None, :, None] * W[None, None, :]
    na = inp.ql.shape[0]
    U = inp.ql.T[:, :, None] * inp.ql.T[:, None, :]                  # [l][a][b]
    T1 = np.tensordot(C, U, axes=([2], [0]))                         # [l1][l2][a3][b3]
    T2 = np.tensordot(T1, U, axes=([1], [0]))                        # [l1][a3][b3][a2][b2]
    T3 = np.tensordot(U, T2, axes=([0], [0]))                        # [a1][b1][a3][b3][a2][b2]
    G = T3.transpose(0, 1, 4, 5, 2, 3)
    ta = inp.tri_a
    return G[ta[:, 0][:, None], ta[:, 0][None, :], ta[:, 1][:, None], ta[:, 1][None, :],
             ta[:, 2][:, None], ta[:, 2][None, :]]


# ---- r rules (Modal3D algorithmic change, Eq. (hermite)) -------------------

def r_rule_integral(rule: str, r, y) -> float:
    """Integral of y(r) over [r[0], r[-1]] from its samples, interval by
    interval.  "trapezoid": the chord of each interval.  "hermite": the cubic
    Hermite interpolant of Eq. (hermite) on each interval [r_k, r_{k+1}],

        p = h00(t) y_k + h10(t) D p'_k + h01(t) y_{k+1} + h11(t) D p'_{k+1},
        t = (r - r_k) / D,  D = r_{k+1} - r_k,
        h00 = 2t^3 - 3t^2 + 1, h10 = t^3 - 2t^2 + t, h01 = -2t^3 + 3t^2,
        h11 = t^3 - t^2,

    with D on both derivative terms (the printed equation drops it on the
    second), the derivative at r_k taken as the chord slope of interval k and,
    at the last node, as that of the last interval.  Each cubic is integrated
    by 3-point Gauss-Legendre in t, which is exact for it."""
    r = np.asarray(r, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = r.size
    total = 0.0
    if rule == "trapezoid":
        for k in range(n - 1):
            total += 0.5 * (r[k + 1] - r[k]) * (y[k] + y[k + 1])
        return total
    if rule != "hermite":
        raise ValueError(rule)
    slope = [(y[k + 1] - y[k]) / (r[k + 1] - r[k]) for k in range(n - 1)]
    slope.append(slope[-1])                       # the last node
    tq = 0.5 + 0.5 * np.array([-math.sqrt(0.6), 0.0, math.sqrt(0.6)])
    wq = 0.5 * np.array([5.0, 8.0, 5.0]) / 9.0    # on [0, 1]
    for k in range(n - 1):
        D = r[k + 1] - r[k]
        for t, wt in zip(tq, wq):
            p = ((2 * t**3 - 3 * t**2 + 1) * y[k] + (t**3 - 2 * t**2 + t) * D * slope[k]
                 + (-2 * t**3 + 3 * t**2) * y[k + 1] + (t**3 - t**2) * D * slope[k + 1])
            total += D * wt * p
    return total


# ---- Eq. (3D): the direct sum over l-triples (Modal3D) ----------------------

def threej000_sq_gosper(l1: int, l2: int, l3: int) -> float:
    """The Gosper-factorial approximation of (l1 l2 l3; 0 0 0)^2 that
    Eq. (3D) carries (its h^2 divided by prod(2l+1) / (4 pi)): with
    L = l1 + l2 + l3 and L_i = L - 2 l_i,

        (2/pi) (L + 1/3) / ((L + 1) prod_i (L_i + 1/3))
             * sqrt(prod_i (L_i + 1/6) / (L + 1/6)),

    zero unless the triangle and parity conditions hold."""
    L = l1 + l2 + l3
    if L % 2 or l3 > l1 + l2 or l1 > l2 + l3 or l2 > l1 + l3:
        return 0.0
    Li = (L - 2 * l1, L - 2 * l2, L - 2 * l3)
    num = (L + 1.0 / 3.0) * math.sqrt((Li[0] + 1.0 / 6.0) * (Li[1] + 1.0 / 6.0) * (Li[2] + 1.0 / 6.0)
                                      / (L + 1.0 / 6.0))
    den = (L + 1.0) * (Li[0] + 1.0 / 3.0) * (Li[1] + 1.0 / 3.0) * (Li[2] + 1.0 / 3.0)
    return 2.0 / math.pi * num / den


def gamma_3d(inp, weight: str = "exact", beta_arr=None) -> np.ndarray:
    """Gamma' of Eq. (3D), summed the way the equation and Listing 2 lay it
    out: over sorted triples l1 <= l2 <= l3 <= min(l1 + l2, lmax) with an even
    sum, each counted with the number of distinct orderings of the triple
    (the summand of the symmetric form is symmetric in the l_i), of

        h^2 / (v1 v2 v3 sqrt(C1 C2 C3)) = w_l1 w_l2 w_l3 (3j)^2 / (4 pi)

    times the late-time product and the r integral of the primordial one.
    Symmetric lists: both products summed over the six permutations, and the
    1/36 of the two symmetrisations (Eq. (3D)'s 1/(72 pi^2) with the
    Gosper form of h^2).  Ordered lists: the plain products
    qbar_a1(l1) qbar_a2(l2) qbar_a3(l3) and beta_p1 beta_p2 beta_p3, summed
    over every distinct ordering of the sorted triple.  weight: "exact"
    (exact 3j, integer arithmetic) or "gosper" (the approximation printed in
    Eq. (3D))."""
    import itertools
    c = inp.cfg
    if beta_arr is None:
        beta_arr = beta(inp)
    w3j = threej000_sq if weight == "exact" else threej000_sq_gosper
    wl = weights_l(inp)
    x_r = inp.wr * inp.r ** 2                                   # r weights with r^2
    ta, tp = inp.tri_a, inp.tri_p
    sym = c.kind == "symmetric"
    perms = list(itertools.permutations(range(3)))
    out = np.zeros((ta.shape[0], tp.shape[0]))
    for l1 in range(c.lmin, c.lmax + 1):
        for l2 in range(l1, c.lmax + 1):
            for l3 in range(l2 + l1 % 2, min(l1 + l2, c.lmax) + 1, 2):
                ls = (l1, l2, l3)
                wt = w3j(*ls)
                if wt == 0.0:
                    continue
                i = [l - c.lmin for l in ls]
                h2 = wl[i[0]] * wl[i[1]] * wl[i[2]] * wt / (4.0 * math.pi)
                q = inp.ql[:, i].T                               # [3][na]
                b = beta_arr[:, i, :].transpose(1, 0, 2)         # [3][np][nr]
                orders = set(itertools.permutations(ls)) if not sym else {ls}
                for lo in orders:
                    # resolve repeated values: map each slot to a position of ls
                    pos, used = [], set()
                    for x in lo:
                        k = next(k for k in range(3) if ls[k] == x and k not in used)
                        used.add(k)
                        pos.append(k)
                    if sym:
                        Q = sum(q[s[0], ta[:, 0]] * q[s[1], ta[:, 1]] * q[s[2], ta[:, 2]] for s in perms)
                        X = sum((b[s[0], tp[:, 0]] * b[s[1], tp[:, 1]] * b[s[2], tp[:, 2]]) @ x_r
                                for s in perms)
                        mult = len(set(itertools.permutations(ls)))
                        out += (mult * h2 / 36.0) * np.outer(Q, X)
                    else:
                        Q = q[pos[0], ta[:, 0]] * q[pos[1], ta[:, 1]] * q[pos[2], ta[:, 2]]
                        X = (b[pos[0], tp[:, 0]] * b[pos[1], tp[:, 1]] * b[pos[2], tp[:, 2]]) @ x_r
                        out += h2 * np.outer(Q, X)
    return out
