"""Seeded synthetic inputs for the separable bispectrum projection.

This module builds the *inputs* of the projection (grids, quadrature
weights on the k and r grids, a synthetic transfer table Delta_l(k), a
synthetic power spectrum C_l, the two 1-D mode bases and the mode-triple
lists).  It holds none of the projection's arithmetic: it never forms
j_l tables, beta, S or Gamma, and it is shared, unchanged, by the test
oracle and by the GPU path so that both see bit-identical inputs.

The physical inputs of the paper (Planck transfer functions, its
optimised mode basis and its pre-computed n -> ijk list, Appendix) are not
available; the synthetic stand-ins below have the shapes and value
structure of the paper's workloads (l_max ~ 2000-4000, ~200-600 radial
points clustered at the last-scattering distance r ~ 14000 Mpc, thousands
of Gauss-Legendre mu nodes, tens of 1-D modes per side; Sec. 2.1 and
Sec. 3.1.3).

Library routines used here (numpy Legendre-series evaluation for the
bases, scipy's spherical Bessel function for the *shape* of the synthetic
transfer table, scipy's normal quantile for the clustered r grid) are
input-construction only.
"""
from __future__ import annotations

import dataclasses
import numpy as np

SEED = 150308809
R_STAR = 14000.0          # last-scattering distance (Mpc) the r grid clusters on


@dataclasses.dataclass(frozen=True)
class Config:
    """One workload: sizes, ranges and damping scales."""
    name: str
    lmax: int
    nk: int
    kmin: float
    kmax: float
    nr: int
    r_kind: str            # "uniform" or "gauss"
    r_lo: float            # uniform: lower end; gauss: unused
    r_hi: float            # uniform: upper end; gauss: unused
    r_sigma: float         # gauss: width of the density (Mpc)
    nmu: int
    k_damp: float
    l_damp: float
    n1: int                # Np = Na
    kind: str              # "ordered" or "symmetric"
    seed_index: int        # c in SEED + 10 c + {1, 2, 3}
    lmin: int = 2
    v_power: float = 1.0 / 6.0

    @property
    def L(self) -> int:
        return self.lmax - self.lmin + 1

    @property
    def noise_seed(self) -> int:
        return SEED + 10 * self.seed_index + 1

    @property
    def weight_seed(self) -> int:
        return SEED + 10 * self.seed_index + 2

    @property
    def pick_seed(self) -> int:
        return SEED + 10 * self.seed_index + 3


# The five standard workloads.  Values the workload descriptions leave
# open are pinned here (k range of the lmax=2500 case, the lmax=1000 case's
# k range and damping scales, and sigma_r = 300 Mpc for every clustered
# grid).
CONFIGS = {
    1: Config("lmax64_ordered_n8", 64, 256, 1e-4, 0.05, 32, "uniform", 13500.0, 14500.0, 0.0,
              97, 0.02, 50.0, 8, "ordered", 1),
    2: Config("lmax500_ordered_n16", 500, 1000, 1e-5, 0.1, 200, "gauss", 0.0, 0.0, 300.0,
              752, 0.02, 400.0, 16, "ordered", 2),
    3: Config("lmax2500_symmetric_n30", 2500, 2000, 1e-5, 0.3, 400, "gauss", 0.0, 0.0, 300.0,
              3752, 0.15, 1500.0, 30, "symmetric", 3),
    4: Config("lmax1000_symmetric_n20", 1000, 1500, 1e-5, 0.12, 300, "gauss", 0.0, 0.0, 300.0,
              1502, 0.06, 600.0, 20, "symmetric", 4),
    5: Config("lmax4000_symmetric_n40", 4000, 3000, 1e-5, 0.3, 600, "gauss", 0.0, 0.0, 300.0,
              6002, 0.25, 2500.0, 40, "symmetric", 5),
}


def workload(name: str) -> Config:
    """A standard workload by its name (e.g. "lmax2500_symmetric_n30")."""
    for c in CONFIGS.values():
        if c.name == name:
            return c
    raise KeyError(name)


def small_config(lmax=40, nk=120, nr=20, nmu=None, n1=8, kind="symmetric", seed_index=90,
                 kmin=1e-4, kmax=0.05, r_kind="uniform", k_damp=0.02, l_damp=None,
                 v_power=1.0 / 6.0) -> Config:
    """A reduced workload of the same structure, for fast tests."""
    if nmu is None:
        nmu = (3 * lmax + 2) // 2 + 1      # one above the exactness minimum
    if l_damp is None:
        l_damp = 0.8 * lmax
    return Config(f"small_l{lmax}_n{n1}_{kind}", lmax, nk, kmin, kmax, nr, r_kind,
                  13500.0, 14500.0, 300.0, nmu, k_damp, l_damp, n1, kind, seed_index,
                  v_power=v_power)


def trapezoid_weights(x: np.ndarray) -> np.ndarray:
    """Trapezoid-rule weights on arbitrary ascending nodes (an input rule:
    the projection itself takes its k and r weights as given)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    w = np.zeros(n)
    if n == 1:
        return w
    d = np.diff(x)
    w[0] = 0.5 * d[0]
    w[-1] = 0.5 * d[-1]
    w[1:-1] = 0.5 * (d[:-1] + d[1:])
    return w


def _legendre_basis(t: np.ndarray, n: int) -> np.ndarray:
    """Rows P_i(t), i < n, via numpy's Legendre-series evaluation."""
    from numpy.polynomial import legendre as npleg
    out = np.empty((n, t.size))
    for i in range(n):
        c = np.zeros(i + 1)
        c[i] = 1.0
        out[i] = npleg.legval(t, c)
    return out


def sym_triples(n: int) -> np.ndarray:
    """Sorted triples i <= j <= k ordered by (k, j, i): 000, 001, 011, 111,
    002, 012, ... (the example mode list of the Appendix)."""
    out = []
    for k in range(n):
        for j in range(k + 1):
            for i in range(j + 1):
                out.append((i, j, k))
    return np.array(out, dtype=np.int32).reshape(-1, 3)


def ordered_triples(n: int) -> np.ndarray:
    """All n^3 ordered triples, row index a1*n^2 + a2*n + a3."""
    g = np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij"), -1)
    return g.reshape(-1, 3).astype(np.int32)


@dataclasses.dataclass
class Inputs:
    cfg: Config
    k: np.ndarray
    wk: np.ndarray
    r: np.ndarray
    wr: np.ndarray
    cl: np.ndarray        # [L]
    delta: np.ndarray     # [L][nk]
    qk: np.ndarray        # [np][nk]
    ql: np.ndarray        # [na][L]
    tri_a: np.ndarray     # [ta][3] int32
    tri_p: np.ndarray     # [tp][3] int32

    @property
    def ells(self) -> np.ndarray:
        return np.arange(self.cfg.lmin, self.cfg.lmax + 1)


def r_grid(cfg: Config) -> np.ndarray:
    if cfg.r_kind == "uniform":
        return np.linspace(cfg.r_lo, cfg.r_hi, cfg.nr)
    from scipy.special import ndtri
    q = (np.arange(cfg.nr) + 0.5) / cfg.nr
    return R_STAR + cfg.r_sigma * ndtri(q)


def make_inputs(cfg: Config, with_delta: bool = True) -> Inputs:
    """Deterministic inputs for a workload (seeded; see module docstring)."""
    from scipy.special import spherical_jn
    ells = np.arange(cfg.lmin, cfg.lmax + 1)
    k = np.geomspace(cfg.kmin, cfg.kmax, cfg.nk)
    wk = trapezoid_weights(k)
    r = r_grid(cfg)
    wr = trapezoid_weights(r)
    lf = ells.astype(np.float64)
    cl = 1e3 / (lf * (lf + 1.0)) * np.exp(-(lf / cfg.l_damp) ** 2)
    if with_delta:
        rng = np.random.Generator(np.random.PCG64(cfg.noise_seed))
        eps = rng.standard_normal((cfg.L, cfg.nk))
        shape = spherical_jn(ells[:, None], k[None, :] * R_STAR)
        delta = shape * np.exp(-(k[None, :] / cfg.k_damp) ** 2) * (1.0 + 0.05 * eps)
    else:
        delta = np.zeros((cfg.L, cfg.nk))
    t = np.log(k / cfg.kmin) / np.log(cfg.kmax / cfg.kmin)
    qk = _legendre_basis(2.0 * t - 1.0, cfg.n1)
    s = 2.0 * (ells - cfg.lmin) / (cfg.lmax - cfg.lmin) - 1.0
    ql = _legendre_basis(s, cfg.n1)
    tri = ordered_triples(cfg.n1) if cfg.kind == "ordered" else sym_triples(cfg.n1)
    return Inputs(cfg, k, wk, r, wr, np.ascontiguousarray(cl), np.ascontiguousarray(delta),
                  np.ascontiguousarray(qk), np.ascontiguousarray(ql), tri.copy(), tri.copy())


def loss_weights(cfg: Config, ta: int, tp: int) -> np.ndarray:
    """Seeded N(0,1) weight matrix W of the scalar loss sum (Gamma * W)^2."""
    rng = np.random.Generator(np.random.PCG64(cfg.weight_seed))
    return rng.standard_normal((ta, tp))


def pick_entries(cfg: Config, shape, count: int, seed_offset: int = 0) -> np.ndarray:
    """Seeded distinct flat indices into an array of the given shape."""
    rng = np.random.Generator(np.random.PCG64(cfg.pick_seed + seed_offset))
    n = int(np.prod(shape))
    return np.sort(rng.choice(n, size=min(count, n), replace=False))
