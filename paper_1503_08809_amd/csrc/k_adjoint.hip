// Adjoint of the projection: the gradient of a scalar loss L of Gamma with
// respect to the primordial basis q_p(k) and the transfer table Delta_l(k),
// given G = dL/dGamma.  The forward stages are differentiated in reverse
// order (Eq. (2D) -> Eq. (legendre) -> Appendix projected modes); the j_l
// tables are regenerated in l chunks, never stored.
//
// Step d.  Gamma is a sum of entries of T[u1,u2,u3] = Sum_z St_u1 St_u2 St_u3
// (St = W^(1/3) S), so with H the symmetric tensor of dL/dT,
//     dL/dSt_u(z) = 3 Sum_{v,w} H[u,v,w] St_v(z) St_w(z).
// Here H is evaluated entry by entry from G (each entry gathers the Gamma
// entries it feeds; no atomics) straight into the operand order of the
// kernels (k_adjoint_fac64.hip, k_adjoint_fac.hip) as
// Hc[u][(v,w)] = 3 c_vw H[u,v,w] over pairs v <= w, and dL/dS = W^(1/3) dL/dSt.
// Step c.  betahat_p(l, r) = Sum_{a, mu} [w_l qbar_a(l) P_l(mu)] Shat_ap(r, mu):
//   per p and per parity of l, one GEMM with the (a, mu >= 0) depth, a
//   generated A operand and the mu-symmetrised dL/dS as B operand.
// Step b.  Ahat_l[p, k] = Sum_r betahat_p(l, r) j_l(k r) per l on regenerated
//   j_l chunks; then dq_p(k) = Sum_l c_k Delta_l(k) Ahat_l[p, k] and
//   dDelta_l(k) = c_k Sum_p q_p(k) Ahat_l[p, k], c_k = (2/pi) wk k^2, with the
//   l chunks accumulated in a fixed order (deterministic).
#include "gemm64.hpp"

#include <algorithm>

namespace mp {
namespace {
using gemm::run;

// ---- H from G -----------------------------------------------------------------
// number of orderings of a triple that leave it unchanged
__device__ __forceinline__ int fixers(int a, int b, int c)
{
    if (a == b && b == c) return 6;
    if (a == b || b == c || a == c) return 2;
    return 1;
}

__device__ __forceinline__ void sort3(int &a, int &b, int &c)
{
    int lo = min(a, min(b, c)), hi = max(a, max(b, c));
    b = a + b + c - lo - hi;
    a = lo;
    c = hi;
}

// H[u1,u2,u3] (symmetric) for rows u = a * np + p
__device__ double adj_h(int kind, int np, int na, const int *__restrict__ inv_a, const int *__restrict__ inv_p,
                        const double *__restrict__ G, int tp, int u1, int u2, int u3)
{
    const int al[3] = {u1 / np, u2 / np, u3 / np};
    const int rh[3] = {u1 % np, u2 % np, u3 % np};
    double h = 0.0;
    if (kind == MODAL_GAMMA_ORDERED) {
        // Gamma_ord[n, m] = T(u(a1,p1), u(a2,p2), u(a3,p3)) / (8 pi): the six
        // orderings of (u1, u2, u3) each name at most one (n, m)
        const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
#pragma unroll
        for (int s = 0; s < 6; ++s) {
            const int *pi = perm[s];
            const int n = inv_a[(al[pi[0]] * na + al[pi[1]]) * na + al[pi[2]]];
            const int m = inv_p[(rh[pi[0]] * np + rh[pi[1]]) * np + rh[pi[2]]];
            if (n >= 0 && m >= 0) h += G[(size_t)n * tp + m];
        }
        h *= 1.0 / (6.0 * 8.0 * kPi);
    } else {
        // Gamma_sym sums over every pairing of a with p, so H depends only on
        // the sorted a and sorted p triples, with their fixer counts
        int a0 = al[0], a1 = al[1], a2 = al[2], p0 = rh[0], p1 = rh[1], p2 = rh[2];
        sort3(a0, a1, a2);
        sort3(p0, p1, p2);
        const int n = inv_a[(a0 * na + a1) * na + a2];
        const int m = inv_p[(p0 * np + p1) * np + p2];
        if (n >= 0 && m >= 0)
            h = G[(size_t)n * tp + m] * fixers(a0, a1, a2) * fixers(p0, p1, p2) * (1.0 / (6.0 * 48.0 * kPi));
    }
    return h;
}

__device__ __forceinline__ uint32_t bf16_bits(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

// Hc[u][(v,w)] = 3 c_vw H[u,v,w] (c = 2 for v < w, 1 for v = w), split into
// BF16 hi and lo, for the factored mixed kernel: per v, the w steps from the one
// holding v to the last ([v_step_offset(v) + ws'][row block of 256][row
// tile][hi/lo][lane], lane: row 16-tile + lane % 16, w = 32 ws + 8 (lane / 16)
// .. + 7); entries with w < v are zero.  blockIdx.y = v.
__global__ void k_build_hc_fac(int kind, int U, int np, int na, const int *__restrict__ inv_a,
                               const int *__restrict__ inv_p, const double *__restrict__ G, int tp, int nws,
                               int nib, uint4 *__restrict__ Hc)
{
    const int v = blockIdx.y;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = (int)(e & 63), rt = (int)((e >> 6) & 15);
    const int64_t r = e >> 10;
    const int ib = (int)(r % nib), wsr = (int)(r / nib);
    const int ws = (v >> 5) + wsr;
    if (ws >= nws) return;
    const int u = ib * 256 + rt * 16 + (lane & 15);
    float x[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int w = 32 * ws + 8 * (lane >> 4) + q;
        double h = 0.0;
        if (u < U && w < U && w >= v)
            h = (w > v ? 6.0 : 3.0) * adj_h(kind, np, na, inv_a, inv_p, G, tp, u, v, w);
        x[q] = (float)h;
    }
    uint32_t hi[4], lo[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t h0 = bf16_bits(x[2 * q]), h1 = bf16_bits(x[2 * q + 1]);
        hi[q] = h0 | (h1 << 16);
        lo[q] = bf16_bits(x[2 * q] - __uint_as_float(h0 << 16)) |
                (bf16_bits(x[2 * q + 1] - __uint_as_float(h1 << 16)) << 16);
    }
    const int64_t st = v_step_offset(v, nws) + wsr;
    uint4 *o = Hc + (((size_t)st * nib + ib) * 16 + rt) * 128 + lane;
    o[0] = make_uint4(hi[0], hi[1], hi[2], hi[3]);
    o[64] = make_uint4(lo[0], lo[1], lo[2], lo[3]);
}

// The same Hc in FP64 for the FP64 factored kernel: per v, the 16-wide w
// steps from the one holding v to the last ([v_step_offset16(v) + ws'][row
// block of 128][row tile 8][k pair 2][lane][2]; lane: row 16 tile + lane % 16,
// w = 16 ws + 4 k + lane / 16 with k = 2 (k pair) + the last index), so that
// one row tile is 2 KB in a row and a lane's two k of one pair are adjacent;
// entries with w < v are zero.  blockIdx.y = v.
__global__ void k_build_hc_fac64(int kind, int U, int np, int na, const int *__restrict__ inv_a,
                                 const int *__restrict__ inv_p, const double *__restrict__ G, int tp, int nws,
                                 int nib, double *__restrict__ Hc)
{
    const int v = blockIdx.y;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int el = (int)(e & 1), lane = (int)((e >> 1) & 63), kp = (int)((e >> 7) & 1), rt = (int)((e >> 8) & 7);
    const int64_t r = e >> 11;
    const int ib = (int)(r % nib), wsr = (int)(r / nib);
    const int ws = (v >> 4) + wsr;
    if (ws >= nws) return;
    const int u = ib * 128 + rt * 16 + (lane & 15);
    const int w = 16 * ws + 4 * (2 * kp + el) + (lane >> 4);
    double h = 0.0;
    if (u < U && w < U && w >= v) h = (w > v ? 6.0 : 3.0) * adj_h(kind, np, na, inv_a, inv_p, G, tp, u, v, w);
    Hc[((size_t)(v_step_offset16(v, nws) + wsr) * nib + ib) * 2048 + (e & 2047)] = h;
}

// ---- betahat ------------------------------------------------------------------
// The same contraction using the mu parity of P_l at nodes symmetric about
// 0: Sum_mu P_l(mu) X(mu) = Sum_{mu >= 0} P_l(mu) [X(mu) + (-1)^l X(-mu)]
// (the node mu = 0, if any, counted once), so the rows l of one parity are
// one product over (a, mu >= 0): half the work.  Rows li0, li0 + 2, ...
// n / d for 0 <= n < 2^31 and 1 <= d < 10^6 without an integer division:
// n / d is formed in FP64 with absolute error below 2^-22, and the offset
// 2^-20 < 1 / d lifts exact quotients clear of it without reaching the next
// integer.
struct DivBy {
    int d;
    double inv;
    __device__ int quot(int n) const { return (int)((double)n * inv + 0x1p-20); }
};

// The mu fold of X = W^(1/3) dL/dSt, in place, once for both parities: for
// each row u, r and node pair (+mu, -mu) = (ioff + jj, nh - 1 - jj), the
// position of +mu receives X(+mu) + X(-mu) and the position of -mu receives
// X(+mu) - X(-mu); the node mu = 0 (odd nmu: its own mirror) keeps X(0).
__global__ void k_fold_mu(int U, int nr, int ldmu, int nh, int ioff, int64_t upad, const double *__restrict__ wz,
                          double *__restrict__ Shat)
{
    const int64_t n = (int64_t)U * nr * nh;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int jj = (int)(e % nh);
        const int64_t t = e / nh;
        const int r = (int)(t % nr);
        const int64_t u = t / nr;
        const int64_t zp = (int64_t)r * ldmu + ioff + jj, zm = (int64_t)r * ldmu + nh - 1 - jj;
        const int64_t ip = (((zp >> 5) * upad + u) << 5) + (zp & 31);
        const double xp = wz[zp] * Shat[ip];
        if (zp == zm) {
            Shat[ip] = xp;
        } else {
            const int64_t im = (((zm >> 5) * upad + u) << 5) + (zm & 31);
            const double xm = wz[zm] * Shat[im];
            Shat[ip] = xp + xm;
            Shat[im] = xp - xm;
        }
    }
}

struct BetaHatParOp {
    static constexpr bool a_k_fast = true;    // (a, mu >= 0) with mu contiguous
    static constexpr bool b_k_fast = true;
    int M, N, K;                              // rows of this parity, nr, na * nh
    int np, ldmu, nh, ioff, L, li0;
    DivBy bynh;                               // kk -> (a, mu index)
    int odd;                                  // l odd for these rows
    int64_t upad;
    const double *wl, *ql, *P, *Shat;
    double *bhat;
    struct RawA { double w, q, p; };
    struct RawB { double x, c; };
    __device__ RawA fa(int, int m, int kk) const
    {
        const int ia = bynh.quot(kk), jj = kk - ia * nh, li = li0 + 2 * m;
        return RawA{wl[li], ql[(size_t)ia * L + li], P[(size_t)li * ldmu + ioff + jj]};
    }
    __device__ double ma(const RawA &v) const { return v.w * v.q * v.p; }
    // X(+mu) + (-1)^l X(-mu) from the folded array: at the position of +mu
    // for even l, of -mu for odd l; at the node mu = 0 X counts once, and
    // only for even l
    __device__ RawB fb(int p, int kk, int r) const
    {
        const int ia = bynh.quot(kk), jj = kk - ia * nh;
        const size_t u = (size_t)ia * np + p;
        const int zo = odd ? nh - 1 - jj : ioff + jj;
        const int64_t z = (int64_t)r * ldmu + zo;
        return RawB{Shat[(((size_t)(z >> 5) * upad + u) << 5) + (z & 31)], odd && ioff + jj == zo ? 0.0 : 1.0};
    }
    __device__ double mb(const RawB &v) const { return v.c * v.x; }
    __device__ void store(int p, int m, int r, double v) const
    {
        bhat[((size_t)p * L + li0 + 2 * m) * N + r] = v;
    }
};

// ---- Ahat per l chunk -------------------------------------------------------------
struct AhatOp {
    static constexpr bool a_k_fast = true;    // bhat[p][l][r]
    static constexpr bool b_k_fast = false;   // J[l][r][k]: k contiguous
    int M, N, K;                              // np, nk, nr
    int l0, lmin, L;
    const double *bhat, *J;
    double *Ahat;                             // [l - l0][p][k]
    using RawA = double;
    using RawB = double;
    __device__ RawA fa(int b, int p, int r) const { return bhat[((size_t)p * L + (l0 + b - lmin)) * K + r]; }
    __device__ double ma(RawA v) const { return v; }
    __device__ RawB fb(int b, int r, int k) const { return J[((size_t)b * K + r) * N + k]; }
    __device__ double mb(RawB v) const { return v; }
    __device__ void store(int b, int p, int k, double v) const { Ahat[((size_t)b * M + p) * N + k] = v; }
};

// One thread per (row, k): rows 0..np-1 accumulate dq_p(k) over the chunk's
// l values (in a fixed order, added to the running sum of earlier chunks),
// rows np..np+nl-1 write dDelta_l(k) for the chunk's l values.
__global__ void k_dq_ddelta(int nl, int l0, int lmin, int np, int nk, const double *__restrict__ k,
                            const double *__restrict__ wk, const double *__restrict__ qk,
                            const double *__restrict__ delta, const double *__restrict__ Ahat,
                            double *__restrict__ dq, double *__restrict__ dd, int first)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int row = blockIdx.y;
    if (i >= nk) return;
    const double ck = (2.0 / kPi) * wk[i] * k[i] * k[i];
    if (row < np) {
        if (!dq) return;
        const int p = row;
        double acc = 0.0;
        for (int b = nl - 1; b >= 0; --b)
            acc += delta[(size_t)(l0 + b - lmin) * nk + i] * Ahat[((size_t)b * np + p) * nk + i];
        dq[(size_t)p * nk + i] = (first ? 0.0 : dq[(size_t)p * nk + i]) + ck * acc;
    } else {
        if (!dd) return;
        const int b = row - np;
        double acc = 0.0;
        for (int p = 0; p < np; ++p) acc += qk[(size_t)p * nk + i] * Ahat[((size_t)b * np + p) * nk + i];
        dd[(size_t)(l0 + b - lmin) * nk + i] = ck * acc;
    }
}

}  // namespace

hipError_t launch_build_hc_fac(int kind, int U, int np, int na, const int *inv_a, const int *inv_p,
                               const double *G, int tp, int nib, uint4 *Hc, hipStream_t s)
{
    const int nws = (U + 31) / 32;
    const int64_t n = (int64_t)nws * nib * 16 * 64;
    if (U > 65535) return hipErrorInvalidValue;     // grid y limit
    hipLaunchKernelGGL(k_build_hc_fac, dim3((unsigned)((n + 255) / 256), (unsigned)U), dim3(256), 0, s, kind, U,
                       np, na, inv_a, inv_p, G, tp, nws, nib, Hc);
    return hipGetLastError();
}

hipError_t launch_build_hc_fac64(int kind, int U, int np, int na, const int *inv_a, const int *inv_p,
                                 const double *G, int tp, int nib, double *Hc, hipStream_t s)
{
    const int nws = (U + 15) / 16;
    const int64_t n = (int64_t)nws * nib * 2048;
    if (U > 65535) return hipErrorInvalidValue;     // grid y limit
    if ((n + 255) / 256 > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_build_hc_fac64, dim3((unsigned)((n + 255) / 256), (unsigned)U), dim3(256), 0, s, kind, U,
                       np, na, inv_a, inv_p, G, tp, nws, nib, Hc);
    return hipGetLastError();
}

hipError_t launch_betahat(int na, int np, int nr, int nmu, int ldmu, int L, int lmin, int64_t upad,
                          const double *wl, const double *ql, const double *P, double *Shat,
                          const double *wz, double *bhat, hipStream_t s)
{
    const int nh = (nmu + 1) / 2, ioff = nmu - nh;
    {
        const int64_t n = (int64_t)na * np * nr * nh;
        const int64_t blocks = std::min<int64_t>((n + 255) / 256, 1 << 20);
        if (blocks > 0)
            hipLaunchKernelGGL(k_fold_mu, dim3((unsigned)blocks), dim3(256), 0, s, na * np, nr, ldmu, nh, ioff, upad,
                               wz, Shat);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    // rows of each parity of l: li with (lmin + li) even, then odd
    for (int par = 0; par < 2; ++par) {
        const int li0 = (par - lmin) & 1;
        const int rows = L > li0 ? (L - li0 + 1) / 2 : 0;
        if (rows == 0) continue;
        BetaHatParOp op{rows, nr, na * nh, np, ldmu, nh, ioff, L, li0, DivBy{nh, 1.0 / nh}, par,
                        upad, wl, ql, P, Shat, bhat};
        const hipError_t e = run(op, np, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_ahat(int nl, int l0, int lmin, int L, int np, int nk, int nr, const double *bhat,
                       const double *J, double *Ahat, hipStream_t s)
{
    AhatOp op{np, nk, nr, l0, lmin, L, bhat, J, Ahat};
    return run(op, nl, s);
}

hipError_t launch_dq_ddelta(int nl, int l0, int lmin, int np, int nk, const double *k, const double *wk,
                            const double *qk, const double *delta, const double *Ahat, double *dq,
                            double *dd, int first, hipStream_t s)
{
    if (np + nl > 65535) return hipErrorInvalidValue;       // grid y limit
    hipLaunchKernelGGL(k_dq_ddelta, dim3((nk + 127) / 128, np + nl), dim3(128), 0, s, nl, l0, lmin, np, nk, k,
                       wk, qk, delta, Ahat, dq, dd, first);
    return hipGetLastError();
}

}  // namespace mp
