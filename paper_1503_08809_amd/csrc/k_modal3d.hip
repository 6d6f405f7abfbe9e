// Eq. (3D) (Modal3D): Gamma' from the direct sum over l-triples with h^2
// from the Wigner symbol (exact, or the Gosper form the equation prints), no
// mu integral.
//
// With G_u(l, r) = w_l qbar_a(l) beta_p(l, r), u = a * np + p, the moment
// tensor of the triple products is
//
//   T(u1, u2, u3) = Sum_r wr r^2 Sum_{l1 l2 l3} K(l1, l2, l3) G_u1(l1, r) G_u2(l2, r) G_u3(l3, r),
//   K = 2 (l1 l2 l3; 0 0 0)^2
//
// (the same tensor as the mu moments of Eq. (2D), since the Gauss-Legendre
// integral of P_l1 P_l2 P_l3 is 2 (3j)^2), and Gamma' is its gather over the
// mode lists with 1/(8 pi) (ordered) or the six-term permanent and 1/(48 pi)
// (symmetric).  It is contracted one l at a time, for each l1:
//   A_r(l2, u3) = Sum_l3 K(l1, l2, l3) G_u3(l3, r)          (stage 1)
//   B_r(u2, u3) = Sum_l2 G_u2(l2, r) A_r(l2, u3)            (stage 2)
//   T(u1, u2, u3) += Sum_r wr r^2 G_u1(l1, r) B_r(u2, u3)   (stage 3)
// B_r is symmetric in (u2, u3) and T in all three: stage 2 forms one
// triangle of B_r, packed u2-major, and stage 3 forms T only for rows
// u1 below the end of each 128-wide block of u2 (u1 <= u2 <= u3 is read).
// The l index is stored parity-sorted (even l first): for a given l1, K is
// non-zero only where l1 + l2 + l3 is even, so stage 1 is two dense products
// of half size (one per parity of l2).  The three stages run on the FP64
// matrix-core GEMM (k_dgemm.hip; stage 2 in its packed-triangle form); this
// file holds the operand builders and the gather.
#include "internal.hpp"

#include <algorithm>
#include <cmath>

namespace mp {
namespace {

__device__ __forceinline__ int l_of(int lp, int nE, int lE0, int lO0)
{
    return lp < nE ? lE0 + 2 * lp : lO0 + 2 * (lp - nE);
}

// G[(rb * U + u) * L + l'] for the r batch [r0, r0 + nrb).
__global__ void k_build_g3(int L, int nE, int lE0, int lO0, int lmin, int nr, int np, int na, int r0,
                           int nrb, const double *__restrict__ wl, const double *__restrict__ ql,
                           const double *__restrict__ beta, double *__restrict__ G)
{
    const int U = na * np;
    const int64_t n = (int64_t)L * nrb * U;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int lp = (int)(i % L);
        const int64_t col = i / L;
        const int u = (int)(col % U), rb = (int)(col / U);
        const int a = u / np, p = u % np;
        const int li = l_of(lp, nE, lE0, lO0) - lmin;
        G[i] = wl[li] * ql[(size_t)a * L + li] * beta[((size_t)p * L + li) * nr + r0 + rb];
    }
}

// (l1 l2 l3; 0 0 0)^2 at l3 = |l1 - l2|: with b = max, s = min,
// C(b, s)^2 / ((2b + 1) C(2b, 2s)) = Prod_{j=1..s} (2j - 1)(b - j + 1) / (j (2b - 2j + 1)) / (2b + 1),
// a product of factors of order one.  V[b (b + 1) / 2 + s] holds it for
// 0 <= s <= b <= lmax: one thread per b runs the product over s.
__global__ void k_start3(int lmax, double *__restrict__ V)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b > lmax) return;
    double *row = V + (size_t)b * (b + 1) / 2;
    double v = 1.0 / (2.0 * b + 1.0);
    row[0] = v;
    for (int j = 1; j <= b; ++j) {
        v *= ((2.0 * j - 1.0) * (double)(b - j + 1)) / ((double)j * (2.0 * b - 2.0 * j + 1.0));
        row[j] = v;
    }
}

// (3j)^2 at l3 + 2 over (3j)^2 at l3 (same l1, l2), from the factorial form
// with g = (l1 + l2 + l3) / 2 and L_i = 2g - 2 l_i at l3:
// 2 (L1 + 1)(L2 + 1)(g + 1) L3 / ((L3 - 1)(2g + 3)(L1 + 2)(L2 + 2)).
__device__ __forceinline__ double threej_sq_step(int l1, int l2, int l3)
{
    const double g = 0.5 * (l1 + l2 + l3);
    const double L1 = (double)(l2 + l3 - l1), L2 = (double)(l1 + l3 - l2), L3 = (double)(l1 + l2 - l3);
    return 2.0 * (L1 + 1.0) * (L2 + 1.0) * (g + 1.0) * L3 / ((L3 - 1.0) * (2.0 * g + 3.0) * (L1 + 2.0) * (L2 + 2.0));
}

__device__ __forceinline__ double threej_sq_gosper(int l1, int l2, int l3)
{
    const double L = (double)(l1 + l2 + l3);
    const double L1 = L - 2.0 * l1, L2 = L - 2.0 * l2, L3 = L - 2.0 * l3;
    const double num = (L + 1.0 / 3.0) *
                       sqrt((L1 + 1.0 / 6.0) * (L2 + 1.0 / 6.0) * (L3 + 1.0 / 6.0) / (L + 1.0 / 6.0));
    const double den = (L + 1.0) * (L1 + 1.0 / 3.0) * (L2 + 1.0 / 3.0) * (L3 + 1.0 / 3.0);
    return 2.0 / kPi * num / den;
}

// K[i3 * n2 + i2] = 2 (l1 l2 l3; 000)^2 with l2 = l20 + 2 i2, l3 = l30 + 2 i3
// (l20, l30 of two parity classes with l1 + l2 + l3 even); zero outside
// the triangle |l1 - l2| <= l3 <= l1 + l2.  One thread per l2 walks l3 upward
// from |l1 - l2| with the step ratio (exact) or evaluates the Gosper form.
// Both parity classes of l2 in one launch: blockIdx.y is the class of l2
// (0 even, 1 odd), K[class] its block.
struct K3Args {
    int l1, gosper;
    int l0[2], n[2];          // first l and count of each parity class
    const double *V;
    double *K[2];
};

__global__ void k_build_k3(K3Args a)
{
    const int c2 = blockIdx.y, c3 = (a.l1 & 1) ^ c2;
    const int n2 = a.n[c2], n3 = a.n[c3];
    const int i2 = blockIdx.x * blockDim.x + threadIdx.x;
    if (i2 >= n2 || n3 == 0) return;
    const int l1 = a.l1, l20 = a.l0[c2], l30 = a.l0[c3], gosper = a.gosper;
    const double *__restrict__ V = a.V;
    double *__restrict__ K = a.K[c2];
    const int l2 = l20 + 2 * i2;
    const int lo = abs(l1 - l2), hi = l1 + l2;
    int lc = lo;
    const int b = max(l1, l2);
    double v = gosper ? 0.0 : V[(size_t)b * (b + 1) / 2 + min(l1, l2)];
    for (int i3 = 0; i3 < n3; ++i3) {
        const int l3 = l30 + 2 * i3;
        double out = 0.0;
        if (l3 >= lo && l3 <= hi) {
            if (gosper) {
                out = 2.0 * threej_sq_gosper(l1, l2, l3);
            } else {
                while (lc < l3) {
                    v *= threej_sq_step(l1, l2, lc);
                    lc += 2;
                }
                out = 2.0 * v;
            }
        }
        K[(size_t)i3 * n2 + i2] = out;
    }
}

// C[rb * U + u] = wr r^2 G(l1', rb * U + u).
__global__ void k_c3(int L, int lp1, int U, int r0, int nrb, const double *__restrict__ r,
                     const double *__restrict__ wr, const double *__restrict__ G, double *__restrict__ C)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= U * nrb) return;
    const int rb = i / U;
    const double x = r[r0 + rb];
    C[i] = wr[r0 + rb] * x * x * G[(size_t)i * L + lp1];
}

// Packed pair index of (u2 <= u3), u2-major: the pairs of one u2 are
// contiguous, from u2 U - u2 (u2 - 1) / 2.
__device__ __forceinline__ int64_t pair3(int U, int u2, int u3)
{
    return (int64_t)u2 * U - (int64_t)u2 * (u2 - 1) / 2 + (u3 - u2);
}

// Zero rows [row0, row0 + nrows) of every column of a column-major matrix
// with leading dimension ld and ncols columns.
__global__ void k_zero_rows3(int64_t ld, int row0, int nrows, int64_t ncols, double *__restrict__ A)
{
    const int64_t n = (int64_t)nrows * ncols;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        A[(i / nrows) * ld + row0 + i % nrows] = 0.0;
}

// Gamma[n][m] from T(u1, u2, u3), fully symmetric, held for u1 <= u2 <= u3
// at T[u1 + U pair3(u2, u3)].
__global__ void k_gather3(int kind, int ta, int tp, const int *__restrict__ tri_a, const int *__restrict__ tri_p,
                          int np, int U, const double *__restrict__ T, double *__restrict__ gamma)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= (int64_t)ta * tp) return;
    const int n = (int)(i / tp), m = (int)(i % tp);
    const int a0 = tri_a[3 * n] * np, a1 = tri_a[3 * n + 1] * np, a2 = tri_a[3 * n + 2] * np;
    const int p0 = tri_p[3 * m], p1 = tri_p[3 * m + 1], p2 = tri_p[3 * m + 2];
    auto at = [&](int x, int y, int z) {
        int s0 = a0 + x, s1 = a1 + y, s2 = a2 + z, t;
        if (s0 > s1) { t = s0; s0 = s1; s1 = t; }
        if (s1 > s2) { t = s1; s1 = s2; s2 = t; }
        if (s0 > s1) { t = s0; s0 = s1; s1 = t; }
        return T[(size_t)s0 + (size_t)U * pair3(U, s1, s2)];
    };
    if (kind == MODAL_GAMMA_ORDERED) {
        gamma[i] = at(p0, p1, p2) / (8.0 * kPi);
        return;
    }
    const double s = at(p0, p1, p2) + at(p0, p2, p1) + at(p1, p0, p2) + at(p1, p2, p0) + at(p2, p0, p1) +
                     at(p2, p1, p0);
    gamma[i] = s / (48.0 * kPi);
}

}  // namespace

hipError_t launch_build_g3(int L, int nE, int lE0, int lO0, int lmin, int nr, int np, int na, int r0, int nrb,
                           const double *wl, const double *ql, const double *beta, double *G, hipStream_t s)
{
    const int64_t n = (int64_t)L * nrb * na * np;
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_build_g3, dim3(blocks), dim3(256), 0, s, L, nE, lE0, lO0, lmin, nr, np, na, r0, nrb,
                       wl, ql, beta, G);
    return hipGetLastError();
}

hipError_t launch_start3(int lmax, double *V, hipStream_t s)
{
    hipLaunchKernelGGL(k_start3, dim3((lmax + 64) / 64), dim3(64), 0, s, lmax, V);
    return hipGetLastError();
}

hipError_t launch_build_k3(int l1, const int l0[2], const int n[2], int gosper, const double *V, double *K0,
                           double *K1, hipStream_t s)
{
    const int nmax = std::max(n[0], n[1]);
    if (nmax <= 0) return hipSuccess;
    K3Args a{l1, gosper, {l0[0], l0[1]}, {n[0], n[1]}, V, {K0, K1}};
    hipLaunchKernelGGL(k_build_k3, dim3((nmax + 63) / 64, 2), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_c3(int L, int lp1, int U, int r0, int nrb, const double *r, const double *wr, const double *G,
                     double *C, hipStream_t s)
{
    const int n = U * nrb;
    hipLaunchKernelGGL(k_c3, dim3((n + 255) / 256), dim3(256), 0, s, L, lp1, U, r0, nrb, r, wr, G, C);
    return hipGetLastError();
}

hipError_t launch_zero_rows3(int64_t ld, int row0, int nrows, int64_t ncols, double *A, hipStream_t s)
{
    const int64_t n = (int64_t)nrows * ncols;
    if (n <= 0) return hipSuccess;
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_zero_rows3, dim3(blocks), dim3(256), 0, s, ld, row0, nrows, ncols, A);
    return hipGetLastError();
}

hipError_t launch_gather3(int kind, int ta, int tp, const int *tri_a, const int *tri_p, int np, int U,
                          const double *T, double *gamma, hipStream_t s)
{
    const int64_t n = (int64_t)ta * tp;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather3, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, kind, ta, tp, tri_a,
                       tri_p, np, U, T, gamma);
    return hipGetLastError();
}

}  // namespace mp
