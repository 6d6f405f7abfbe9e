// Steps b and c: the k contraction (beta) and the l contraction (S) as FP64
// matrix-core GEMMs (v_mfma_f64_16x16x4f64), 64x64 output tiles per
// 256-thread workgroup, 16-deep K tiles staged through LDS with the next
// tile prefetched into registers while the current one is multiplied.
//
// Step b (Appendix, projected modes; times 2/pi), one GEMM per l:
//   beta_p(l, r) = Sum_k [Delta_l(k) j_l(k r)] * [(2/pi) wk k^2 q_p(k)]
//   rows r, columns p, depth k.  The first factor comes from the Bessel
//   emit pass (already multiplied by Delta_l(k)); the second is formed on
//   load.
// Step c (Sec. 2.2, Eq. (legendre)), one GEMM per pair u = (a, p):
//   S_ap(r, mu) = Sum_l [w_l qbar_a(l) beta_p(l, r)] * P_l(mu)
//   rows r, columns mu, depth l; the first factor is formed on load.  The
//   epilogue optionally multiplies by the cube root of the quadrature weight
//   W(r, mu) = wr r^2 wmu, so that the triple product of three scaled rows
//   carries W once, and then writes the rows z-blocked: St[z / 32][u][z % 32]
//   with z = r * ldmu + mu, so that one 32-wide z step of every row is one
//   contiguous slab (the triple-product kernels read a few hundred rows per
//   step; with whole rows contiguous each step would touch a few hundred
//   pages).
#include "gemm64.hpp"

namespace mp {
namespace {
using gemm::run;

// ---- step b ----------------------------------------------------------------
struct BetaOp {
    static constexpr bool a_k_fast = true;    // Jd[l][r][k]
    static constexpr bool b_k_fast = true;    // qk[p][k]
    int M, N, K;                              // nr, np, nk
    int l0, lmin, L;
    const double *Jd, *k, *wk, *qk;
    double *beta;
    __device__ double a(int b, int m, int kk) const { return Jd[((size_t)b * M + m) * K + kk]; }
    __device__ double bv(int, int kk, int n) const
    {
        const double kv = k[kk];
        return (2.0 / kPi) * wk[kk] * kv * kv * qk[(size_t)n * K + kk];
    }
    __device__ void store(int b, int m, int n, double v) const
    {
        beta[((size_t)n * L + (l0 + b - lmin)) * M + m] = v;
    }
};

// ---- step c ----------------------------------------------------------------
struct SOp {
    static constexpr bool a_k_fast = false;   // beta[p][l][r]: r contiguous
    static constexpr bool b_k_fast = false;   // P[l][mu]: mu contiguous
    int M, N, K;                              // nr, ldmu, L
    int np, nmu, ldP;
    const double *wl, *ql, *beta, *P, *wz;
    double *S;
    int64_t upad;                             // > 0: z-blocked output (see below)
    __device__ double a(int u, int m, int l) const
    {
        const int ia = u / np, ip = u % np;
        return wl[l] * ql[(size_t)ia * K + l] * beta[((size_t)ip * K + l) * M + m];
    }
    __device__ double bv(int, int l, int n) const { return P[(size_t)l * ldP + n]; }
    __device__ void store(int u, int m, int n, double v) const
    {
        if (upad > 0) {
            // z-blocked rows: St[z / 32][u][z % 32], z = r * ldmu + mu
            const int64_t z = (int64_t)m * N + n;
            const size_t o = (((size_t)(z >> 5) * upad + u) << 5) + (z & 31);
            S[o] = (n < nmu) ? v * wz[z] : 0.0;
            return;
        }
        S[((size_t)u * M + m) * N + n] = (n < nmu) ? v : 0.0;
    }
};

__global__ void k_weights_l(int L, int lmin, double v_power, const double *__restrict__ cl,
                            double *__restrict__ wl)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L) return;
    const double l2 = 2.0 * (lmin + i) + 1.0;
    wl[i] = pow(l2, 1.0 - v_power) / sqrt(cl[i]);
}

__global__ void k_cbrt_weights(int nr, int nmu, int ldmu, const double *__restrict__ r,
                               const double *__restrict__ wr, const double *__restrict__ wmu,
                               double *__restrict__ wz)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)nr * ldmu) return;
    const int ir = (int)(i / ldmu), im = (int)(i % ldmu);
    wz[i] = (im < nmu) ? cbrt(wr[ir] * r[ir] * r[ir] * wmu[im]) : 0.0;
}

__global__ void k_s_import(int64_t nu, int64_t upad, int nr, int nmu, int ldmu,
                           const double *__restrict__ S, const double *__restrict__ wz,
                           double *__restrict__ St)
{
    // caller layout S[u][r][nmu] -> z-blocked St[z / 32][u][z % 32], scaled
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ldz = (int64_t)nr * ldmu;
    const int64_t n = nu * ldz;
    if (i >= n) return;
    const int64_t u = i / ldz, z = i % ldz;
    const int ir = (int)(z / ldmu), im = (int)(z % ldmu);
    St[(((z >> 5) * upad + u) << 5) + (z & 31)] =
        (im < nmu) ? S[(u * nr + ir) * nmu + im] * wz[z] : 0.0;
}

}  // namespace

hipError_t launch_beta_gemm(int nl, int l0, int lmin, int L, int nk, int nr, int np,
                            const double *Jd, const double *k, const double *wk, const double *qk,
                            double *beta, hipStream_t s)
{
    BetaOp op{nr, np, nk, l0, lmin, L, Jd, k, wk, qk, beta};
    return run(op, nl, s);
}

hipError_t launch_s_gemm(int na, int np, int nr, int nmu, int ldmu, int L, const double *wl,
                         const double *ql, const double *beta, const double *P, int ldP,
                         const double *wz, int64_t upad, double *S, hipStream_t s)
{
    if (upad > 0 && (!wz || ldmu % 32 != 0)) return hipErrorInvalidValue;
    SOp op{nr, ldmu, L, np, nmu, ldP, wl, ql, beta, P, wz, S, upad};
    return run(op, na * np, s);
}

hipError_t launch_weights_l(int L, int lmin, double v_power, const double *cl, double *wl,
                            hipStream_t s)
{
    hipLaunchKernelGGL(k_weights_l, dim3((L + 255) / 256), dim3(256), 0, s, L, lmin, v_power, cl, wl);
    return hipGetLastError();
}

hipError_t launch_cbrt_weights(int nr, int nmu, int ldmu, const double *r, const double *wr,
                               const double *wmu, double *wz, hipStream_t s)
{
    const int64_t n = (int64_t)nr * ldmu;
    hipLaunchKernelGGL(k_cbrt_weights, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, nr, nmu,
                       ldmu, r, wr, wmu, wz);
    return hipGetLastError();
}

hipError_t launch_s_import(int64_t nu, int64_t upad, int nr, int nmu, int ldmu, const double *S,
                           const double *wz, double *St, hipStream_t s)
{
    if (ldmu % 32 != 0) return hipErrorInvalidValue;
    const int64_t n = nu * nr * ldmu;
    hipLaunchKernelGGL(k_s_import, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, nu, upad, nr, nmu,
                       ldmu, S, wz, St);
    return hipGetLastError();
}

}  // namespace mp
