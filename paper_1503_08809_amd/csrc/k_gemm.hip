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
using gemm::d4;

// ---- step b ----------------------------------------------------------------
struct BetaOp {
    static constexpr bool a_k_fast = true;    // Jd[l][r][k]
    static constexpr bool b_k_fast = true;    // qk[p][k]
    int M, N, K;                              // nr, np, nk
    int l0, lmin, L;
    const double *Jd, *k, *wk, *qk;
    double *beta;
    using RawA = double;
    struct RawB { double k, wk, q; };
    __device__ RawA fa(int b, int m, int kk) const { return Jd[((size_t)b * M + m) * K + kk]; }
    __device__ double ma(RawA v) const { return v; }
    __device__ RawB fb(int, int kk, int n) const { return RawB{k[kk], wk[kk], qk[(size_t)n * K + kk]}; }
    __device__ double mb(const RawB &v) const { return (2.0 / kPi) * v.wk * v.k * v.k * v.q; }
    __device__ void store(int b, int m, int n, double v) const
    {
        beta[((size_t)n * L + (l0 + b - lmin)) * M + m] = v;
    }
};

// ---- step c with mu parity ---------------------------------------------------
// At nodes symmetric about 0, P_l(-mu) = (-1)^l P_l(mu), so with
// E = Sum_{l even} A P_l(mu) and O = Sum_{l odd} A P_l(mu) over mu >= 0 only,
// S(+mu) = E + O and S(-mu) = E - O: half the work of the plain product.
// Rows m = u * nr + r (all (a, p) pairs and radial points in one index),
// columns j over the nh = ceil(nmu / 2) nodes mu >= 0, depth l.  Each 16-l
// tile is stored in LDS with its even-l entries first, so that two 4-deep
// matrix-core steps feed E and two feed O.  Workgroup tile 128 x 64, each
// wave 32 rows x 64 columns with E and O accumulators.
constexpr int SP_BM = 128, SP_BN = 64, SP_BK = 16;

template <bool ZB>   // ZB: z-blocked output scaled by wz, else plain [u][r][ldmu]
__global__ __launch_bounds__(256, 2) void k_s_parity(int na, int np, int nr, int nmu, int ldmu, int L, int lmin,
                                                  const double *__restrict__ wl, const double *__restrict__ ql,
                                                  const double *__restrict__ beta, const double *__restrict__ P,
                                                  int ldP, const double *__restrict__ wz, int64_t upad,
                                                  double *__restrict__ S)
{
    __shared__ double As[SP_BK][SP_BM + 1];
    __shared__ double Bs[SP_BK][SP_BN + 1];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int M = na * np * nr;
    const int nh = (nmu + 1) / 2, ioff = nmu - nh;
    const int m0 = blockIdx.x * SP_BM, j0 = blockIdx.y * SP_BN;

    // staging map: A 128 x 16 (8 per thread, rows fastest), B 16 x 64 (4 per
    // thread); a thread's A row is fixed for the whole l loop
    double ra[8], rb[4];
    auto slot = [&](int kk) { return ((lmin + kk) & 1) * 8 + (kk >> 1); };
    const int mrow = m0 + (t & 127);
    const bool rowok = mrow < M;
    const double *grow = nullptr, *brow = nullptr;
    {
        const int m = rowok ? mrow : 0;
        const int u = m / nr, r = m % nr, ia = u / np, ip = u % np;
        grow = ql + (size_t)ia * L;                 // wl is folded in below
        brow = beta + (size_t)ip * L * nr + r;
    }
    auto load = [&](int k0) {
        // clamped loads times a 0/1 factor (a select with a loaded operand is
        // compiled to a branch with its own wait for memory)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int l = k0 + (t >> 7) + 2 * i, lc = min(l, L - 1);
            ra[i] = wl[lc] * grow[lc] * brow[(size_t)lc * nr] * ((rowok && l < L) ? 1.0 : 0.0);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int j = j0 + (t & 63), kk = (t >> 6) + 4 * i, l = k0 + kk;
            rb[i] = P[(size_t)min(l, L - 1) * ldP + ioff + min(j, nh - 1)] * ((j < nh && l < L) ? 1.0 : 0.0);
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int kk = (t >> 7) + 2 * i;
            As[slot(kk)][t & 127] = ra[i];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int kk = (t >> 6) + 4 * i;
            Bs[slot(kk)][t & 63] = rb[i];
        }
    };

    d4 aE[2][4], aO[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            aE[i][j] = d4{0.0, 0.0, 0.0, 0.0};
            aO[i][j] = d4{0.0, 0.0, 0.0, 0.0};
        }
    const int ktiles = (L + SP_BK - 1) / SP_BK;
    load(0);
    for (int kt = 0; kt < ktiles; ++kt) {
        __syncthreads();
        stash();
        __syncthreads();
        if (kt + 1 < ktiles) load((kt + 1) * SP_BK);
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int kr = ks * 4 + (lane >> 4);
            double av[2], bv[4];
#pragma unroll
            for (int i = 0; i < 2; ++i) av[i] = As[kr][wave * 32 + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 4; ++j) bv[j] = Bs[kr][j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (ks < 2) aE[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], aE[i][j], 0, 0, 0);
                    else        aO[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], aO[i][j], 0, 0, 0);
                }
        }
    }
    // epilogue: S(+mu) = E + O at node ioff + j, S(-mu) = E - O at node nh - 1 - j.
    // The quadrature factors are loaded first, clamped and unconditionally, so
    // that their loads overlap instead of each waiting inside a branch.
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int m = m0 + wave * 32 + i * 16 + 4 * q + (lane >> 4);
            const int mc = min(m, M - 1);
            const int u = mc / nr, r = mc % nr;
            double fp[4], fm[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int jj = min(j0 + j * 16 + (lane & 15), nh - 1);
                fp[j] = ZB ? wz[(int64_t)r * ldmu + ioff + jj] : 1.0;
                fm[j] = ZB ? wz[(int64_t)r * ldmu + nh - 1 - jj] : 1.0;
            }
            if (m >= M) continue;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int jj = j0 + j * 16 + (lane & 15);
                if (jj >= nh) continue;
                const double e = aE[i][j][q], o = aO[i][j][q];
                const int ip = ioff + jj, im = nh - 1 - jj;
                if (ZB) {
                    const int64_t zp = (int64_t)r * ldmu + ip, zm = (int64_t)r * ldmu + im;
                    S[(((size_t)(zp >> 5) * upad + u) << 5) + (zp & 31)] = (e + o) * fp[j];
                    if (im != ip) S[(((size_t)(zm >> 5) * upad + u) << 5) + (zm & 31)] = (e - o) * fm[j];
                } else {
                    S[((size_t)u * nr + r) * ldmu + ip] = e + o;
                    if (im != ip) S[((size_t)u * nr + r) * ldmu + im] = e - o;
                }
            }
        }
}

// zero the mu padding (nodes nmu..ldmu) of z-blocked rows
__global__ void k_zero_mu_pad(int U, int nr, int nmu, int ldmu, int64_t upad, double *__restrict__ S)
{
    const int pad = ldmu - nmu;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)U * nr * pad) return;
    const int u = (int)(i / ((int64_t)nr * pad));
    const int rem = (int)(i % ((int64_t)nr * pad));
    const int r = rem / pad, mu = nmu + rem % pad;
    const int64_t z = (int64_t)r * ldmu + mu;
    S[(((size_t)(z >> 5) * upad + u) << 5) + (z & 31)] = 0.0;
}

__global__ void k_weights_l(int L, int lmin, double v_power, const double *__restrict__ cl,
                            double *__restrict__ wl)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L) return;
    const double l2 = 2.0 * (lmin + i) + 1.0;
    wl[i] = pow(l2, 1.0 - v_power) / (cl ? sqrt(cl[i]) : 1.0);     // cl NULL: C_l = 1
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

hipError_t launch_s_parity(int na, int np, int nr, int nmu, int ldmu, int L, int lmin, const double *wl,
                          const double *ql, const double *beta, const double *P, int ldP, const double *wz,
                          int64_t upad, double *S, hipStream_t s)
{
    if (upad > 0 && (!wz || ldmu % 32 != 0)) return hipErrorInvalidValue;
    const int M = na * np * nr, nh = (nmu + 1) / 2;
    dim3 grid((M + SP_BM - 1) / SP_BM, (nh + SP_BN - 1) / SP_BN);
    if (upad > 0)
        hipLaunchKernelGGL(k_s_parity<true>, grid, dim3(256), 0, s, na, np, nr, nmu, ldmu, L, lmin, wl, ql, beta,
                           P, ldP, wz, upad, S);
    else
        hipLaunchKernelGGL(k_s_parity<false>, grid, dim3(256), 0, s, na, np, nr, nmu, ldmu, L, lmin, wl, ql, beta,
                           P, ldP, wz, upad, S);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || upad == 0 || ldmu == nmu) return e;
    const int64_t n = (int64_t)na * np * nr * (ldmu - nmu);
    hipLaunchKernelGGL(k_zero_mu_pad, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, na * np, nr, nmu, ldmu,
                       upad, S);
    return hipGetLastError();
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
