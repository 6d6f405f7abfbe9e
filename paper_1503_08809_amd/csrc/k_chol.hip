// The small kernels of the blocked Cholesky solve behind the full Gamma =
// <Q, Q>^-1 Gamma' (Appendix): the factorisation of one diagonal block and
// the triangular solves of many short vectors against one diagonal block.
// The large updates between blocks run on the FP64 GEMM (k_dgemm.hip); the
// host drives the block loop (api.hip).  Blocks are at most 64 x 64; all
// matrices column major.
#include "internal.hpp"

namespace mp {
namespace {

constexpr int NB = 64;

// In-place Cholesky A = L L^T of one jb x jb block (jb <= 64), lower
// triangle, one wave: the block in LDS, one column at a time (scale the
// column by the square root of its pivot, then subtract its outer product
// from the trailing block).  A pivot that is not positive and finite sets
// *info = 1 (the matrix is not positive definite); the rest of the block is
// still written, with whatever the arithmetic gives.
__global__ __launch_bounds__(64) void k_potrf_block(int jb, double *__restrict__ A, int64_t lda,
                                                    int *__restrict__ info)
{
    __shared__ double S[NB][NB + 1];
    const int t = threadIdx.x;
    for (int j = 0; j < jb; ++j)
        if (t < jb) S[t][j] = A[(size_t)j * lda + t];
    __syncthreads();
    bool bad = false;
    for (int k = 0; k < jb; ++k) {
        const double piv = S[k][k];
        const bool ok = piv > 0.0 && isfinite(piv);
        bad |= !ok;
        const double d = sqrt(ok ? piv : 1.0);
        __syncthreads();
        if (t >= k && t < jb) S[t][k] = t == k ? d : S[t][k] / d;
        __syncthreads();
        if (t > k && t < jb) {
            const double a = S[t][k];
            for (int j = k + 1; j <= t; ++j) S[t][j] -= a * S[j][k];
        }
        __syncthreads();
    }
    for (int j = 0; j < jb; ++j)
        if (t < jb && t >= j) A[(size_t)j * lda + t] = S[t][j];
    if (t == 0 && bad) info[0] = 1;
}

// rows vectors x_i (element j of x_i at X[i xr + j xc]) overwritten by the
// solution of x L^T = x (backward = 0: forward substitution,
//     x_j = (x_j - Sum_{p<j} x_p L[j][p]) / L[j][j])
// or of x L = x (backward = 1: backward substitution,
//     x_j = (x_j - Sum_{p>j} x_p L[p][j]) / L[j][j]),
// L the lower jb x jb block at Lb (leading dimension ldl).  One thread per
// vector, 64 per workgroup; the block and the vectors staged in LDS.
__global__ __launch_bounds__(64) void k_trsm_rows(int rows, int jb, const double *__restrict__ Lb, int64_t ldl,
                                                  double *__restrict__ X, int64_t xr, int64_t xc, int backward)
{
    __shared__ double Ls[NB][NB + 1];
    __shared__ double Xs[NB][NB + 1];
    const int t = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * NB + t;
    for (int j = 0; j < jb; ++j)
        if (t < jb) Ls[t][j] = Lb[(size_t)j * ldl + t];
    if (i < rows)
        for (int j = 0; j < jb; ++j) Xs[t][j] = X[i * xr + j * xc];
    __syncthreads();
    if (i >= rows) return;
    if (!backward) {
        for (int j = 0; j < jb; ++j) {
            double s = Xs[t][j];
            for (int p = 0; p < j; ++p) s -= Xs[t][p] * Ls[j][p];
            Xs[t][j] = s / Ls[j][j];
        }
    } else {
        for (int j = jb - 1; j >= 0; --j) {
            double s = Xs[t][j];
            for (int p = j + 1; p < jb; ++p) s -= Xs[t][p] * Ls[p][j];
            Xs[t][j] = s / Ls[j][j];
        }
    }
    for (int j = 0; j < jb; ++j) X[i * xr + j * xc] = Xs[t][j];
}

}  // namespace

int chol_block() { return NB; }

hipError_t launch_potrf_block(int jb, double *A, int64_t lda, int *info, hipStream_t s)
{
    if (jb <= 0) return hipSuccess;
    if (jb > NB || lda < jb) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_potrf_block, dim3(1), dim3(64), 0, s, jb, A, lda, info);
    return hipGetLastError();
}

hipError_t launch_trsm_rows(int rows, int jb, const double *L, int64_t ldl, double *X, int64_t xr, int64_t xc,
                            int backward, hipStream_t s)
{
    if (rows <= 0 || jb <= 0) return hipSuccess;
    if (jb > NB || ldl < jb) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_trsm_rows, dim3((unsigned)((rows + NB - 1) / NB)), dim3(64), 0, s, rows, jb, L, ldl, X,
                       xr, xc, backward);
    return hipGetLastError();
}

}  // namespace mp
