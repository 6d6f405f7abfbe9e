// Plain column-major FP64 GEMM on the matrix cores (v_mfma_f64_16x16x4f64),
// for the contractions of Eq. (3D) and the blocked Cholesky solve of the
// full Gamma:
//
//     C_b = alpha op(A_b) op(B_b) + beta C_b,   b = 0 .. batch - 1,
//     op(A)(m, k) = ta ? A[k + m lda] : A[m + k lda],
//     op(B)(k, n) = tb ? B[n + k ldb] : B[k + n ldb],
//     C(m, n) = C[m + n ldc],  X_b = X + b * stride_X.
//
// Workgroup: 256 threads, one 128 x 128 output tile; each of the four waves
// holds 64 x 64 (4 x 4 tiles of 16 x 16, 64 FP64 accumulators per lane).
// K runs in 16-deep tiles staged through LDS, two buffers: the next tile's
// loads are issued before the current tile's matrix-core work and written
// to the other buffer after it, one barrier per tile.  Loads outside the
// matrix are clamped into it and multiplied by 0 (no branch, so the compiler
// keeps every load of a tile in flight together).  Tiles are dealt to the 8
// XCDs in contiguous runs (M tile fastest), so the tiles that share a column
// block of op(B) run on one XCD and read it through one L2.
//
// FP64 16x16x4 operand layouts: A 16 x 4, lane l holds A[l % 16][l / 16];
// B 4 x 16, lane l holds B[l / 16][l % 16]; result 16 x 16, lane l element
// q holds C[4 q + l / 16][l % 16].
#include "internal.hpp"

namespace mp {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int TM = 128, TN = 128, TK = 16;
constexpr int LDS_LD = TM + 1;                // padded LDS row (doubles)

struct DgemmArgs {
    int m, n, k, batch;
    double alpha, beta;
    const double *A;
    int64_t lda, sA;
    const double *B;
    int64_t ldb, sB;
    double *C;
    int64_t ldc, sC;
};

template <bool TA, bool TB>
__global__ __launch_bounds__(256, 2) void k_dgemm(DgemmArgs g)
{
    __shared__ double As[2][TK][LDS_LD];
    __shared__ double Bs[2][TK][LDS_LD];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int M = g.m, N = g.n, K = g.k;
    const int mt = (M + TM - 1) / TM, nt = (N + TN - 1) / TN;
    const int64_t ntiles = (int64_t)mt * nt * g.batch;
    const int64_t bid = blockIdx.x;
    if (bid >= ntiles) return;
    int64_t tile;
    {
        const int64_t x = bid & 7, idx = bid >> 3;
        const int64_t base = ntiles >> 3, rem = ntiles & 7;
        tile = x * base + (x < rem ? x : rem) + idx;
    }
    const int b = (int)(tile / ((int64_t)mt * nt));
    const int rest = (int)(tile % ((int64_t)mt * nt));
    const int m0 = (rest % mt) * TM, n0 = (rest / mt) * TN;
    const double *A = g.A + (size_t)b * g.sA;
    const double *B = g.B + (size_t)b * g.sB;
    double *C = g.C + (size_t)b * g.sC;

    // staging map: 8 values of A and 8 of B per thread and K tile.  The
    // loads only load (clamped into the matrix); which values lie outside
    // it is kept as bits and applied when the tile is written to LDS, after
    // the matrix-core work: a select on a loaded value at the load would
    // make the compiler wait for each load in turn.
    double ra[8], rb[8];
    uint32_t okm = 0;                         // bit i: A value i inside, bit 8 + i: B value i
    auto load = [&](int k0) {
        okm = 0;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            int m, kk;
            if (TA) { kk = t % TK; m = t / TK + 16 * i; }
            else    { m = t % TM;  kk = t / TM + 2 * i; }
            const int gm = m0 + m, gk = k0 + kk;
            const int cm = min(gm, M - 1), ck = min(gk, K - 1);
            ra[i] = TA ? A[(size_t)cm * g.lda + ck] : A[(size_t)ck * g.lda + cm];
            okm |= (uint32_t)(gm < M && gk < K) << i;
            int n, k2;
            if (TB) { n = t % TN;  k2 = t / TN + 2 * i; }
            else    { k2 = t % TK; n = t / TK + 16 * i; }
            const int gn = n0 + n, gk2 = k0 + k2;
            const int cn = min(gn, N - 1), ck2 = min(gk2, K - 1);
            rb[i] = TB ? B[(size_t)ck2 * g.ldb + cn] : B[(size_t)cn * g.ldb + ck2];
            okm |= (uint32_t)(gn < N && gk2 < K) << (8 + i);
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            int m, kk;
            if (TA) { kk = t % TK; m = t / TK + 16 * i; }
            else    { m = t % TM;  kk = t / TM + 2 * i; }
            As[buf][kk][m] = (okm >> i) & 1 ? ra[i] : 0.0;
            int n, k2;
            if (TB) { n = t % TN;  k2 = t / TN + 2 * i; }
            else    { k2 = t % TK; n = t / TK + 16 * i; }
            Bs[buf][k2][n] = (okm >> (8 + i)) & 1 ? rb[i] : 0.0;
        }
    };

    d4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

    const int ktiles = (K + TK - 1) / TK;
    if (ktiles > 0) {
        load(0);
        stash(0);
    }
    __syncthreads();
    for (int kt = 0; kt < ktiles; ++kt) {
        const int buf = kt & 1;
        const bool more = kt + 1 < ktiles;
        if (more) load((kt + 1) * TK);
#pragma unroll
        for (int ks = 0; ks < TK / 4; ++ks) {
            const int kr = ks * 4 + (lane >> 4);
            double av[4], bv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) av[i] = As[buf][kr][wm * 64 + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 4; ++j) bv[j] = Bs[buf][kr][wn * 64 + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
        }
        // the other buffer was last read in tile kt - 1, before the barrier
        // that ended it
        if (more) stash(buf ^ 1);
        __syncthreads();
    }

    const double alpha = g.alpha, beta = g.beta;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int m = m0 + wm * 64 + i * 16 + 4 * q + (lane >> 4);
                const int n = n0 + wn * 64 + j * 16 + (lane & 15);
                if (m < M && n < N) {
                    double *p = C + (size_t)n * g.ldc + m;
                    const double v = alpha * acc[i][j][q];
                    *p = beta == 0.0 ? v : v + beta * *p;
                }
            }
}

}  // namespace

hipError_t launch_dgemm(bool ta, bool tb, int m, int n, int k, double alpha, const double *A, int64_t lda,
                        int64_t sA, const double *B, int64_t ldb, int64_t sB, double beta, double *C,
                        int64_t ldc, int64_t sC, int batch, hipStream_t s)
{
    if (m < 0 || n < 0 || k < 0 || batch < 0) return hipErrorInvalidValue;
    if (m == 0 || n == 0 || batch == 0) return hipSuccess;
    if (ldc < m || lda < (ta ? k : m) || ldb < (tb ? n : k)) return hipErrorInvalidValue;
    const int64_t tiles = (int64_t)((m + TM - 1) / TM) * ((n + TN - 1) / TN) * batch;
    if (tiles > INT32_MAX) return hipErrorInvalidValue;
    DgemmArgs g{m, n, k, batch, alpha, beta, A, lda, sA, B, ldb, sB, C, ldc, sC};
    const dim3 grid((unsigned)tiles), block(256);
    if (!ta && !tb)     hipLaunchKernelGGL((k_dgemm<false, false>), grid, block, 0, s, g);
    else if (ta && !tb) hipLaunchKernelGGL((k_dgemm<true, false>), grid, block, 0, s, g);
    else if (!ta && tb) hipLaunchKernelGGL((k_dgemm<false, true>), grid, block, 0, s, g);
    else                hipLaunchKernelGGL((k_dgemm<true, true>), grid, block, 0, s, g);
    return hipGetLastError();
}

}  // namespace mp
