// Plain column-major FP64 GEMM on the matrix cores (v_mfma_f64_16x16x4f64),
// for the contractions of Eq. (3D) and the blocked Cholesky solve of the
// full Gamma:
//
//     C_b = alpha op(A_b) op(B_b) + beta C_b,   b = 0 .. batch - 1,
//     op(A)(m, k) = ta ? A[k + m lda] : A[m + k lda],
//     op(B)(k, n) = tb ? B[n + k ldb] : B[k + n ldb],
//     C(m, n) = C[m + n ldc],  X_b = X + b * stride_X.
//
// A packed variant computes only the tiles on or below the diagonal of a
// square C and stores the entries m >= n as u2-major pairs,
// C_b[n m_total - n (n - 1) / 2 + (m - n)] (the upper triangle of C^T, which
// is what Eq. (3D) keeps of its symmetric B_r).
//
// Workgroup: 256 threads, one T x T output tile (T = 64 or 128); each of the
// four waves holds (T/2) x (T/2) in 16 x 16 matrix-core tiles.  K runs in
// 16-deep tiles staged through LDS, two buffers: the next tile's loads are
// issued before the current tile's matrix-core work and written to the other
// buffer after it, one barrier per tile.  Loads outside the matrix are
// clamped into it and zeroed only when written to LDS (no branch, so every
// load of a tile stays in flight together).  Tiles are dealt to the 8 XCDs
// in contiguous runs (M tile fastest), so the tiles that share a column
// block of op(B) run on one XCD and read it through one L2.
//
// FP64 16x16x4 operand layouts: A 16 x 4, lane l holds A[l % 16][l / 16];
// B 4 x 16, lane l holds B[l / 16][l % 16]; result 16 x 16, lane l element
// q holds D[4 q + l / 16][l % 16].  The product is formed as
// op(B)^T op(A)^T = C^T, so that lane l holds C[m = l % 16][n = 4 q + l / 16]:
// the 16 lanes of a group write 16 consecutive rows of one column of the
// column-major C (128 bytes) instead of 4.
#include "internal.hpp"

namespace mp {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int TK = 16;

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

// tile index (m tile, n tile, batch) of workgroup bid
template <bool PACKED>
__device__ __forceinline__ void tile_of(int64_t bid, int mt, int nt, int64_t ntiles, int &tm, int &tn, int &b)
{
    const int64_t x = bid & 7, idx = bid >> 3;
    const int64_t base = ntiles >> 3, rem = ntiles & 7;
    const int64_t tile = x * base + (x < rem ? x : rem) + idx;
    if (!PACKED) {
        b = (int)(tile / ((int64_t)mt * nt));
        const int rest = (int)(tile % ((int64_t)mt * nt));
        tm = rest % mt;
        tn = rest / mt;
    } else {
        // tiles tm >= tn of an mt x mt grid, column by column: column tn
        // holds mt - tn tiles
        const int per = mt * (mt + 1) / 2;
        b = (int)(tile / per);
        int rest = (int)(tile % per);
        tn = 0;
        while (rest >= mt - tn) {
            rest -= mt - tn;
            ++tn;
        }
        tm = tn + rest;
    }
}

template <int T, bool TA, bool TB, bool PACKED>
__global__ __launch_bounds__(256, 2) void k_dgemm(DgemmArgs g)
{
    constexpr int LD = T + 1;                 // padded LDS row (doubles)
    constexpr int NL = T * TK / 256;          // values of each operand per thread and K tile
    constexpr int WT = T / 32;                // 16 x 16 tiles per wave along m and n
    __shared__ double As[2][TK][LD];
    __shared__ double Bs[2][TK][LD];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int M = g.m, N = g.n, K = g.k;
    const int mt = (M + T - 1) / T, nt = (N + T - 1) / T;
    const int64_t ntiles = PACKED ? (int64_t)mt * (mt + 1) / 2 * g.batch : (int64_t)mt * nt * g.batch;
    const int64_t bid = blockIdx.x;
    if (bid >= ntiles) return;
    int tm, tn, b;
    tile_of<PACKED>(bid, mt, nt, ntiles, tm, tn, b);
    const int m0 = tm * T, n0 = tn * T;
    const double *A = g.A + (size_t)b * g.sA;
    const double *B = g.B + (size_t)b * g.sB;
    double *C = g.C + (size_t)b * g.sC;

    // staging map: NL values of A and NL of B per thread and K tile.  The
    // loads only load (clamped into the matrix); which values lie outside
    // it is kept as bits and applied when the tile is written to LDS, after
    // the matrix-core work: a select on a loaded value at the load would
    // make the compiler wait for each load in turn.
    double ra[NL], rb[NL];
    uint32_t okm = 0;                         // bit i: A value i inside, bit 16 + i: B value i
    auto amap = [&](int i, int &m, int &kk) {
        if (TA) { kk = t % TK; m = t / TK + 16 * i; }
        else    { m = t % T;   kk = t / T + (256 / T) * i; }
    };
    auto bmap = [&](int i, int &n, int &k2) {
        if (TB) { n = t % T;   k2 = t / T + (256 / T) * i; }
        else    { k2 = t % TK; n = t / TK + 16 * i; }
    };
    auto load = [&](int k0) {
        okm = 0;
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            int m, kk;
            amap(i, m, kk);
            const int gm = m0 + m, gk = k0 + kk;
            const int cm = min(gm, M - 1), ck = min(gk, K - 1);
            ra[i] = TA ? A[(size_t)cm * g.lda + ck] : A[(size_t)ck * g.lda + cm];
            okm |= (uint32_t)(gm < M && gk < K) << i;
            int n, k2;
            bmap(i, n, k2);
            const int gn = n0 + n, gk2 = k0 + k2;
            const int cn = min(gn, N - 1), ck2 = min(gk2, K - 1);
            rb[i] = TB ? B[(size_t)ck2 * g.ldb + cn] : B[(size_t)cn * g.ldb + ck2];
            okm |= (uint32_t)(gn < N && gk2 < K) << (16 + i);
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            int m, kk;
            amap(i, m, kk);
            As[buf][kk][m] = (okm >> i) & 1 ? ra[i] : 0.0;
            int n, k2;
            bmap(i, n, k2);
            Bs[buf][k2][n] = (okm >> (16 + i)) & 1 ? rb[i] : 0.0;
        }
    };

    // acc[j][i]: the 16 x 16 tile (n block j, m block i) of C^T
    d4 acc[WT][WT];
#pragma unroll
    for (int i = 0; i < WT; ++i)
#pragma unroll
        for (int j = 0; j < WT; ++j) acc[j][i] = d4{0.0, 0.0, 0.0, 0.0};

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
            double av[WT], bv[WT];
#pragma unroll
            for (int i = 0; i < WT; ++i) av[i] = As[buf][kr][wm * (T / 2) + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < WT; ++j) bv[j] = Bs[buf][kr][wn * (T / 2) + j * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < WT; ++j)
#pragma unroll
                for (int i = 0; i < WT; ++i)
                    acc[j][i] = __builtin_amdgcn_mfma_f64_16x16x4f64(bv[j], av[i], acc[j][i], 0, 0, 0);
        }
        // the other buffer was last read in tile kt - 1, before the barrier
        // that ended it
        if (more) stash(buf ^ 1);
        __syncthreads();
    }

    const double alpha = g.alpha, beta = g.beta;
#pragma unroll
    for (int j = 0; j < WT; ++j)
#pragma unroll
        for (int i = 0; i < WT; ++i)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int m = m0 + wm * (T / 2) + i * 16 + (lane & 15);
                const int n = n0 + wn * (T / 2) + j * 16 + 4 * q + (lane >> 4);
                const double v = alpha * acc[j][i][q];
                if (!PACKED) {
                    if (m < M && n < N) {
                        double *p = C + (size_t)n * g.ldc + m;
                        *p = beta == 0.0 ? v : v + beta * *p;
                    }
                } else if (m < M && n <= m) {
                    C[(int64_t)n * M - (int64_t)n * (n - 1) / 2 + (m - n)] = v;
                }
            }
}

template <int T, bool PACKED>
hipError_t launch_t(bool ta, bool tb, const DgemmArgs &g, int64_t tiles, hipStream_t s)
{
    const dim3 grid((unsigned)tiles), block(256);
    if (!ta && !tb)     hipLaunchKernelGGL((k_dgemm<T, false, false, PACKED>), grid, block, 0, s, g);
    else if (ta && !tb) hipLaunchKernelGGL((k_dgemm<T, true, false, PACKED>), grid, block, 0, s, g);
    else if (!ta && tb) hipLaunchKernelGGL((k_dgemm<T, false, true, PACKED>), grid, block, 0, s, g);
    else                hipLaunchKernelGGL((k_dgemm<T, true, true, PACKED>), grid, block, 0, s, g);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_dgemm(bool ta, bool tb, int m, int n, int k, double alpha, const double *A, int64_t lda,
                        int64_t sA, const double *B, int64_t ldb, int64_t sB, double beta, double *C,
                        int64_t ldc, int64_t sC, int batch, hipStream_t s, int tile)
{
    if (m < 0 || n < 0 || k < 0 || batch < 0 || (tile != 64 && tile != 128)) return hipErrorInvalidValue;
    if (m == 0 || n == 0 || batch == 0) return hipSuccess;
    if (ldc < m || lda < (ta ? k : m) || ldb < (tb ? n : k)) return hipErrorInvalidValue;
    const int64_t tiles = (int64_t)((m + tile - 1) / tile) * ((n + tile - 1) / tile) * batch;
    if (tiles > INT32_MAX) return hipErrorInvalidValue;
    DgemmArgs g{m, n, k, batch, alpha, beta, A, lda, sA, B, ldb, sB, C, ldc, sC};
    return tile == 64 ? launch_t<64, false>(ta, tb, g, tiles, s) : launch_t<128, false>(ta, tb, g, tiles, s);
}

hipError_t launch_dgemm_packed_lower(bool ta, bool tb, int m, int k, const double *A, int64_t lda, int64_t sA,
                                     const double *B, int64_t ldb, int64_t sB, double *P, int64_t sP, int batch,
                                     hipStream_t s)
{
    constexpr int T = 64;
    if (m < 0 || k < 0 || batch < 0) return hipErrorInvalidValue;
    if (m == 0 || batch == 0) return hipSuccess;
    if (lda < (ta ? k : m) || ldb < (tb ? m : k) || sP < (int64_t)m * (m + 1) / 2) return hipErrorInvalidValue;
    const int64_t mt = (m + T - 1) / T;
    const int64_t tiles = mt * (mt + 1) / 2 * batch;
    if (tiles > INT32_MAX) return hipErrorInvalidValue;
    DgemmArgs g{m, m, k, batch, 1.0, 0.0, A, lda, sA, B, ldb, sB, P, m, sP};
    return launch_t<T, true>(ta, tb, g, tiles, s);
}

}  // namespace mp
