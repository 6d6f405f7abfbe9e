// Generic FP64 matrix-core GEMM used by the contraction stages: 64x64 output
// tiles per 256-thread workgroup (four waves, each 32x32 = 2x2 tiles of
// v_mfma_f64_16x16x4f64), 16-deep K tiles staged through LDS with the next
// tile prefetched into registers.  Operands and the epilogue come from an Op
// (see below), so generated operands and fused epilogues cost no extra pass.
//
// FP64 16x16x4 operand layouts: A 16x4, lane l holds A[l % 16][l / 16];
// B 4x16, lane l holds B[l / 16][l % 16]; result 16x16, lane l element q
// holds C[4 q + l / 16][l % 16].
#pragma once

#include "internal.hpp"

namespace mp {
namespace gemm {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 16;
constexpr int LDA = BM + 1, LDB = BN + 1;

// Op interface.  Operands are formed from loaded values in two phases: every
// load of the next K tile is issued first (fa, fb: loads only), and the
// arithmetic that forms the operand (ma, mb) runs when the tile is written
// to LDS, after the matrix-core work of the current tile, so the loads of a
// generated operand never wait for one another.
//   static constexpr bool a_k_fast, b_k_fast;   // which index is contiguous in memory
//   int M, N, K;
//   RawA fa(int b, int m, int k) const;   double ma(const RawA &) const;
//   RawB fb(int b, int k, int n) const;   double mb(const RawB &) const;
//   void store(int b, int m, int n, double v) const;
template <class Op>
__global__ __launch_bounds__(256) void k_gemm64(Op op)
{
    __shared__ double As[BK][LDA];
    __shared__ double Bs[BK][LDB];
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int M = op.M, N = op.N, K = op.K;
    // 1-D grid of (M tile, N tile, batch) tiles, M tile fastest.  Workgroups
    // go to the 8 XCDs round-robin; each XCD takes a contiguous range of
    // tiles, so the M tiles that share one B column block run on one XCD and
    // read it through the same L2.
    const int mt = (M + BM - 1) / BM, nt = (N + BN - 1) / BN;
    const int ntiles = mt * nt * gridDim.y;
    const int bid = blockIdx.x + gridDim.x * blockIdx.y;
    if (bid >= ntiles) return;
    const int tile = [&] {
        const int x = bid & 7, idx = bid >> 3;
        const int base = ntiles >> 3, rem = ntiles & 7;
        return x * base + (x < rem ? x : rem) + idx;
    }();
    const int b = tile / (mt * nt);
    const int m0 = (tile % mt) * BM, n0 = ((tile / mt) % nt) * BN;

    typename Op::RawA ra[4];
    typename Op::RawB rb[4];
    double fa[4], fb[4];                      // 1 inside the matrix, 0 outside
    auto load = [&](int k0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            int m, k;
            if (Op::a_k_fast) { k = t % BK; m = t / BK + 16 * i; }
            else              { m = t % BM; k = t / BM + 4 * i; }
            // clamped (always in-range) loads, zeroed by a 0/1 factor: a
            // guarded load, or a select with a loaded operand, is compiled to
            // a branch with its own wait for memory
            const int gm = m0 + m, gk = k0 + k;
            ra[i] = op.fa(b, min(gm, M - 1), min(gk, K - 1));
            fa[i] = (gm < M && gk < K) ? 1.0 : 0.0;
            int n, kk;
            if (Op::b_k_fast) { kk = t % BK; n = t / BK + 16 * i; }
            else              { n = t % BN; kk = t / BN + 4 * i; }
            const int gn = n0 + n, gk2 = k0 + kk;
            rb[i] = op.fb(b, min(gk2, K - 1), min(gn, N - 1));
            fb[i] = (gn < N && gk2 < K) ? 1.0 : 0.0;
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            int m, k;
            if (Op::a_k_fast) { k = t % BK; m = t / BK + 16 * i; }
            else              { m = t % BM; k = t / BM + 4 * i; }
            As[k][m] = op.ma(ra[i]) * fa[i];
            int n, kk;
            if (Op::b_k_fast) { kk = t % BK; n = t / BK + 16 * i; }
            else              { n = t % BN; kk = t / BN + 4 * i; }
            Bs[kk][n] = op.mb(rb[i]) * fb[i];
        }
    };

    d4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

    const int ktiles = (K + BK - 1) / BK;
    if (ktiles > 0) load(0);
    for (int kt = 0; kt < ktiles; ++kt) {
        __syncthreads();
        stash();
        __syncthreads();
        if (kt + 1 < ktiles) load((kt + 1) * BK);
#pragma unroll
        for (int ks = 0; ks < BK / 4; ++ks) {
            const int kr = ks * 4 + (lane >> 4);
            double av[2], bv[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) av[i] = As[kr][wm * 32 + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 2; ++j) bv[j] = Bs[kr][wn * 32 + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int m = m0 + wm * 32 + i * 16 + 4 * q + (lane >> 4);
                const int n = n0 + wn * 32 + j * 16 + (lane & 15);
                if (m < M && n < N) op.store(b, m, n, acc[i][j][q]);
            }
}


template <class Op>
inline hipError_t run(const Op &op, int batches, hipStream_t s)
{
    if (op.M <= 0 || op.N <= 0 || batches <= 0) return hipSuccess;
    const int64_t per = (int64_t)((op.M + BM - 1) / BM) * ((op.N + BN - 1) / BN);
    if (per * batches > INT32_MAX) return hipErrorInvalidValue;
    // grid x * y covers the tiles of all batches (y = batches)
    dim3 grid((unsigned)per, (unsigned)batches);
    hipLaunchKernelGGL(k_gemm64<Op>, grid, dim3(256), 0, s, op);
    return hipGetLastError();
}


}  // namespace gemm
}  // namespace mp
