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
// Workgroup: one BT x BT output tile.  K runs in 16-deep steps whose
// operands are copied from memory straight into LDS (buffer_load ... lds, no
// registers) through a ring of slots, one array per slot, one barrier per
// step; every LDS read is 16 bytes per lane and all of a step's reads are
// issued before its copies.  BT = 64: four waves of 32 x 32, two slots
// (copies one step ahead, 32 KB, four workgroups per CU); BT = 128: eight
// waves of 64 (m) x 32 (n), three slots (copies two steps ahead, 96 KB, one
// workgroup per CU).
//
// LDS layout of an operand in a slot, by how it lies in memory:
//  * free index (m of op(A), n of op(B)) contiguous: rows [k][BT]; a lane
//    reads two adjacent free indices, which feed the even and the odd one of
//    a pair of 16-wide matrix-core tiles (tile 2p + e holds the free indices
//    32 p + 2 r + e, r = 0..15);
//  * k contiguous: [BT][k pair][2], the pair index XOR-swizzled by
//    (free index / 2) mod 8 (a copy's 8 lanes of one free index read one
//    128-byte run; the 16 free indices of a read fall in distinct banks); a
//    lane reads the two k of one pair, which feed two consecutive
//    matrix-core steps.
// Inside a step the 16 k are taken in the order k = 2 (4 j + g) + e for
// matrix-core step 2 j + e and lane group g (lane / 16), in both operands,
// so that a 16-byte read serves either form.  Values outside the matrix are
// read as zero (their buffer offset is out of range), except the second k of
// a pair that straddles an odd K, which is zeroed in registers.
//
// FP64 16x16x4 operand layouts: A 16 x 4, lane l holds A[l % 16][l / 16];
// B 4 x 16, lane l holds B[l / 16][l % 16]; result 16 x 16, lane l element
// q holds D[4 q + l / 16][l % 16].  The product is formed as
// op(B)^T op(A)^T = C^T, so that a lane's results lie along m, the
// contiguous index of the column-major C.
#include "internal.hpp"

#include <type_traits>

namespace mp {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

constexpr int KS = 16;                         // k per step
constexpr int kBufWord3 = 0x00020000;          // descriptor word 3: 32-bit data format, raw access
constexpr uint32_t kOut = 0x80000000u;         // a buffer offset past every record: reads zero
constexpr int kRecords = 0x7ffffff0;           // bytes a descriptor admits
// leading dimensions up to this keep every copy's byte offset inside one
// step below kRecords (128 rows of the k-contiguous form)
constexpr int64_t kMaxLd = kRecords / (8 * 128) - 1;

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

__device__ __forceinline__ void dma16(__amdgpu_buffer_rsrc_t rs, uint32_t voff, void *lds_base)
{
    __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void *)lds_base, 16, voff, 0,
                                             0, 0);
}

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

// One operand's copies: instruction i (of BT / 8 per step) moves 1 KB, lane
// `lane` 16 bytes.  Returns the lane's byte offset from the operand's step
// origin (k = k0, free index = the tile's first); kk and f are the lane's
// first k and free index inside the step.
template <int BT>
__device__ __forceinline__ uint32_t copy_offset(bool free, int i, int lane, int64_t ld, int &kk, int &f)
{
    const int e = i * 128 + 2 * lane;                  // first value of the lane in the slot part
    if (free) {
        kk = e / BT;
        f = e % BT;
        return (uint32_t)(((int64_t)kk * ld + f) * 8);
    }
    // k contiguous: 16-byte position q = f * 8 + (pair ^ ((f >> 1) & 7)), so
    // that the 8 lanes of one f read one 128-byte run and the 16 f a
    // matrix-core read takes fall in 16 different bank groups
    const int q = e / 2;
    f = q / 8;
    kk = 2 * ((q % 8) ^ ((f >> 1) & 7));
    return (uint32_t)(((int64_t)f * ld + kk) * 8);
}

template <int BT, bool TA, bool TB, bool PACKED>
__global__ __launch_bounds__(BT == 128 ? 512 : 256)
__attribute__((amdgpu_waves_per_eu(BT == 128 ? 2 : 4))) void k_dgemm(DgemmArgs g)
{
    constexpr int NW = BT == 128 ? 8 : 4;          // waves
    constexpr int WGN = NW / 2;                     // wave columns along n (two wave rows along m)
    constexpr int WM = BT / 2, WN = BT / WGN;       // wave tile
    constexpr int TMt = WM / 16, TNt = WN / 16;     // matrix-core tiles per wave along m and n
    constexpr bool AF = !TA, BF = TB;               // free index contiguous in memory
    constexpr int NI = BT / 8;                      // copies per operand and step (1 KB each)
    constexpr int NDMA = 2 * NI / NW;               // copies per wave and step
    constexpr int SLOT = 2 * KS * BT;               // doubles per slot: A part, then B part
    constexpr int NSL = BT == 128 ? 3 : 2;          // ring slots (copies NSL - 1 steps ahead)
    static_assert(TMt % 2 == 0 && TNt % 2 == 0 && NDMA * NW == 2 * NI && NDMA <= 15, "shape");
    __shared__ d2 ring0[SLOT / 2], ring1[SLOT / 2], ring2[NSL == 3 ? SLOT / 2 : 1];

    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int wm = wave & 1, wn = wave >> 1;
    const int M = g.m, N = g.n, K = g.k;
    const int mt = (M + BT - 1) / BT, nt = (N + BT - 1) / BT;
    const int64_t ntiles = PACKED ? (int64_t)mt * (mt + 1) / 2 * g.batch : (int64_t)mt * nt * g.batch;
    const int64_t bid = blockIdx.x;
    if (bid >= ntiles) return;
    int tm, tn, b;
    tile_of<PACKED>(bid, mt, nt, ntiles, tm, tn, b);
    // uniform over the workgroup: kept in scalar registers
    tm = __builtin_amdgcn_readfirstlane(tm);
    tn = __builtin_amdgcn_readfirstlane(tn);
    b = __builtin_amdgcn_readfirstlane(b);
    const int m0 = tm * BT, n0 = tn * BT;
    const double *Ab = g.A + (size_t)b * g.sA;
    const double *Bb = g.B + (size_t)b * g.sB;
    double *C = g.C + (size_t)b * g.sC;

    // this wave's copies: instructions wave * NDMA .. + NDMA - 1 of the 2 NI,
    // A's first, then B's, so that each wave copies from one operand only.
    // Per copy: the lane's byte offset from the step origin (or an offset
    // past every record where its free index lies outside the matrix) and
    // its first k inside the step.
    const bool wA = wave * NDMA < NI;
    const int i0 = wA ? wave * NDMA : wave * NDMA - NI;
    const bool fr = wA ? AF : BF;
    const int64_t ld = wA ? g.lda : g.ldb;
    const int f0 = wA ? m0 : n0, F = wA ? M : N;
    uint32_t coff[NDMA];
    int ck[NDMA];
#pragma unroll
    for (int c = 0; c < NDMA; ++c) {
        int kk, f;
        const uint32_t o = copy_offset<BT>(fr, i0 + c, lane, ld, kk, f);
        coff[c] = f0 + f < F ? o : kOut;
        ck[c] = kk;
    }
    const int nsteps = (K + KS - 1) / KS;
    // the operand's origin at step s is base0 + 16 s kst elements from its
    // matrix, whose last element is ext - 1
    const double *P = wA ? Ab : Bb;
    const int64_t ext = wA ? (TA ? (int64_t)(M - 1) * g.lda + K : (int64_t)(K - 1) * g.lda + M)
                           : (TB ? (int64_t)(K - 1) * g.ldb + N : (int64_t)(N - 1) * g.ldb + K);
    const int64_t base0 = fr ? f0 : (int64_t)f0 * ld;
    const int64_t kst = fr ? ld : 1;
    const int dpart = (wA ? 0 : KS * BT) + i0 * 128;       // doubles into the slot
    auto issue = [&](int s, d2 *r) {
        const int k0 = min(s, nsteps - 1) * KS;
        const int64_t org = base0 + (int64_t)k0 * kst;
        // the descriptor admits the operand's bytes from the step origin to
        // its last element, so that no copy reads outside the matrix
        const int64_t bytes = (ext - org) * 8;
        const int rec = bytes < kRecords ? (int)bytes : kRecords;
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void *)(P + org), 0, rec, kBufWord3);
        double *d = reinterpret_cast<double *>(r) + dpart;
        if (k0 + KS <= K) {
#pragma unroll
            for (int c = 0; c < NDMA; ++c) dma16(rs, coff[c], d + c * 128);
        } else {
#pragma unroll
            for (int c = 0; c < NDMA; ++c) dma16(rs, k0 + ck[c] < K ? coff[c] : kOut, d + c * 128);
        }
    };

    // 16-byte position of (free index f, k pair p) in the k-contiguous form
    auto kpos = [](int f, int p) { return f * 8 + (p ^ ((f >> 1) & 7)); };
    // operand reads of a step: lane (r = lane % 16, group gg = lane / 16)
    const int r16 = lane & 15, gg = lane >> 4;
    d4 acc[TNt][TMt];
#pragma unroll
    for (int j = 0; j < TNt; ++j)
#pragma unroll
        for (int i = 0; i < TMt; ++i) acc[j][i] = d4{0.0, 0.0, 0.0, 0.0};

    int s = 0;
    auto step = [&](auto slot) -> bool {
        constexpr int S = decltype(slot)::value;
        const d2 *const rg = S == 0 ? ring0 : (S == 1 ? ring1 : ring2);
        d2 *const rn = NSL == 2 ? (S == 0 ? ring1 : ring0) : (S == 0 ? ring2 : (S == 1 ? ring0 : ring1));
        // this wave's copies of step s are done once at most the next step's
        // NDMA are outstanding (with two slots: none)
        __builtin_amdgcn_s_waitcnt(0x0f70 | (NSL == 3 ? NDMA : 0));     // vmcnt(NDMA) or vmcnt(0)
        __builtin_amdgcn_s_barrier();
        const double *ra = reinterpret_cast<const double *>(rg);
        const double *rb = ra + KS * BT;
        // a[j][x][e2]: m side; b[j][y][e2]: n side.  For the free form x (y)
        // runs over tile pairs and e2 over the pair's even / odd tile at k
        // step 2 j + e; for the k form x (y) runs over tiles and e2 over the
        // two k steps 2 j, 2 j + 1.
        d2 a[2][2][TMt], bv[2][2][TNt];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            if (AF) {
#pragma unroll
                for (int e = 0; e < 2; ++e)
#pragma unroll
                    for (int p = 0; p < TMt / 2; ++p)
                        a[j][e][p] = *reinterpret_cast<const d2 *>(ra + (2 * (4 * j + gg) + e) * BT + wm * WM + 32 * p +
                                                                   2 * r16);
            } else {
#pragma unroll
                for (int i = 0; i < TMt; ++i)
                    a[j][0][i] = *reinterpret_cast<const d2 *>(ra + kpos(wm * WM + 16 * i + r16, 4 * j + gg) * 2);
            }
            if (BF) {
#pragma unroll
                for (int e = 0; e < 2; ++e)
#pragma unroll
                    for (int p = 0; p < TNt / 2; ++p)
                        bv[j][e][p] = *reinterpret_cast<const d2 *>(rb + (2 * (4 * j + gg) + e) * BT + wn * WN + 32 * p +
                                                                    2 * r16);
            } else {
#pragma unroll
                for (int i = 0; i < TNt; ++i)
                    bv[j][0][i] = *reinterpret_cast<const d2 *>(rb + kpos(wn * WN + 16 * i + r16, 4 * j + gg) * 2);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        issue(s + NSL - 1, rn);
        __builtin_amdgcn_sched_barrier(0);
        // the second k of a pair straddling an odd K lies outside the matrix
        const int k0 = s * KS;
        if (k0 + KS > K) {
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const bool out = k0 + 2 * (4 * j + gg) + 1 >= K;
                if (!AF)
#pragma unroll
                    for (int i = 0; i < TMt; ++i) a[j][0][i].y = out ? 0.0 : a[j][0][i].y;
                if (!BF)
#pragma unroll
                    for (int i = 0; i < TNt; ++i) bv[j][0][i].y = out ? 0.0 : bv[j][0][i].y;
            }
        }
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 2; ++e)
#pragma unroll
                for (int y = 0; y < TNt; ++y)
#pragma unroll
                    for (int x = 0; x < TMt; ++x) {
                        const double av = AF ? a[j][e][x >> 1][x & 1] : a[j][0][x][e];
                        const double bw = BF ? bv[j][e][y >> 1][y & 1] : bv[j][0][y][e];
                        acc[y][x] = __builtin_amdgcn_mfma_f64_16x16x4f64(bw, av, acc[y][x], 0, 0, 0);
                    }
        return ++s < nsteps;
    };
    if (nsteps > 0) {
        issue(0, ring0);
        if (NSL == 3) issue(1, ring1);
        for (;;) {
            if (!step(std::integral_constant<int, 0>())) break;
            if (!step(std::integral_constant<int, 1>())) break;
            if constexpr (NSL == 3)
                if (!step(std::integral_constant<int, 2>())) break;
        }
    }
    // no copy into this workgroup's LDS may outlive it
    __builtin_amdgcn_s_waitcnt(0x0f70);                                 // vmcnt(0)

    // lane l element q of tile (y, x): n side row 4 q + gg, m side column r16
    auto mof = [&](int x) { return m0 + wm * WM + (AF ? 32 * (x >> 1) + 2 * r16 + (x & 1) : 16 * x + r16); };
    auto nof = [&](int y, int q) {
        const int rr = 4 * q + gg;
        return n0 + wn * WN + (BF ? 32 * (y >> 1) + 2 * rr + (y & 1) : 16 * y + rr);
    };
    const double alpha = g.alpha, beta = g.beta;
#pragma unroll
    for (int y = 0; y < TNt; ++y)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int n = nof(y, q);
#pragma unroll
            for (int x = 0; x < TMt; ++x) {
                const int m = mof(x);
                const double v = alpha * acc[y][x][q];
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
}

template <int BT, bool PACKED>
hipError_t launch_t(bool ta, bool tb, const DgemmArgs &g, int64_t tiles, hipStream_t s)
{
    const dim3 grid((unsigned)tiles), block(BT == 128 ? 512 : 256);
    if (!ta && !tb)     hipLaunchKernelGGL((k_dgemm<BT, false, false, PACKED>), grid, block, 0, s, g);
    else if (ta && !tb) hipLaunchKernelGGL((k_dgemm<BT, true, false, PACKED>), grid, block, 0, s, g);
    else if (!ta && tb) hipLaunchKernelGGL((k_dgemm<BT, false, true, PACKED>), grid, block, 0, s, g);
    else                hipLaunchKernelGGL((k_dgemm<BT, true, true, PACKED>), grid, block, 0, s, g);
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
    if (lda > kMaxLd || ldb > kMaxLd) return hipErrorInvalidValue;
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
    if (lda > kMaxLd || ldb > kMaxLd) return hipErrorInvalidValue;
    const int64_t mt = (m + T - 1) / T;
    const int64_t tiles = mt * (mt + 1) / 2 * batch;
    if (tiles > INT32_MAX) return hipErrorInvalidValue;
    DgemmArgs g{m, m, k, batch, 1.0, 0.0, A, lda, sA, B, ldb, sB, P, m, sP};
    return launch_t<T, true>(ta, tb, g, tiles, s);
}

}  // namespace mp
