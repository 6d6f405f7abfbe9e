// Step d adjoint, mixed precision: dL/dSt from the symmetric tensor H of
// dL/dT (T the third moments of the W^(1/3)-scaled S rows, see
// k_triple_mx.hip), as
//     Shat_u(z) = 3 Sum_{v,w} H[u,v,w] St_v(z) St_w(z)
//               = Sum_{v <= w} Hc[u][(v,w)] St_v(z) St_w(z),
//     Hc[u][(v,w)] = 3 c_vw H[u,v,w],  c_vw = 2 (v < w), 1 (v = w).
// This is a product with a generated right operand: rows u, columns z, depth
// the pairs (v, w).  Pairs come in blocks of 16 x 16 (v block <= w block;
// inside a diagonal block Hc is zero for v > w), 32 pairs per matrix-core
// step.  It costs three times the forward product (each unique triple feeds
// three outputs) and, unlike the forward, reduces over pairs, not z.
//
// Work decomposition: a workgroup owns the output tile of 128 rows u times
// 256 values z and runs over every pair block.  Hc is stored pre-split
// (BF16 hi, lo) in the matrix-core A-operand order, so one 128 x 256-pair
// block is a contiguous 128 KB read; tasks are ordered (row block, z tile)
// and dealt to the XCDs in contiguous runs, so the workgroups of one XCD
// stream the same Hc blocks through their shared L2.  The operand
// St_v(z) St_w(z) is formed in FP32 from the 32 source rows of the pair
// block (staged in LDS once per block), split into BF16 hi and lo, and
// shared through LDS by the eight waves (double-buffered per step).
//
// Arithmetic: A_lo B_hi + A_hi B_lo + A_hi B_hi per term on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation over kFlush pair blocks,
// then added to the FP64 output (each workgroup owns its tile: a plain
// read-modify-write, deterministic).
#include "internal.hpp"

#include <algorithm>

namespace mp {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));

constexpr int AI = 256;            // output rows per workgroup
constexpr int RB = 4;              // 16-row tiles per wave
constexpr int TW = 4;              // 16-wide column tiles per wave
constexpr int PB = 16;             // pair block: 16 v x 16 w
constexpr int KS = PB * PB / 32;   // 32-pair steps per pair block
constexpr int ZT = 128;            // z values per workgroup
constexpr int NCT = ZT / 16;       // 16-wide column tiles
constexpr int ZBW = ZT / 32;       // z blocks of 32 per workgroup
constexpr int kFlush = 32;         // pair blocks per FP32 partial sum
constexpr int SJ_LD = ZT + 4;      // padded LDS rows (floats)
constexpr int SK_LD = PB + 4;

__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_s_waitcnt(0xc07f);       // lgkmcnt(0) only: global loads stay in flight
    __builtin_amdgcn_s_barrier();
}

// x = hi + lo for two values a, b: hi and lo are BF16 roundings to nearest
// even (v_cvt_pk_bf16_f32), packed as (a, b) halves of h and l.
__device__ __forceinline__ void split2(float a, float b, uint32_t &h, uint32_t &l)
{
    const bf2 hv = {(__bf16)a, (__bf16)b};
    h = __builtin_bit_cast(uint32_t, hv);
    asm("" : "+v"(h));                        // keep one conversion: unpack h itself below
    const bf2 lv = {(__bf16)(a - __uint_as_float(h << 16)), (__bf16)(b - __uint_as_float(h & 0xffff0000u))};
    l = __builtin_bit_cast(uint32_t, lv);
}

__device__ __forceinline__ bf8 as_bf8(uint4 v)
{
    bf8 r;
    __builtin_memcpy(&r, &v, sizeof(r));
    return r;
}

struct AdjArgs {
    const int2 *pblocks;    // (v block, w block), v block <= w block
    int npb;
    int nib;                // row blocks of AI
    int nzt;                // z tiles of ZT
    int U;                  // rows holding data (rows >= U are zero)
    int64_t upad;           // rows per z block of the z-blocked layouts
};

__global__ __launch_bounds__(512) void k_adj_bt(AdjArgs A, const float *__restrict__ S32,
                                                const uint4 *__restrict__ Hc, double *__restrict__ Shat)
{
    __shared__ float SrcJ[2][PB][SJ_LD];      // [pair-block parity][v local][z]
    __shared__ float SrcK[2][ZT][SK_LD];      // [pair-block parity][z][w local]
    __shared__ uint4 Bb[2][NCT][2][64];       // [step parity][column tile][hi/lo][lane]

    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int rg = wave & 3, ch = wave >> 2;   // 64-row group, 4-tile column half
    // tasks (row block, z tile), row block outer, dealt to the 8 XCDs in
    // contiguous runs
    const int ntasks = A.nib * A.nzt;
    const int task = [&] {
        const int x = blockIdx.x & 7, idx = blockIdx.x >> 3;
        const int base = ntasks >> 3, rem = ntasks & 7;
        return x * base + (x < rem ? x : rem) + idx;
    }();
    const int ib = task / A.nzt, zt = task % A.nzt;
    const int64_t zb0 = (int64_t)zt * ZBW;
    const int u0 = ib * AI + rg * 16 * RB;
    const bool active = u0 < A.U;              // wave-uniform: some row holds data

    f4 acc[RB][TW];
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < TW; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

    // ---- staging of a pair block's 32 source rows over the z tile: 1024
    // float4, two per thread.  Part 0, the v rows: a wave covers two rows'
    // 128 z (contiguous LDS writes); part 1, the w rows: consecutive lanes
    // take consecutive rows, so the transposed LDS writes spread over banks.
    auto sload1 = [&](int pb, int i) -> f4 {
        const int2 b = A.pblocks[pb];
        int grow, z4;
        if (i == 0) { grow = b.x * PB + (t >> 5); z4 = t & 31; }
        else        { grow = b.y * PB + (t & 15); z4 = t >> 4; }
        return *reinterpret_cast<const f4 *>(S32 + (((zb0 + (z4 >> 3)) * A.upad + grow) << 5) + 4 * (z4 & 7));
    };
    auto sstore1 = [&](int sb, int i, f4 v) {
        if (i == 0) {
            *reinterpret_cast<f4 *>(&SrcJ[sb][t >> 5][4 * (t & 31)]) = v;
        } else {
            const int zl = 4 * (t >> 4), row = t & 15;
#pragma unroll
            for (int e = 0; e < 4; ++e) SrcK[sb][zl + e][row] = v[e];
        }
    };
    // ---- operand of step ks of the pair block staged in SrcJ/K[sb]: column
    // tile `wave`.  Lane: z = tile * 16 + lane % 16, v local = 2 ks + lane /
    // 32, w local = 8 ((lane / 16) % 2) + e (matrix-core depth index
    // 8 (lane / 16) + e of the step).  The LDS reads are issued early (gread)
    // and the products formed later (gwrite), under matrix-core work.
    float gsv;
    f4 gw0, gw1;
    auto gread = [&](int sb, int ks) {
        const int vl = 2 * ks + (lane >> 5), wh = ((lane >> 4) & 1) * 8;
        const int zl = wave * 16 + (lane & 15);
        gsv = SrcJ[sb][vl][zl];
        gw0 = *reinterpret_cast<const f4 *>(&SrcK[sb][zl][wh]);
        gw1 = *reinterpret_cast<const f4 *>(&SrcK[sb][zl][wh + 4]);
    };
    auto gwrite = [&](int bb) {
        float v[8];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            v[e] = gsv * gw0[e];
            v[4 + e] = gsv * gw1[e];
        }
        uint32_t h[4], l[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) split2(v[2 * e], v[2 * e + 1], h[e], l[e]);
        Bb[bb][wave][0][lane] = make_uint4(h[0], h[1], h[2], h[3]);
        Bb[bb][wave][1][lane] = make_uint4(l[0], l[1], l[2], l[3]);
    };
    // ---- A fragments (Hc) of step (pb, ks) for this wave's row tiles:
    // Hc[pb][ib][ks][row tile][hi/lo][lane]
    uint4 ah[RB], al[RB];
    auto aload = [&](int pb, int ks) {
        const uint4 *p = Hc + ((((size_t)pb * A.nib + ib) * KS + ks) * (AI / 16) + RB * rg) * 128 + lane;
#pragma unroll
        for (int i = 0; i < RB; ++i) {
            ah[i] = p[i * 128];
            al[i] = p[i * 128 + 64];
        }
    };

    // ---- output: this wave's tiles (row tile i, column tile TW ch + j) at
    // Shat[zb][u][32], u = u0 + 16 i + 4 (lane / 16) + q, z = 16 (TW ch + j) + lane % 16
    const int zl0 = ch * 16 * TW + (lane & 15);
    auto flush = [&](bool first) {
#pragma unroll
        for (int i = 0; i < RB; ++i) {
            const int ub = u0 + 16 * i + 4 * (lane >> 4);
            double old[TW][4];
#pragma unroll
            for (int j = 0; j < TW; ++j) {
                const int zl = zl0 + 16 * j;
                const double *p = Shat + ((((zb0 + (zl >> 5)) * A.upad + ub) << 5) + (zl & 31));
#pragma unroll
                for (int q = 0; q < 4; ++q) old[j][q] = first ? 0.0 : p[q * 32];
            }
#pragma unroll
            for (int j = 0; j < TW; ++j) {
                const int zl = zl0 + 16 * j;
                double *p = Shat + ((((zb0 + (zl >> 5)) * A.upad + ub) << 5) + (zl & 31));
#pragma unroll
                for (int q = 0; q < 4; ++q) p[q * 32] = old[j][q] + (double)acc[i][j][q];
            }
        }
#pragma unroll
        for (int i = 0; i < RB; ++i)
#pragma unroll
            for (int j = 0; j < TW; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    };

    const int npb = A.npb;
    // prologue: sources of pair block 0, operand of step (0, 0), A of (0, 0)
    {
        const f4 v0 = sload1(0, 0), v1 = sload1(0, 1);
        sstore1(0, 0, v0);
        sstore1(0, 1, v1);
    }
    lds_barrier();
    gread(0, 0);
    gwrite(0);
    aload(0, 0);
    lds_barrier();
    f4 sreg = f4{0.f, 0.f, 0.f, 0.f};

    int since_flush = 0;
    bool first = true;
    for (int pb = 0; pb < npb; ++pb) {
        const int sb = pb & 1;
#pragma unroll 1
        for (int ks = 0; ks < KS; ++ks) {
            const int bb = ks & 1;             // KS is even: step parity = ks parity
            // the step after this one: next ks, or step 0 of the next pair block
            const bool last_step = ks == KS - 1;
            const int nsb = last_step ? sb ^ 1 : sb, nks = last_step ? 0 : ks + 1;
            const bool has_next = !(last_step && pb + 1 == npb);
            if (has_next) gread(nsb, nks);
            if (active) {
                // B fragments one tile ahead of their matrix-core use
                uint4 bh = Bb[bb][ch * TW][0][lane], bl = Bb[bb][ch * TW][1][lane];
#pragma unroll
                for (int j = 0; j < TW; ++j) {
                    uint4 nbh = bh, nbl = bl;
                    if (j + 1 < TW) {
                        nbh = Bb[bb][ch * TW + j + 1][0][lane];
                        nbl = Bb[bb][ch * TW + j + 1][1][lane];
                    }
                    const bf8 h8 = as_bf8(bh), l8 = as_bf8(bl);
#pragma unroll
                    for (int i = 0; i < RB; ++i)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf8(al[i]), h8, acc[i][j], 0, 0, 0);
#pragma unroll
                    for (int i = 0; i < RB; ++i)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf8(ah[i]), l8, acc[i][j], 0, 0, 0);
#pragma unroll
                    for (int i = 0; i < RB; ++i)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf8(ah[i]), h8, acc[i][j], 0, 0, 0);
                    // operand of the next step
                    if (j == 1 && has_next) gwrite(bb ^ 1);
                    __builtin_amdgcn_sched_barrier(0);
                    bh = nbh;
                    bl = nbl;
                }
            } else if (has_next) {
                gwrite(bb ^ 1);
            }
            // sources of pair block pb + 1 into the other buffer (its last
            // reader formed this block's first operand): one float4 per thread
            // per step, loaded in steps 0 and 1 and stored one step later, well
            // before step KS - 1 forms the next block's operand
            if (pb + 1 < npb) {
                if (ks == 1 || ks == 2) sstore1(sb ^ 1, ks - 1, sreg);
                if (ks <= 1) sreg = sload1(pb + 1, ks);
            }
            if (last_step && (++since_flush == kFlush || pb + 1 == npb)) {
                if (active) flush(first);
                since_flush = 0;
                first = false;
            }
            // A fragments of the next step (the other wave of the SIMD covers
            // their latency)
            if (has_next) aload(last_step ? pb + 1 : pb, nks);
            lds_barrier();
        }
    }
}

}  // namespace

hipError_t launch_adj_triple_mixed(const int2 *pblocks, int npb, int U, int64_t upad, int64_t nzb,
                                   const float *S32, const uint4 *Hc, double *Shat, hipStream_t s)
{
    if (upad % AI != 0 || upad < U || nzb % ZBW != 0 || npb <= 0) return hipErrorInvalidValue;
    AdjArgs a;
    a.pblocks = pblocks;
    a.npb = npb;
    a.nib = (int)(upad / AI);
    a.nzt = (int)(nzb / ZBW);
    a.U = U;
    a.upad = upad;
    const int64_t ntasks = (int64_t)a.nib * a.nzt;
    if (ntasks == 0) return hipSuccess;
    if (ntasks > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_adj_bt, dim3((unsigned)ntasks), dim3(512), 0, s, a, S32, Hc, Shat);
    return hipGetLastError();
}

// FP32 copy of the first n values of St, zeros up to ntot (the z tail that
// completes the last z tile)
__global__ void k_f32_copy(int64_t n, int64_t ntot, const double *__restrict__ St, float *__restrict__ S32)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ntot;
         i += (int64_t)gridDim.x * blockDim.x)
        S32[i] = i < n ? (float)St[i] : 0.f;
}

hipError_t launch_f32_copy(int64_t n, int64_t ntot, const double *St, float *S32, hipStream_t s)
{
    const int64_t blocks = std::min<int64_t>((ntot + 255) / 256, 1 << 20);
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_f32_copy, dim3((unsigned)blocks), dim3(256), 0, s, n, ntot, St, S32);
    return hipGetLastError();
}

static_assert(kZBlockPad % ZBW == 0, "z tiles must divide the z-block padding");
static_assert(kRowPad % AI == 0, "row blocks must divide the row padding");
int adj_rowblock_mixed() { return AI; }

}  // namespace mp
