// Step d adjoint in FP64: the same product as the mixed kernel,
//     Shat_u(z) = Sum_{v <= w} Hc[u][(v,w)] St_v(z) St_w(z),
//     Hc[u][(v,w)] = 3 c_vw H[u,v,w]  (c = 2 for v < w, 1 for v = w),
// on v_mfma_f64_16x16x4f64 with FP64 accumulation over every pair.
//
// A workgroup owns the output tile of 128 rows u times 128 values z and runs
// over the pair blocks (16 v x 16 w, v block <= w block); a super-step is one
// v of the block (16 pairs = four 4-deep matrix-core steps).  Hc is stored
// in the A-operand order, [pair block][row block][v][step][row tile][lane],
// so a wave's fragments of one super-step are eight coalesced loads.  The
// operand St_v(z) St_w(z) of a super-step (16 pairs x 128 z) is formed once
// per workgroup from the block's 32 source rows (staged in LDS per pair
// block, double-buffered) and shared through LDS (double-buffered per
// super-step).  Eight waves: wave w owns rows 32 (w % 4) .. + 31 and column
// tiles 4 (w / 4) .. + 3.  Tasks (row block, z tile) are ordered row block
// first and dealt to the XCDs in contiguous runs, so one XCD's workgroups
// stream the same Hc blocks through their L2.
#include "internal.hpp"

#include <algorithm>

namespace mp {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int AI = 128;            // output rows per workgroup
constexpr int PB = 16;             // pair block: 16 v x 16 w
constexpr int ZT = 128;            // z values per workgroup
constexpr int NCT = ZT / 16;       // column tiles
constexpr int ZBW = ZT / 32;       // z blocks of 32 per workgroup
constexpr int SLD = ZT + 2;        // padded LDS rows (doubles)

__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_s_waitcnt(0xc07f);       // lgkmcnt(0) only: global loads stay in flight
    __builtin_amdgcn_s_barrier();
}

struct AdjArgs {
    const int2 *pblocks;
    int npb, nib, nzt, U;
    int64_t upad;
};

__global__ __launch_bounds__(512) void k_adj_f64(AdjArgs A, const double *__restrict__ St,
                                                 const double *__restrict__ Hc, double *__restrict__ Shat)
{
    __shared__ double Src[2][2 * PB][SLD];    // [pair-block parity][v rows, then w rows][z]
    __shared__ double Bb[2][4][NCT][64];      // [super-step parity][step][column tile][lane]

    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int rg = wave & 3, ch = wave >> 2;
    const int ntasks = A.nib * A.nzt;
    const int task = [&] {
        const int x = blockIdx.x & 7, idx = blockIdx.x >> 3;
        const int base = ntasks >> 3, rem = ntasks & 7;
        return x * base + (x < rem ? x : rem) + idx;
    }();
    const int ib = task / A.nzt, zt = task % A.nzt;
    const int64_t zb0 = (int64_t)zt * ZBW;
    const int u0 = ib * AI + rg * 32;
    const bool active = u0 < A.U;

    d4 acc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

    // staging: 32 rows x 128 z = 2048 double2, four per thread; a wave covers
    // one row (64 double2 = 128 z)
    double2 sreg[4];
    auto sload = [&](int pb) {
        const int2 b = A.pblocks[pb];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int f = t + 512 * i, row = f >> 6, zq = f & 63;
            const int grow = row < PB ? b.x * PB + row : b.y * PB + row - PB;
            sreg[i] = *reinterpret_cast<const double2 *>(St + (((zb0 + (zq >> 4)) * A.upad + grow) << 5) +
                                                         2 * (zq & 15));
        }
    };
    auto sstore = [&](int sb) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int f = t + 512 * i;
            *reinterpret_cast<double2 *>(&Src[sb][f >> 6][2 * (f & 63)]) = sreg[i];
        }
    };
    // operand of super-step sv (v local = sv, pairs (sv, w) for w = 0..15):
    // step kk, column tile ct, lane -> St_v(z) St_w(z) with w = 4 kk + lane / 16,
    // z = 16 ct + lane % 16.  Wave w forms the (kk, ct) combinations 4 w .. 4 w + 3.
    auto bgen = [&](int sb, int sv, int bb) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int cmb = 4 * wave + q, kk = cmb >> 3, ct = cmb & 7;
            const int zl = 16 * ct + (lane & 15), wl = 4 * kk + (lane >> 4);
            Bb[bb][kk][ct][lane] = Src[sb][sv][zl] * Src[sb][PB + wl][zl];
        }
    };
    // A fragments of super-step (pb, sv): Hc[pb][ib][sv][kk][row tile][lane]
    double a[4][2];
    auto aload = [&](int pb, int sv) {
        const double *p = Hc + (((size_t)pb * A.nib + ib) * PB + sv) * (4 * 8 * 64) + (2 * rg) * 64 + lane;
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
#pragma unroll
            for (int i = 0; i < 2; ++i) a[kk][i] = p[kk * 512 + i * 64];
    };

    const int npb = A.npb;
    sload(0);
    sstore(0);
    lds_barrier();
    bgen(0, 0, 0);
    aload(0, 0);
    sload(npb > 1 ? 1 : 0);
    lds_barrier();

    for (int pb = 0; pb < npb; ++pb) {
        const int sb = pb & 1;
#pragma unroll 1
        for (int sv = 0; sv < PB; ++sv) {
            const int bb = sv & 1;             // PB is even: super-step parity = sv parity
            const bool last = sv == PB - 1;
            const int nsb = last ? sb ^ 1 : sb, nsv = last ? 0 : sv + 1;
            const bool has_next = !(last && pb + 1 == npb);
            if (active) {
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    double b[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) b[j] = Bb[bb][kk][4 * ch + j][lane];
#pragma unroll
                    for (int i = 0; i < 2; ++i)
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kk][i], b[j], acc[i][j], 0, 0, 0);
                    if (kk == 1 && has_next) bgen(nsb, nsv, bb ^ 1);
                }
            } else if (has_next) {
                bgen(nsb, nsv, bb ^ 1);
            }
            // sources of pair block pb + 1 into the other buffer (free since the
            // operand of this block's first super-step was formed), then the
            // loads of pair block pb + 2's sources
            if (sv == PB / 2) {
                sstore(sb ^ 1);
                sload(pb + 2 < npb ? pb + 2 : npb - 1);
            }
            if (has_next) aload(last ? pb + 1 : pb, nsv);
            lds_barrier();
        }
    }
    if (!active) return;
    // D lane l element q: row 4 q + l / 16, column l % 16
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int zl = 16 * (4 * ch + j) + (lane & 15);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int u = u0 + 16 * i + 4 * q + (lane >> 4);
                Shat[(((zb0 + (zl >> 5)) * A.upad + u) << 5) + (zl & 31)] = acc[i][j][q];
            }
        }
}

}  // namespace

hipError_t launch_adj_triple_f64(const int2 *pblocks, int npb, int U, int64_t upad, int64_t nzb,
                                 const double *St, const double *Hc, double *Shat, hipStream_t s)
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
    hipLaunchKernelGGL(k_adj_f64, dim3((unsigned)ntasks), dim3(512), 0, s, a, St, Hc, Shat);
    return hipGetLastError();
}

static_assert(kZBlockPad % ZBW == 0, "z tiles must divide the z-block padding");
int adj_rowblock() { return AI; }

}  // namespace mp
