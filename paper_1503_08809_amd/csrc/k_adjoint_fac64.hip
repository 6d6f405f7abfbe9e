// Step d adjoint in FP64, in factored form (the same decomposition as the
// mixed kernel in k_adjoint_fac.hip):
//     dL/dSt_u(z) = Sum_v St_v(z) D_v[u](z),  D_v[u](z) = Sum_{w >= v} Hc[u][(v,w)] St_w(z),
// with Hc[u][(v,w)] = 3 c_vw H[u,v,w] (c = 2 for v < w, 1 for v = w; see
// k_adjoint.hip).  Each D_v is a plain product on v_mfma_f64_16x16x4f64 whose
// right operand is the S rows themselves, so no product operand is formed;
// its columns are scaled by St_v(z) and summed over v in FP64 registers, and
// the tile is written once at the end.
//
// A workgroup owns a block of rows u x a tile of z values and runs over v, and
// for each v over the 16-wide w steps from the one holding v to the last (four
// 4-deep matrix-core steps each).  Both operands of a step are copied from
// memory straight into LDS (buffer_load ... lds, no registers) two steps ahead
// through a ring of three slots (issued after the step's LDS reads), one
// barrier per step: the step's Hc rows (2 KB per 16-row tile, stored in the
// matrix-core A order) and its 16 S rows at the workgroup's z (gathered from
// the z-blocked layout row by row).  All LDS reads are 16 bytes per lane, so
// that none is merged into a paired read the compiler can no longer tell
// apart from the copies in flight.
//
// Two shapes of one kernel:
//  * full row blocks: 128 rows x 128 z, eight waves of 32 rows (two row tiles)
//    x 64 z (four column tiles);
//  * the last, partial row block: up to four live row tiles x 256 z, each
//    wave all of them x 32 z, so that its cost follows its live rows (a full
//    block's shape would keep one SIMD as busy as in a full block).
#include "internal.hpp"

#include <algorithm>
#include <type_traits>

namespace mp {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

constexpr int AI = 128;            // rows per row block (the Hc block)
constexpr int KW = 16;             // w per step
constexpr int SLOT_A = AI * KW;    // doubles of Hc per step and row block

// LDS DMA in buffer form: each lane's 16 bytes land at lds_base + 16 lane
// (see k_adjoint_fac.hip for why the buffer form)
__device__ __forceinline__ void dma16(__amdgpu_buffer_rsrc_t rs, uint32_t voff, void *lds_base)
{
    __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void *)lds_base, 16, voff, 0,
                                             0, 0);
}
constexpr int kBufWord3 = 0x00020000;         // descriptor word 3: 32-bit data format, raw access

struct Fac64Args {
    int U, nws;
    int nib;        // row blocks of Hc
    int nblk;       // row blocks of this launch (from ib0)
    int ib0;        // first row block
    int rt0;        // first row tile inside the block (partial block)
    int nzt;        // z tiles
    int64_t upad;
};

// RB row tiles x TW column tiles per wave; NRG row groups of waves (the other
// 8 / NRG wave groups split the z tile).  TW is even: column tiles 2 p and
// 2 p + 1 of a wave hold the even and odd z of one 32-wide run, so a lane's two
// B values are adjacent.
template <int RB, int TW, int NRG>
__global__ __launch_bounds__(512) void k_adj_fac64(Fac64Args A, const double *__restrict__ St,
                                                   const double *__restrict__ Hc, double *__restrict__ Shat)
{
    constexpr int NCG = 8 / NRG;                 // column groups
    constexpr int ZT = 16 * TW * NCG;            // z per workgroup
    constexpr int ZBW = ZT / 32;                 // z blocks of 32 per workgroup
    constexpr int NRT = RB * NRG;                // row tiles of the workgroup
    constexpr int BPR = ZT / 128;                // 1 KB copies per S row
    constexpr int NDMA = 2 + 2 * BPR;            // copies per wave and step
    constexpr int SLOT = SLOT_A + KW * ZT;
    static_assert(TW % 2 == 0 && NRT <= 8 && NCG * NRG == 8, "tile shape");
    static_assert(NDMA <= 15, "vmcnt field");
    // ring of three steps, one array per slot (so that the compiler sees that
    // copies into one slot never alias reads of another): Hc row tiles
    // [row tile][k pair][lane][2], then the S rows [w][z]
    __shared__ d2 ring0[SLOT / 2], ring1[SLOT / 2], ring2[SLOT / 2];

    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int rg = wave % NRG, ch = wave / NRG;
    const int ntasks = A.nblk * A.nzt;
    const int task = [&] {
        const int x = blockIdx.x & 7, idx = blockIdx.x >> 3;
        const int base = ntasks >> 3, rem = ntasks & 7;
        return x * base + (x < rem ? x : rem) + idx;
    }();
    // consecutive tasks (co-resident on one XCD) take the row blocks of one
    // z tile in turn
    const int ib = A.ib0 + task % A.nblk, zt = task / A.nblk;
    const int64_t zb0 = (int64_t)zt * ZBW;
    const int u0 = ib * AI + (A.rt0 + rg * RB) * 16;
    const bool active = u0 < A.U;
    const int U = A.U, nws = A.nws;
    const int64_t nsteps = v_step_offset16(U, nws);
    const uint32_t voff = (uint32_t)lane * 16;

    // this wave's copies of a step: Hc row tile A.rt0 + wave (2 KB; none past
    // the workgroup's row tiles: the range is empty and the base stays inside
    // the row block) and S rows w0 + 2 wave, w0 + 2 wave + 1 in 1 KB pieces of
    // 128 z (a lane: z = 2 lane, 2 lane + 1 of the piece)
    const uint32_t arec = wave < NRT ? 2048u : 0u;
    const int arow = min(A.rt0 + wave, AI / 16 - 1);
    const uint32_t bvoff = (uint32_t)(((lane >> 4) * A.upad * 32 + 2 * (lane & 15)) * 8);
    const uint32_t bpiece = (uint32_t)(4 * A.upad * 32 * 8);
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void *)(St + zb0 * A.upad * 32), 0,
                                          (int)(ZBW * A.upad * 32 * sizeof(double)), kBufWord3);
    auto issue = [&](int64_t st, int ws, d2 *r) {
        const double *a = Hc + ((size_t)st * A.nib + ib) * SLOT_A + (size_t)arow * 256;
        const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc((void *)a, 0, (int)arec, kBufWord3);
        dma16(ra, voff, r + wave * 128);
        dma16(ra, voff + 1024, r + wave * 128 + 64);
        const int w = KW * ws + 2 * wave;
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int pc = 0; pc < BPR; ++pc)
                dma16(rs, bvoff + (uint32_t)((w + h) * 32 * 8) + pc * bpiece,
                      r + SLOT_A / 2 + ((2 * wave + h) * ZT + 128 * pc) / 2);
    };
    // a lane's columns: tile 2 p + e is z = zl0 + 32 p + e of the z tile
    const int zl0 = ch * 16 * TW + 2 * (lane & 15);
    auto zidx = [&](int zl, int row) -> int64_t { return (((zb0 + (zl >> 5)) * A.upad + row) << 5) + (zl & 31); };
    auto svload = [&](int v, d2 (&sv)[TW / 2]) {
#pragma unroll
        for (int p = 0; p < TW / 2; ++p) sv[p] = *reinterpret_cast<const d2 *>(St + zidx(zl0 + 32 * p, v));
    };

    d4 out[RB][TW], D[RB][TW];
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < TW; ++j) {
            out[i][j] = d4{0.0, 0.0, 0.0, 0.0};
            D[i][j] = d4{0.0, 0.0, 0.0, 0.0};
        }

    // the step sequence: v = 0.., for each v the w steps v / 16 .. nws - 1;
    // (iv, iws) runs two steps ahead of (v, ws) to issue the copies
    int iv = 0, iws = 0;
    int64_t ist = 0;
    auto advance = [&](int &vv, int &ww) {
        if (ww == nws - 1) { ++vv; ww = vv >> 4; } else { ++ww; }
    };
    // past the last step the copies repeat it (into a slot no step reads),
    // so that every step issues exactly NDMA per wave
    auto issue_next = [&](d2 *r) {
        issue(ist, iws, r);
        if (ist + 1 < nsteps) {
            ++ist;
            advance(iv, iws);
        }
    };
    issue_next(ring0);
    issue_next(ring1);
    d2 svd[TW / 2];
    svload(0, svd);

    int v = 0, ws = 0;
    int64_t st = 0;
    auto step = [&](auto slot) -> bool {
        constexpr int S = decltype(slot)::value;
        const d2 *const r = S == 0 ? ring0 : (S == 1 ? ring1 : ring2);
        d2 *const rn = S == 0 ? ring2 : (S == 1 ? ring0 : ring1);
        // this wave's copies of step st are done once at most the next step's
        // NDMA are outstanding (loads complete in order; any younger St_v
        // loads only make this stricter)
        __builtin_amdgcn_s_waitcnt(0x0f70 | NDMA);                      // vmcnt(NDMA)
        __builtin_amdgcn_s_barrier();
        const bool vlast = ws == nws - 1;
        // all of this step's operands are read first: copies issued before an
        // LDS read that the compiler cannot prove disjoint make it wait for
        // them in full.  A lane l: row 16 tile + l % 16, w = 4 k + l / 16
        // (k = 2 pair + e); B lane l: w = 4 k + l / 16, z as above.
        d2 a[RB][2], b[4][TW / 2];
        if (active) {
#pragma unroll
            for (int i = 0; i < RB; ++i)
#pragma unroll
                for (int kp = 0; kp < 2; ++kp) a[i][kp] = r[((RB * rg + i) * 2 + kp) * 64 + lane];
            const d2 *bl = r + SLOT_A / 2 + ((lane >> 4) * ZT + zl0) / 2;
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int p = 0; p < TW / 2; ++p) b[k][p] = bl[(4 * k * ZT + 32 * p) / 2];
        }
        __builtin_amdgcn_sched_barrier(0);
        issue_next(rn);
        __builtin_amdgcn_sched_barrier(0);
        if (active) {
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int i = 0; i < RB; ++i)
#pragma unroll
                    for (int j = 0; j < TW; ++j)
                        D[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i][k >> 1][k & 1], b[k][j >> 1][j & 1],
                                                                       D[i][j], 0, 0, 0);
            if (vlast) {
                // D_v is complete: out += St_v(z) D_v(z), then D = 0
#pragma unroll
                for (int i = 0; i < RB; ++i)
#pragma unroll
                    for (int j = 0; j < TW; ++j) {
                        out[i][j] += svd[j >> 1][j & 1] * D[i][j];
                        D[i][j] = d4{0.0, 0.0, 0.0, 0.0};
                    }
            }
        }
        if (vlast && v + 1 < U) svload(v + 1, svd);
        advance(v, ws);
        return ++st < nsteps;
    };
    for (;;) {
        if (!step(std::integral_constant<int, 0>())) break;
        if (!step(std::integral_constant<int, 1>())) break;
        if (!step(std::integral_constant<int, 2>())) break;
    }
    // no copy into this workgroup's LDS may outlive it
    __builtin_amdgcn_s_waitcnt(0x0f70);                                 // vmcnt(0)
    if (!active) return;
    // D lane l element q: row 4 q + l / 16, column l % 16 (z as above)
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int p = 0; p < TW / 2; ++p)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int u = u0 + 16 * i + 4 * q + (lane >> 4);
                *reinterpret_cast<d2 *>(Shat + zidx(zl0 + 32 * p, u)) = d2{out[i][2 * p][q], out[i][2 * p + 1][q]};
            }
}

template <int RB, int TW, int NRG>
hipError_t launch_shape(const Fac64Args &a, int64_t nzb, const double *St, const double *Hc, double *Shat,
                        hipStream_t s)
{
    constexpr int ZBW = TW * (8 / NRG) / 2;
    Fac64Args b = a;
    b.nzt = (int)(nzb / ZBW);
    const int64_t ntasks = (int64_t)b.nblk * b.nzt;
    if (ntasks == 0) return hipSuccess;
    if (ntasks > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_adj_fac64<RB, TW, NRG>), dim3((unsigned)ntasks), dim3(512), 0, s, b, St, Hc, Shat);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_adj_fac64(int U, int64_t upad, int64_t nzb, const double *St, const double *Hc, double *Shat,
                            hipStream_t s)
{
    // z tiles of 128 (full blocks) and 256 (partial block) values
    if (upad % AI != 0 || upad < U || nzb % 8 != 0 || U <= 0) return hipErrorInvalidValue;
    // the copies of S rows address up to 8 z blocks of upad rows in one
    // buffer descriptor (32-bit byte range)
    if ((int64_t)8 * upad * 32 * (int64_t)sizeof(double) > INT32_MAX) return hipErrorInvalidValue;
    Fac64Args a;
    a.U = U;
    a.nws = (U + KW - 1) / KW;
    a.nib = (int)(upad / AI);
    a.upad = upad;
    a.nzt = 0;
    // full row blocks; a last block with eight live row tiles counts as full
    const int nfull = U / AI, tail_tiles = (U - nfull * AI + 15) / 16;
    const bool tail_full = tail_tiles == AI / 16;
    a.ib0 = 0;
    a.nblk = nfull + (tail_full ? 1 : 0);
    a.rt0 = 0;
    hipError_t e = launch_shape<2, 4, 4>(a, nzb, St, Hc, Shat, s);
    if (e != hipSuccess || tail_full) return e;
    // the partial block, in chunks of at most four row tiles
    a.ib0 = nfull;
    a.nblk = 1;
    for (int rt0 = 0; rt0 < tail_tiles && e == hipSuccess; rt0 += 4) {
        a.rt0 = rt0;
        switch (std::min(4, tail_tiles - rt0)) {
        case 1: e = launch_shape<1, 2, 1>(a, nzb, St, Hc, Shat, s); break;
        case 2: e = launch_shape<2, 2, 1>(a, nzb, St, Hc, Shat, s); break;
        case 3: e = launch_shape<3, 2, 1>(a, nzb, St, Hc, Shat, s); break;
        default: e = launch_shape<4, 2, 1>(a, nzb, St, Hc, Shat, s); break;
        }
    }
    return e;
}

static_assert(kZBlockPad % 8 == 0, "z tiles must divide the z-block padding");
static_assert(kRowPad % AI == 0, "row blocks must divide the row padding");
int adj_fac64_rowblock() { return AI; }

}  // namespace mp
