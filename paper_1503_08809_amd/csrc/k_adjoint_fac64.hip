// Step d adjoint in FP64, in factored form (the same decomposition as the
// mixed kernel in k_adjoint_fac.hip):
//     dL/dSt_u(z) = Sum_v St_v(z) D_v[u](z),  D_v[u](z) = Sum_{w >= v} Hc[u][(v,w)] St_w(z),
// with Hc[u][(v,w)] = 3 c_vw H[u,v,w] (c = 2 for v < w, 1 for v = w; see
// k_adjoint.hip).  Each D_v is a plain product on v_mfma_f64_16x16x4f64 whose
// right operand is the S rows themselves, so no product operand is formed;
// its columns are scaled by St_v(z) and summed over v in FP64 registers, and
// the tile is written once at the end.
//
// A workgroup owns 128 rows u x 128 values z and runs over v, and for each v
// over the 16-wide w steps from the one holding v to the last (four 4-deep
// matrix-core steps each).  Eight waves: wave w owns rows 32 (w % 4) .. + 31
// (two row tiles) and column tiles 4 (w / 4) .. + 3 (16 z each).  Both
// operands of a step are copied from memory straight into LDS (buffer_load
// ... lds, no registers) two steps ahead through a ring of three slots (issued
// after the step's LDS reads), one barrier per step: Hc (16 KB, stored in the matrix-core A order) and the 16
// S rows of the step at the workgroup's 128 z (16 KB, gathered from the
// z-blocked layout row by row, one padded LDS row each).
#include "internal.hpp"

#include <algorithm>
#include <type_traits>

namespace mp {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int AI = 128;            // output rows per workgroup
constexpr int RB = 2;              // 16-row tiles per wave
constexpr int TW = 4;              // 16-wide column tiles per wave
constexpr int ZT = 128;            // z values per workgroup
constexpr int ZBW = ZT / 32;       // z blocks of 32 per workgroup
constexpr int KW = 16;             // w per step
constexpr int BLD = ZT + 2;        // padded LDS row of B (doubles)

// LDS DMA in buffer form: each lane's 16 bytes land at lds_base + 16 lane
// (see k_adjoint_fac.hip for why the buffer form)
__device__ __forceinline__ void dma16(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff, void *lds_base)
{
    __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void *)lds_base, 16, voff, soff,
                                             0, 0);
}
constexpr int kBufWord3 = 0x00020000;         // descriptor word 3: 32-bit data format, raw access

constexpr int RING = 3;
constexpr int SLOT_A = AI * KW;               // doubles of Hc per slot
constexpr int SLOT = SLOT_A + KW * BLD;       // + the 16 S rows

struct Fac64Args {
    int U, nws, nib, nzt;
    int64_t upad;
};

__global__ __launch_bounds__(512) void k_adj_fac64(Fac64Args A, const double *__restrict__ St,
                                                   const double *__restrict__ Hc, double *__restrict__ Shat)
{
    // ring of three steps, one array per slot (so that the compiler sees that
    // copies into one slot never alias reads of another): Hc as
    // [k step][row tile][lane], then the S rows [w][z] with padded rows
    __shared__ double ring0[SLOT], ring1[SLOT], ring2[SLOT];

    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int rg = wave & 3, ch = wave >> 2;
    const int ntasks = A.nib * A.nzt;
    const int task = [&] {
        const int x = blockIdx.x & 7, idx = blockIdx.x >> 3;
        const int base = ntasks >> 3, rem = ntasks & 7;
        return x * base + (x < rem ? x : rem) + idx;
    }();
    // consecutive tasks (co-resident on one XCD) take the row blocks of one
    // z tile in turn
    const int ib = task % A.nib, zt = task / A.nib;
    const int64_t zb0 = (int64_t)zt * ZBW;
    const int u0 = ib * AI + rg * 16 * RB;
    const bool active = u0 < A.U;
    const int U = A.U, nws = A.nws;
    const int64_t nsteps = v_step_offset16(U, nws);
    const uint32_t voff = (uint32_t)lane * 16;

    // this wave's copies of a step: 2 KB of Hc (bytes 2 KB wave ..) and the S
    // rows w0 + 2 wave, w0 + 2 wave + 1 (a lane: z = 2 lane, 2 lane + 1)
    const uint32_t bvoff = (uint32_t)(((lane >> 4) * A.upad * 32 + 2 * (lane & 15)) * 8);
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void *)(St + zb0 * A.upad * 32), 0,
                                          (int)(ZBW * A.upad * 32 * sizeof(double)), kBufWord3);
    auto issue = [&](int64_t st, int ws, double *r) {
        const double *a = Hc + ((size_t)st * A.nib + ib) * SLOT_A + (size_t)wave * 256;
        const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc((void *)a, 0, 2048, kBufWord3);
        dma16(ra, voff, 0, r + wave * 256);
        dma16(ra, voff, 1024, r + wave * 256 + 128);
        const int w = KW * ws + 2 * wave;
        dma16(rs, bvoff, (uint32_t)(w * 32 * 8), r + SLOT_A + (2 * wave) * BLD);
        dma16(rs, bvoff, (uint32_t)((w + 1) * 32 * 8), r + SLOT_A + (2 * wave + 1) * BLD);
    };
    // St_v at this lane's columns: z = zb0 * 32 + 16 (TW ch + j) + lane % 16
    const int zl0 = ch * 16 * TW + (lane & 15);
    auto svload = [&](int v, double (&sv)[TW]) {
#pragma unroll
        for (int j = 0; j < TW; ++j) {
            const int zl = zl0 + 16 * j;
            sv[j] = St[(((zb0 + (zl >> 5)) * A.upad + v) << 5) + (zl & 31)];
        }
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
    // so that every step issues exactly four per wave
    auto issue_next = [&](double *r) {
        issue(ist, iws, r);
        if (ist + 1 < nsteps) {
            ++ist;
            advance(iv, iws);
        }
    };
    issue_next(ring0);
    issue_next(ring1);
    double svd[TW];
    svload(0, svd);

    int v = 0, ws = 0;
    int64_t st = 0;
    auto step = [&](auto slot) -> bool {
        constexpr int S = decltype(slot)::value;
        const double *const r = S == 0 ? ring0 : (S == 1 ? ring1 : ring2);
        double *const rn = S == 0 ? ring2 : (S == 1 ? ring0 : ring1);
        // this wave's copies of step st are done once at most the next step's
        // four are outstanding (loads complete in order; any younger St_v
        // loads only make this stricter)
        __builtin_amdgcn_s_waitcnt(0x0f74);                             // vmcnt(4)
        __builtin_amdgcn_s_barrier();
        const bool vlast = ws == nws - 1;
        // all of this step's operands are read first: copies issued before
        // an LDS read that the compiler cannot prove disjoint make it wait for
        // them in full.  A lane l: row 16 tile + l % 16, w = 4 k + l / 16;
        // B lane l: w = 4 k + l / 16, z = 16 tile + l % 16.
        double a[KW / 4][RB], b[KW / 4][TW];
        if (active) {
            const double *bl = r + SLOT_A + (lane >> 4) * BLD + ch * 16 * TW + (lane & 15);
#pragma unroll
            for (int k = 0; k < KW / 4; ++k) {
#pragma unroll
                for (int i = 0; i < RB; ++i) a[k][i] = r[(k * (AI / 16) + RB * rg + i) * 64 + lane];
#pragma unroll
                for (int j = 0; j < TW; ++j) b[k][j] = bl[4 * k * BLD + 16 * j];
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        issue_next(rn);
        __builtin_amdgcn_sched_barrier(0);
        if (active) {
#pragma unroll
            for (int k = 0; k < KW / 4; ++k)
#pragma unroll
                for (int i = 0; i < RB; ++i)
#pragma unroll
                    for (int j = 0; j < TW; ++j)
                        D[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[k][i], b[k][j], D[i][j], 0, 0, 0);
            if (vlast) {
                // D_v is complete: out += St_v(z) D_v(z), then D = 0
#pragma unroll
                for (int i = 0; i < RB; ++i)
#pragma unroll
                    for (int j = 0; j < TW; ++j) {
                        out[i][j] += svd[j] * D[i][j];
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
    // D lane l element q: row 4 q + l / 16, column l % 16
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < TW; ++j) {
            const int zl = zl0 + 16 * j;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int u = u0 + 16 * i + 4 * q + (lane >> 4);
                Shat[(((zb0 + (zl >> 5)) * A.upad + u) << 5) + (zl & 31)] = out[i][j][q];
            }
        }
}

}  // namespace

hipError_t launch_adj_fac64(int U, int64_t upad, int64_t nzb, const double *St, const double *Hc, double *Shat,
                            hipStream_t s)
{
    if (upad % AI != 0 || upad < U || nzb % ZBW != 0 || U <= 0) return hipErrorInvalidValue;
    // the copies of S rows address up to ZBW z blocks of upad rows in one
    // buffer descriptor (32-bit byte range)
    if ((int64_t)ZBW * upad * 32 * (int64_t)sizeof(double) > INT32_MAX) return hipErrorInvalidValue;
    Fac64Args a;
    a.U = U;
    a.nws = (U + KW - 1) / KW;
    a.nib = (int)(upad / AI);
    a.nzt = (int)(nzb / ZBW);
    a.upad = upad;
    const int64_t ntasks = (int64_t)a.nib * a.nzt;
    if (ntasks == 0) return hipSuccess;
    if (ntasks > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_adj_fac64, dim3((unsigned)ntasks), dim3(512), 0, s, a, St, Hc, Shat);
    return hipGetLastError();
}

static_assert(kZBlockPad % ZBW == 0, "z tiles must divide the z-block padding");
static_assert(kRowPad % AI == 0, "row blocks must divide the row padding");
static_assert(KW == 2 * 8, "each wave copies two S rows per step");
int adj_fac64_rowblock() { return AI; }

}  // namespace mp
