// Step d adjoint, mixed precision, in factored form.  With Hc the tensor of
// dL/dT over pairs v <= w (Hc[u][(v,w)] = 3 c_vw H[u,v,w], c = 2 for v < w,
// 1 for v = w; see k_adjoint.hip),
//     dL/dSt_u(z) = Sum_{v <= w} Hc[u][(v,w)] St_v(z) St_w(z)
//                 = Sum_v St_v(z) D_v[u](z),   D_v[u](z) = Sum_{w >= v} Hc[u][(v,w)] St_w(z).
// Each D_v is a plain matrix product (rows u, columns z, depth w) whose right
// operand is the S rows themselves, stored once pre-split in the matrix-core
// B-operand order, so no product operand has to be formed; its columns are
// then scaled by St_v(z) and summed over v in registers.  The work is the
// same as the pair form (each (u, v, w <= ...) term once).
//
// A workgroup owns 256 rows u x 128 values z and runs over v, and for each v
// over the 32-wide w steps from the one holding v to the last.  Eight waves:
// wave w owns rows 64 (w % 4) .. + 63 and column tiles 4 (w / 4) .. + 3
// (16 z each); per step it issues 4 x 4 tiles x 3 products.  Both operands of
// a step (A: Hc, 256 rows x 32 w, 32 KB; B: the pre-split rows, 32 w x 128 z,
// 16 KB) are copied from memory straight into LDS (buffer_load ... lds, no
// registers) two steps ahead through a ring of three slots, one barrier per
// step; each wave reads its operands in the order its matrix-core operations
// take them, so the first starts once three reads are back, and issues its
// copies for the step after next behind its first row tile's operations.  Hc is ordered
// [v][w step][row block]; the workgroups of one XCD take the row blocks of
// neighbouring z tiles in turn, so each Hc tile and each block of split rows
// is read through one L2 by several of them.
//
// Arithmetic: A_lo B_hi + A_hi B_lo + A_hi B_hi per term on
// v_mfma_f32_16x16x32_bf16, FP32 sums over w (D_v) and over up to kFlushV
// values of v, then added to the FP64 output (each workgroup owns its tile:
// a plain read-modify-write, deterministic).
#include "internal.hpp"

#include <algorithm>
#include <type_traits>

namespace mp {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int AI = 256;            // output rows per workgroup
constexpr int RB = 4;              // 16-row tiles per wave
constexpr int TW = 4;              // 16-wide column tiles per wave
constexpr int ZT = 128;            // z values per workgroup
constexpr int NCT = ZT / 16;       // column tiles per workgroup
constexpr int ZBW = ZT / 32;       // z blocks of 32 per workgroup
constexpr int kFlushV = 64;        // values of v per FP32 partial sum

__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_s_waitcnt(0xc07f);       // lgkmcnt(0) only: global loads stay in flight
    __builtin_amdgcn_s_barrier();
}

__device__ __forceinline__ bf8 as_bf8(uint4 v)
{
    bf8 r;
    __builtin_memcpy(&r, &v, sizeof(r));
    return r;
}

__device__ __forceinline__ uint32_t bf16_rne_bits(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

struct FacArgs {
    int U, nws, nib, nzt;
    int64_t upad;
};

// LDS DMA in buffer form (buffer_load_dwordx4 ... lds): each lane's 16 bytes
// land at lds_base + 16 lane, so one instruction moves one 1 KB operand half
// (hi or lo) of a fragment, already in the order the lanes read it back.  The
// buffer form, unlike the global one, lets the compiler keep counting the LDS
// reads issued before it exactly, so a matrix-core operation waits only for
// its own operands.  `rs` covers the wave's bytes of the step (reads outside
// it return zero); `soff` selects the fragment inside it.
__device__ __forceinline__ void dma16(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff, uint4 *lds_base)
{
    __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void *)lds_base, 16, voff, soff,
                                             0, 0);
}
constexpr int kBufWord3 = 0x00020000;         // descriptor word 3: 32-bit data format, raw access

constexpr int RING = 3;                       // steps in flight (LDS slots)
constexpr int SLOT_A = (AI / 16) * 128;       // uint4 of A (Hc) per slot: row tiles x hi/lo x lanes
constexpr int SLOT_B = NCT * 128;             // uint4 of B per slot
constexpr int SLOT = SLOT_A + SLOT_B;

__global__ __launch_bounds__(512) void k_adj_fac(FacArgs A, const double *__restrict__ St,
                                                 const uint4 *__restrict__ SB, const uint4 *__restrict__ Hc,
                                                 double *__restrict__ Shat)
{
    // ring of RING steps, one array per slot (so that the compiler sees that
    // loads into one slot never alias reads of another): [A row tile][hi/lo]
    // [lane], then [B column tile][hi/lo][lane]
    __shared__ uint4 ring0[SLOT], ring1[SLOT], ring2[SLOT];
    static_assert(RING == 3, "three ring slots");

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
    // z tile in turn: the XCD's workgroups share both operand streams
    const int ib = task % A.nib, zt = task / A.nib;
    const int64_t zb0 = (int64_t)zt * ZBW;
    const int u0 = ib * AI + rg * 16 * RB;
    const bool active = u0 < A.U;
    const int U = A.U, nws = A.nws;
    const int64_t nsteps = v_step_offset(U, nws);

    f4 out[RB][TW], D[RB][TW];
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < TW; ++j) {
            out[i][j] = f4{0.f, 0.f, 0.f, 0.f};
            D[i][j] = f4{0.f, 0.f, 0.f, 0.f};
        }

    // this wave's share of a step's operands (6 DMA instructions): A row
    // tiles 2 wave, 2 wave + 1 and B column tile `wave`, hi and lo each
    const uint4 *bsrc = SB + ((size_t)(zb0 + (wave >> 1)) * nws * 2 + (wave & 1)) * 128;
    const uint32_t voff = (uint32_t)lane * 16;
    auto issue = [&](int64_t st, int ws, uint4 *r) {
        const uint4 *a = Hc + (((size_t)st * A.nib + ib) * (AI / 16) + 2 * wave) * 128;
        const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc((void *)a, 0, 4096, kBufWord3);
        dma16(ra, voff, 0, r + (2 * wave) * 128);
        dma16(ra, voff, 1024, r + (2 * wave) * 128 + 64);
        dma16(ra, voff, 2048, r + (2 * wave + 1) * 128);
        dma16(ra, voff, 3072, r + (2 * wave + 1) * 128 + 64);
        const __amdgpu_buffer_rsrc_t rb =
            __builtin_amdgcn_make_buffer_rsrc((void *)(bsrc + (size_t)ws * 256), 0, 2048, kBufWord3);
        dma16(rb, voff, 0, r + SLOT_A + wave * 128);
        dma16(rb, voff, 1024, r + SLOT_A + wave * 128 + 64);
    };
    // St_v at this lane's columns (FP32): z = zb0 * 32 + 16 (TW ch + j) + lane % 16
    const int zl0 = ch * 16 * TW + (lane & 15);
    auto svload = [&](int v, double (&sv)[TW]) {
#pragma unroll
        for (int j = 0; j < TW; ++j) {
            const int zl = zl0 + 16 * j;
            sv[j] = St[(((zb0 + (zl >> 5)) * A.upad + v) << 5) + (zl & 31)];
        }
    };
    // output rows u = u0 + 16 i + 4 (lane / 16) + q, columns as above
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
                for (int q = 0; q < 4; ++q) p[q * 32] = old[j][q] + (double)out[i][j][q];
            }
        }
#pragma unroll
        for (int i = 0; i < RB; ++i)
#pragma unroll
            for (int j = 0; j < TW; ++j) out[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    };

    // the step sequence: v = 0.., for each v the w steps v / 32 .. nws - 1;
    // (iv, iws) runs RING - 1 steps ahead of (v, ws) to issue the loads
    int iv = 0, iws = 0;
    int64_t ist = 0;
    auto advance = [&](int &vv, int &ww) {
        if (ww == nws - 1) { ++vv; ww = vv >> 5; } else { ++ww; }
    };
    // past the last step the loads repeat it (into a slot no step reads), so
    // that every step issues exactly six
    auto issue_next = [&](uint4 *r) {
        issue(ist, iws, r);
        if (ist + 1 < nsteps) {
            ++ist;
            advance(iv, iws);
        }
    };
    issue_next(ring0);
    issue_next(ring1);
    double svd[TW];                           // St_v of the next epilogue, converted at use
    svload(0, svd);

    int v = 0, ws = 0, since = 0;
    int64_t st = 0;
    bool first = true;
    // one step from ring slot S, refilling slot (S + 2) % 3; false when done
    auto step = [&](auto slot) -> bool {
        constexpr int S = decltype(slot)::value;
        uint4 *const r = S == 0 ? ring0 : (S == 1 ? ring1 : ring2);
        uint4 *const rn = S == 0 ? ring2 : (S == 1 ? ring0 : ring1);
        // this wave's loads of step st are done once at most the next step's
        // six are outstanding (loads complete in order; any younger St_v
        // loads only make this stricter)
        __builtin_amdgcn_s_waitcnt(0x0f76);                             // vmcnt(6)
        __builtin_amdgcn_s_barrier();
        const bool vlast = ws == nws - 1;
        uint4 ah[RB], al[RB], fh[TW], fl[TW];
        auto rows = [&](int i) {
#pragma unroll
            for (int j = 0; j < TW; ++j)
                D[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf8(al[i]), as_bf8(fh[j]), D[i][j], 0, 0, 0);
#pragma unroll
            for (int j = 0; j < TW; ++j)
                D[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf8(ah[i]), as_bf8(fl[j]), D[i][j], 0, 0, 0);
#pragma unroll
            for (int j = 0; j < TW; ++j)
                D[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf8(ah[i]), as_bf8(fh[j]), D[i][j], 0, 0, 0);
        };
        if (active) {
            // in the order the matrix-core operations take them
            al[0] = r[(RB * rg) * 128 + 64 + lane];
#pragma unroll
            for (int j = 0; j < TW; ++j) fh[j] = r[SLOT_A + (TW * ch + j) * 128 + lane];
            ah[0] = r[(RB * rg) * 128 + lane];
#pragma unroll
            for (int j = 0; j < TW; ++j) fl[j] = r[SLOT_A + (TW * ch + j) * 128 + 64 + lane];
#pragma unroll
            for (int i = 1; i < RB; ++i) {
                al[i] = r[(RB * rg + i) * 128 + 64 + lane];
                ah[i] = r[(RB * rg + i) * 128 + lane];
            }
            rows(0);
        }
        // every wave is past step st - 1: its slot can be refilled.  Issued
        // after this step's LDS reads (so that no wait the compiler places
        // before those reads covers these loads) and after the first row
        // tile's operations (so that no wave waits for the copy queue before
        // its first operation).
        __builtin_amdgcn_sched_barrier(0);
        issue_next(rn);
        __builtin_amdgcn_sched_barrier(0);
        if (active) {
#pragma unroll
            for (int i = 1; i < RB; ++i) rows(i);
            if (vlast) {
                // D_v is complete: out += St_v(z) D_v(z), then D = 0
#pragma unroll
                for (int i = 0; i < RB; ++i)
#pragma unroll
                    for (int j = 0; j < TW; ++j) {
                        out[i][j] += (float)svd[j] * D[i][j];
                        D[i][j] = f4{0.f, 0.f, 0.f, 0.f};
                    }
            }
        }
        if (vlast) {
            const bool lastv = v + 1 == U;
            if (++since == kFlushV || lastv) {
                if (active) flush(first);
                since = 0;
                first = false;
            }
            if (!lastv) svload(v + 1, svd);
        }
        advance(v, ws);
        return ++st < nsteps;
    };
    for (;;) {
        if (!step(std::integral_constant<int, 0>())) break;
        if (!step(std::integral_constant<int, 1>())) break;
        if (!step(std::integral_constant<int, 2>())) break;
    }
    // no copy into this workgroup's LDS may outlive it (the last steps issue
    // copies that no step reads)
    __builtin_amdgcn_s_waitcnt(0x0f70);                                 // vmcnt(0)
}

// St pre-split in the B-operand order of the 16x16x32 BF16 matrix-core step:
// SB[(zb * nws + ws) * 2 + half][hi/lo][lane], lane l holding rows
// w = 32 ws + 8 (l / 16) + e (e = 0..7) at z = 32 zb + 16 half + l % 16.
__global__ void k_split_b(int64_t nzb, int nws, int64_t upad, const double *__restrict__ St,
                          uint4 *__restrict__ SB)
{
    const int64_t n = nzb * nws * 2 * 64;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int lane = (int)(e & 63), half = (int)((e >> 6) & 1);
        const int64_t f = e >> 7;
        const int ws = (int)(f % nws);
        const int64_t zb = f / nws;
        const int zz = 16 * half + (lane & 15);
        const int w0 = 32 * ws + 8 * (lane >> 4);
        uint32_t h[4], l[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double x0 = St[((zb * upad + w0 + 2 * q) << 5) + zz];
            const double x1 = St[((zb * upad + w0 + 2 * q + 1) << 5) + zz];
            const uint32_t h0 = bf16_rne_bits((float)x0), h1 = bf16_rne_bits((float)x1);
            const float r0 = (float)(x0 - (double)__uint_as_float(h0 << 16));
            const float r1 = (float)(x1 - (double)__uint_as_float(h1 << 16));
            h[q] = h0 | (h1 << 16);
            l[q] = bf16_rne_bits(r0) | (bf16_rne_bits(r1) << 16);
        }
        uint4 *o = SB + ((f * 2 + half) << 7) + lane;
        o[0] = make_uint4(h[0], h[1], h[2], h[3]);
        o[64] = make_uint4(l[0], l[1], l[2], l[3]);
    }
}

}  // namespace

hipError_t launch_split_b(int64_t nzb, int U, int64_t upad, const double *St, uint4 *SB, hipStream_t s)
{
    const int nws = (U + 31) / 32;
    const int64_t n = nzb * nws * 2 * 64;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 1 << 20);
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_split_b, dim3((unsigned)blocks), dim3(256), 0, s, nzb, nws, upad, St, SB);
    return hipGetLastError();
}

hipError_t launch_adj_fac(int U, int64_t upad, int64_t nzb, const double *St, const uint4 *SB, const uint4 *Hc,
                          double *Shat, hipStream_t s)
{
    if (upad % AI != 0 || upad < U || nzb % ZBW != 0 || U <= 0) return hipErrorInvalidValue;
    FacArgs a;
    a.U = U;
    a.nws = (U + 31) / 32;
    a.nib = (int)(upad / AI);
    a.nzt = (int)(nzb / ZBW);
    a.upad = upad;
    const int64_t ntasks = (int64_t)a.nib * a.nzt;
    if (ntasks == 0) return hipSuccess;
    if (ntasks > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_adj_fac, dim3((unsigned)ntasks), dim3(512), 0, s, a, St, SB, Hc, Shat);
    return hipGetLastError();
}

static_assert(kZBlockPad % ZBW == 0, "z tiles must divide the z-block padding");
static_assert(kRowPad % AI == 0, "row blocks must divide the row padding");
int adj_fac_rowblock() { return AI; }

}  // namespace mp
