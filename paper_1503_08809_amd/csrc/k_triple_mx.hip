// Step d, mixed precision: the unique third moments
//     T[i <= j <= k] = Sum_z St_i(z) St_j(z) St_k(z)
// of the W^(1/3)-scaled S rows (Eq. (2D); see k_triple.hip for how Gamma is
// assembled from T) on BF16 matrix cores with split operands.
//
// Work decomposition: block triples.  A workgroup task is (ib, jb, kb): the
// 128 rows i of block ib times the 16 x 16 pairs (j, k) of blocks jb, kb,
// i.e. 32768 moments.  The column operand St_j(z) St_k(z) of all 256 pairs
// is generated from only 32 source rows, and the 128 A rows are shared by
// every task of the same ib; tasks are ordered (ib, jb, kb) and dealt to
// the XCDs in contiguous runs so that co-resident workgroups read the same A
// rows through one L2.  Only tasks holding some i <= j <= k are launched;
// inside one, only the row blocks holding some i <= j (rounded up to an
// even count) are multiplied, and the remaining out-of-order entries are
// computed but never read.
//
// Arithmetic: each value x is split as x = hi + lo with hi the BF16 rounding
// of x and lo the BF16 rounding of the remainder; a term A B is formed by
// v_mfma_f32_16x16x32_bf16 as A_lo B_hi + A_hi B_lo + A_hi B_hi (the dropped
// A_lo B_lo is ~2^-16 of the term).  The A rows are split once in memory;
// the product operand St_j St_k is formed in FP32 and split per step, its
// remainder taken from the exact product by a fused multiply-add.  Each r's
// mu sum accumulates in FP32 in the matrix-core accumulators; when it is
// complete it is added to the FP64 r sum held in T (each task owns its
// outputs: a plain read-modify-write, no atomics, deterministic).  The mu
// sum of an r is always complete before it enters the r sum (Sec. 2.2).
//
// Four waves per workgroup, two workgroups per CU (one wave of each per
// SIMD, so that the barriers of the two fall at different times).  Wave w
// owns the 4 pair tiles j = 4 w .. + 3 (k = the 16 k of the task) for all
// 128 rows, and generates exactly those tiles itself, straight into the
// registers that the matrix cores take as B operands: no pair tile passes
// through LDS.  The A fragments of a step (the task's 128 rows, split, 16 KB)
// are copied from memory straight into LDS (buffer_load ... lds, four
// instructions per wave) one step ahead into the other of two buffers, and
// every wave reads all 8 row blocks of them.  Per 32-wide z step a wave
// issues up to 8 row blocks x 4 pair tiles x 3 products = 96 matrix-core
// operations, row block by row block (12 operations ordered product by
// product over the four tiles, so that dependent operations on one
// accumulator are four apart), reading the next block's fragments while the
// current one is multiplied; then generates its tiles of the next step from
// the staged source rows (double-buffered in LDS, two rows per thread,
// loaded three steps ahead); one barrier per step.  Sharing the generated
// tiles through LDS instead (waves of 32 rows x all 16 tiles) would read
// twice the operand bytes from LDS per step.
#include "internal.hpp"

#include <algorithm>
#include <type_traits>

namespace mp {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));

constexpr int BI = 128, BJ = 16, BK = 16;     // rows per task along i, j, k
constexpr int NT = BJ;                        // pair tiles per task: (j, k0..k0+15)
constexpr int KZ = 32;                        // z values per step
constexpr int SRC_ROWS = BJ + BK;             // staged source rows per step
constexpr int SRC_LD = KZ + 4;                // padded LDS row (floats)
constexpr int TASK_SIZE = BI * BJ * BK;       // moments per task

// The products p = x y, q = u w split as p = hi + lo: hi the BF16 rounding of
// the FP32 product, lo the BF16 rounding of the exact remainder x y - hi
// (one fused multiply-add, so the product's own rounding error is kept).
__device__ __forceinline__ void split_prod2(float x, float y, float u, float w, uint32_t &h, uint32_t &l)
{
    const bf2 hv = {(__bf16)(x * y), (__bf16)(u * w)};
    h = __builtin_bit_cast(uint32_t, hv);
    asm("" : "+v"(h));                        // keep one conversion: unpack h itself below
    const bf2 lv = {(__bf16)__builtin_fmaf(x, y, -__uint_as_float(h << 16)),
                    (__bf16)__builtin_fmaf(u, w, -__uint_as_float(h & 0xffff0000u))};
    l = __builtin_bit_cast(uint32_t, lv);
}

__device__ __forceinline__ bf8 as_bf8(uint4 v)
{
    bf8 r;
    __builtin_memcpy(&r, &v, sizeof(r));
    return r;
}

__device__ __forceinline__ int task_of_block(int bid, int ntasks)
{
    const int x = bid & 7, idx = bid >> 3;     // workgroups go to the 8 XCDs round-robin
    const int base = ntasks >> 3, rem = ntasks & 7;
    return x * base + (x < rem ? x : rem) + idx;
}

struct BTArgs {
    const int4 *tasks;      // (ib, jb, kb, -)
    int ntasks;
    int64_t upad;           // rows per z block of the z-blocked S layout
    int64_t nsteps;         // z steps (nr * nmu_pad / 32)
    int kpr;                // steps per r
};

// Offset of moment (i, j, k) inside its task block; the 4 values a lane holds
// for one matrix-core tile are contiguous.
__device__ __host__ __forceinline__ int bt_offset(int il, int jl, int kl)
{
    const int rb16 = il >> 4, row = il & 15;
    const int lane = kl + 16 * (row >> 2), q = row & 3;
    return ((rb16 * NT + jl) * 64 + lane) * 4 + q;
}

__device__ __forceinline__ void dma16(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff, uint4 *lds_base)
{
    __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void *)lds_base, 16, voff, soff,
                                             0, 0);
}
constexpr int kBufWord3 = 0x00020000;         // descriptor word 3: 32-bit data format, raw access
constexpr int NRB = BI / 16;                  // row blocks per task
constexpr int TQ = 4;                         // pair tiles per wave
constexpr int ASLOT = NRB * 128;              // uint4 per A buffer: [row block][hi/lo][lane]

__global__ __launch_bounds__(256, 2) void k_triple_bt(BTArgs A, const float *__restrict__ S32,
                                                   const uint16_t *__restrict__ SA,
                                                   double *__restrict__ T)
{
    __shared__ float Src[2][SRC_ROWS][SRC_LD];
    __shared__ uint4 abuf0[ASLOT], abuf1[ASLOT];

    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int task = task_of_block(blockIdx.x, A.ntasks);
    const int4 tk = A.tasks[task];
    const int j0 = tk.y * BJ, k0 = tk.z * BK;
    const int n = lane & 15, zg = lane >> 4;
    // row blocks holding some i <= j0 + BJ - 1 (at least one: tasks are
    // launched only then), rounded up to even
    const int live = min(NRB, (j0 + BJ - 1 - tk.x * BI) / 16 + 1);
    const int nl = min(NRB, (live + 1) & ~1);

    f4 acc[NRB][TQ];
#pragma unroll
    for (int i = 0; i < NRB; ++i)
#pragma unroll
        for (int j = 0; j < TQ; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

    // A fragments of step s (the task's 128 rows, split, 16 KB) copied into
    // LDS: this wave copies row blocks 2 wave, 2 wave + 1, hi and lo each;
    // lane (n, zg) takes row 16 rb + n, 8-z group zg at byte
    // ((row * 4 + zg) * 32) (hi) and + 16 (lo) of the task's rows
    const size_t astep = (size_t)A.upad << 6;                     // uint16 per step
    const uint32_t avoff = (uint32_t)(n * 4 + zg) * 32;
    auto acopy = [&](int64_t s, uint4 *buf) {
        const uint16_t *base = SA + (size_t)s * astep + (size_t)tk.x * BI * 64;
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void *)base, 0, BI * 128, kBufWord3);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int rb = 2 * wave + h;
            dma16(rs, avoff, rb * 2048, buf + (rb * 2) * 64);
            dma16(rs, avoff, rb * 2048 + 16, buf + (rb * 2 + 1) * 64);
        }
    };
    // source rows: local 0..15 = j0.., 16..31 = k0..; 32 rows x 16 float2,
    // two per thread, rows srow and 16 + srow
    const int srow = t >> 4, sq = t & 15;
    const uint32_t soff0 = ((uint32_t)(j0 + srow) << 5) + 2 * sq;
    const uint32_t soff1 = ((uint32_t)(k0 + srow) << 5) + 2 * sq;
    const size_t sstep = (size_t)A.upad << 5;
    float2 sreg0 = make_float2(0.f, 0.f), sreg1 = sreg0;
    auto sload = [&](int64_t s) {
        sreg0 = *reinterpret_cast<const float2 *>(S32 + (size_t)s * sstep + soff0);
        sreg1 = *reinterpret_cast<const float2 *>(S32 + (size_t)s * sstep + soff1);
    };
    auto sstore = [&](int buf) {
        *reinterpret_cast<float2 *>(&Src[buf][srow][2 * sq]) = sreg0;
        *reinterpret_cast<float2 *>(&Src[buf][BJ + srow][2 * sq]) = sreg1;
    };
    // this wave's pair tiles j = 4 wave + q (q < 4), k = k0 + n: generated in
    // registers as the matrix-core B operands (hi, lo)
    uint4 bh[TQ], bl[TQ];
    auto bgen = [&](int buf) {
        const float *pk = &Src[buf][BJ + n][8 * zg];
#pragma unroll
        for (int q = 0; q < TQ; ++q) {
            const f4 k0v = *reinterpret_cast<const f4 *>(pk), k1v = *reinterpret_cast<const f4 *>(pk + 4);
            const float *pj = &Src[buf][4 * wave + q][8 * zg];
            const f4 j0v = *reinterpret_cast<const f4 *>(pj), j1v = *reinterpret_cast<const f4 *>(pj + 4);
            float jv[8], kv[8];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                jv[e] = j0v[e];
                jv[4 + e] = j1v[e];
                kv[e] = k0v[e];
                kv[4 + e] = k1v[e];
            }
            uint32_t h[4], l[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) split_prod2(jv[2 * e], kv[2 * e], jv[2 * e + 1], kv[2 * e + 1], h[e], l[e]);
            bh[q] = make_uint4(h[0], h[1], h[2], h[3]);
            bl[q] = make_uint4(l[0], l[1], l[2], l[3]);
        }
    };

    // output tile (row block rb, pair tile 4 wave + q) at
    // T + task * TASK_SIZE + ((rb * NT + 4 wave + q) * 64 + lane) * 4
    double *tbase = T + (size_t)task * TASK_SIZE + (size_t)(4 * wave) * 256;
    const uint32_t toff = (uint32_t)lane * 4;

    const int64_t nsteps = A.nsteps, last = nsteps - 1;
    sload(0);
    sstore(0);
    sload(nsteps > 1 ? 1 : 0);
    sstore(1);
    acopy(0, abuf0);
    __builtin_amdgcn_s_waitcnt(0xc07f);                                 // lgkmcnt(0)
    __builtin_amdgcn_s_barrier();
    bgen(0);
    sload(nsteps > 2 ? 2 : last);

    int kin = 0;
    bool first = true;
    int64_t s = 0;
    // one step with parity P (A buffer P, sources of step s + 1 in Src[1 - P])
    // over NL row blocks; false when done
    auto step = [&](auto par, auto rows) -> bool {
        constexpr int P = decltype(par)::value;
        constexpr int NL = decltype(rows)::value;
        const uint4 *ab = P ? abuf1 : abuf0;
        uint4 *abn = P ? abuf0 : abuf1;
        // this step's A copies and every wave's source stores are complete
        __builtin_amdgcn_s_waitcnt(0x0070);                             // vmcnt(0) lgkmcnt(0)
        __builtin_amdgcn_s_barrier();
        sstore(P);                                                      // sources of step s + 2
        sload(s + 3 < last ? s + 3 : last);
        // A of step s + 1.  An LDS read that the compiler cannot tell apart
        // from a copy's destination gets a wait for all copies in front of
        // it; here the compiler issues this step's operand reads (buffer P)
        // ahead of the copies (buffer 1 - P) and waits for none of them
        acopy(s + 1 < last ? s + 1 : last, abn);
        // row block by row block, the next block's fragments read while this
        // one's 12 matrix-core operations run (product by product over the
        // four tiles, so that dependent operations are four apart)
        uint4 ah = ab[lane], al = ab[64 + lane];
#pragma unroll
        for (int rb = 0; rb < NL; ++rb) {
            uint4 nh, nl2;
            if (rb + 1 < NL) {
                nh = ab[((rb + 1) * 2) * 64 + lane];
                nl2 = ab[((rb + 1) * 2 + 1) * 64 + lane];
            }
#pragma unroll
            for (int q = 0; q < TQ; ++q)
                acc[rb][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf8(al), as_bf8(bh[q]), acc[rb][q], 0, 0, 0);
#pragma unroll
            for (int q = 0; q < TQ; ++q)
                acc[rb][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf8(ah), as_bf8(bl[q]), acc[rb][q], 0, 0, 0);
#pragma unroll
            for (int q = 0; q < TQ; ++q)
                acc[rb][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf8(ah), as_bf8(bh[q]), acc[rb][q], 0, 0, 0);
            if (rb + 1 < NL) {
                ah = nh;
                al = nl2;
            }
        }
        bgen(1 - P);                                                    // operands of step s + 1
        if (++kin == A.kpr) {
            // this r's mu sum is complete: add it to the FP64 r sum in T
            kin = 0;
            uint32_t to = toff;
            asm volatile("" : "+v"(to));
#pragma unroll
            for (int rb = 0; rb < NL; ++rb)
#pragma unroll
                for (int qh = 0; qh < TQ; qh += 2) {
                    double2 old[2][2];
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        const double2 *p =
                            reinterpret_cast<const double2 *>(tbase + to + (uint32_t)((rb * NT + qh + q) << 8));
                        old[q][0] = first ? make_double2(0.0, 0.0) : p[0];
                        old[q][1] = first ? make_double2(0.0, 0.0) : p[1];
                    }
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        double2 *p = reinterpret_cast<double2 *>(tbase + to + (uint32_t)((rb * NT + qh + q) << 8));
                        const f4 a = acc[rb][qh + q];
                        p[0] = make_double2(old[q][0].x + (double)a[0], old[q][0].y + (double)a[1]);
                        p[1] = make_double2(old[q][1].x + (double)a[2], old[q][1].y + (double)a[3]);
                    }
                }
#pragma unroll
            for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
                for (int q = 0; q < TQ; ++q) acc[rb][q] = f4{0.f, 0.f, 0.f, 0.f};
            first = false;
        }
        return ++s < nsteps;
    };
    auto run = [&](auto rows) {
        for (;;) {
            if (!step(std::integral_constant<int, 0>(), rows)) break;
            if (!step(std::integral_constant<int, 1>(), rows)) break;
        }
    };
    switch (nl) {
    case 2: run(std::integral_constant<int, 2>()); break;
    case 4: run(std::integral_constant<int, 4>()); break;
    case 6: run(std::integral_constant<int, 6>()); break;
    default: run(std::integral_constant<int, 8>()); break;
    }
    // no copy into this workgroup's LDS may outlive it
    __builtin_amdgcn_s_waitcnt(0x0f70);                                 // vmcnt(0)
}

// ---- gather ---------------------------------------------------------------
__device__ __forceinline__ double bt_get(int a, int b, int c, const int *__restrict__ tidx, int njb,
                                         int nkb, const double *__restrict__ T)
{
    const int lo = min(a, min(b, c)), hi = max(a, max(b, c));
    const int mid = a + b + c - lo - hi;
    const int task = tidx[((lo / BI) * njb + mid / BJ) * nkb + hi / BK];
    return T[(size_t)task * TASK_SIZE + bt_offset(lo % BI, mid % BJ, hi % BK)];
}

__global__ void k_gather_bt(int kind, int ta, int tp, const int *__restrict__ tri_a,
                            const int *__restrict__ tri_p, int np, const int *__restrict__ tidx,
                            int njb, int nkb, const double *__restrict__ T, double *__restrict__ gamma)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)ta * tp) return;
    const int n = (int)(e / tp), m = (int)(e % tp);
    const int a0 = tri_a[3 * n] * np, a1 = tri_a[3 * n + 1] * np, a2 = tri_a[3 * n + 2] * np;
    const int p0 = tri_p[3 * m], p1 = tri_p[3 * m + 1], p2 = tri_p[3 * m + 2];
    double v;
    if (kind == MODAL_GAMMA_ORDERED) {
        v = bt_get(a0 + p0, a1 + p1, a2 + p2, tidx, njb, nkb, T) * (1.0 / (8.0 * kPi));
    } else {
        v = bt_get(a0 + p0, a1 + p1, a2 + p2, tidx, njb, nkb, T) +
            bt_get(a0 + p0, a1 + p2, a2 + p1, tidx, njb, nkb, T) +
            bt_get(a0 + p1, a1 + p0, a2 + p2, tidx, njb, nkb, T) +
            bt_get(a0 + p1, a1 + p2, a2 + p0, tidx, njb, nkb, T) +
            bt_get(a0 + p2, a1 + p0, a2 + p1, tidx, njb, nkb, T) +
            bt_get(a0 + p2, a1 + p1, a2 + p0, tidx, njb, nkb, T);
        v *= 1.0 / (48.0 * kPi);
    }
    gamma[e] = v;
}

}  // namespace

hipError_t build_bt_plan(int U, BTPlan &plan, std::string &err, DevArena *arena)
{
    free_bt_plan(plan);
    plan.U = U;
    plan.nib = (U + BI - 1) / BI;
    plan.njb = (U + BJ - 1) / BJ;
    plan.nkb = (U + BK - 1) / BK;
    std::vector<int> tidx((size_t)plan.nib * plan.njb * plan.nkb, -1);
    std::vector<int4> tasks;
    for (int ib = 0; ib < plan.nib; ++ib)
        for (int jb = 0; jb < plan.njb; ++jb) {
            const int jmax = std::min(jb * BJ + BJ - 1, U - 1);
            if (ib * BI > jmax) continue;
            for (int kb = 0; kb < plan.nkb; ++kb) {
                if (jb * BJ > kb * BK + BK - 1) continue;
                tidx[((size_t)ib * plan.njb + jb) * plan.nkb + kb] = (int)tasks.size();
                tasks.push_back(make_int4(ib, jb, kb, 0));
            }
        }
    plan.ntasks = (int)tasks.size();
    plan.tsize = (int64_t)plan.ntasks * TASK_SIZE;
    plan.borrowed = arena != nullptr;
    auto get = [&](void **p, size_t nb) { return arena ? arena->take(p, nb) : hipMalloc(p, nb); };
    hipError_t e = get((void **)&plan.tasks, sizeof(int4) * std::max<size_t>(tasks.size(), 1));
    if (e == hipSuccess && !tasks.empty())
        e = hipMemcpy(plan.tasks, tasks.data(), sizeof(int4) * tasks.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = get((void **)&plan.tidx, sizeof(int) * tidx.size());
    if (e == hipSuccess)
        e = hipMemcpy(plan.tidx, tidx.data(), sizeof(int) * tidx.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        err = std::string("block-triple plan upload: ") + hipGetErrorString(e);
        free_bt_plan(plan);
    }
    return e;
}

void free_bt_plan(BTPlan &p)
{
    if (p.borrowed) {
        p = BTPlan{};
        return;
    }
    (void)hipFree(p.tasks);
    (void)hipFree(p.tidx);
    p = BTPlan{};
}

hipError_t launch_triple_bt(const BTPlan &plan, int64_t upad, int64_t ldz, int nmu_pad,
                            const float *S32, const uint16_t *SA, double *T, hipStream_t s)
{
    if (nmu_pad % KZ != 0 || ldz % nmu_pad != 0 || upad % BI != 0 || upad < plan.U)
        return hipErrorInvalidValue;
    if (plan.ntasks == 0) return hipSuccess;
    BTArgs a;
    a.tasks = plan.tasks;
    a.ntasks = plan.ntasks;
    a.upad = upad;
    a.nsteps = ldz / KZ;
    a.kpr = nmu_pad / KZ;
    hipLaunchKernelGGL(k_triple_bt, dim3(plan.ntasks), dim3(256), 0, s, a, S32, SA, T);
    return hipGetLastError();
}

hipError_t launch_gather_bt(int kind, int ta, int tp, const int *tri_a, const int *tri_p, int np,
                            const BTPlan &plan, const double *T, double *gamma, hipStream_t s)
{
    const int64_t n = (int64_t)ta * tp;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_bt, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, kind, ta, tp,
                       tri_a, tri_p, np, plan.tidx, plan.njb, plan.nkb, T, gamma);
    return hipGetLastError();
}

}  // namespace mp
