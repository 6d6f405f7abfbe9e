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
// inside one, waves whose 32 rows all exceed the largest j skip the matrix
// work, and the remaining out-of-order entries are computed but never read.
//
// Arithmetic: each value x is split as x = hi + lo with hi the BF16 rounding
// of x and lo the BF16 rounding of the remainder; a term A B is formed by
// v_mfma_f32_16x16x32_bf16 as A_lo B_hi + A_hi B_lo + A_hi B_hi (the dropped
// A_lo B_lo is ~2^-16 of the term).  The A rows are split once in memory;
// the product operand St_j St_k is formed in FP32 and split per step.  Each
// r's mu sum accumulates in FP32 in the matrix-core accumulators; when it
// is complete it is added to the FP64 r sum held in T (each task owns its
// outputs: a plain read-modify-write, no atomics, deterministic).  The mu
// sum of an r is always complete before it enters the r sum (Sec. 2.2).
//
// Four waves per workgroup, two workgroups per CU (one wave of each per
// SIMD, so that the barriers of the two fall at different times): wave w
// owns rows 32 w .. + 31 of the task and all 16 pair tiles, so each A row
// is loaded by one wave only.  Per 32-wide z step a wave issues 2 row
// blocks x 16 pair tiles x 3 products = 96 matrix-core operations, two pair
// tiles at a time (12 operations ordered product by product, so that
// dependent operations on one accumulator are four apart), reading the next
// two tiles from LDS while the current two are multiplied; generates 4 of
// the 16 pair tiles for the next step (its k rows read once for all four)
// and shares them through LDS (double-buffered, one barrier per step); loads
// its A fragments straight from memory two steps ahead (two register sets);
// and all threads stage the 32 source rows of the step after next, two rows
// each.  A wave whose rows all exceed the task's largest j runs the same
// steps (staging, generation, barriers) in a loop of its own without the
// matrix-core work: a branch inside the step would make the compiler copy
// the 128 accumulator registers and spill.
#include "internal.hpp"

#include <algorithm>
#include <type_traits>

namespace mp {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));

constexpr int BI = 128, BJ = 16, BK = 16;     // rows per task along i, j, k
constexpr int RB = 2;                         // 16-row blocks per wave
constexpr int TW = 16;                        // pair tiles per wave
constexpr int NT = BJ;                        // pair tiles per task: (j, k0..k0+15)
constexpr int KZ = 32;                        // z values per step
constexpr int SRC_ROWS = BJ + BK;             // staged source rows per step
constexpr int SRC_LD = KZ + 4;                // padded LDS row (floats)
constexpr int TASK_SIZE = BI * BJ * BK;       // moments per task

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

__global__ __launch_bounds__(256, 2) void k_triple_bt(BTArgs A, const float *__restrict__ S32,
                                                   const uint16_t *__restrict__ SA,
                                                   double *__restrict__ T)
{
    __shared__ float Src[2][SRC_ROWS][SRC_LD];
    __shared__ uint4 Bb[2][NT][2][64];        // [buf][tile][hi/lo][lane]

    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int rg = wave;                       // row group (32 rows)
    const int task = task_of_block(blockIdx.x, A.ntasks);
    const int4 tk = A.tasks[task];
    const int i0 = tk.x * BI + rg * 16 * RB;   // this wave's rows
    const int j0 = tk.y * BJ, k0 = tk.z * BK;
    const int n = lane & 15, zg = lane >> 4;
    const bool active = i0 <= j0 + BJ - 1;     // some row <= some j (wave-uniform)

    f4 acc[RB][TW];
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < TW; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

    // A fragments of step s: row i0 + 16 i + n, 8-z group zg, at
    // SA[((s * upad + row) * 4 + zg) * 16]; 32-bit lane offsets from a
    // wave-uniform base keep the addressing in scalar registers plus one VGPR
    const uint32_t aoff = ((uint32_t)(i0 + n) * 4 + zg) << 4;     // uint16 units
    const size_t astep = (size_t)A.upad << 6;
    // two sets: step s uses set s % 2, whose loads were issued two steps ahead
    uint4 ah0[RB], al0[RB], ah1[RB], al1[RB];
    auto aload = [&](int64_t s, uint4 (&ah)[RB], uint4 (&al)[RB]) {
        const uint16_t *base = SA + (size_t)s * astep;
#pragma unroll
        for (int i = 0; i < RB; ++i) {
            const uint4 *p = reinterpret_cast<const uint4 *>(base + aoff + (uint32_t)(i * 16 * 64));
            ah[i] = p[0];
            al[i] = p[1];
        }
    };
    // source rows: local 0..15 = j0.., 16..31 = k0..; 32 rows x 16 float2,
    // two per thread, rows srow and 16 + srow (every thread, so that no
    // branch leaves the compiler unable to count this wave's outstanding
    // loads)
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
    // this wave generates pair tiles 4 wave .. + 3 (tile = j local); the k
    // values (this lane's k row, 8 z) are read once for all four
    f4 k0v, k1v;
    auto bgen_k = [&](int buf) {
        const float *pk = &Src[buf][BJ + n][8 * zg];
        k0v = *reinterpret_cast<const f4 *>(pk);
        k1v = *reinterpret_cast<const f4 *>(pk + 4);
    };
    auto bgen_tile = [&](int buf, int q) {
        const int tile = 4 * wave + q;
        const float *pj = &Src[buf][tile][8 * zg];
        const f4 j0v = *reinterpret_cast<const f4 *>(pj), j1v = *reinterpret_cast<const f4 *>(pj + 4);
        float v[8];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            v[e] = j0v[e] * k0v[e];
            v[4 + e] = j1v[e] * k1v[e];
        }
        uint32_t h[4], l[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) split2(v[2 * e], v[2 * e + 1], h[e], l[e]);
        Bb[buf][tile][0][lane] = make_uint4(h[0], h[1], h[2], h[3]);
        Bb[buf][tile][1][lane] = make_uint4(l[0], l[1], l[2], l[3]);
    };

    // this wave's output: tile jl = j of row block rb16 = RB rg + i at
    // T + task * TASK_SIZE + ((rb16 * NT + jl) * 64 + lane) * 4
    double *tbase = T + (size_t)task * TASK_SIZE + (size_t)(rg * RB * NT) * 256;
    const uint32_t toff = (uint32_t)lane * 4;

    const int64_t nsteps = A.nsteps, last = nsteps - 1;
    sload(0);
    sstore(0);
    sload(nsteps > 1 ? 1 : 0);
    sstore(1);
    lds_barrier();
    bgen_k(0);
    bgen_tile(0, 0);
    bgen_tile(0, 1);
    bgen_tile(0, 2);
    bgen_tile(0, 3);
    sload(nsteps > 2 ? 2 : last);
    aload(0, ah0, al0);
    aload(nsteps > 1 ? 1 : 0, ah1, al1);
    lds_barrier();

    int kin = 0;
    bool first = true;
    int64_t s = 0;
    // one step with parity P (LDS buffers and A set P), with or without the
    // matrix-core work; false when done
    auto step = [&](auto par, auto act) -> bool {
        constexpr int P = decltype(par)::value;
        constexpr bool work = decltype(act)::value;
        constexpr int buf = P;
        uint4(&ah)[RB] = P ? ah1 : ah0;
        uint4(&al)[RB] = P ? al1 : al0;
        // past the last step these clamp to it; their results are never used
        sstore(buf);                                       // sources of step s + 2
        sload(s + 3 < last ? s + 3 : last);
        if constexpr (work) {
            // pairs of pair tiles: the operands of pair p + 1 are read while
            // pair p's 12 matrix-core operations run, ordered product by
            // product over both tiles and both row blocks so that dependent
            // operations on one accumulator are four apart; this wave's 4
            // pair tiles of step s + 1 are generated after pairs 1, 3, 5 and
            // 7 (VALU work under the matrix cores)
            uint4 ch[2], cl[2], nh[2], nl[2];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                ch[q] = Bb[buf][q][0][lane];
                cl[q] = Bb[buf][q][1][lane];
            }
#pragma unroll
            for (int p = 0; p < TW / 2; ++p) {
                if (p + 1 < TW / 2) {
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        nh[q] = Bb[buf][2 * p + 2 + q][0][lane];
                        nl[q] = Bb[buf][2 * p + 2 + q][1][lane];
                    }
                }
#pragma unroll
                for (int q = 0; q < 2; ++q)
#pragma unroll
                    for (int i = 0; i < RB; ++i)
                        acc[i][2 * p + q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf8(al[i]), as_bf8(ch[q]), acc[i][2 * p + q], 0, 0, 0);
#pragma unroll
                for (int q = 0; q < 2; ++q)
#pragma unroll
                    for (int i = 0; i < RB; ++i)
                        acc[i][2 * p + q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf8(ah[i]), as_bf8(cl[q]), acc[i][2 * p + q], 0, 0, 0);
#pragma unroll
                for (int q = 0; q < 2; ++q)
#pragma unroll
                    for (int i = 0; i < RB; ++i)
                        acc[i][2 * p + q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf8(ah[i]), as_bf8(ch[q]), acc[i][2 * p + q], 0, 0, 0);
                if (p == 1) bgen_k(buf ^ 1);
                if ((p & 1) == 1) bgen_tile(buf ^ 1, p >> 1);      // operand of step s + 1
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    ch[q] = nh[q];
                    cl[q] = nl[q];
                }
            }
        } else {
            bgen_k(buf ^ 1);
            bgen_tile(buf ^ 1, 0);
            bgen_tile(buf ^ 1, 1);
            bgen_tile(buf ^ 1, 2);
            bgen_tile(buf ^ 1, 3);
        }
        if (++kin == A.kpr) {
            // this r's mu sum is complete: add it to the FP64 r sum in T,
            // four tiles at a time with their loads issued first
            kin = 0;
            if constexpr (work) {
                // opaque copy: keeps the compiler from hoisting every tile
                // address out of the z loop
                uint32_t to = toff;
                asm volatile("" : "+v"(to));
#pragma unroll
                for (int i = 0; i < RB; ++i)
#pragma unroll
                    for (int jh = 0; jh < TW; jh += 4) {
                        double2 old[4][2];
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const double2 *p = reinterpret_cast<const double2 *>(
                                tbase + to + (uint32_t)((i * NT + jh + j) << 8));
                            old[j][0] = first ? make_double2(0.0, 0.0) : p[0];
                            old[j][1] = first ? make_double2(0.0, 0.0) : p[1];
                        }
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            double2 *p = reinterpret_cast<double2 *>(tbase + to + (uint32_t)((i * NT + jh + j) << 8));
                            const f4 a = acc[i][jh + j];
                            p[0] = make_double2(old[j][0].x + (double)a[0], old[j][0].y + (double)a[1]);
                            p[1] = make_double2(old[j][1].x + (double)a[2], old[j][1].y + (double)a[3]);
                        }
                    }
            }
#pragma unroll
            for (int i = 0; i < RB; ++i)
#pragma unroll
                for (int j = 0; j < TW; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
            first = false;
        }
        // A fragments of step s + 2 into the set this step has finished with
        aload(s + 2 < last ? s + 2 : last, ah, al);
        lds_barrier();
        return ++s < nsteps;
    };
    if (active) {
        for (;;) {
            if (!step(std::integral_constant<int, 0>(), std::true_type())) break;
            if (!step(std::integral_constant<int, 1>(), std::true_type())) break;
        }
    } else {
        for (;;) {
            if (!step(std::integral_constant<int, 0>(), std::false_type())) break;
            if (!step(std::integral_constant<int, 1>(), std::false_type())) break;
        }
    }
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
