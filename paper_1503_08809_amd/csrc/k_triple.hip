// Step d: the triple-product quadrature of Eq. (2D).
//
// With the S rows pre-scaled by the cube root of the quadrature weight
// (St_u(z) = W(z)^(1/3) S_u(z), z = (r, mu), u = (a, p)), every entry of the
// ordered and the symmetric Gamma is built from the third moments
//
//     T[u1, u2, u3] = Sum_z St_u1(z) St_u2(z) St_u3(z),
//
// a tensor symmetric in (u1, u2, u3): the ordered Gamma entry for
// (a1 a2 a3),(p1 p2 p3) is T at u_s = (a_s, p_s) over 8 pi, and the
// symmetric entry is the sum of the six T values of the permanent over
// 48 pi.  Only the unique entries i <= j <= k are computed (one sixth of the
// dense work); a gather kernel then assembles Gamma.
//
// The unique entries form a matrix product over z: rows i, columns the pairs
// (j <= k), and the column operand St_j(z) St_k(z) generated on the fly.
// Pairs are listed by (j, k); 16 consecutive pairs make a column tile, and a
// 16-row block i0..i0+15 is needed for a tile only when i0 <= max j of the
// tile.  Tiles are packed T[tile][row block][16][16].
//
// A workgroup task is (group of column tiles whose pairs touch a bounded set
// of distinct rows, row super-block).  z runs over the whole range inside one
// workgroup: no split-K, no atomics, deterministic results.
//
// FP64 path (k_triple_f64): v_mfma_f64_16x16x4f64.  Tasks are 8 column tiles
// x 128 rows; per 16-wide z chunk the workgroup stages the 128 A rows and
// the group's rows in LDS (double-buffered, next chunk prefetched into
// registers); each of the four waves owns 64 rows x 64 pairs.
//
// The mixed-precision kernel is in k_triple_mx.hip; this file also holds the
// FP64 copy and BF16 split of the scaled rows that it reads.
#include "internal.hpp"

#include <algorithm>
#include <cstring>
#include <type_traits>

namespace mp {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

// ---- shapes -----------------------------------------------------------------
constexpr int F64_ROWBLOCK = 128, F64_TILES = 8, F64_GROUP_ROWS = 160;

constexpr int ZC = 16;                       // z values per staged chunk (FP64)
constexpr int LDSA = F64_ROWBLOCK + 1;       // padded LDS row lengths (doubles)
constexpr int LDSG = F64_GROUP_ROWS + 1;

__device__ __forceinline__ int task_of_block(int bid, int ntasks)
{
    // Workgroups are dealt to the 8 XCDs round-robin; give each XCD a
    // contiguous run of tasks so neighbouring tasks (which share S rows)
    // share an L2.
    const int x = bid & 7, idx = bid >> 3;
    const int base = ntasks >> 3, rem = ntasks & 7;
    return x * base + (x < rem ? x : rem) + idx;
}

struct TripleArgs {
    const int *tile_maxj;
    const int64_t *tile_off;
    const int *group_tile0;
    const int *group_rows;
    const int *group_nrows;
    const unsigned short *pair_lj, *pair_lk;
    const int2 *tasks;
    int ntasks;
    int group_cap;
    int64_t upad;          // rows per z block of the z-blocked S layout
    int64_t nz;            // z values (nr * nmu_pad)
};

// Barrier for LDS traffic only: unlike __syncthreads() it does not wait for
// outstanding global loads, so prefetches stay in flight across it.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_s_waitcnt(0xc07f);      // lgkmcnt(0); vmcnt and expcnt unconstrained
    __builtin_amdgcn_s_barrier();
}

// ============================================================================
// FP64
// ============================================================================
__global__ __launch_bounds__(256, 2) void k_triple_f64(TripleArgs A, const double *__restrict__ St,
                                                       double *__restrict__ T)
{
    __shared__ double Sa[2][ZC][LDSA];
    __shared__ double Sg[2][ZC][LDSG];

    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int task = task_of_block(blockIdx.x, A.ntasks);
    const int2 tk = A.tasks[task];
    const int g = tk.x, rb = tk.y;
    const int t0 = A.group_tile0[g], nt = A.group_tile0[g + 1] - t0;
    const int *grow = A.group_rows + (size_t)g * A.group_cap;
    const int row0 = rb * F64_ROWBLOCK;

    // this lane's four pairs (one per column tile of the wave); tiles past the
    // group's end and row blocks past a tile's max j are computed (their
    // operands are valid rows) but never stored
    int lj[4], lk[4];
    unsigned mask = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int tj = wn * 4 + j;
        lj[j] = 0;
        lk[j] = 0;
        if (tj < nt) {
            const int q = (t0 + tj) * 16 + (lane & 15);
            lj[j] = A.pair_lj[q];
            lk[j] = A.pair_lk[q];
            const int mj = A.tile_maxj[t0 + tj];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (row0 + wm * 64 + i * 16 <= mj) mask |= 1u << (i * 4 + j);
        }
    }
    mask = __builtin_amdgcn_readfirstlane(mask);
    const bool active = mask != 0;               // wave-uniform

    d4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

    // staging: A rows 128 x 16 z = 1024 double2 (4 per thread); group rows
    // (padded to 160 with valid row indices) x 16 z = 1280 double2 (5 per
    // thread).  Row offsets are fixed for the whole z loop.
    size_t aoff[4], goff[5];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int idx = t + 256 * i;
        aoff[i] = ((size_t)(row0 + (idx >> 3)) << 5) + 2 * (idx & 7);
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        const int idx = t + 256 * i;
        goff[i] = ((size_t)grow[idx >> 3] << 5) + 2 * (idx & 7);
    }
    double2 pa[4], pg[5];
    auto gload = [&](int64_t z0) {
        // z-blocked rows: element (row, z) at ((z / 32) * upad + row) * 32 + z % 32
        const double *base = St + (((size_t)(z0 >> 5) * A.upad) << 5) + (z0 & 31);
#pragma unroll
        for (int i = 0; i < 4; ++i) pa[i] = *reinterpret_cast<const double2 *>(base + aoff[i]);
#pragma unroll
        for (int i = 0; i < 5; ++i) pg[i] = *reinterpret_cast<const double2 *>(base + goff[i]);
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int idx = t + 256 * i;
            const int row = idx >> 3, zp = idx & 7;
            Sa[buf][2 * zp][row] = pa[i].x;
            Sa[buf][2 * zp + 1][row] = pa[i].y;
        }
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            const int idx = t + 256 * i;
            const int row = idx >> 3, zp = idx & 7;
            Sg[buf][2 * zp][row] = pg[i].x;
            Sg[buf][2 * zp + 1][row] = pg[i].y;
        }
    };

    const int64_t nchunks = A.nz / ZC;
    gload(0);
    lstore(0);
    lds_barrier();
    for (int64_t c = 0; c < nchunks; ++c) {
        const int buf = (int)(c & 1);
        if (c + 1 < nchunks) gload((c + 1) * ZC);
        if (active) {
#pragma unroll
            for (int ks = 0; ks < ZC / 4; ++ks) {
                const int z = ks * 4 + (lane >> 4);
                double av[4], bv[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) av[i] = Sa[buf][z][wm * 64 + i * 16 + (lane & 15)];
#pragma unroll
                for (int j = 0; j < 4; ++j) bv[j] = Sg[buf][z][lj[j]] * Sg[buf][z][lk[j]];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
            }
        }
        if (c + 1 < nchunks) lstore(buf ^ 1);
        lds_barrier();
    }

    // FP64 16x16x4 result layout: lane l, element q -> row 4q + l/16, column l%16
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (!(mask & (1u << (i * 4 + j)))) continue;
            const int tile = t0 + wn * 4 + j;
            const int blk = (row0 + wm * 64 + i * 16) >> 4;
            double *dst = T + ((size_t)(A.tile_off[tile] + blk) << 8);
#pragma unroll
            for (int q = 0; q < 4; ++q) dst[(4 * q + (lane >> 4)) * 16 + (lane & 15)] = acc[i][j][q];
        }
}

// ---- operands of the mixed kernel ------------------------------------------
__device__ __forceinline__ uint32_t bf16_rne_bits(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

__global__ void k_split_bf16(int64_t nblk, const double *__restrict__ St, float *__restrict__ S32,
                             uint16_t *__restrict__ SA)
{
    // one thread per 8 consecutive values (the same 8 z of one row in the
    // z-blocked layout): FP32 copy, and BF16 high parts of the FP32 values
    // with the BF16 rounding of the FP64 remainders
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nblk) return;
    const double *src = St + i * 8;
    float f[8];
    uint32_t h[4], l[4];
#pragma unroll
    for (int e = 0; e < 8; ++e) f[e] = (float)src[e];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const double x0 = src[2 * e], x1 = src[2 * e + 1];
        const uint32_t h0 = bf16_rne_bits(f[2 * e]), h1 = bf16_rne_bits(f[2 * e + 1]);
        const float r0 = (float)(x0 - (double)__uint_as_float(h0 << 16));
        const float r1 = (float)(x1 - (double)__uint_as_float(h1 << 16));
        h[e] = h0 | (h1 << 16);
        l[e] = bf16_rne_bits(r0) | (bf16_rne_bits(r1) << 16);
    }
    float4 *o32 = reinterpret_cast<float4 *>(S32 + i * 8);
    o32[0] = make_float4(f[0], f[1], f[2], f[3]);
    o32[1] = make_float4(f[4], f[5], f[6], f[7]);
    uint4 *oa = reinterpret_cast<uint4 *>(SA + i * 16);
    oa[0] = make_uint4(h[0], h[1], h[2], h[3]);
    oa[1] = make_uint4(l[0], l[1], l[2], l[3]);
}

// ---- gather ---------------------------------------------------------------
__device__ __forceinline__ double tget(int a, int b, int c, int U, const int64_t *__restrict__ toff,
                                       const double *__restrict__ T)
{
    // sort a <= b <= c
    int lo = min(a, min(b, c)), hi = max(a, max(b, c));
    int mid = a + b + c - lo - hi;
    const int64_t q = (int64_t)mid * U - (int64_t)mid * (mid - 1) / 2 + (hi - mid);
    const int64_t tile = q >> 4;
    const int n = (int)(q & 15);
    return T[((size_t)(toff[tile] + (lo >> 4)) << 8) + ((lo & 15) << 4) + n];
}

__global__ void k_gather(int kind, int ta, int tp, const int *__restrict__ tri_a,
                         const int *__restrict__ tri_p, int np, int U,
                         const int64_t *__restrict__ toff, const double *__restrict__ T,
                         double *__restrict__ gamma)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)ta * tp) return;
    const int n = (int)(e / tp), m = (int)(e % tp);
    const int a0 = tri_a[3 * n] * np, a1 = tri_a[3 * n + 1] * np, a2 = tri_a[3 * n + 2] * np;
    const int p0 = tri_p[3 * m], p1 = tri_p[3 * m + 1], p2 = tri_p[3 * m + 2];
    double v;
    if (kind == MODAL_GAMMA_ORDERED) {
        v = tget(a0 + p0, a1 + p1, a2 + p2, U, toff, T) * (1.0 / (8.0 * kPi));
    } else {
        v = tget(a0 + p0, a1 + p1, a2 + p2, U, toff, T) + tget(a0 + p0, a1 + p2, a2 + p1, U, toff, T)
          + tget(a0 + p1, a1 + p0, a2 + p2, U, toff, T) + tget(a0 + p1, a1 + p2, a2 + p0, U, toff, T)
          + tget(a0 + p2, a1 + p0, a2 + p1, U, toff, T) + tget(a0 + p2, a1 + p1, a2 + p0, U, toff, T);
        v *= 1.0 / (48.0 * kPi);
    }
    gamma[e] = v;
}

}  // namespace

// ---- plan -----------------------------------------------------------------
void triple_f64_shape(int &rb, int &tpg, int &gr)
{
    rb = F64_ROWBLOCK;
    tpg = F64_TILES;
    gr = F64_GROUP_ROWS;
}

hipError_t build_triple_plan(int U, int rowblock, int tiles_per_group, int group_cap,
                             TriplePlan &plan, std::string &err, DevArena *arena)
{
    free_triple_plan(plan);
    plan.U = U;
    plan.rowblock = rowblock;
    plan.tiles_per_group = tiles_per_group;
    plan.group_rows = group_cap;
    plan.npairs = (int64_t)U * (U + 1) / 2;
    plan.ntiles = (int)((plan.npairs + 15) / 16);
    const int nt = plan.ntiles;
    std::vector<int> pj((size_t)nt * 16, 0), pk((size_t)nt * 16, 0);
    {
        int64_t q = 0;
        for (int j = 0; j < U; ++j)
            for (int k = j; k < U; ++k, ++q) {
                pj[q] = j;
                pk[q] = k;
            }
        for (; q < (int64_t)nt * 16; ++q) { pj[q] = 0; pk[q] = 0; }   // padding pairs
    }
    std::vector<int> maxj(nt);
    std::vector<int64_t> toff(nt);
    int64_t acc = 0;
    for (int t = 0; t < nt; ++t) {
        int64_t last = std::min<int64_t>((int64_t)t * 16 + 15, plan.npairs - 1);
        maxj[t] = pj[last];
        toff[t] = acc;
        acc += maxj[t] / 16 + 1;
    }
    plan.tsize = acc * 256;

    // groups of <= tiles_per_group tiles touching <= group_cap distinct rows
    std::vector<int> gt0, grows, gn;
    std::vector<unsigned short> lj((size_t)nt * 16), lk((size_t)nt * 16);
    std::vector<int> stamp(U, -1), local(U, 0);
    int t = 0;
    while (t < nt) {
        const int g = (int)gt0.size();
        gt0.push_back(t);
        std::vector<int> rows;
        int ntg = 0;
        while (t < nt && ntg < tiles_per_group) {
            int seen[32];
            int ns = 0;
            for (int e = 0; e < 16; ++e) {
                for (int v : {pj[(size_t)t * 16 + e], pk[(size_t)t * 16 + e]}) {
                    if (stamp[v] == g) continue;
                    bool dup = false;
                    for (int s = 0; s < ns; ++s) dup |= (seen[s] == v);
                    if (!dup) seen[ns++] = v;
                }
            }
            if ((int)rows.size() + ns > group_cap) break;
            for (int s = 0; s < ns; ++s) {
                stamp[seen[s]] = g;
                local[seen[s]] = (int)rows.size();
                rows.push_back(seen[s]);
            }
            for (int e = 0; e < 16; ++e) {
                lj[(size_t)t * 16 + e] = (unsigned short)local[pj[(size_t)t * 16 + e]];
                lk[(size_t)t * 16 + e] = (unsigned short)local[pk[(size_t)t * 16 + e]];
            }
            ++t;
            ++ntg;
        }
        gn.push_back((int)rows.size());
        rows.resize(group_cap, 0);
        grows.insert(grows.end(), rows.begin(), rows.end());
    }
    plan.ngroups = (int)gt0.size();
    gt0.push_back(nt);
    std::vector<int2> tasks;
    for (int g = 0; g < plan.ngroups; ++g) {
        int mj = 0;
        for (int tt = gt0[g]; tt < gt0[g + 1]; ++tt) mj = std::max(mj, maxj[tt]);
        for (int rb = 0; rb <= mj / rowblock; ++rb) tasks.push_back(make_int2(g, rb));
    }
    // row block major: the workgroups co-resident on one XCD (contiguous task
    // runs) share their 128 A rows, and neighbouring groups part of their rows
    std::stable_sort(tasks.begin(), tasks.end(), [](int2 a, int2 b) { return a.y < b.y; });
    plan.ntasks = (int)tasks.size();
    plan.borrowed = arena != nullptr;

    hipError_t e = hipSuccess;
    auto up = [&](auto *&dst, const auto &src) {
        using T = std::remove_cv_t<std::remove_reference_t<decltype(src[0])>>;
        if (e != hipSuccess) return;
        const size_t nb = sizeof(T) * std::max<size_t>(src.size(), 1);
        e = arena ? arena->take((void **)&dst, nb) : hipMalloc((void **)&dst, nb);
        if (e == hipSuccess && !src.empty())
            e = hipMemcpy(dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice);
    };
    up(plan.tile_maxj, maxj);
    up(plan.tile_off, toff);
    up(plan.group_tile0, gt0);
    up(plan.group_rows_idx, grows);
    up(plan.group_nrows, gn);
    up(plan.pair_lj, lj);
    up(plan.pair_lk, lk);
    up(plan.tasks, tasks);
    if (e != hipSuccess) {
        err = std::string("triple plan upload: ") + hipGetErrorString(e);
        free_triple_plan(plan);
    }
    return e;
}

void free_triple_plan(TriplePlan &p)
{
    if (p.borrowed) {
        p = TriplePlan{};
        return;
    }
    (void)hipFree(p.tile_maxj);
    (void)hipFree(p.tile_off);
    (void)hipFree(p.group_tile0);
    (void)hipFree(p.group_rows_idx);
    (void)hipFree(p.group_nrows);
    (void)hipFree(p.pair_lj);
    (void)hipFree(p.pair_lk);
    (void)hipFree(p.tasks);
    p = TriplePlan{};
}

static TripleArgs args_of(const TriplePlan &p, int64_t upad, int64_t nz)
{
    TripleArgs a;
    a.tile_maxj = p.tile_maxj;
    a.tile_off = p.tile_off;
    a.group_tile0 = p.group_tile0;
    a.group_rows = p.group_rows_idx;
    a.group_nrows = p.group_nrows;
    a.pair_lj = p.pair_lj;
    a.pair_lk = p.pair_lk;
    a.tasks = p.tasks;
    a.ntasks = p.ntasks;
    a.group_cap = p.group_rows;
    a.upad = upad;
    a.nz = nz;
    return a;
}

hipError_t launch_triple_f64(const TriplePlan &plan, int64_t upad, int64_t ldz, const double *St,
                             double *T, hipStream_t s)
{
    if (ldz % 32 != 0 || upad % F64_ROWBLOCK != 0 || upad < plan.U || plan.rowblock != F64_ROWBLOCK ||
        plan.tiles_per_group != F64_TILES || plan.group_rows != F64_GROUP_ROWS)
        return hipErrorInvalidValue;
    if (plan.ntasks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_triple_f64, dim3(plan.ntasks), dim3(256), 0, s, args_of(plan, upad, ldz), St, T);
    return hipGetLastError();
}

hipError_t launch_split_bf16(int64_t n, const double *St, float *S32, uint16_t *SA, hipStream_t s)
{
    if (n % 8 != 0) return hipErrorInvalidValue;
    const int64_t nb = n / 8;
    hipLaunchKernelGGL(k_split_bf16, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, nb, St, S32, SA);
    return hipGetLastError();
}

hipError_t launch_gather(int kind, int ta, int tp, const int *tri_a, const int *tri_p, int np,
                         const TriplePlan &plan, const double *T, double *gamma, hipStream_t s)
{
    const int64_t n = (int64_t)ta * tp;
    hipLaunchKernelGGL(k_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, kind, ta, tp,
                       tri_a, tri_p, np, plan.U, plan.tile_off, T, gamma);
    return hipGetLastError();
}

}  // namespace mp
