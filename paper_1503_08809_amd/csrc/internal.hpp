// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/modalproj.h"

namespace mp {

constexpr double kPi = 3.14159265358979323846264338327950288;

// Padding of the mu axis inside the library: each r holds a whole number of
// 16-wide z chunks (zeros past nmu), so an r boundary never falls inside a
// chunk of the triple-product kernels.
constexpr int kMuPad = 32;
inline int pad_to(int n, int m) { return (n + m - 1) / m * m; }

struct Error {
    modal_status st;
    std::string msg;
};

// A bump allocator over caller-provided device memory: the no-allocation
// entry point serves its workspace and plans from it instead of hipMalloc.
struct DevArena {
    char *base = nullptr;
    size_t cap = 0, used = 0;
    // p = the next `bytes` (256-byte aligned); hipErrorOutOfMemory when the
    // arena is full
    hipError_t take(void **p, size_t bytes)
    {
        const size_t off = (used + 255) & ~(size_t)255;
        if (bytes > cap || off > cap - bytes) return hipErrorOutOfMemory;
        *p = base + off;
        used = off + bytes;
        return hipSuccess;
    }
};

// ---- launchers (one per kernel family) --------------------------------
// Step a: grids and tables.
hipError_t launch_gauss_legendre(int n, double *x, double *w, hipStream_t s);
// The same rule computed on the host (host arrays, no device).
void gauss_legendre_host(int n, double *x, double *w);
hipError_t launch_legendre_table(int lmax, int lout0, int nmu, int ld, const double *mu,
                                 double *P, hipStream_t s);

// Spherical Bessel functions by Miller's downward recurrence.  The x value of
// item i is xs[i] (table mode) or k[i % nk] * r[i / nk] (beta mode, xs == NULL).
struct BesselState {
    double *f0, *f1;     // f_l and f_{l+1} at the next l to emit
    int *e;              // rescale count at that point
    double *c;           // normalisation in the final frame
    int *efin;           // rescale count at l = 0
};
hipError_t launch_bessel_prepare(int64_t nitems, const double *xs, const double *k, int nk,
                                 const double *r, int lfirst, BesselState st, hipStream_t s);
// Emit l = lhi down to llo (inclusive) into out[(l - llo) * ld_l + i] scaled by
// rowscale[(l - lrow0) * nk + i % nk] when rowscale != NULL.
hipError_t launch_bessel_chunk(int64_t nitems, const double *xs, const double *k, int nk,
                               const double *r, int lhi, int llo, BesselState st,
                               double *out, int64_t ld_l, const double *rowscale, int lrow0,
                               hipStream_t s);

// Step b: beta[p][l - lmin][r] for l in [l0, l0 + nl) from the emitted chunk
// Jd[l - l0][k][r] = Delta_l(k) j_l(k r).
hipError_t launch_beta_gemm(int nl, int l0, int lmin, int L, int nk, int nr, int np,
                            const double *Jd, const double *k, const double *wk,
                            const double *qk, double *beta, hipStream_t s);

// Step c: S rows.  Row u = a * np + p holds, for each r, ldmu values (zero
// past nmu), computed with the mu parity of P_l at nodes symmetric about 0
// (half the work of the plain product); ldP is the row length of P (nodes
// ascending).  upad == 0: caller layout S[u][r][ldmu], unscaled.  upad > 0:
// scaled by wz[z] (the cube root of the quadrature weight) and z-blocked,
// St[z / 32][u][z % 32] with z = r * ldmu + mu and upad rows per block.
hipError_t launch_s_parity(int na, int np, int nr, int nmu, int ldmu, int L, int lmin, const double *wl,
                          const double *ql, const double *beta, const double *P, int ldP, const double *wz,
                          int64_t upad, double *S, hipStream_t s);
// w_l = (2l+1)^(1 - v_power) / sqrt(C_l); cl == NULL reads C_l = 1
hipError_t launch_weights_l(int L, int lmin, double v_power, const double *cl, double *wl,
                            hipStream_t s);
hipError_t launch_cbrt_weights(int nr, int nmu, int ldmu, const double *r, const double *wr,
                               const double *wmu, double *wz, hipStream_t s);
// S in the caller's layout [u][r][nmu] -> scaled, z-blocked rows.
hipError_t launch_s_import(int64_t nu, int64_t upad, int nr, int nmu, int ldmu, const double *S,
                           const double *wz, double *St, hipStream_t s);

// Step d: unique third moments T[i<=j<=k] = Sum_z St_i St_j St_k of the
// z-blocked rows St[z / 32][Upad][32] (Upad = rows padded to kRowPad).
// A plan lists the 16-pair column tiles, their packing offsets in T (shared
// by every plan of the same U), and the workgroup tasks of one kernel shape:
// groups of `tiles_per_group` column tiles touching at most `group_rows`
// distinct rows, times row super-blocks of `rowblock` rows.
struct TriplePlan {
    int U = 0;                 // number of S rows (na * np)
    int rowblock = 0, tiles_per_group = 0, group_rows = 0;
    int64_t npairs = 0;        // U (U + 1) / 2
    int ntiles = 0;            // 16-pair column tiles
    int ngroups = 0;
    int ntasks = 0;
    int64_t tsize = 0;         // doubles in the tile-packed T
    // device arrays
    int *tile_maxj = nullptr;  // [ntiles]
    int64_t *tile_off = nullptr; // [ntiles] offset in 16x16 blocks
    int *group_tile0 = nullptr;  // [ngroups + 1]
    int *group_rows_idx = nullptr; // [ngroups][group_rows]
    int *group_nrows = nullptr;  // [ngroups]
    unsigned short *pair_lj = nullptr; // [ntiles * 16] local row of j in its group
    unsigned short *pair_lk = nullptr; // [ntiles * 16]
    int2 *tasks = nullptr;       // [ntasks] (group, row super-block)
    bool borrowed = false;       // arrays live in a DevArena (never freed)
};
// S rows are allocated padded to a multiple of kRowPad (>= every rowblock),
// and the z blocks of 32 to a multiple of kZBlockPad (zero past the data).
constexpr int kRowPad = 256;
constexpr int kZBlockPad = 8;
// arena != NULL: the plan's device arrays are taken from it (no hipMalloc)
hipError_t build_triple_plan(int U, int rowblock, int tiles_per_group, int group_rows,
                             TriplePlan &plan, std::string &err, DevArena *arena = nullptr);
void free_triple_plan(TriplePlan &plan);
// shape of the FP64 kernel
void triple_f64_shape(int &rowblock, int &tiles_per_group, int &group_rows);

hipError_t launch_triple_f64(const TriplePlan &plan, int64_t upad, int64_t ldz,
                             const double *St, double *T, hipStream_t s);
// Block-triple plan of the mixed kernel: tasks (ib, jb, kb) of 128 x 16 x 16
// rows, the task index of every block triple (-1 if it holds no i <= j <= k),
// and T packed per task.  The kernel reads S32, the FP32 copy of the scaled
// rows (z-blocked like St), and SA, their BF16 (hi, lo) split packed per 8 z
// values ([z / 32][Upad][4][8 hi, 8 lo]); each r holds nmu_pad z values (a
// multiple of 32).
struct BTPlan {
    int U = 0;
    int nib = 0, njb = 0, nkb = 0;
    int ntasks = 0;
    int64_t tsize = 0;         // doubles of T
    int4 *tasks = nullptr;     // device [ntasks]
    int *tidx = nullptr;       // device [nib][njb][nkb]
    bool borrowed = false;     // arrays live in a DevArena (never freed)
};
hipError_t build_bt_plan(int U, BTPlan &plan, std::string &err, DevArena *arena = nullptr);
void free_bt_plan(BTPlan &plan);
hipError_t launch_triple_bt(const BTPlan &plan, int64_t upad, int64_t ldz, int nmu_pad,
                            const float *S32, const uint16_t *SA, double *T, hipStream_t s);
hipError_t launch_gather_bt(int kind, int ta, int tp, const int *tri_a, const int *tri_p, int np,
                            const BTPlan &plan, const double *T, double *gamma, hipStream_t s);
// Elementwise over the n values (a multiple of 8): S32 and SA as above.
hipError_t launch_split_bf16(int64_t n, const double *St, float *S32, uint16_t *SA,
                             hipStream_t s);

// Adjoint stages (k_adjoint*.hip).  Step d: dL/dSt_u(z) = Sum_{v <= w}
// Hc[u][(v,w)] St_v(z) St_w(z), Hc built from G in each kernel's operand
// order.  Shat and St are z-blocked with nzb z blocks (a multiple of
// kZBlockPad, zero past the data); rows >= U of Shat are left unwritten.
// Factored mixed adjoint of step d (k_adjoint_fac.hip): for every v, the w
// steps (32 wide) from the one holding v to the last; Hc is stored per
// (v, w step) as [v_step_offset(v) + ws - v / 32][row block of 256][row
// tile][hi/lo][lane] (uint4, 2048 per step and row block), and St pre-split in
// the B-operand order (SB, uint4, 128 per z block of 32, w step and half).
__host__ __device__ inline int64_t v_step_offset(int v, int nws)
{
    const int64_t a = v >> 5, b = v & 31;      // Sum_{v' < v} (nws - v' / 32)
    return 32 * (a * nws - a * (a - 1) / 2) + b * (nws - a);
}
int adj_fac_rowblock();
// FP64 factored adjoint of step d (k_adjoint_fac64.hip): the same order with
// 16-wide w steps; Hc in FP64 per (v, w step) as [step][row block of 128]
// [k step 4][row tile 8][lane] (2048 doubles per step and row block).
__host__ __device__ inline int64_t v_step_offset16(int v, int nws)
{
    const int64_t a = v >> 4, b = v & 15;      // Sum_{v' < v} (nws - v' / 16)
    return 16 * (a * nws - a * (a - 1) / 2) + b * (nws - a);
}
int adj_fac64_rowblock();
hipError_t launch_build_hc_fac64(int kind, int U, int np, int na, const int *inv_a, const int *inv_p,
                                 const double *G, int tp, int nib, double *Hc, hipStream_t s);
hipError_t launch_adj_fac64(int U, int64_t upad, int64_t nzb, const double *St, const double *Hc, double *Shat,
                            hipStream_t s);
hipError_t launch_build_hc_fac(int kind, int U, int np, int na, const int *inv_a, const int *inv_p,
                               const double *G, int tp, int nib, uint4 *Hc, hipStream_t s);
hipError_t launch_split_b(int64_t nzb, int U, int64_t upad, const double *St, uint4 *SB, hipStream_t s);
hipError_t launch_adj_fac(int U, int64_t upad, int64_t nzb, const double *St, const uint4 *SB,
                          const uint4 *Hc, double *Shat, hipStream_t s);
// dL/dbeta from dL/dSt (z-blocked; folded over +-mu and scaled by wz in place)
hipError_t launch_betahat(int na, int np, int nr, int nmu, int ldmu, int L, int lmin, int64_t upad,
                          const double *wl, const double *ql, const double *P, double *Shat,
                          const double *wz, double *bhat, hipStream_t s);
hipError_t launch_ahat(int nl, int l0, int lmin, int L, int np, int nk, int nr, const double *bhat,
                       const double *J, double *Ahat, hipStream_t s);
hipError_t launch_dq_ddelta(int nl, int l0, int lmin, int np, int nk, const double *k, const double *wk,
                            const double *qk, const double *delta, const double *Ahat, double *dq,
                            double *dd, int first, hipStream_t s);

// Gather Gamma entries from T.
// Eq. (3D) (k_modal3d.hip): operand G[(rb U + u) L + l'] (l' parity-sorted,
// even l first) for r in [r0, r0 + nrb); the band of 2 (3j)^2 for one l1 and
// one pair of parity classes, K[i3 n2 + i2]; the r weights times the row l1'
// of G, C[rb U + u]; and the gather of Gamma' from T(u1 <= u2 <= u3).
hipError_t launch_build_g3(int L, int nE, int lE0, int lO0, int lmin, int nr, int np, int na, int r0, int nrb,
                           const double *wl, const double *ql, const double *beta, double *G, hipStream_t s);
hipError_t launch_start3(int lmax, double *V, hipStream_t s);
hipError_t launch_build_k3(int l1, const int l0[2], const int n[2], int gosper, const double *V, double *K0,
                           double *K1, hipStream_t s);
hipError_t launch_c3(int L, int lp1, int U, int r0, int nrb, const double *r, const double *wr, const double *G,
                     double *C, hipStream_t s);
hipError_t launch_zero_rows3(int64_t ld, int row0, int nrows, int64_t ncols, double *A, hipStream_t s);
hipError_t launch_gather3(int kind, int ta, int tp, const int *tri_a, const int *tri_p, int np, int U,
                          const double *T, double *gamma, hipStream_t s);

// Column-major FP64 matrix-core GEMM (k_dgemm.hip), strided batches:
// C_b = alpha op(A_b) op(B_b) + beta C_b with op(A)(m, k) = ta ? A[k + m lda]
// : A[m + k lda], op(B)(k, n) = tb ? B[n + k ldb] : B[k + n ldb]; tile = 64
// or 128 (the output tile edge of a workgroup).
hipError_t launch_dgemm(bool ta, bool tb, int m, int n, int k, double alpha, const double *A, int64_t lda,
                        int64_t sA, const double *B, int64_t ldb, int64_t sB, double beta, double *C,
                        int64_t ldc, int64_t sC, int batch, hipStream_t s, int tile = 128);
// The square m x m product C = op(A) op(B) (k deep) on and below its
// diagonal only, stored as u2-major pairs: P_b[n m - n (n - 1) / 2 + (m' - n)]
// = C(m', n) for m' >= n (sP >= m (m + 1) / 2 doubles per batch).
hipError_t launch_dgemm_packed_lower(bool ta, bool tb, int m, int k, const double *A, int64_t lda, int64_t sA,
                                     const double *B, int64_t ldb, int64_t sB, double *P, int64_t sP, int batch,
                                     hipStream_t s);

// Blocked Cholesky pieces (k_chol.hip): factor one diagonal block (at most
// chol_block() wide; *info = 1 if it is not positive definite), and solve
// rows vectors (element j of vector i at X[i xr + j xc]) against the lower
// block L: x L^T = x (backward = 0) or x L = x (backward = 1).
int chol_block();
hipError_t launch_potrf_block(int jb, double *A, int64_t lda, int *info, hipStream_t s);
hipError_t launch_trsm_rows(int rows, int jb, const double *L, int64_t ldl, double *X, int64_t xr, int64_t xc,
                            int backward, hipStream_t s);

hipError_t launch_gather(int kind, int ta, int tp, const int *tri_a, const int *tri_p,
                         int np, const TriplePlan &plan, const double *T, double *gamma,
                         hipStream_t s);

}  // namespace mp
