// C ABI of the separable projection: argument checks, workspace, host/device
// staging, and the order of the stages (Sec. 2.2, Eq. (2D) and
// Eq. (legendre); Appendix, projected modes).  No exception or abort crosses
// the boundary: every entry point returns a modal_status.
#include "internal.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>

using namespace mp;

// ---- the no-allocation scratch ---------------------------------------------
// modal_gamma_noalloc serves every buffer it needs from this array instead of
// hipMalloc.  Each device holds its own copy, whose device address is looked
// up once per device (modal_create) and kept in g_scratch_ptr; host code only
// ever uses that address, never the array's name.  Calls on one device share
// it: two such calls that overlap on one device race.
constexpr size_t kScratchBytes = (size_t)MODAL_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxScratchDevices] = {};

namespace {

thread_local std::string g_last_error;   // for calls without a usable context

enum Slot {
    W_MU, W_WMU, W_P, W_WL, W_WZ, W_BSTATE, W_JCHUNK, W_BETA, W_ST, W_T,
    W_S32, W_SH, W_SL, W_GAMMA,
    W_INVA, W_INVP, W_H, W_SHAT, W_BHAT, W_AHAT, W_DQ, W_DD, W_GRAM, W_INFO,
    W_G3, W_A3, W_C3, W_K3, W_T3, W_P3, W_V3, W_FLAG,
    W_IN0, NSLOTS = W_IN0 + 16
};

struct Buf {
    void *p = nullptr;
    size_t n = 0;
};

struct Grid {
    const double *k, *wk, *r, *wr, *mu, *wmu;
};

// Steps a-c of the forward projection: GL rule, Legendre table, weights,
// beta (Bessel chunks) and the scaled, z-blocked S rows.
struct Forward {
    Grid G;
    const double *delta, *qk, *cl, *ql;
    double *P, *wl, *wz, *beta, *St;
};

// The forward tables of the last modal_gamma (or recomputing
// modal_gamma_backward) call, kept for a later modal_gamma_backward when the
// caller has enabled reuse: valid only until any other call, and only for the
// same grid and problem (every field, pointers included).
struct FwdCache {
    bool valid = false, was_valid = false;
    modal_grid g{};
    modal_problem p{};
    Forward f{};
    int next_in = 0;                   // host-input slots its staging used
};

bool same_inputs(const modal_grid &a, const modal_grid &b)
{
    return a.lmin == b.lmin && a.lmax == b.lmax && a.nk == b.nk && a.k == b.k && a.wk == b.wk && a.nr == b.nr &&
           a.r == b.r && a.wr == b.wr && a.nmu == b.nmu && a.mu == b.mu && a.wmu == b.wmu &&
           a.allow_inexact_gl == b.allow_inexact_gl;
}

bool same_inputs(const modal_problem &a, const modal_problem &b)
{
    return a.delta == b.delta && a.cl == b.cl && a.np == b.np && a.qk == b.qk && a.na == b.na && a.ql == b.ql &&
           a.v_power == b.v_power && a.kind == b.kind && a.ta == b.ta && a.tri_a == b.tri_a && a.tp == b.tp &&
           a.tri_p == b.tri_p;
}

}  // namespace

struct modal_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    Buf ws[NSLOTS];
    size_t limit = 0;
    int next_in = 0;
    TriplePlan plan64;                 // triple-product plan of the FP64 kernel
    BTPlan planbt;                     // block-triple plan of the mixed kernel
    bool timing = false;
    bool reuse_fwd = false;            // modal_set_forward_reuse
    FwdCache fwd;
    // per stage: a pool of (start, end) event pairs; the first `used` belong
    // to the last call (chunked stages record one pair per chunk)
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[MODAL_NSTAGES];
    int used[MODAL_NSTAGES] = {};
    // no-allocation mode (modal_gamma_noalloc): every workspace slot and plan
    // comes from the device's scratch array through a bump arena
    bool arena_on = false;
    DevArena arena;
    void *aslot_p[NSLOTS] = {};
    size_t aslot_n[NSLOTS] = {};
    TriplePlan aplan64;                // plans built in the arena (borrowed)
    BTPlan aplanbt;
};

namespace {

struct Fail {
    modal_status st;
};

[[noreturn]] void fail(modal_ctx c, modal_status st, const std::string &msg)
{
    if (c) c->err = msg;
    g_last_error = msg;
    throw Fail{st};
}

void hipck(modal_ctx c, hipError_t e, const char *what)
{
    if (e != hipSuccess) {
        const modal_status st = (e == hipErrorOutOfMemory) ? MODAL_ERR_OOM : MODAL_ERR_DEVICE;
        fail(c, st, std::string(what) + ": " + hipGetErrorString(e));
    }
}

size_t held_bytes(modal_ctx c)
{
    size_t s = 0;
    for (auto &b : c->ws) s += b.n;
    return s;
}

void *ws_get(modal_ctx c, int slot, size_t bytes)
{
    if (bytes == 0) bytes = 8;
    if (c->arena_on) {
        if (c->aslot_n[slot] >= bytes) return c->aslot_p[slot];
        void *p = nullptr;
        if (c->arena.take(&p, bytes) != hipSuccess)
            fail(c, MODAL_ERR_OOM,
                 "the problem needs more than the " + std::to_string(kScratchBytes) +
                     "-byte no-allocation scratch (use modal_gamma)");
        c->aslot_p[slot] = p;
        c->aslot_n[slot] = bytes;
        return p;
    }
    Buf &b = c->ws[slot];
    if (b.n >= bytes) return b.p;
    if (c->limit && held_bytes(c) - b.n + bytes > c->limit)
        fail(c, MODAL_ERR_OOM, "workspace limit exceeded (" + std::to_string(bytes) + " bytes requested)");
    if (b.p) {
        hipck(c, hipStreamSynchronize(c->stream), "sync before realloc");
        (void)hipFree(b.p);
        b.p = nullptr;
        b.n = 0;
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(c, MODAL_ERR_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    b.p = p;
    b.n = bytes;
    return p;
}

// Device-visible copy of a caller array (the caller's pointer itself if it is
// device memory of this context's device).
bool is_device_ptr(modal_ctx c, const void *p)
{
    hipPointerAttribute_t a;
    hipError_t e = hipPointerGetAttributes(&a, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    if (a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged) {
        if (a.device != c->device) fail(c, MODAL_ERR_INVALID_ARG, "device pointer of another device");
        return true;
    }
    return false;
}

template <class T>
const T *dev_in(modal_ctx c, const T *p, size_t count)
{
    if (!p || count == 0) return p;
    if (is_device_ptr(c, p)) return p;
    if (c->arena_on)
        fail(c, MODAL_ERR_INVALID_ARG, "modal_gamma_noalloc takes device arrays only (a host array needs staging)");
    if (c->next_in >= 16) fail(c, MODAL_ERR_INVALID_ARG, "too many host inputs");
    T *d = (T *)ws_get(c, W_IN0 + c->next_in++, sizeof(T) * count);
    hipck(c, hipMemcpyAsync(d, p, sizeof(T) * count, hipMemcpyHostToDevice, c->stream), "H2D");
    return d;
}

template <class T>
std::vector<T> host_copy(modal_ctx c, const T *p, size_t count)
{
    std::vector<T> v(count);
    if (count == 0) return v;
    if (is_device_ptr(c, p)) {
        hipck(c, hipMemcpyAsync(v.data(), p, sizeof(T) * count, hipMemcpyDeviceToHost, c->stream), "D2H");
        hipck(c, hipStreamSynchronize(c->stream), "sync");
    } else {
        std::memcpy(v.data(), p, sizeof(T) * count);
    }
    return v;
}

struct OutBuf {
    double *dev = nullptr;
    double *host = nullptr;
    size_t count = 0;
};

OutBuf dev_out(modal_ctx c, double *p, size_t count, int slot)
{
    OutBuf o;
    o.count = count;
    if (count == 0) {
        o.dev = p;
        return o;
    }
    if (is_device_ptr(c, p)) {
        o.dev = p;
    } else {
        if (c->arena_on)
            fail(c, MODAL_ERR_INVALID_ARG, "modal_gamma_noalloc takes device arrays only (a host output needs staging)");
        o.host = p;
        o.dev = (double *)ws_get(c, slot, sizeof(double) * count);
    }
    return o;
}

void finish_out(modal_ctx c, const OutBuf &o)
{
    if (o.host && o.count) {
        hipck(c, hipMemcpyAsync(o.host, o.dev, sizeof(double) * o.count, hipMemcpyDeviceToHost, c->stream),
              "D2H");
        hipck(c, hipStreamSynchronize(c->stream), "sync");
    }
}

struct StageTimer {
    modal_ctx c;
    int st;
    hipEvent_t end = nullptr;
    StageTimer(modal_ctx c_, int s) : c(c_), st(s)
    {
        if (!c->timing || c->arena_on) return;      // events are not made in no-allocation mode
        auto &pool = c->ev[st];
        if (c->used[st] == (int)pool.size()) {
            hipEvent_t a = nullptr, b = nullptr;
            hipck(c, hipEventCreate(&a), "event create");
            if (hipEventCreate(&b) != hipSuccess) {
                (void)hipEventDestroy(a);
                fail(c, MODAL_ERR_DEVICE, "event create");
            }
            pool.emplace_back(a, b);
        }
        auto &pr = pool[c->used[st]++];
        hipck(c, hipEventRecord(pr.first, c->stream), "event");
        end = pr.second;
    }
    ~StageTimer()
    {
        if (end) (void)hipEventRecord(end, c->stream);
    }
};

// Fill kernel (no memset nodes: callers may capture these streams).
__global__ void k_zero(double *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

void zero(modal_ctx c, double *p, int64_t n)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, p, n);
    hipck(c, hipGetLastError(), "zero fill");
}

// flag[0] = 1 if any of the n values is not finite (every writer stores the
// same value, so the unordered stores need no atomics); flag is cleared by
// the caller with the fill kernel first.
__global__ void k_flag_nonfinite(const double *__restrict__ p, int64_t n, int *__restrict__ flag)
{
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        bad |= !isfinite(p[i]);
    if (bad) flag[0] = 1;
}

__global__ void k_zero_int(int *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// Zero the padding rows U..upad of every 32-wide z block of a z-blocked array.
__global__ void k_zero_pad_rows(double *St, int64_t nzb, int64_t upad, int64_t U)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (upad - U) * 32;
    if (i >= nzb * per) return;
    const int64_t zb = i / per, rem = i % per;
    St[(zb * upad + U) * 32 + rem] = 0.0;
}

void zero_pad_rows(modal_ctx c, double *St, int64_t ldz, int64_t upad, int64_t U)
{
    const int64_t n = (ldz / 32) * (upad - U) * 32;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_zero_pad_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, St,
                       ldz / 32, upad, U);
    hipck(c, hipGetLastError(), "zero fill");
}

// ---- validation -------------------------------------------------------------
struct Dims {
    int L, nk, nr, nmu, ldmu, np, na, U;
};

void need(modal_ctx c, bool ok, modal_status st, const char *msg)
{
    if (!ok) fail(c, st, msg);
}

Dims check_grid(modal_ctx c, const modal_grid *g, bool need_mu_rule)
{
    need(c, g != nullptr, MODAL_ERR_INVALID_ARG, "grid is NULL");
    need(c, g->lmin >= 0 && g->lmax >= g->lmin, MODAL_ERR_SHAPE, "need 0 <= lmin <= lmax");
    need(c, g->lmax <= 20000, MODAL_ERR_SHAPE, "lmax above 20000");
    need(c, g->nk >= 1 && g->nr >= 1 && g->nmu >= 1, MODAL_ERR_SHAPE, "nk, nr, nmu must be >= 1");
    need(c, g->k && g->wk && g->r && g->wr, MODAL_ERR_INVALID_ARG, "k, wk, r, wr must be non-NULL");
    need(c, (g->mu == nullptr) == (g->wmu == nullptr), MODAL_ERR_INVALID_ARG,
         "mu and wmu must both be given or both be NULL");
    if (need_mu_rule && !g->allow_inexact_gl) {
        const int64_t nmin = (3 * (int64_t)g->lmax + 2) / 2;     // ceil((3 lmax + 1) / 2)
        need(c, g->nmu >= nmin, MODAL_ERR_SHAPE,
             "nmu below ceil((3 lmax + 1)/2): the mu rule would not be exact (set allow_inexact_gl)");
    }
    {
        auto hk = host_copy(c, g->k, (size_t)g->nk);
        auto hr = host_copy(c, g->r, (size_t)g->nr);
        double km = 0.0, rm = 0.0;
        for (double v : hk) {
            need(c, v > 0.0 && std::isfinite(v), MODAL_ERR_NUMERIC, "k must be finite and > 0");
            km = std::max(km, v);
        }
        for (double v : hr) {
            need(c, v > 0.0 && std::isfinite(v), MODAL_ERR_NUMERIC, "r must be finite and > 0");
            rm = std::max(rm, v);
        }
        need(c, km * rm < 1e6, MODAL_ERR_SHAPE, "k r above 1e6: Bessel recurrence range not supported");
    }
    Dims d{};
    d.L = g->lmax - g->lmin + 1;
    d.nk = g->nk;
    d.nr = g->nr;
    d.nmu = g->nmu;
    d.ldmu = pad_to(g->nmu, kMuPad);
    return d;
}

// Every value of a caller array (host or device) must be finite: a NaN or an
// infinity in Delta, q or qbar would otherwise run through every stage and
// surface only as a non-finite Gamma.  Device arrays are scanned by a kernel
// on the context's stream (one flag read back); host arrays on the host.
void check_finite(modal_ctx c, const double *p, size_t n, const char *msg)
{
    if (!p || n == 0) return;
    if (!is_device_ptr(c, p)) {
        for (size_t i = 0; i < n; ++i) need(c, std::isfinite(p[i]), MODAL_ERR_NUMERIC, msg);
        return;
    }
    int *flag = (int *)ws_get(c, W_FLAG, sizeof(int));
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, c->stream, flag, 1);
    hipck(c, hipGetLastError(), "zero fill");
    const int64_t blocks = std::min<int64_t>(4096, ((int64_t)n + 255) / 256);
    hipLaunchKernelGGL(k_flag_nonfinite, dim3((unsigned)blocks), dim3(256), 0, c->stream, p, (int64_t)n, flag);
    hipck(c, hipGetLastError(), "finiteness scan");
    int h = 0;
    hipck(c, hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, c->stream), "D2H");
    hipck(c, hipStreamSynchronize(c->stream), "sync");
    need(c, h == 0, MODAL_ERR_NUMERIC, msg);
}

void check_problem(modal_ctx c, const modal_problem *p, Dims &d, bool need_delta, bool need_tri,
                   bool scan_values = true)
{
    need(c, p != nullptr, MODAL_ERR_INVALID_ARG, "problem is NULL");
    need(c, p->np >= 1 && p->na >= 1, MODAL_ERR_SHAPE, "np and na must be >= 1");
    need(c, (int64_t)p->np * p->na <= 8192, MODAL_ERR_SHAPE, "np * na above 8192");
    need(c, p->cl && p->ql, MODAL_ERR_INVALID_ARG, "cl and ql must be non-NULL");
    if (need_delta) need(c, p->delta && p->qk, MODAL_ERR_INVALID_ARG, "delta and qk must be non-NULL");
    need(c, std::isfinite(p->v_power), MODAL_ERR_NUMERIC, "v_power not finite");
    d.np = p->np;
    d.na = p->na;
    d.U = p->np * p->na;
    auto cl = host_copy(c, p->cl, (size_t)d.L);
    for (double v : cl) need(c, v > 0.0 && std::isfinite(v), MODAL_ERR_NUMERIC, "C_l must be finite and > 0");
    if (scan_values) check_finite(c, p->ql, (size_t)d.na * d.L, "qbar_a(l) must be finite");
    if (need_delta && scan_values) {
        check_finite(c, p->delta, (size_t)d.L * d.nk, "Delta_l(k) must be finite");
        check_finite(c, p->qk, (size_t)d.np * d.nk, "q_p(k) must be finite");
    }
    if (need_tri) {
        need(c, p->kind == MODAL_GAMMA_ORDERED || p->kind == MODAL_GAMMA_SYMMETRIC, MODAL_ERR_INVALID_ARG,
             "kind must be MODAL_GAMMA_ORDERED or MODAL_GAMMA_SYMMETRIC");
        need(c, p->ta >= 0 && p->tp >= 0, MODAL_ERR_SHAPE, "ta, tp must be >= 0");
        need(c, p->ta == 0 || p->tri_a, MODAL_ERR_INVALID_ARG, "tri_a is NULL");
        need(c, p->tp == 0 || p->tri_p, MODAL_ERR_INVALID_ARG, "tri_p is NULL");
        auto ta = host_copy(c, p->tri_a, (size_t)p->ta * 3);
        for (int v : ta) need(c, v >= 0 && v < p->na, MODAL_ERR_SHAPE, "tri_a entry outside [0, na)");
        auto tp = host_copy(c, p->tri_p, (size_t)p->tp * 3);
        for (int v : tp) need(c, v >= 0 && v < p->np, MODAL_ERR_SHAPE, "tri_p entry outside [0, np)");
    }
}

void check_prec(modal_ctx c, modal_precision prec)
{
    need(c, prec == MODAL_FP64 || prec == MODAL_MIXED, MODAL_ERR_INVALID_ARG, "unknown precision");
}

template <class F>
modal_status guarded(modal_ctx c, F &&f)
{
    if (!c) {
        g_last_error = "context is NULL";
        return MODAL_ERR_INVALID_ARG;
    }
    c->next_in = 0;
    // any call may overwrite the workspace: only modal_gamma and
    // modal_gamma_backward set the forward tables valid again
    c->fwd.was_valid = c->fwd.valid;
    c->fwd.valid = false;
    try {
        hipError_t e = hipSetDevice(c->device);
        if (e != hipSuccess) fail(c, MODAL_ERR_DEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
        if (c->timing)
            for (int s = 0; s < MODAL_NSTAGES; ++s) c->used[s] = 0;
        f();
        return MODAL_OK;
    } catch (const Fail &x) {
        return x.st;
    } catch (const std::bad_alloc &) {
        c->err = g_last_error = "host allocation failed";
        return MODAL_ERR_OOM;
    } catch (...) {
        c->err = g_last_error = "internal error";
        return MODAL_ERR_DEVICE;
    }
}

// ---- shared pipeline pieces ---------------------------------------------------

Grid stage_grid(modal_ctx c, const modal_grid *g, const Dims &d)
{
    Grid G;
    G.k = dev_in(c, g->k, d.nk);
    G.wk = dev_in(c, g->wk, d.nk);
    G.r = dev_in(c, g->r, d.nr);
    G.wr = dev_in(c, g->wr, d.nr);
    if (g->mu) {
        G.mu = dev_in(c, g->mu, d.nmu);
        G.wmu = dev_in(c, g->wmu, d.nmu);
    } else {
        StageTimer tm(c, MODAL_STAGE_GL);
        double *mu = (double *)ws_get(c, W_MU, sizeof(double) * d.nmu);
        double *wmu = (double *)ws_get(c, W_WMU, sizeof(double) * d.nmu);
        hipck(c, launch_gauss_legendre(d.nmu, mu, wmu, c->stream), "gauss_legendre");
        G.mu = mu;
        G.wmu = wmu;
    }
    return G;
}

// beta[p][l][r] into `beta` (device).
void run_beta(modal_ctx c, const modal_grid *g, const Dims &d, const Grid &G, const double *delta,
              const double *qk, double *beta)
{
    const int64_t nitems = (int64_t)d.nk * d.nr;
    BesselState st;
    char *sb = (char *)ws_get(c, W_BSTATE, (size_t)nitems * 40);
    st.f0 = (double *)sb;
    st.f1 = st.f0 + nitems;
    st.c = st.f1 + nitems;
    st.e = (int *)(st.c + nitems);
    st.efin = st.e + nitems;
    const size_t per_l = (size_t)nitems * sizeof(double);
    int cl = (int)std::max<size_t>(1, std::min<size_t>((size_t)d.L, ((size_t)512 << 20) / per_l));
    double *jd = (double *)ws_get(c, W_JCHUNK, per_l * cl);
    {
        StageTimer tm(c, MODAL_STAGE_BESSEL);
        hipck(c, launch_bessel_prepare(nitems, nullptr, G.k, d.nk, G.r, g->lmax, st, c->stream),
              "bessel prepare");
    }
    for (int lhi = g->lmax; lhi >= g->lmin; lhi -= cl) {
        const int llo = std::max(g->lmin, lhi - cl + 1);
        {
            StageTimer tm(c, MODAL_STAGE_BESSEL);
            hipck(c, launch_bessel_chunk(nitems, nullptr, G.k, d.nk, G.r, lhi, llo, st, jd, nitems,
                                         delta + (size_t)(llo - g->lmin) * d.nk, llo, c->stream),
                  "bessel chunk");
        }
        StageTimer tm(c, MODAL_STAGE_BETA);
        hipck(c, launch_beta_gemm(lhi - llo + 1, llo, g->lmin, d.L, d.nk, d.nr, d.np, jd, G.k, G.wk, qk,
                                  beta, c->stream),
              "beta gemm");
    }
}

// rowscale pointer arithmetic above: the emit kernel indexes
// rowscale[(l - lrow0) * nk + k] with lrow0 = llo, so the pointer is offset to
// row llo of delta.

Forward run_forward(modal_ctx c, const modal_grid *g, const modal_problem *p, const Dims &d)
{
    Forward f;
    f.G = stage_grid(c, g, d);
    f.delta = dev_in(c, p->delta, (size_t)d.L * d.nk);
    f.qk = dev_in(c, p->qk, (size_t)d.np * d.nk);
    f.cl = dev_in(c, p->cl, (size_t)d.L);
    f.ql = dev_in(c, p->ql, (size_t)d.na * d.L);
    // (a) Legendre table at the nodes, weights
    f.P = (double *)ws_get(c, W_P, sizeof(double) * (size_t)d.L * d.ldmu);
    f.wl = (double *)ws_get(c, W_WL, sizeof(double) * d.L);
    const int64_t ldz = (int64_t)d.nr * d.ldmu;
    f.wz = (double *)ws_get(c, W_WZ, sizeof(double) * ldz);
    {
        StageTimer tm(c, MODAL_STAGE_LEGENDRE);
        hipck(c, launch_legendre_table(g->lmax, g->lmin, d.nmu, d.ldmu, f.G.mu, f.P, c->stream), "legendre");
    }
    // (a, b) Bessel functions and the k contraction
    f.beta = (double *)ws_get(c, W_BETA, sizeof(double) * (size_t)d.np * d.L * d.nr);
    run_beta(c, g, d, f.G, f.delta, f.qk, f.beta);
    // (c) the l contraction, scaled rows
    // St holds whole groups of kZBlockPad z blocks; the blocks past ldz are
    // zero (the adjoint kernels work on whole z tiles)
    const int Upad = pad_to(d.U, kRowPad);
    const int64_t nzb = ldz / 32, nzbp = (nzb + kZBlockPad - 1) / kZBlockPad * kZBlockPad;
    f.St = (double *)ws_get(c, W_ST, sizeof(double) * (size_t)Upad * nzbp * 32);
    zero(c, f.St + (size_t)nzb * Upad * 32, (nzbp - nzb) * Upad * 32);
    {
        StageTimer tm(c, MODAL_STAGE_S);
        hipck(c, launch_weights_l(d.L, g->lmin, p->v_power, f.cl, f.wl, c->stream), "weights");
        hipck(c, launch_cbrt_weights(d.nr, d.nmu, d.ldmu, f.G.r, f.G.wr, f.G.wmu, f.wz, c->stream),
              "cbrt weights");
        // the padding rows U..Upad of every z block must read as zero
        zero_pad_rows(c, f.St, ldz, Upad, d.U);
        hipck(c, launch_s_parity(d.na, d.np, d.nr, d.nmu, d.ldmu, d.L, g->lmin, f.wl, f.ql, f.beta, f.P, d.ldmu,
                                 f.wz, Upad, f.St, c->stream),
              "S gemm");
    }
    return f;
}

const TriplePlan &ensure_plan64(modal_ctx c, int U)
{
    if (c->arena_on) {          // built in the scratch for this call only
        int rb, tpg, gr;
        triple_f64_shape(rb, tpg, gr);
        std::string err;
        hipck(c, hipStreamSynchronize(c->stream), "sync");
        hipError_t e = build_triple_plan(U, rb, tpg, gr, c->aplan64, err, &c->arena);
        if (e != hipSuccess)
            fail(c, e == hipErrorOutOfMemory ? MODAL_ERR_OOM : MODAL_ERR_DEVICE, err + " (no-allocation scratch)");
        return c->aplan64;
    }
    TriplePlan &pl = c->plan64;
    if (pl.U == U && pl.tasks) return pl;
    int rb, tpg, gr;
    triple_f64_shape(rb, tpg, gr);
    std::string err;
    hipck(c, hipStreamSynchronize(c->stream), "sync");
    hipError_t e = build_triple_plan(U, rb, tpg, gr, pl, err);
    if (e != hipSuccess) fail(c, e == hipErrorOutOfMemory ? MODAL_ERR_OOM : MODAL_ERR_DEVICE, err);
    return pl;
}

const BTPlan &ensure_planbt(modal_ctx c, int U)
{
    if (c->arena_on) {          // built in the scratch for this call only
        std::string err;
        hipck(c, hipStreamSynchronize(c->stream), "sync");
        hipError_t e = build_bt_plan(U, c->aplanbt, err, &c->arena);
        if (e != hipSuccess)
            fail(c, e == hipErrorOutOfMemory ? MODAL_ERR_OOM : MODAL_ERR_DEVICE, err + " (no-allocation scratch)");
        return c->aplanbt;
    }
    BTPlan &pl = c->planbt;
    if (pl.U == U && pl.tasks) return pl;
    std::string err;
    hipck(c, hipStreamSynchronize(c->stream), "sync");
    hipError_t e = build_bt_plan(U, pl, err);
    if (e != hipSuccess) fail(c, e == hipErrorOutOfMemory ? MODAL_ERR_OOM : MODAL_ERR_DEVICE, err);
    return pl;
}

// Triple products from the z-blocked scaled rows St ([ldz/32][Upad][32]) and gather.
void run_triple_gather(modal_ctx c, const modal_problem *p, const Dims &d, modal_precision prec,
                       double *St, double *gamma)
{
    const int64_t ldz = (int64_t)d.nr * d.ldmu;
    const int64_t upad = pad_to(d.U, kRowPad);
    const int *ta = dev_in(c, p->tri_a, (size_t)p->ta * 3);
    const int *tp = dev_in(c, p->tri_p, (size_t)p->tp * 3);
    if (prec == MODAL_FP64) {
        const TriplePlan &plan = ensure_plan64(c, d.U);
        double *T = (double *)ws_get(c, W_T, sizeof(double) * (size_t)plan.tsize);
        {
            StageTimer tm(c, MODAL_STAGE_TRIPLE);
            hipck(c, launch_triple_f64(plan, upad, ldz, St, T, c->stream), "triple f64");
        }
        if ((int64_t)p->ta * p->tp == 0) return;
        StageTimer tm(c, MODAL_STAGE_GATHER);
        hipck(c, launch_gather(p->kind, p->ta, p->tp, ta, tp, d.np, plan, T, gamma, c->stream), "gather");
        return;
    }
    const BTPlan &plan = ensure_planbt(c, d.U);
    double *T = (double *)ws_get(c, W_T, sizeof(double) * (size_t)plan.tsize);
    const size_t n = (size_t)upad * ldz;
    float *s32 = (float *)ws_get(c, W_S32, sizeof(float) * n);
    uint16_t *sa = (uint16_t *)ws_get(c, W_SH, 2 * sizeof(uint16_t) * n);
    {
        StageTimer tm(c, MODAL_STAGE_PREP);
        hipck(c, launch_split_bf16((int64_t)n, St, s32, sa, c->stream), "split");
    }
    {
        StageTimer tm(c, MODAL_STAGE_TRIPLE);
        hipck(c, launch_triple_bt(plan, upad, ldz, d.ldmu, s32, sa, T, c->stream), "triple mixed");
    }
    if ((int64_t)p->ta * p->tp == 0) return;
    StageTimer tm(c, MODAL_STAGE_GATHER);
    hipck(c, launch_gather_bt(p->kind, p->ta, p->tp, ta, tp, d.np, plan, T, gamma, c->stream), "gather");
}

// The late-time Gram matrix <Q_n, Q_m> over tri_a x tri_a (Appendix; the
// inner product of Sec. 2.1 with h^2 as the mu integral of Sec. 2.2): the
// same l contraction and triple products as Eq. (2D), with qbar_b(l) in place
// of beta_p(l, r), weights (2l+1) / v_l^2 (no C_l) and one radial point of
// unit weight (no r integral).  The qbar table [na][L] is the beta layout
// [np][L][nr] for np = na, nr = 1.
void run_gram(modal_ctx c, const modal_grid *g, const modal_problem *p, const Dims &d, modal_precision prec,
              double *gram)
{
    static const double one = 1.0;
    Dims dg = d;
    dg.nr = 1;
    dg.np = d.na;
    dg.U = d.na * d.na;
    const Grid G = stage_grid(c, g, d);
    const double *ql = dev_in(c, p->ql, (size_t)d.na * d.L);
    const double *r1 = dev_in(c, &one, 1), *wr1 = dev_in(c, &one, 1);
    double *P = (double *)ws_get(c, W_P, sizeof(double) * (size_t)d.L * d.ldmu);
    double *wl = (double *)ws_get(c, W_WL, sizeof(double) * d.L);
    const int64_t ldz = dg.ldmu;
    double *wz = (double *)ws_get(c, W_WZ, sizeof(double) * ldz);
    const int Upad = pad_to(dg.U, kRowPad);
    const int64_t nzb = ldz / 32, nzbp = (nzb + kZBlockPad - 1) / kZBlockPad * kZBlockPad;
    double *St = (double *)ws_get(c, W_ST, sizeof(double) * (size_t)Upad * nzbp * 32);
    zero(c, St + (size_t)nzb * Upad * 32, (nzbp - nzb) * Upad * 32);
    {
        StageTimer tm(c, MODAL_STAGE_LEGENDRE);
        hipck(c, launch_legendre_table(g->lmax, g->lmin, d.nmu, d.ldmu, G.mu, P, c->stream), "legendre");
    }
    {
        StageTimer tm(c, MODAL_STAGE_S);
        hipck(c, launch_weights_l(d.L, g->lmin, 2.0 * p->v_power, nullptr, wl, c->stream), "weights");
        hipck(c, launch_cbrt_weights(1, d.nmu, d.ldmu, r1, wr1, G.wmu, wz, c->stream), "cbrt weights");
        zero_pad_rows(c, St, ldz, Upad, dg.U);
        hipck(c, launch_s_parity(d.na, d.na, 1, d.nmu, d.ldmu, d.L, g->lmin, wl, ql, ql, P, d.ldmu, wz, Upad, St,
                                 c->stream),
              "Gram rows");
    }
    modal_problem pg = *p;
    pg.np = p->na;
    pg.tp = p->ta;
    pg.tri_p = p->tri_a;
    run_triple_gather(c, &pg, dg, prec, St, gram);
}

// Gamma' of Eq. (3D) with the exact (threej = MODAL_3J_EXACT) or Gosper
// symbol: the moment tensor T contracted one l at a time (k_modal3d.hip),
// then gathered; the three contractions per l1 run on the in-tree FP64
// matrix-core GEMM (k_dgemm.hip) with 64-wide output tiles (measured at
// lmax = 1000: 3.57 s per call against 3.80 s with 128-wide tiles in
// stages 1 and 3, whose row counts are 128 and up to U).  The r axis is taken in balanced batches
// of at most nrb points, nrb the largest count whose batch operands fit the
// batch budget (8 GiB, or a quarter of the workspace limit when one is set).
constexpr int kRowChunk3d = 128;
constexpr int kU2Block3d = 128;
constexpr size_t kBatchBudget3d = (size_t)8 << 30;

// bytes of the batch operands (G, A, packed B_r, C) per radial point
size_t batch_bytes_per_r3d(int L, int U)
{
    const size_t NT = (size_t)U * (U + 1) / 2;
    return sizeof(double) * (2 * (size_t)L * U + NT + (size_t)U);
}

void dg(modal_ctx c, hipError_t e, const char *what) { hipck(c, e, what); }

void run_gamma_3d(modal_ctx c, const modal_grid *g, const modal_problem *p, const Dims &d, int threej,
                  double *gamma)
{
    Grid G{};
    G.k = dev_in(c, g->k, d.nk);
    G.wk = dev_in(c, g->wk, d.nk);
    G.r = dev_in(c, g->r, d.nr);
    G.wr = dev_in(c, g->wr, d.nr);
    const double *delta = dev_in(c, p->delta, (size_t)d.L * d.nk);
    const double *qk = dev_in(c, p->qk, (size_t)d.np * d.nk);
    const double *cl = dev_in(c, p->cl, (size_t)d.L);
    const double *ql = dev_in(c, p->ql, (size_t)d.na * d.L);
    double *beta = (double *)ws_get(c, W_BETA, sizeof(double) * (size_t)d.np * d.L * d.nr);
    run_beta(c, g, d, G, delta, qk, beta);
    double *wl = (double *)ws_get(c, W_WL, sizeof(double) * d.L);
    hipck(c, launch_weights_l(d.L, g->lmin, p->v_power, cl, wl, c->stream), "weights");

    const int L = d.L, U = d.U;
    // parity classes of l in [lmin, lmax]: even first in the l' order
    const int lE0 = g->lmin + (g->lmin & 1), lO0 = g->lmin + 1 - (g->lmin & 1);
    const int nE = lE0 <= g->lmax ? (g->lmax - lE0) / 2 + 1 : 0;
    const int nO = lO0 <= g->lmax ? (g->lmax - lO0) / 2 + 1 : 0;
    const int l0c[2] = {lE0, lO0}, nc[2] = {nE, nO}, offc[2] = {0, nE};
    const size_t per_r = (size_t)L * U * sizeof(double);
    size_t budget = kBatchBudget3d;
    if (c->limit) budget = std::min(budget, c->limit / 4);
    const size_t nrb_max = std::max<size_t>(1, std::min<size_t>((size_t)d.nr, budget / batch_bytes_per_r3d(L, U)));
    const int nbatch = (int)((d.nr + nrb_max - 1) / nrb_max);
    const int nrb = (d.nr + nbatch - 1) / nbatch;
    double *Gb = (double *)ws_get(c, W_G3, per_r * nrb);
    double *Ab = (double *)ws_get(c, W_A3, per_r * nrb);
    double *Cb = (double *)ws_get(c, W_C3, sizeof(double) * (size_t)U * nrb);
    // the symbol blocks of both parity classes of l2 for one l1
    const size_t kblk = std::max<size_t>(1, (size_t)std::max(nE, nO) * std::max(nE, nO));
    double *Kb = (double *)ws_get(c, W_K3, sizeof(double) * 2 * kblk);
    // T over the (u2 <= u3) pairs, packed u2-major: NT = U (U + 1) / 2
    // columns, of which only the rows u1 <= u2 are formed and read
    const int NT = U * (U + 1) / 2;
    double *Pb = (double *)ws_get(c, W_P3, sizeof(double) * (size_t)NT * nrb);
    const size_t tn = (size_t)U * NT;
    double *T = (double *)ws_get(c, W_T3, sizeof(double) * tn);
    zero(c, T, (int64_t)tn);
    // start values of the symbol bands, (l1 l2 |l1 - l2|; 000)^2 by max and min
    double *V = (double *)ws_get(c, W_V3, sizeof(double) * ((size_t)g->lmax + 1) * (g->lmax + 2) / 2);
    hipck(c, launch_start3(g->lmax, V, c->stream), "Eq. (3D) band starts");
    for (int r0 = 0; r0 < d.nr; r0 += nrb) {
        const int nb = std::min(nrb, d.nr - r0);
        {
            StageTimer tm(c, MODAL_STAGE_PREP);     // one interval per r batch
            hipck(c, launch_build_g3(L, nE, lE0, lO0, g->lmin, d.nr, d.np, d.na, r0, nb, wl, ql, beta, Gb,
                                     c->stream),
                  "Eq. (3D) operand");
        }
        StageTimer tm(c, MODAL_STAGE_TRIPLE);
        for (int l1 = g->lmin; l1 <= g->lmax; ++l1) {
            const int p1 = l1 & 1;
            hipck(c, launch_build_k3(l1, l0c, nc, threej == MODAL_3J_GOSPER, V, Kb, Kb + kblk, c->stream),
                  "Eq. (3D) symbols");
            // stage 1: A_r(l2, u) = Sum_l3 K(l2, l3) G_r(l3, u), per parity
            // class of l2 (class 0 = even l, 1 = odd l; l3 has the parity of
            // l1 + l2)
            for (int par2 = 0; par2 < 2; ++par2) {
                const int par3 = (p1 + par2) & 1;
                const int n2 = nc[par2], n3 = nc[par3];
                if (n2 == 0) continue;
                if (n3 == 0) {      // no l3 of the needed parity at all
                    hipck(c, launch_zero_rows3(L, offc[par2], n2, (int64_t)nb * U, Ab, c->stream), "Eq. (3D) empty rows");
                    continue;
                }
                const double *Kp = Kb + (par2 ? kblk : 0);
                // rows in chunks, each multiplied only over the l3 columns its
                // triangles reach: |l1 - l2| <= l3 <= l1 + l2 (half the block
                // on average)
                for (int i2a = 0; i2a < n2; i2a += kRowChunk3d) {
                    const int i2b = std::min(n2, i2a + kRowChunk3d);
                    const int l2a = l0c[par2] + 2 * i2a, l2b = l0c[par2] + 2 * (i2b - 1);
                    const int lo = l1 < l2a ? l2a - l1 : (l1 > l2b ? l1 - l2b : 0);
                    const int hi = l1 + l2b;
                    const int c0 = std::max(0, (lo - l0c[par3] + 1) / 2);
                    const int c1 = hi < l0c[par3] ? -1 : std::min(n3 - 1, (hi - l0c[par3]) / 2);
                    if (c1 < c0) {      // no triangle reaches an l3 of this class
                        hipck(c, launch_zero_rows3(L, offc[par2] + i2a, i2b - i2a, (int64_t)nb * U, Ab, c->stream),
                              "Eq. (3D) empty rows");
                        continue;
                    }
                    dg(c, launch_dgemm(false, false, i2b - i2a, nb * U, c1 - c0 + 1, 1.0, Kp + (size_t)c0 * n2 + i2a,
                                       n2, 0, Gb + offc[par3] + c0, L, 0, 0.0, Ab + offc[par2] + i2a, L, 0, 1,
                                       c->stream, 64),
                       "Eq. (3D) stage 1");
                }
            }
            // stage 2: B_r = G_r^T A_r is symmetric (K is symmetric in l2,
            // l3): only its upper triangle u <= v, formed as the lower one of
            // B_r^T = A_r^T G_r and written straight into the u2-major pairs
            dg(c, launch_dgemm_packed_lower(true, false, U, L, Ab, L, (int64_t)U * L, Gb, L, (int64_t)U * L, Pb, NT,
                                            nb, c->stream),
               "Eq. (3D) stage 2");
            const int lp1 = p1 == 0 ? (l1 - lE0) / 2 : nE + (l1 - lO0) / 2;
            hipck(c, launch_c3(L, lp1, U, r0, nb, G.r, G.wr, Gb, Cb, c->stream), "Eq. (3D) radial weights");
            // stage 3: T(u1, (u2, u3)) += Sum_r C_r(u1) B_r(u2, u3), for u1
            // below the end of each u2 block: u1 <= u2 <= u3 is all the
            // gather reads
            for (int b0 = 0; b0 < U; b0 += kU2Block3d) {
                const int b1 = std::min(U, b0 + kU2Block3d);
                const int64_t t0 = (int64_t)b0 * U - (int64_t)b0 * (b0 - 1) / 2;
                const int64_t t1 = (int64_t)b1 * U - (int64_t)b1 * (b1 - 1) / 2;
                dg(c, launch_dgemm(false, true, b1, (int)(t1 - t0), nb, 1.0, Cb, U, 0, Pb + t0, NT, 0, 1.0,
                                   T + (size_t)t0 * U, U, 0, 1, c->stream, 64),
                   "Eq. (3D) stage 3");
            }
        }
    }
    const int *ta = dev_in(c, p->tri_a, (size_t)p->ta * 3);
    const int *tp = dev_in(c, p->tri_p, (size_t)p->tp * 3);
    hipck(c, launch_gather3(p->kind, p->ta, p->tp, ta, tp, d.np, U, T, gamma, c->stream), "Eq. (3D) gather");
}

// x (row-major [n][m], on the device) := gram^-1 x, gram SPD [n][n] (on the
// device, overwritten by its Cholesky factor).  Read column major, x is its
// transpose X' (m x n), and X' gram^-1 = X' L^-T L^-1 for gram = L L^T: two
// triangular solves from the right.  All in-tree: a right-looking blocked
// Cholesky (64-wide diagonal blocks factored in LDS, the panel below solved
// row by row, the trailing block updated on the FP64 GEMM), then each
// triangular solve blocked the same way (the columns of one block solved
// per row of X' against the diagonal block, the rest by GEMM updates).
void solve_gram(modal_ctx c, int n, int m, double *gram, double *x)
{
    if (n == 0 || m == 0) return;
    const int nb = chol_block();
    int *info = (int *)ws_get(c, W_INFO, sizeof(int));
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, c->stream, info, 1);
    hipck(c, hipGetLastError(), "zero fill");
    double *A = gram;
    for (int j0 = 0; j0 < n; j0 += nb) {
        const int jb = std::min(nb, n - j0), j1 = j0 + jb, rest = n - j1;
        double *D = A + (size_t)j0 * n + j0;
        hipck(c, launch_potrf_block(jb, D, n, info, c->stream), "Cholesky diagonal block");
        if (rest == 0) break;
        // panel: A21 := A21 L11^-T, one row of A21 per vector
        double *P = A + (size_t)j0 * n + j1;
        hipck(c, launch_trsm_rows(rest, jb, D, n, P, 1, n, 0, c->stream), "Cholesky panel");
        // trailing block: A22 -= A21 A21^T
        hipck(c, launch_dgemm(false, true, rest, rest, jb, -1.0, P, n, 0, P, n, 0, 1.0, A + (size_t)j1 * n + j1, n,
                              0, 1, c->stream),
              "Cholesky update");
    }
    int hinfo = 0;
    hipck(c, hipMemcpyAsync(&hinfo, info, sizeof(hinfo), hipMemcpyDeviceToHost, c->stream), "D2H");
    hipck(c, hipStreamSynchronize(c->stream), "synchronise");
    need(c, hinfo == 0, MODAL_ERR_NUMERIC, "the Gram matrix <Q, Q> is not positive definite");
    // X' := X' L^-T: block columns forward, X'_J -= X'_{<J} L_{J,<J}^T, then
    // the diagonal block
    for (int j0 = 0; j0 < n; j0 += nb) {
        const int jb = std::min(nb, n - j0);
        if (j0 > 0)
            hipck(c, launch_dgemm(false, true, m, jb, j0, -1.0, x, m, 0, A + j0, n, 0, 1.0, x + (size_t)j0 * m, m, 0,
                                  1, c->stream),
                  "triangular solve update");
        hipck(c, launch_trsm_rows(m, jb, A + (size_t)j0 * n + j0, n, x + (size_t)j0 * m, 1, m, 0, c->stream),
              "triangular solve");
    }
    // X' := X' L^-1: block columns backward, X'_J -= X'_{>J} L_{>J,J}, then
    // the diagonal block
    const int last = (n - 1) / nb * nb;
    for (int j0 = last; j0 >= 0; j0 -= nb) {
        const int jb = std::min(nb, n - j0), j1 = j0 + jb;
        if (j1 < n)
            hipck(c, launch_dgemm(false, false, m, jb, n - j1, -1.0, x + (size_t)j1 * m, m, 0, A + (size_t)j0 * n + j1,
                                  n, 0, 1.0, x + (size_t)j0 * m, m, 0, 1, c->stream),
                  "triangular solve update");
        hipck(c, launch_trsm_rows(m, jb, A + (size_t)j0 * n + j0, n, x + (size_t)j0 * m, 1, m, 1, c->stream),
              "triangular solve");
    }
}

}  // namespace

// ============================================================================
extern "C" {

modal_status modal_create(modal_ctx *out, int device, void *hip_stream)
{
    if (!out) {
        g_last_error = "out is NULL";
        return MODAL_ERR_INVALID_ARG;
    }
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n <= 0) {
        (void)hipGetLastError();
        g_last_error = "no HIP device available";
        return MODAL_ERR_DEVICE;
    }
    if (device < 0 || device >= n) {
        g_last_error = "device index out of range";
        return MODAL_ERR_DEVICE;
    }
    e = hipSetDevice(device);
    if (e != hipSuccess) {
        g_last_error = std::string("hipSetDevice: ") + hipGetErrorString(e);
        return MODAL_ERR_DEVICE;
    }
    {
        // the device address of this device's scratch array, once per device
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (device < kMaxScratchDevices && !g_scratch_ptr[device]) {
            void *p = nullptr;
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p) {
                g_last_error = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
                return MODAL_ERR_DEVICE;
            }
            g_scratch_ptr[device] = p;
        }
    }
    modal_ctx c = new (std::nothrow) modal_ctx_s;
    if (!c) {
        g_last_error = "host allocation failed";
        return MODAL_ERR_OOM;
    }
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    *out = c;
    return MODAL_OK;
}

modal_status modal_destroy(modal_ctx c)
{
    if (!c) return MODAL_OK;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (auto &b : c->ws) (void)hipFree(b.p);
    free_triple_plan(c->plan64);
    free_bt_plan(c->planbt);
    for (auto &pool : c->ev)
        for (auto &pr : pool) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
    delete c;
    return MODAL_OK;
}

modal_status modal_set_stream(modal_ctx c, void *hip_stream)
{
    if (!c) return MODAL_ERR_INVALID_ARG;
    const hipStream_t s = (hipStream_t)hip_stream;
    if (s == c->stream) return MODAL_OK;
    // work already queued on the old stream (which may still read or write
    // the workspace) is ordered before anything the new stream runs next
    c->next_in = 0;
    try {
        hipck(c, hipSetDevice(c->device), "hipSetDevice");
        hipEvent_t ev = nullptr;
        hipck(c, hipEventCreateWithFlags(&ev, hipEventDisableTiming), "event create");
        hipError_t e = hipEventRecord(ev, c->stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, ev, 0);
        (void)hipEventDestroy(ev);
        hipck(c, e, "ordering the new stream after the old one");
    } catch (const Fail &x) {
        return x.st;
    }
    c->stream = s;
    return MODAL_OK;
}

const char *modal_status_str(modal_status s)
{
    switch (s) {
    case MODAL_OK: return "ok";
    case MODAL_ERR_INVALID_ARG: return "invalid argument";
    case MODAL_ERR_SHAPE: return "shape or index out of range";
    case MODAL_ERR_OOM: return "out of device memory";
    case MODAL_ERR_DEVICE: return "device or HIP runtime error";
    case MODAL_ERR_NUMERIC: return "invalid numeric input";
    case MODAL_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char *modal_last_error(modal_ctx c)
{
    if (c) return c->err.c_str();
    return g_last_error.c_str();
}

modal_status modal_set_workspace_limit(modal_ctx c, size_t bytes)
{
    if (!c) return MODAL_ERR_INVALID_ARG;
    c->limit = bytes;
    return MODAL_OK;
}

modal_status modal_set_forward_reuse(modal_ctx c, int on)
{
    if (!c) return MODAL_ERR_INVALID_ARG;
    c->reuse_fwd = on != 0;
    return MODAL_OK;
}

modal_status modal_enable_timing(modal_ctx c, int on)
{
    if (!c) return MODAL_ERR_INVALID_ARG;
    c->timing = on != 0;
    for (int s = 0; s < MODAL_NSTAGES; ++s) c->used[s] = 0;
    return MODAL_OK;
}

modal_status modal_stage_times(modal_ctx c, double *ms, int n)
{
    if (!c || !ms || n < MODAL_NSTAGES) return MODAL_ERR_INVALID_ARG;
    // not `guarded`: that would reset the per-call event counts
    c->err.clear();
    if (hipSetDevice(c->device) != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess) {
        c->err = g_last_error = "stream synchronisation failed";
        return MODAL_ERR_DEVICE;
    }
    for (int s = 0; s < MODAL_NSTAGES; ++s) {
        ms[s] = 0.0;
        if (!c->timing) continue;
        for (int i = 0; i < c->used[s]; ++i) {
            float v = 0.f;
            if (hipEventElapsedTime(&v, c->ev[s][i].first, c->ev[s][i].second) != hipSuccess) {
                c->err = g_last_error = "hipEventElapsedTime failed";
                return MODAL_ERR_DEVICE;
            }
            ms[s] += v;
        }
    }
    return MODAL_OK;
}

modal_status modal_stage_counts(modal_ctx c, int32_t *counts, int n)
{
    if (!c || !counts || n < MODAL_NSTAGES) return MODAL_ERR_INVALID_ARG;
    for (int s = 0; s < MODAL_NSTAGES; ++s) counts[s] = c->timing ? c->used[s] : 0;
    return MODAL_OK;
}

modal_status modal_workspace_bytes(modal_ctx c, const modal_grid *g, const modal_problem *p,
                                   modal_precision prec, size_t *bytes)
{
    return guarded(c, [&] {
        c->fwd.valid = c->fwd.was_valid;          // reads no device memory
        need(c, bytes != nullptr, MODAL_ERR_INVALID_ARG, "bytes is NULL");
        check_prec(c, prec);
        Dims d = check_grid(c, g, false);
        check_problem(c, p, d, true, false, false);
        const size_t Upad = (size_t)pad_to(d.U, kRowPad);
        const size_t z = (size_t)d.nr * d.ldmu;
        const size_t nitems = (size_t)d.nk * d.nr;
        size_t cl = std::max<size_t>(1, std::min<size_t>((size_t)d.L, ((size_t)512 << 20) / (nitems * 8)));
        const size_t npairs = (size_t)d.U * (d.U + 1) / 2;
        const size_t tsize = (npairs + 15) / 16 * ((size_t)d.U / 16 + 1) * 256;   // upper bound
        size_t b = 0;
        b += 2 * d.nmu * 8 + (size_t)d.L * d.ldmu * 8 + d.L * 8 + z * 8;
        b += nitems * 40 + cl * nitems * 8 + (size_t)d.np * d.L * d.nr * 8;
        b += Upad * ((z / 32 + kZBlockPad - 1) / kZBlockPad * kZBlockPad) * 32 * 8 + tsize * 8;
        if (prec == MODAL_MIXED) b += Upad * z * 8;   // FP32 copy + BF16 split
        *bytes = b;
    });
}

modal_status modal_gauss_legendre(modal_ctx c, int32_t n, double *x, double *w)
{
    if (!c) {
        // host rule, host arrays: no context and no device needed
        if (n < 1) {
            g_last_error = "n must be >= 1";
            return MODAL_ERR_SHAPE;
        }
        if (!x || !w) {
            g_last_error = "x, w must be non-NULL";
            return MODAL_ERR_INVALID_ARG;
        }
        try {
            gauss_legendre_host(n, x, w);
        } catch (...) {
            g_last_error = "host Gauss-Legendre rule failed (thread start)";
            return MODAL_ERR_DEVICE;
        }
        return MODAL_OK;
    }
    return guarded(c, [&] {
        need(c, n >= 1, MODAL_ERR_SHAPE, "n must be >= 1");
        need(c, x && w, MODAL_ERR_INVALID_ARG, "x, w must be non-NULL");
        OutBuf ox = dev_out(c, x, n, W_MU), ow = dev_out(c, w, n, W_WMU);
        {
            StageTimer tm(c, MODAL_STAGE_GL);
            hipck(c, launch_gauss_legendre(n, ox.dev, ow.dev, c->stream), "gauss_legendre");
        }
        finish_out(c, ox);
        finish_out(c, ow);
    });
}

modal_status modal_legendre_table(modal_ctx c, int32_t lmax, int32_t nmu, const double *mu, double *P)
{
    return guarded(c, [&] {
        need(c, lmax >= 0 && lmax <= 20000 && nmu >= 1, MODAL_ERR_SHAPE, "need 0 <= lmax <= 20000, nmu >= 1");
        need(c, mu && P, MODAL_ERR_INVALID_ARG, "mu, P must be non-NULL");
        const double *dmu = dev_in(c, mu, nmu);
        OutBuf o = dev_out(c, P, (size_t)(lmax + 1) * nmu, W_P);
        {
            StageTimer tm(c, MODAL_STAGE_LEGENDRE);
            hipck(c, launch_legendre_table(lmax, 0, nmu, nmu, dmu, o.dev, c->stream), "legendre");
        }
        finish_out(c, o);
    });
}

modal_status modal_sph_bessel_table(modal_ctx c, int32_t lmax, int64_t nx, const double *x, double *J)
{
    return guarded(c, [&] {
        need(c, lmax >= 0 && lmax <= 20000 && nx >= 1, MODAL_ERR_SHAPE, "need 0 <= lmax <= 20000, nx >= 1");
        need(c, x && J, MODAL_ERR_INVALID_ARG, "x, J must be non-NULL");
        auto hx = host_copy(c, x, (size_t)nx);
        for (double v : hx)
            need(c, v >= 0.0 && v < 1e6, MODAL_ERR_NUMERIC, "x must be finite, >= 0 and < 1e6");
        const double *dx = dev_in(c, x, (size_t)nx);
        BesselState st;
        char *sb = (char *)ws_get(c, W_BSTATE, (size_t)nx * 40);
        st.f0 = (double *)sb;
        st.f1 = st.f0 + nx;
        st.c = st.f1 + nx;
        st.e = (int *)(st.c + nx);
        st.efin = st.e + nx;
        OutBuf o = dev_out(c, J, (size_t)(lmax + 1) * nx, W_JCHUNK);
        StageTimer tm(c, MODAL_STAGE_BESSEL);
        hipck(c, launch_bessel_prepare(nx, dx, nullptr, 1, nullptr, lmax, st, c->stream), "bessel prepare");
        hipck(c, launch_bessel_chunk(nx, dx, nullptr, 1, nullptr, lmax, 0, st, o.dev, nx, nullptr, 0, c->stream),
              "bessel emit");
        finish_out(c, o);
    });
}

modal_status modal_beta(modal_ctx c, const modal_grid *g, const modal_problem *p, modal_precision prec,
                        double *beta)
{
    return guarded(c, [&] {
        check_prec(c, prec);
        need(c, beta != nullptr, MODAL_ERR_INVALID_ARG, "beta is NULL");
        Dims d = check_grid(c, g, false);
        check_problem(c, p, d, true, false);
        Grid G = stage_grid(c, g, d);
        const double *delta = dev_in(c, p->delta, (size_t)d.L * d.nk);
        const double *qk = dev_in(c, p->qk, (size_t)d.np * d.nk);
        OutBuf o = dev_out(c, beta, (size_t)d.np * d.L * d.nr, W_BETA);
        run_beta(c, g, d, G, delta, qk, o.dev);
        finish_out(c, o);
    });
}

modal_status modal_S(modal_ctx c, const modal_grid *g, const modal_problem *p, modal_precision prec,
                     const double *beta, double *S)
{
    return guarded(c, [&] {
        check_prec(c, prec);
        need(c, beta && S, MODAL_ERR_INVALID_ARG, "beta, S must be non-NULL");
        Dims d = check_grid(c, g, false);
        check_problem(c, p, d, false, false);
        Grid G = stage_grid(c, g, d);
        const double *dbeta = dev_in(c, beta, (size_t)d.np * d.L * d.nr);
        const double *cl = dev_in(c, p->cl, (size_t)d.L);
        const double *ql = dev_in(c, p->ql, (size_t)d.na * d.L);
        double *P = (double *)ws_get(c, W_P, sizeof(double) * (size_t)d.L * d.nmu);
        double *wl = (double *)ws_get(c, W_WL, sizeof(double) * d.L);
        {
            StageTimer tm(c, MODAL_STAGE_LEGENDRE);
            hipck(c, launch_legendre_table(g->lmax, g->lmin, d.nmu, d.nmu, G.mu, P, c->stream), "legendre");
        }
        OutBuf o = dev_out(c, S, (size_t)d.U * d.nr * d.nmu, W_ST);
        StageTimer tm(c, MODAL_STAGE_S);
        hipck(c, launch_weights_l(d.L, g->lmin, p->v_power, cl, wl, c->stream), "weights");
        hipck(c, launch_s_parity(d.na, d.np, d.nr, d.nmu, d.nmu, d.L, g->lmin, wl, ql, dbeta, P, d.nmu, nullptr, 0,
                                 o.dev, c->stream),
              "S gemm");
        finish_out(c, o);
    });
}

modal_status modal_gamma_from_S(modal_ctx c, const modal_grid *g, const modal_problem *p,
                                modal_precision prec, const double *S, double *gamma)
{
    return guarded(c, [&] {
        check_prec(c, prec);
        Dims d = check_grid(c, g, false);
        check_problem(c, p, d, false, true);
        need(c, S != nullptr, MODAL_ERR_INVALID_ARG, "S is NULL");
        need(c, gamma != nullptr || (int64_t)p->ta * p->tp == 0, MODAL_ERR_INVALID_ARG, "gamma is NULL");
        Grid G = stage_grid(c, g, d);
        const double *dS = dev_in(c, S, (size_t)d.U * d.nr * d.nmu);
        const int Upad = pad_to(d.U, kRowPad);
        const int64_t ldz = (int64_t)d.nr * d.ldmu;
        double *wz = (double *)ws_get(c, W_WZ, sizeof(double) * ldz);
        double *St = (double *)ws_get(c, W_ST, sizeof(double) * (size_t)Upad * ldz);
        OutBuf o = dev_out(c, gamma, (size_t)p->ta * p->tp, W_GAMMA);
        {
            StageTimer tm(c, MODAL_STAGE_S);
            hipck(c, launch_cbrt_weights(d.nr, d.nmu, d.ldmu, G.r, G.wr, G.wmu, wz, c->stream), "weights");
            zero_pad_rows(c, St, ldz, Upad, d.U);
            hipck(c, launch_s_import(d.U, Upad, d.nr, d.nmu, d.ldmu, dS, wz, St, c->stream), "S import");
        }
        run_triple_gather(c, p, d, prec, St, o.dev);
        finish_out(c, o);
    });
}

modal_status modal_gamma(modal_ctx c, const modal_grid *g, const modal_problem *p, modal_precision prec,
                         double *gamma)
{
    return guarded(c, [&] {
        check_prec(c, prec);
        Dims d = check_grid(c, g, true);
        check_problem(c, p, d, true, true);
        need(c, gamma != nullptr || (int64_t)p->ta * p->tp == 0, MODAL_ERR_INVALID_ARG, "gamma is NULL");
        OutBuf o = dev_out(c, gamma, (size_t)p->ta * p->tp, W_GAMMA);
        Forward f = run_forward(c, g, p, d);
        const int fwd_in = c->next_in;
        // (d) triple products and Gamma
        run_triple_gather(c, p, d, prec, f.St, o.dev);
        finish_out(c, o);
        c->fwd = FwdCache{true, false, *g, *p, f, fwd_in};
    });
}

modal_status modal_gamma_noalloc(modal_ctx c, const modal_grid *g, const modal_problem *p, modal_precision prec,
                                 double *gamma)
{
    return guarded(c, [&] {
        void *base = nullptr;
        {
            std::lock_guard<std::mutex> lk(g_scratch_mu);
            if (c->device < kMaxScratchDevices) base = g_scratch_ptr[c->device];
        }
        need(c, base != nullptr, MODAL_ERR_DEVICE, "no no-allocation scratch on this device");
        // arena mode for this call only (also on an error exit)
        struct Scope {
            modal_ctx c;
            ~Scope() { c->arena_on = false; }
        } scope{c};
        c->arena = DevArena{(char *)base, kScratchBytes, 0};
        for (int i = 0; i < NSLOTS; ++i) {
            c->aslot_p[i] = nullptr;
            c->aslot_n[i] = 0;
        }
        c->arena_on = true;
        check_prec(c, prec);
        Dims d = check_grid(c, g, true);
        check_problem(c, p, d, true, true);
        need(c, gamma != nullptr || (int64_t)p->ta * p->tp == 0, MODAL_ERR_INVALID_ARG, "gamma is NULL");
        OutBuf o = dev_out(c, gamma, (size_t)p->ta * p->tp, W_GAMMA);
        Forward f = run_forward(c, g, p, d);
        run_triple_gather(c, p, d, prec, f.St, o.dev);
        // the forward tables live in the shared scratch: never kept for reuse
    });
}

modal_status modal_gram(modal_ctx c, const modal_grid *g, const modal_problem *p, modal_precision prec,
                        double *gram)
{
    return guarded(c, [&] {
        check_prec(c, prec);
        Dims d = check_grid(c, g, true);
        modal_problem pc = *p;                // the Gram matrix reads tri_a only
        pc.tp = 0;
        pc.tri_p = nullptr;
        check_problem(c, &pc, d, false, true);
        need(c, (int64_t)p->na * p->na <= 8192, MODAL_ERR_SHAPE, "na * na above 8192");
        need(c, gram != nullptr || p->ta == 0, MODAL_ERR_INVALID_ARG, "gram is NULL");
        OutBuf o = dev_out(c, gram, (size_t)p->ta * p->ta, W_GRAM);
        run_gram(c, g, &pc, d, prec, o.dev);
        finish_out(c, o);
    });
}

modal_status modal_gamma_modal(modal_ctx c, const modal_grid *g, const modal_problem *p, modal_precision prec,
                               double *gamma)
{
    return guarded(c, [&] {
        check_prec(c, prec);
        Dims d = check_grid(c, g, true);
        check_problem(c, p, d, true, true);
        need(c, (int64_t)p->na * p->na <= 8192, MODAL_ERR_SHAPE, "na * na above 8192");
        need(c, gamma != nullptr || (int64_t)p->ta * p->tp == 0, MODAL_ERR_INVALID_ARG, "gamma is NULL");
        OutBuf o = dev_out(c, gamma, (size_t)p->ta * p->tp, W_GAMMA);
        // Gamma' = <Q, Q~> in the requested precision
        Forward f = run_forward(c, g, p, d);
        run_triple_gather(c, p, d, prec, f.St, o.dev);
        // <Q, Q> in FP64 (its cost is that of one radial point), then the solve
        double *gm = (double *)ws_get(c, W_GRAM, sizeof(double) * (size_t)p->ta * p->ta);
        run_gram(c, g, p, d, MODAL_FP64, gm);
        solve_gram(c, p->ta, p->tp, gm, o.dev);
        finish_out(c, o);
    });
}

modal_status modal_gamma_backward(modal_ctx c, const modal_grid *g, const modal_problem *p,
                                  modal_precision prec, const double *dgamma, double *dqk, double *ddelta)
{
    return guarded(c, [&] {
        check_prec(c, prec);
        Dims d = check_grid(c, g, true);
        check_problem(c, p, d, true, true);
        const int64_t ng = (int64_t)p->ta * p->tp;
        need(c, dgamma != nullptr || ng == 0, MODAL_ERR_INVALID_ARG, "dgamma is NULL");
        need(c, dqk != nullptr || ddelta != nullptr, MODAL_ERR_INVALID_ARG, "dqk and ddelta are both NULL");
        // inverse maps of the mode lists (ordered: the triple; symmetric: its sorted form)
        std::vector<int> inva((size_t)d.na * d.na * d.na, -1), invp((size_t)d.np * d.np * d.np, -1);
        auto fill = [&](const int32_t *tri, int n, int base, std::vector<int> &inv, const char *which) {
            auto h = host_copy(c, tri, (size_t)n * 3);
            for (int i = 0; i < n; ++i) {
                int t0 = h[3 * i], t1 = h[3 * i + 1], t2 = h[3 * i + 2];
                if (p->kind == MODAL_GAMMA_SYMMETRIC) {
                    int lo = std::min(t0, std::min(t1, t2)), hi = std::max(t0, std::max(t1, t2));
                    t1 = t0 + t1 + t2 - lo - hi;
                    t0 = lo;
                    t2 = hi;
                }
                int &slot = inv[((size_t)t0 * base + t1) * base + t2];
                if (slot >= 0)
                    fail(c, MODAL_ERR_SHAPE, std::string("the adjoint needs distinct triples in ") + which);
                slot = i;
            }
        };
        fill(p->tri_a, p->ta, d.na, inva, "tri_a");
        fill(p->tri_p, p->tp, d.np, invp, "tri_p");

        // the forward tables: those of the previous call when the caller has
        // enabled reuse and that call was a forward on the same grid and
        // problem (its staged host inputs are kept: staging continues after
        // them), else recomputed
        const bool reuse = c->reuse_fwd && c->fwd.was_valid && same_inputs(c->fwd.g, *g) &&
                           same_inputs(c->fwd.p, *p);
        if (reuse) c->next_in = c->fwd.next_in;
        const double *dG = dev_in(c, dgamma, (size_t)ng);
        OutBuf oq = dev_out(c, dqk, dqk ? (size_t)d.np * d.nk : 0, W_DQ);
        OutBuf od = dev_out(c, ddelta, ddelta ? (size_t)d.L * d.nk : 0, W_DD);
        const Forward f = reuse ? c->fwd.f : run_forward(c, g, p, d);
        const int fwd_in = reuse ? c->fwd.next_in : c->next_in;
        const int64_t ldz = (int64_t)d.nr * d.ldmu;
        const int64_t upad = pad_to(d.U, kRowPad);

        // (d) adjoint: dL/dSt (z-blocked like St) from dL/dT
        int *dinva = (int *)ws_get(c, W_INVA, sizeof(int) * inva.size());
        int *dinvp = (int *)ws_get(c, W_INVP, sizeof(int) * invp.size());
        hipck(c, hipMemcpyAsync(dinva, inva.data(), sizeof(int) * inva.size(), hipMemcpyHostToDevice, c->stream),
              "H2D");
        hipck(c, hipMemcpyAsync(dinvp, invp.data(), sizeof(int) * invp.size(), hipMemcpyHostToDevice, c->stream),
              "H2D");
        // z blocks of the output: whole z tiles of the kernel (St is zero past ldz)
        const int64_t nzb = ldz / 32, nzbp = (nzb + kZBlockPad - 1) / kZBlockPad * kZBlockPad;
        double *Shat = (double *)ws_get(c, W_SHAT, sizeof(double) * (size_t)nzbp * upad * 32);
        if (prec == MODAL_MIXED) {
            const int nib = (int)(upad / adj_fac_rowblock()), nws = (d.U + 31) / 32;
            uint4 *Hc = (uint4 *)ws_get(c, W_H, sizeof(uint4) * (size_t)v_step_offset(d.U, nws) * nib * 2048);
            uint4 *sb = (uint4 *)ws_get(c, W_S32, sizeof(uint4) * (size_t)nzbp * nws * 256);
            {
                StageTimer tm(c, MODAL_STAGE_ADJ_PREP);
                hipck(c, launch_build_hc_fac(p->kind, d.U, d.np, d.na, dinva, dinvp, dG, p->tp, nib, Hc, c->stream),
                      "build Hc");
                hipck(c, launch_split_b(nzbp, d.U, upad, f.St, sb, c->stream), "split S");
            }
            StageTimer tm(c, MODAL_STAGE_ADJ_TRIPLE);
            hipck(c, launch_adj_fac(d.U, upad, nzbp, f.St, sb, Hc, Shat, c->stream), "dL/dS");
        } else {
            const int nib = (int)(upad / adj_fac64_rowblock()), nws = (d.U + 15) / 16;
            double *Hc = (double *)ws_get(c, W_H, sizeof(double) * (size_t)v_step_offset16(d.U, nws) * nib * 2048);
            {
                StageTimer tm(c, MODAL_STAGE_ADJ_PREP);
                hipck(c, launch_build_hc_fac64(p->kind, d.U, d.np, d.na, dinva, dinvp, dG, p->tp, nib, Hc,
                                               c->stream),
                      "build Hc");
            }
            StageTimer tm(c, MODAL_STAGE_ADJ_TRIPLE);
            hipck(c, launch_adj_fac64(d.U, upad, nzbp, f.St, Hc, Shat, c->stream), "dL/dS");
        }
        // (c) adjoint
        double *bhat = (double *)ws_get(c, W_BHAT, sizeof(double) * (size_t)d.np * d.L * d.nr);
        {
            StageTimer tm(c, MODAL_STAGE_ADJ_S);
            hipck(c, launch_betahat(d.na, d.np, d.nr, d.nmu, d.ldmu, d.L, g->lmin, upad, f.wl, f.ql, f.P, Shat,
                                    f.wz, bhat, c->stream),
                  "dL/dbeta");
        }
        // (b) adjoint: j_l regenerated in l chunks
        {
            StageTimer tm(c, MODAL_STAGE_ADJ_BETA);
            const int64_t nitems = (int64_t)d.nk * d.nr;
            BesselState st;
            char *sb = (char *)ws_get(c, W_BSTATE, (size_t)nitems * 40);
            st.f0 = (double *)sb;
            st.f1 = st.f0 + nitems;
            st.c = st.f1 + nitems;
            st.e = (int *)(st.c + nitems);
            st.efin = st.e + nitems;
            const size_t per_l = (size_t)nitems * sizeof(double);
            // l chunks of at most 512 MB of j_l values and 4096 l (grid limits)
            int cl = (int)std::max<size_t>(1, std::min<size_t>({(size_t)d.L, ((size_t)512 << 20) / per_l,
                                                                (size_t)4096}));
            double *jd = (double *)ws_get(c, W_JCHUNK, per_l * cl);
            double *ah = (double *)ws_get(c, W_AHAT, sizeof(double) * (size_t)cl * d.np * d.nk);
            hipck(c, launch_bessel_prepare(nitems, nullptr, f.G.k, d.nk, f.G.r, g->lmax, st, c->stream),
                  "bessel prepare");
            bool first = true;
            for (int lhi = g->lmax; lhi >= g->lmin; lhi -= cl) {
                const int llo = std::max(g->lmin, lhi - cl + 1), nl = lhi - llo + 1;
                hipck(c, launch_bessel_chunk(nitems, nullptr, f.G.k, d.nk, f.G.r, lhi, llo, st, jd, nitems,
                                             nullptr, llo, c->stream),
                      "bessel chunk");
                hipck(c, launch_ahat(nl, llo, g->lmin, d.L, d.np, d.nk, d.nr, bhat, jd, ah, c->stream), "Ahat");
                hipck(c, launch_dq_ddelta(nl, llo, g->lmin, d.np, d.nk, f.G.k, f.G.wk, f.qk, f.delta, ah,
                                          oq.dev, od.dev, first ? 1 : 0, c->stream),
                      "dq, ddelta");
                first = false;
            }
        }
        finish_out(c, oq);
        finish_out(c, od);
        c->fwd = FwdCache{true, false, *g, *p, f, fwd_in};
    });
}

modal_status modal_gamma_3d(modal_ctx c, const modal_grid *g, const modal_problem *p, int32_t threej,
                            double *gamma)
{
    return guarded(c, [&] {
        need(c, threej == MODAL_3J_EXACT || threej == MODAL_3J_GOSPER, MODAL_ERR_INVALID_ARG,
             "threej must be MODAL_3J_EXACT or MODAL_3J_GOSPER");
        need(c, gamma != nullptr, MODAL_ERR_INVALID_ARG, "gamma must be non-NULL");
        Dims d = check_grid(c, g, false);
        check_problem(c, p, d, true, true);
        need(c, d.U <= 1280, MODAL_ERR_SHAPE, "np * na above 1280: the moment tensor (about 4 (np na)^3 bytes) is too large");
        OutBuf o = dev_out(c, gamma, (size_t)p->ta * p->tp, W_GAMMA);
        run_gamma_3d(c, g, p, d, threej, o.dev);
        finish_out(c, o);
    });
}

modal_status modal_r_weights(int32_t rule, int32_t n, const double *r, double *w)
{
    if (!r || !w) {
        g_last_error = "r, w must be non-NULL";
        return MODAL_ERR_INVALID_ARG;
    }
    if (rule != MODAL_R_TRAPEZOID && rule != MODAL_R_HERMITE) {
        g_last_error = "unknown r rule";
        return MODAL_ERR_INVALID_ARG;
    }
    if (n < 2) {
        g_last_error = "a rule needs n >= 2 nodes";
        return MODAL_ERR_SHAPE;
    }
    for (int32_t j = 0; j < n; ++j) {
        if (!std::isfinite(r[j])) {
            g_last_error = "r must be finite";
            return MODAL_ERR_NUMERIC;
        }
        if (j > 0 && !(r[j] > r[j - 1])) {
            g_last_error = "r must be strictly ascending";
            return MODAL_ERR_SHAPE;
        }
    }
    for (int32_t j = 0; j < n; ++j) w[j] = 0.0;
    for (int32_t k = 0; k + 1 < n; ++k) {      // the trapezium part of every interval
        const double h = r[k + 1] - r[k];
        w[k] += 0.5 * h;
        w[k + 1] += 0.5 * h;
    }
    if (rule == MODAL_R_HERMITE) {
        // interval k adds h_k^2 / 12 (d_k - d_{k+1}), d_k = (y_{k+1} - y_k) / h_k
        // the chord slope taken as y'(r_k) (the integrals of the two derivative
        // basis cubics over [0, 1] are +1/12 and -1/12); d_{n-1} = d_{n-2}, so
        // the last interval adds nothing
        for (int32_t k = 0; k + 2 < n; ++k) {
            const double h = r[k + 1] - r[k], h1 = r[k + 2] - r[k + 1];
            const double c = h * h / 12.0;
            w[k] -= c / h;
            w[k + 1] += c / h + c / h1;
            w[k + 2] -= c / h1;
        }
    }
    return MODAL_OK;
}

}  // extern "C"
