// Step a: Gauss-Legendre rule, Legendre table P_l(mu) and spherical Bessel
// functions j_l(x), all FP64.
//
// Gauss-Legendre (Sec. 2.2: the mu integrand P_l1 P_l2 P_l3 is a polynomial,
// so an exact rule reproduces the geometric factor, and the rule itself must
// be accurate).  Each thread refines one non-negative root with Newton's
// method on P_n in double-double arithmetic, starting from Tricomi's
// asymptotic estimate; the weight is 2 / ((1 - x^2) P_n'(x)^2).
//
// Legendre (Eq. (legendre)'s P_l(mu)): Bonnet's three-term recurrence run
// upward in l, one thread per node, writes coalesced along mu.
//
// Spherical Bessel (the j_l(kr) of the projected modes, Appendix): Miller's
// method.  From a start index l_s(x) well above both x and the requested
// l range, the recurrence f_{l-1} = (2l+1)/x f_l - f_{l+1} is run downward
// from (f_{l_s+1}, f_{l_s}) = (0, 1); that direction is stable for the
// minimal solution j_l.  The result is normalised once at the bottom by
// least squares against the closed forms of j_0 and j_1.  Values are kept
// in range by exact power-of-two rescaling (2^-600 whenever |f| > 2^600),
// with the count of rescalings carried so that the emitted
// j_l = f_l c 2^(600 (e_l - e_final)) is exact in the exponent.  Two
// passes: `prepare` runs the whole recurrence to get c and e_final (and
// the state at the first l to emit); `chunk` re-runs the same arithmetic
// over an l range and emits values.  Nothing of size L x Nk x Nr is ever
// stored; chunks are consumed by the k contraction as they are made.
#include "internal.hpp"

#include <algorithm>
#include <cmath>
#include <thread>
#include <vector>

namespace mp {
namespace {

// Double-double arithmetic (value = hi + lo, |lo| <= ulp(hi)/2) for the
// Gauss-Legendre refinement: the nodes near +-1 sit within ~1e-6 of the ends
// at n ~ 6000, where 1 - x^2 in the weight loses ~10 digits if x carries only
// one FP64 rounding.  Carrying the Newton iteration in double-double gives
// nodes and weights correctly rounded to FP64.  The error-free
// transformations below must not be contracted into fused operations, so
// contraction is off from here to the end of the Gauss-Legendre kernel.
#pragma clang fp contract(off)
struct dd {
    double hi, lo;
};
__host__ __device__ __forceinline__ dd two_sum(double a, double b)
{
    const double s = a + b, bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}
__host__ __device__ __forceinline__ dd quick_two_sum(double a, double b)
{
    const double s = a + b;
    return {s, b - (s - a)};
}
__host__ __device__ __forceinline__ dd two_prod(double a, double b)
{
    const double p = a * b;
    return {p, fma(a, b, -p)};
}
__host__ __device__ __forceinline__ dd dd_add(dd x, dd y)
{
    dd s = two_sum(x.hi, y.hi), t = two_sum(x.lo, y.lo);
    s.lo += t.hi;
    s = quick_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return quick_two_sum(s.hi, s.lo);
}
__host__ __device__ __forceinline__ dd dd_neg(dd x) { return {-x.hi, -x.lo}; }
__host__ __device__ __forceinline__ dd dd_mul(dd x, dd y)
{
    dd p = two_prod(x.hi, y.hi);
    p.lo += x.hi * y.lo + x.lo * y.hi;
    return quick_two_sum(p.hi, p.lo);
}
__host__ __device__ __forceinline__ dd dd_mul_d(dd x, double d)
{
    dd p = two_prod(x.hi, d);
    p.lo += x.lo * d;
    return quick_two_sum(p.hi, p.lo);
}
__host__ __device__ __forceinline__ dd dd_div(dd x, dd y)
{
    const double q1 = x.hi / y.hi;
    dd r = dd_add(x, dd_neg(dd_mul_d(y, q1)));
    const double q2 = r.hi / y.hi;
    r = dd_add(r, dd_neg(dd_mul_d(y, q2)));
    const double q3 = r.hi / y.hi;
    dd q = quick_two_sum(q1, q2);
    return dd_add(q, dd{q3, 0.0});
}

// P_n(z) and P_{n-1}(z) by the three-term recurrence, in double-double.
__host__ __device__ void legendre_pair_dd(int n, dd z, dd &pn, dd &pn1)
{
    dd p0{1.0, 0.0}, p1 = z;
    for (int l = 1; l < n; ++l) {
        const dd a = dd_mul_d(dd_mul(z, p1), 2.0 * l + 1.0);
        const dd b = dd_mul_d(p0, (double)l);
        dd p2 = dd_div(dd_add(a, dd_neg(b)), dd{(double)(l + 1), 0.0});
        p0 = p1;
        p1 = p2;
    }
    if (n == 0) {
        pn = {1.0, 0.0};
        pn1 = {0.0, 0.0};
    } else {
        pn = p1;
        pn1 = p0;
    }
}

// The i-th largest root of P_n (i < (n + 1) / 2) and its weight; the same
// code runs in the device kernel and in the host rule (modal_gauss_legendre
// without a context).
__host__ __device__ void gl_root(int n, int i, double &xr, double &wr)
{
    const double dn = (double)n;
    const double th = kPi * (4.0 * i + 3.0) / (4.0 * dn + 2.0);
    dd z{(1.0 - 1.0 / (8.0 * dn * dn) + 1.0 / (8.0 * dn * dn * dn)) * cos(th), 0.0};
    const bool centre = (n % 2 == 1 && i == (n + 1) / 2 - 1);
    if (centre) z = {0.0, 0.0};
    // FP64 Newton to ~1e-13 relative, then two double-double steps (quadratic
    // convergence: ~1e-26, then far below FP64 resolution).  The FP64 steps
    // stop at 1e-13: near a root the FP64 value of P_n carries ~n ulp of
    // rounding noise, so asking for more only repeats steps of noise.
    double zf = z.hi, dzprev = 1.0;
    for (int it = 0; it < 16 && !centre; ++it) {
        double p0 = 1.0, p1 = zf;
        for (int l = 1; l < n; ++l) {
            const double p2 = ((2.0 * l + 1.0) * zf * p1 - (double)l * p0) / (double)(l + 1);
            p0 = p1;
            p1 = p2;
        }
        const double dpf = dn * (zf * p1 - p0) / ((zf - 1.0) * (zf + 1.0));
        const double dz = p1 / dpf;
        zf -= dz;
        if (fabs(dz) <= 1e-13 * fabs(zf) + 1e-300 || fabs(dz) >= dzprev) break;
        dzprev = fabs(dz);
    }
    z = {zf, 0.0};
    dd pn, pn1, dp{1.0, 0.0};
    const dd one{1.0, 0.0};
    for (int it = 0; it < 2 && !centre; ++it) {
        legendre_pair_dd(n, z, pn, pn1);
        // P_n'(z) = n (z P_n - P_{n-1}) / (z^2 - 1)
        const dd num = dd_mul_d(dd_add(dd_mul(z, pn), dd_neg(pn1)), dn);
        const dd den = dd_mul(dd_add(z, dd_neg(one)), dd_add(z, one));
        dp = dd_div(num, den);
        const dd dz = dd_div(pn, dp);
        z = dd_add(z, dd_neg(dz));
    }
    legendre_pair_dd(n, z, pn, pn1);
    {
        const dd num = dd_mul_d(dd_add(dd_mul(z, pn), dd_neg(pn1)), dn);
        const dd den = dd_mul(dd_add(z, dd_neg(one)), dd_add(z, one));
        dp = dd_div(num, den);
    }
    // w = 2 / ((1 - z^2) P_n'(z)^2)
    const dd omz2 = dd_mul(dd_add(one, dd_neg(z)), dd_add(one, z));
    const dd wv = dd_div(dd{2.0, 0.0}, dd_mul(omz2, dd_mul(dp, dp)));
    xr = z.hi + z.lo;
    wr = wv.hi + wv.lo;
}

__global__ void k_gauss_legendre(int n, double *__restrict__ x, double *__restrict__ w)
{
    const int half = (n + 1) / 2;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;   // i-th largest root
    if (i >= half) return;
    double zr, wi;
    gl_root(n, i, zr, wi);
    x[n - 1 - i] = zr;
    w[n - 1 - i] = wi;
    x[i] = -zr;
    w[i] = wi;
}
#pragma clang fp contract(fast)

__global__ void k_legendre_table(int lmax, int lout0, int nmu, int ld, const double *__restrict__ mu,
                                 double *__restrict__ P)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= ld) return;
    if (j >= nmu) {                                      // padding columns
        for (int l = lout0; l <= lmax; ++l) P[(size_t)(l - lout0) * ld + j] = 0.0;
        return;
    }
    const double x = mu[j];
    double pm = 1.0, pc = x;                             // P_0, P_1
    if (lout0 == 0) P[j] = 1.0;
    if (lmax >= 1 && lout0 <= 1) P[(size_t)(1 - lout0) * ld + j] = x;
    for (int l = 1; l < lmax; ++l) {
        const double pn = ((2.0 * l + 1.0) * x * pc - (double)l * pm) / (double)(l + 1);
        pm = pc;
        pc = pn;
        if (l + 1 >= lout0) P[(size_t)(l + 1 - lout0) * ld + j] = pn;
    }
}

// ---- spherical Bessel ---------------------------------------------------
constexpr double kBig = 0x1p600;
constexpr double kBigInv = 0x1p-600;
constexpr double kTinyX = 1e-20;   // below this: j_0 = 1, j_l = 0 (l >= 1)

__device__ __forceinline__ int bessel_start(double x)
{
    // above x + 24 x^(1/3) + 40 the function has fallen below ~1e-30 of its peak
    return (int)ceil(x + 24.0 * cbrt(x) + 40.0);
}

__device__ __forceinline__ void bessel_step(int l, double x, double &fl, double &fl1, int &e)
{
    // (fl, fl1) = (f_l, f_{l+1}) -> (f_{l-1}, f_l)
    const double fm = (2.0 * l + 1.0) / x * fl - fl1;
    fl1 = fl;
    fl = fm;
    if (fabs(fm) > kBig) {
        fl *= kBigInv;
        fl1 *= kBigInv;
        ++e;
    }
}

__device__ __forceinline__ double item_x(int64_t i, const double *xs, const double *k, int nk,
                                         const double *r)
{
    if (xs) return xs[i];
    return k[i % nk] * r[i / nk];
}

__global__ void k_bessel_prepare(int64_t nitems, const double *__restrict__ xs,
                                 const double *__restrict__ k, int nk, const double *__restrict__ r,
                                 int lfirst, BesselState st)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nitems) return;
    const double x = item_x(i, xs, k, nk, r);
    if (!(x >= kTinyX)) {                 // x == 0 (or below the cut): j_0 = 1 only
        st.f0[i] = 0.0;
        st.f1[i] = 0.0;
        st.e[i] = 0;
        st.c[i] = 0.0;
        st.efin[i] = 0;
        return;
    }
    const int ls = bessel_start(x);
    double fl = 1.0, fl1 = 0.0;
    int e = 0;
    if (ls <= lfirst) {                   // the emit pass seeds the recurrence itself
        st.f0[i] = 0.0;
        st.f1[i] = 0.0;
        st.e[i] = 0;
    }
    for (int l = ls; l >= 1; --l) {
        if (l == lfirst) {
            st.f0[i] = fl;
            st.f1[i] = fl1;
            st.e[i] = e;
        }
        bessel_step(l, x, fl, fl1, e);
    }
    if (lfirst == 0 && ls > 0) {
        st.f0[i] = fl;
        st.f1[i] = fl1;
        st.e[i] = e;
    }
    // fl = f_0, fl1 = f_1: least-squares scale against the closed forms
    double j0, j1;
    if (x < 1e-3) {
        const double x2 = x * x;
        j0 = 1.0 - x2 / 6.0 * (1.0 - x2 / 20.0);
        j1 = x / 3.0 * (1.0 - x2 / 10.0 * (1.0 - x2 / 28.0));
    } else {
        double sx, cx;
        sincos(x, &sx, &cx);
        j0 = sx / x;
        j1 = (sx / x - cx) / x;
    }
    const double t = fmax(fabs(fl), fabs(fl1));
    const double a = fl / t, b = fl1 / t;
    st.c[i] = (a * j0 + b * j1) / (a * a + b * b) / t;
    st.efin[i] = e;
}

__global__ void k_bessel_chunk(int64_t nitems, const double *__restrict__ xs,
                               const double *__restrict__ k, int nk, const double *__restrict__ r,
                               int lhi, int llo, BesselState st, double *__restrict__ out,
                               int64_t ld_l, const double *__restrict__ rowscale, int lrow0)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nitems) return;
    const double x = item_x(i, xs, k, nk, r);
    const int ik = (int)(i % nk);
    if (!(x >= kTinyX)) {
        for (int l = lhi; l >= llo; --l) {
            double v = (l == 0) ? 1.0 : 0.0;
            if (rowscale) v *= rowscale[(size_t)(l - lrow0) * nk + ik];
            out[(size_t)(l - llo) * ld_l + i] = v;
        }
        return;
    }
    const int ls = bessel_start(x);
    double fl = st.f0[i], fl1 = st.f1[i];
    int e = st.e[i];
    const double c = st.c[i];
    const int efin = st.efin[i];
    for (int l = lhi; l >= llo; --l) {
        if (l == ls) {
            fl = 1.0;
            fl1 = 0.0;
            e = 0;
        }
        double v = 0.0;
        if (l <= ls) {
            const int de = e - efin;                       // <= 0
            v = (de < -3) ? 0.0 : ldexp(fl * c, 600 * de);
            if (fabs(v) < 1e-300) v = 0.0;
        }
        if (rowscale) v *= rowscale[(size_t)(l - lrow0) * nk + ik];
        out[(size_t)(l - llo) * ld_l + i] = v;
        if (l <= ls && l >= 1) bessel_step(l, x, fl, fl1, e);
    }
    st.f0[i] = fl;
    st.f1[i] = fl1;
    st.e[i] = e;
}

}  // namespace

void gauss_legendre_host(int n, double *x, double *w)
{
    const int half = (n + 1) / 2;
    const int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (int t = 0; t < nth; ++t)
        pool.emplace_back([=] {
            for (int i = t; i < half; i += nth) {
                double zr, wi;
                gl_root(n, i, zr, wi);
                x[n - 1 - i] = zr;
                w[n - 1 - i] = wi;
                x[i] = -zr;
                w[i] = wi;
            }
        });
    for (auto &th : pool) th.join();
}

hipError_t launch_gauss_legendre(int n, double *x, double *w, hipStream_t s)
{
    const int half = (n + 1) / 2;
    hipLaunchKernelGGL(k_gauss_legendre, dim3((half + 63) / 64), dim3(64), 0, s, n, x, w);
    return hipGetLastError();
}

hipError_t launch_legendre_table(int lmax, int lout0, int nmu, int ld, const double *mu, double *P,
                                 hipStream_t s)
{
    hipLaunchKernelGGL(k_legendre_table, dim3((ld + 127) / 128), dim3(128), 0, s, lmax, lout0, nmu,
                       ld, mu, P);
    return hipGetLastError();
}

hipError_t launch_bessel_prepare(int64_t nitems, const double *xs, const double *k, int nk,
                                 const double *r, int lfirst, BesselState st, hipStream_t s)
{
    const int64_t nb = (nitems + 127) / 128;
    hipLaunchKernelGGL(k_bessel_prepare, dim3((unsigned)nb), dim3(128), 0, s, nitems, xs, k, nk, r,
                       lfirst, st);
    return hipGetLastError();
}

hipError_t launch_bessel_chunk(int64_t nitems, const double *xs, const double *k, int nk,
                               const double *r, int lhi, int llo, BesselState st, double *out,
                               int64_t ld_l, const double *rowscale, int lrow0, hipStream_t s)
{
    const int64_t nb = (nitems + 127) / 128;
    hipLaunchKernelGGL(k_bessel_chunk, dim3((unsigned)nb), dim3(128), 0, s, nitems, xs, k, nk, r,
                       lhi, llo, st, out, ld_l, rowscale, lrow0);
    return hipGetLastError();
}

}  // namespace mp
