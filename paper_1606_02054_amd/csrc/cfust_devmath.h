// cfust_devmath.h -- device special functions for the univariate Student t law
// with real degrees of freedom, in the variables the lattice integrand uses.
//
// For u real and dof nu, write s = u / sqrt(nu + u^2) in (-1,1) and
// tau = 1 - |s| in (0,1].  The smaller of T_nu(u) and 1 - T_nu(u) is
//     T_lower(tau) = 1/2 I_z(nu/2, 1/2),   z = 1 - s^2 = tau (2 - tau),
// with I the regularised incomplete beta function.  Working in tau keeps
// both tails to full relative accuracy.
//
// FP64 routines (used by the FP64 mode and to build the FP32 tables):
//   - I_z(a, b) by the continued fraction of DLMF 8.17.22 evaluated with the
//     modified Lentz method, switching to I_z(a,b) = 1 - I_{1-z}(b,a) where
//     the fraction converges slowly;
//   - the quantile by Newton's method on ln T_lower as a function of ln tau
//     (nearly linear in ln tau in the far tail), kept inside a bracket;
//   - digamma by upward recurrence and its asymptotic Bernoulli series
//     (DLMF 5.11.2); lgamma is the device math library's.
// FP32 routines evaluate per-dof piecewise Chebyshev tables of
//   F(tau) = log2 T_lower(tau) - (nu/2) log2 tau     (smooth on [0,1]) and
//   G(lam) = log2 tau(p),  lam = -log2(2p)            (smooth on [0, inf)),
// built on the device from the FP64 routines.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "cfust_common.h"

namespace cfust {

constexpr double LN2 = 0.69314718055994530942;
constexpr double LNSQRTPI = 0.57236494292470008707;  // ln sqrt(pi) = lgamma(1/2)

// ---------------------------------------------------------------- FP64 ------

__device__ inline double dm_digamma(double x) {
    // psi(x) = psi(x + 1) - 1/x; psi(x) ~ ln x - 1/(2x) - sum_k B_2k/(2k x^2k)
    if (!(x > 0.0) || !isfinite(x)) return NAN;   // only positive arguments occur
    double shift = 0.0;
    while (x < 9.0) { shift += 1.0 / x; x += 1.0; }
    const double r = 1.0 / (x * x);
    // B_2k / (2k) for k = 7..1, highest power first
    const double c[7] = {7.0 / 6.0 / 14.0, -691.0 / 2730.0 / 12.0, 5.0 / 66.0 / 10.0,
                         -1.0 / 30.0 / 8.0, 1.0 / 42.0 / 6.0, -1.0 / 30.0 / 4.0, 1.0 / 6.0 / 2.0};
    double sr = c[0];
    for (int k = 1; k < 7; ++k) sr = sr * r + c[k];
    return log(x) - 0.5 / x - sr * r - shift;
}

// ln B(a, 1/2)
__device__ inline double dm_lbeta_half(double a) {
    return lgamma(a) + LNSQRTPI - lgamma(a + 0.5);
}

// Continued fraction K = 1 + d1/(1 + d2/(1 + ...)) of I_x(a,b), DLMF 8.17.22:
// d_{2k+1} = -(a+k)(a+b+k)x/((a+2k)(a+2k+1)), d_{2k} = k(b-k)x/((a+2k-1)(a+2k)).
__device__ inline double dm_beta_cf(double a, double b, double x) {
    const double tiny = 1e-300;
    double f = 1.0, Cc = 1.0, Dd = 0.0;
    for (int j = 1; j < 2000; ++j) {
        const int k = j >> 1;
        const double d = (j & 1) ? -(a + k) * (a + b + k) * x / ((a + 2 * k) * (a + 2 * k + 1))
                                 : k * (b - k) * x / ((a + 2 * k - 1) * (a + 2 * k));
        Dd = 1.0 + d * Dd;
        Dd = fabs(Dd) < tiny ? tiny : Dd;
        Dd = 1.0 / Dd;
        Cc = 1.0 + d / Cc;
        Cc = fabs(Cc) < tiny ? tiny : Cc;
        const double del = Cc * Dd;
        f *= del;
        if (fabs(del - 1.0) < 2e-16) break;
    }
    return f;
}

// ln T_lower given z = tau(2-tau) and zc = (1-tau)^2 = s^2; a = nu/2, lb = ln B(a,1/2).
__device__ inline double dm_lnT_lower(double z, double zc, double a, double lb) {
    if (!(z > 0.0)) return -INFINITY;
    if (!(zc > 0.0)) return -LN2;
    const double lz = log(z), lzc = log(zc);
    if (z < (a + 1.0) / (a + 2.5)) {
        return a * lz + 0.5 * lzc - log(a) - lb - log(dm_beta_cf(a, 0.5, z)) - LN2;
    }
    const double v = exp(0.5 * lzc + a * lz + LN2 - lb) / dm_beta_cf(0.5, a, zc);
    return log1p(-v) - LN2;
}

// H = ln T_lower - a ln z, formed without the cancellation of the two large
// terms where z is small (the values the FP64 tables are fitted to).
__device__ inline double dm_H_lower(double z, double zc, double a, double lb) {
    if (z < (a + 1.0) / (a + 2.5)) return 0.5 * log(zc) - log(a) - lb - log(dm_beta_cf(a, 0.5, z)) - LN2;
    return dm_lnT_lower(z, zc, a, lb) - a * log(z);
}

// Quantile in the tau variable: l = ln tau, tau in (0,1] with
// ln T_lower(tau) = lnq (lnq <= -ln 2).
__device__ inline double dm_l_of_lnq(double lnq, double a, double lb) {
    if (!(lnq < -LN2)) return 0.0;
    if (lnq == -INFINITY) return -INFINITY;
    auto g = [&](double l, double *dg) {
        const double tau = exp(l);
        const double s = -expm1(l);          // 1 - tau
        const double z = tau * (2.0 - tau);
        const double lt = dm_lnT_lower(z, s * s, a, lb);
        // d ln T / d ln tau = tau z^(a-1) / (B(a,1/2) T)
        *dg = exp(l + (a - 1.0) * log(z) - lb - lt - LN2) * 2.0;
        return lt - lnq;
    };
    double hi = 0.0, lo = (lnq + LN2) / a;   // T ~ tau^a h(tau), h(1) = 1/2
    double dg;
    double glo = g(lo, &dg);
    int guard = 0;
    while (glo > 0.0 && guard++ < 2000) { hi = lo; lo = 2.0 * lo - 1.0; glo = g(lo, &dg); }
    double l = lo;
    double gl = glo;
    for (int it = 0; it < 200; ++it) {
        if (gl > 0.0) hi = l; else lo = l;
        double ln = l - gl / dg;
        // a converged Newton step ends the search before the bracket test (a
        // zero step lands on the bracket end and would restart bisection)
        if (fabs(ln - l) <= 4e-16 * fmax(1.0, fabs(l))) { l = ln; break; }
        if (!(ln > lo && ln < hi)) ln = 0.5 * (lo + hi);
        const double step = fabs(ln - l);
        l = ln;
        if (step <= 4e-16 * fmax(1.0, fabs(l)) || hi - lo <= 4e-16 * fmax(1.0, fabs(lo))) break;
        gl = g(l, &dg);
    }
    return l;
}

__device__ inline double dm_tau_of_lnq(double lnq, double a, double lb) {
    return exp(dm_l_of_lnq(lnq, a, lb));
}

// (v + a) / (v + b), with its limit 1 at v = infinity (the normal limit of the
// t laws: every dof ratio of the family tends to 1).
__device__ inline double dm_ratio(double v, double a, double b) {
    return isinf(v) ? 1.0 : (v + a) / (v + b);
}

// log of the univariate t_1 density with scale S (variance-like) and dof v,
// given the log normaliser lnc = lgamma((v+1)/2) - lgamma(v/2) - 1/2 ln(pi v);
// at v = infinity the normal density, lnc = -1/2 ln(2 pi).
__device__ inline double dm_lt1pdf(double x, double S, double v, double lnc) {
    if (isinf(v)) return lnc - 0.5 * log(S) - 0.5 * x * x / S;
    return lnc - 0.5 * log(S) - 0.5 * (v + 1.0) * log1p(x * x / (v * S));
}

__device__ inline double dm_lt1_const(double v) {
    if (isinf(v)) return -0.5 * log(2.0 * M_PI);
    return lgamma(0.5 * (v + 1.0)) - lgamma(0.5 * v) - 0.5 * log(M_PI * v);
}

// ------------------------------------------------ normal limit (FP64) ------

// ln Phi(x) for x <= 0: erfc for moderate x, the scaled erfcx (erfc(t) =
// exp(-t^2) erfcx(t)) in the tail so the log stays finite far past underflow.
__device__ inline double dm_lnPhi_lower(double x) {
    const double t = -x * M_SQRT1_2;                  // >= 0
    if (t < 1.0) return log(0.5 * erfc(t));
    return log(0.5 * erfcx(t)) - t * t;
}

// The z <= 0 with ln Phi(z) = lnq (lnq <= -ln 2): erfcinv start (or the
// asymptotic z ~ -sqrt(-2 lnq - ln(-4 pi lnq)) where exp(lnq) underflows),
// then Newton steps on ln Phi, whose slope is the inverse Mills ratio.
__device__ inline double dm_ninv_lower(double lnq) {
    if (!(lnq < -LN2)) return 0.0;
    if (lnq == -INFINITY) return -INFINITY;
    double z = lnq > -700.0 ? -M_SQRT2 * erfcinv(2.0 * exp(lnq))
                            : -sqrt(-2.0 * lnq - log(-4.0 * M_PI * lnq));
    for (int it = 0; it < 3; ++it) {
        const double lp = dm_lnPhi_lower(z);
        const double slope = exp(-0.5 * z * z - 0.5 * log(2.0 * M_PI) - lp);   // phi(z) / Phi(z)
        const double zn = z - (lp - lnq) / slope;
        if (!(zn <= 0.0) || !isfinite(zn)) break;
        z = zn;
    }
    return z;
}

// Univariate t CDF T_v(x) in FP64 (the one-dimensional T_m).
__device__ inline double dm_tcdf(double x, double v) {
    if (isnan(x)) return x;
    if (isinf(x)) return x > 0 ? 1.0 : 0.0;
    if (isinf(v)) return 0.5 * erfc(-x * M_SQRT1_2);          // normal limit
    const double a = 0.5 * v, lb = dm_lbeta_half(a);
    // s = x / sqrt(v + x^2): z = v/(v+x^2), zc = x^2/(v+x^2)
    double z, zc;
    const double ax = fabs(x);
    if (ax > 1.0) { const double r = (v / ax) / ax; z = r / (1.0 + r); zc = 1.0 / (1.0 + r); }
    else { const double den = v + x * x; z = v / den; zc = x * x / den; }
    const double lo = exp(dm_lnT_lower(z, zc, a, lb));
    return x <= 0.0 ? lo : 1.0 - lo;
}

// ------------------------------------------------- FP64 dof tables ------

// c[0] + sum_k c[k] T_k(x), x in [-1, 1], by Clenshaw's recurrence.
__device__ __forceinline__ double tab64_cheb(const double *c, double x) {
    const double x2 = 2.0 * x;
    double b1 = 0.0, b2 = 0.0;
#pragma unroll
    for (int k = TAB64_NC - 1; k >= 1; --k) {
        const double t = fma(x2, b1, c[k] - b2);
        b2 = b1;
        b1 = t;
    }
    return fma(x, b1, c[0] - b2);
}

// H(tau) = ln T_lower(tau) - a ln(tau (2 - tau)) from the CDF rows of one
// dof's table; tau is clamped into [0, 1] (NaN to 0), so the row index is
// always in range.
__device__ __forceinline__ double tab64_H(const double *tab, double tau) {
    const double pos = fmin(fmax(tau, 0.0), 1.0) * (double)TAB64_CDF_ROWS;
    const int k = min((int)pos, TAB64_CDF_ROWS - 1);
    return tab64_cheb(tab + k * TAB64_NC, 2.0 * (pos - (double)k) - 1.0);
}

// l = ln tau with ln T_lower(tau) = lnq for dof 2a (lb = ln B(a, 1/2)): a
// start from the quantile rows (lambda = -log2(2p) = -1 - lnq / ln 2), or
// past the last row from the tail law T ~ e^H(0) (2 tau)^a, then Newton steps
// on g(l) = H(tau) + a (l + ln(2 - tau)) - lnq, whose slope is
// g'(l) = e^(-lb - H(tau)) / (2 - tau) (the t density in the tau variable).
// One step from the table's start (error ~1e-11) reaches the accuracy of H;
// the tail start takes four.  l is kept <= 0 (tau <= 1).
__device__ inline double tab64_quantile_l(const double *tab, double lnq, double a, double lb) {
    const double zz = fmax(-lnq * (1.0 / LN2) - 1.0, 0.0) + 0.25;
    double l;
    int steps = 1;
    if (zz < TAB64_ZZ_END) {
        const int e = __builtin_amdgcn_frexp_exp(zz);          // zz = mant 2^e, mant in [0.5, 1)
        const double mant = __builtin_amdgcn_frexp_mant(zz);
        l = tab64_cheb(tab + (TAB64_CDF_ROWS + e + 1) * TAB64_NC, 4.0 * mant - 3.0);
    } else {
        l = (lnq - tab64_H(tab, 0.0)) / a - LN2;
        steps = 4;
    }
    for (int it = 0; it < steps; ++it) {
        const double tau = exp(l);
        const double u = 2.0 - tau;
        const double H = tab64_H(tab, tau);
        const double g = H + a * (l + log(u)) - lnq;
        l = fmin(l - g * u * exp(lb + H), 0.0);
    }
    return l;
}

// The root of the same equation solved to rounding on the CDF rows (the
// quantile nodes of the table builds): the tail-law start (at most 0),
// widened until g changes sign, then Newton steps kept inside the bracket
// [lo, 0], bisecting where a step would leave it; relative tolerance 2e-15
// (the rounding noise of g at large |ln p|).  Every loop is bounded.
__device__ inline double tab64_l_solve(const double *tab, double lnq, double a, double lb) {
    if (!(lnq < -LN2)) return 0.0;
    auto g = [&](double l, double *dg) {
        const double tau = exp(l), u = 2.0 - tau, H = tab64_H(tab, tau);
        *dg = exp(-lb - H) / u;
        return H + a * (l + log(u)) - lnq;
    };
    double hi = 0.0, lo = fmin((lnq - tab64_H(tab, 0.0)) / a - LN2, 0.0), dg;
    double glo = g(lo, &dg);
    double l = lo, gl = glo, dgl = dg;     // Newton starts from the bracket end nearest the root
    for (int guard = 0; glo > 0.0 && guard < 64; ++guard) {
        hi = lo; l = lo; gl = glo; dgl = dg;
        lo = 2.0 * lo - 1.0;
        glo = g(lo, &dg);
    }
    dg = dgl;
    for (int it = 0; it < 100; ++it) {
        if (gl > 0.0) hi = l; else lo = l;
        double ln = l - gl / dg;
        if (fabs(ln - l) <= 2e-15 * fmax(1.0, fabs(l))) { l = fmin(ln, 0.0); break; }
        if (!(ln > lo && ln < hi)) ln = 0.5 * (lo + hi);
        const double step = fabs(ln - l);
        l = ln;
        if (step <= 2e-15 * fmax(1.0, fabs(l)) || hi - lo <= 2e-15 * fmax(1.0, fabs(lo))) break;
        gl = g(l, &dg);
    }
    return l;
}

// ---------------------------------------------------------------- FP32 ------

__device__ __forceinline__ float fexp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float flog2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }

__device__ __forceinline__ float tab_poly(const float *row, float x) {
    const float4 lo = *reinterpret_cast<const float4 *>(row);
    const float4 hi = *reinterpret_cast<const float4 *>(row + 4);
    float r = hi.z;
    r = fmaf(r, x, hi.y);
    r = fmaf(r, x, hi.x);
    r = fmaf(r, x, lo.w);
    r = fmaf(r, x, lo.z);
    r = fmaf(r, x, lo.y);
    r = fmaf(r, x, lo.x);
    return r;
}

// Normal limit: log2 Phi(-v), v >= 0, from the CDF rows of the dof-free
// normal table (geometric intervals of v + 1/4; v is clamped to 63.5, where
// the probability is far below any that matters).
__device__ __forceinline__ float tab_ncdf_l2(const float *tab, float v) {
    const float zz = fminf(v, 63.5f) + 0.25f;
    const int e = __builtin_amdgcn_frexp_expf(zz);     // zz = mant 2^e, mant in [0.5, 1)
    const float mant = __builtin_amdgcn_frexp_mantf(zz);
    return tab_poly(tab + 8 * (e + 1), mant);           // rows are polynomials in mant
}

// The same two lookups in the fine layout (rows of 4 coefficients, cubic).
__device__ __forceinline__ float tab_cubic(const float *row, float x) {
    const float4 c = *reinterpret_cast<const float4 *>(row);
    return fmaf(fmaf(fmaf(c.w, x, c.z), x, c.y), x, c.x);
}

// H(tau) at pos = 64 tau (clamped into the table, NaN included).
__device__ __forceinline__ float tabf_cdf_H(const float *tab, float pos) {
    pos = fminf(fmaxf(pos, 0.0f), 63.9999962f);
    const int k = (int)pos;
    return tab_cubic(tab + 4 * k, __builtin_amdgcn_fractf(pos));
}

// H(tau) given x = 1 + tau (clamped into [1, 2), NaN included): the top 6
// mantissa bits of x are the row (the integer part of 64 tau) and the other
// 17 the position inside it, as the float 1 + low 2^-23 in [1, 1 + 1/64),
// position = 64 (that - 1), exact.  No conversion instruction is needed.
static_assert(TABF_CDF_ROWS == 64, "the CDF rows are indexed by 6 mantissa bits");
__device__ __forceinline__ float tabf_cdf_H_1p(const float *tab, float x) {
    x = fminf(fmaxf(x, 1.0f), 1.99999988f);
    const uint32_t bits = __float_as_uint(x);
    const float t = fmaf(__uint_as_float((bits & 0x0001FFFFu) | 0x3F800000u), 64.0f, -64.0f);
    return tab_cubic(reinterpret_cast<const float *>(reinterpret_cast<const char *>(tab) + ((bits >> 13) & 0x3F0u)), t);
}

// log2 tau at l2p = log2 p.  -l2p = lambda + 1, clamped to [1, 512): l2p is
// clamped to [-512, -1) (NaN included) instead, whose biased exponent is
// 127..135, so bits 20..26 (low 4 exponent bits and top 3 mantissa bits) are
// the quantile slot (tabf_inv_slot) with no offset to subtract, and the low
// 20 mantissa bits the position inside it: as the float 1 + low 2^-23 in
// [1, 9/8), position = 8 (that - 1), exact.  Without CLAMP, l2p must be at
// least -512 and at most -1 or log2 of an FP32 p in [0, 1/2] (rounded up to
// 1/2 + ulp at most): log2 p is
// then in [-149, -1] (exponents 127..134, inside the rows), -inf at p = 0
// reads a valid row, and a p just above 1/2 (exponent 126) reads an unused
// zero row, log2 tau = 0, the centre, as it should.
template <bool CLAMP = true>
__device__ __forceinline__ float tabf_inv_G(const float *tab, float l2p) {
    const float zz = CLAMP ? fminf(fmaxf(l2p, -511.999969f), -1.0f) : l2p;
    const uint32_t bits = __float_as_uint(zz);
    const float t = fmaf(__uint_as_float((bits & 0x000FFFFFu) | 0x3F800000u), 8.0f, -8.0f);
    return tab_cubic(reinterpret_cast<const float *>(reinterpret_cast<const char *>(tab + 4 * TABF_CDF_ROWS) +
                                                     ((bits >> 16) & 0x7F0u)), t);
}

// log2 tau from the quantile rows, given l2p = log2 p of the tail probability
// p <= 1/2; the table variable is lam = -log2(2p) = -1 - l2p, clamped to
// [0, INV_LAMBDA_MAX] and offset by 1/4 (both folded into one clamp of
// -3/4 - l2p).
__device__ __forceinline__ float tab_inv_G(const float *tab, float l2p) {
    const float zz = fminf(fmaxf(-0.75f - l2p, 0.25f), INV_LAMBDA_MAX + 0.25f);
    const int e = __builtin_amdgcn_frexp_expf(zz);     // zz = mant 2^e, mant in [0.5, 1)
    const float mant = __builtin_amdgcn_frexp_mantf(zz);
    const int k = e + 1;                               // interval 0..10
    return tab_poly(tab + 8 * (TAB_CDF_ROWS + k), mant);   // rows are polynomials in mant
}

}  // namespace cfust
