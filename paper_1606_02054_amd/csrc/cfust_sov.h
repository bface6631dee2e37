// cfust_sov.h -- the lattice estimate of a multivariate t probability
//     T_m(b; 0, L L^T, nu) = P(Z <= b),  Z ~ t_m(0, L L^T, nu),
// by Genz's separation of variables for the t law: with Z = L Y, the
// coordinates of Y are sampled one after another from their conditional laws
//     Y_i | y_0..y_{i-1} ~ sqrt((nu + S_i)/(nu + i)) t_{nu+i},  S_i = sum_{j<i} y_j^2,
// each truncated to the region that keeps Z_i <= b_i; the integrand is the
// product of the truncation probabilities e_1 ... e_{m-1} (e_0 is the same for
// every point and is factored out).  Coordinate i uses lattice coordinate i.
//
// Both precisions track Q_i = sqrt(nu + S_i), for which the algebra of the
// conditional t collapses to
//     s_i   = num_i / sqrt(L_ii^2 Q_i^2 + num_i^2),  num_i = b_i - sum_{j<i} L_ij y_j,
//     tau_i = 1 - |s_i|  (the argument of the lower-tail probability),
//     y_i   = s'_i Q_{i+1},   Q_{i+1} = Q_i / sqrt(tau'_i (2 - tau'_i)),
// where s'_i, tau'_i belong to the quantile drawn at p = x_i e_i.
// The complement 1 - p = (1 - x_i) e_i + (1 - e_i) is formed from accurate
// complements, so neither tail loses relative accuracy.
#pragma once
#include "cfust_devmath.h"
#include "cfust_kernels.h"

namespace cfust {

// ------------------------------------------------------------ wave helpers --

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

using Lattice = LatticeArgs;

// ------------------------------------------------------------- FP64 path ---

// Lattice coordinate (FP64), the same arithmetic as the definition:
// t = frac(r/N + shift), x = 1 - |2t - 1|, clamped to [2^-24, 1 - 2^-24].
__device__ __forceinline__ void point64(const Lattice &Lt, int s, int k, int j, double &x, double &xb) {
    const unsigned long long r = ((unsigned long long)k * (unsigned long long)Lt.z[j]) % (unsigned long long)Lt.N;
    double t = (double)r / (double)Lt.N + Lt.shifts[s * LATD + j];
    if (t >= 1.0) t -= 1.0;
    double xbv = fabs(2.0 * t - 1.0);
    double xv = 1.0 - xbv;
    const double lo = 1.0 / 16777216.0;
    if (xv < lo) { xv = lo; xbv = 1.0 - lo; }
    if (xv > 1.0 - lo) { xv = 1.0 - lo; xbv = lo; }
    x = xv;
    xb = xbv;
}

// Quantile step shared by all coordinates: given the truncation probability
// (e, eb = 1-e, lne valid when lowt) and the point (x, xb), draw y and update Q.
__device__ __forceinline__ double quantile_step64(double x, double xb, double e, double eb, double lne,
                                                  bool lowt, double a, double lb, double &Q) {
    const double p = x * e;
    const double pb = xb * e + eb;
    const bool lower = lowt || p <= 0.5;
    const double lnq = lowt ? log(x) + lne : log(lower ? p : pb);
    const double tq = dm_tau_of_lnq(lnq, a, lb);
    const double sabs = 1.0 - tq;
    Q *= 1.0 / sqrt(tq * (2.0 - tq));
    return (lower ? -sabs : sabs) * Q;
}

// Per-lane sum over this lane's points of one shift, FP64 arithmetic.
template <int M>
__device__ double sov_lane_sum64(const double *b, const double *L, double nu, const Lattice &Lt, int s,
                                 double e0, double eb0, double lne0, bool low0, int lane) {
    double a[M], lb[M];
#pragma unroll
    for (int i = 0; i < M; ++i) { a[i] = 0.5 * (nu + i); lb[i] = dm_lbeta_half(a[i]); }
    double acc = 0.0;
    for (int k = lane; k < Lt.N; k += 64) {
        double y[M];
        double Q = sqrt(nu);
        double x, xb;
        point64(Lt, s, k, 0, x, xb);
        y[0] = quantile_step64(x, xb, e0, eb0, lne0, low0, a[0], lb[0], Q);
        double f = 1.0;
#pragma unroll
        for (int i = 1; i < M; ++i) {
            double num = b[i];
#pragma unroll
            for (int j = 0; j < i; ++j) num -= L[i * M + j] * y[j];
            const double LQ = L[i * M + i] * Q;
            const double K = LQ * LQ;
            const double R = 1.0 / sqrt(K + num * num);
            const double tau = K * R * R / (1.0 + fabs(num) * R);
            const double sr = num * R;
            const double lt = dm_lnT_lower(tau * (2.0 - tau), sr * sr, a[i], lb[i]);
            const double small = exp(lt);
            const bool lowt = num <= 0.0;
            const double e = lowt ? small : 1.0 - small;
            const double eb = lowt ? 1.0 - small : small;
            f *= e;
            if (f == 0.0) break;
            if (i < M - 1) {
                point64(Lt, s, k, i, x, xb);
                y[i] = quantile_step64(x, xb, e, eb, lt, lowt, a[i], lb[i], Q);
            }
        }
        acc += f;
    }
    return acc;
}

// FP64 integrand with the dof tables (tab: TAB64_DOUBLES per dof, dof nu + i
// for coordinate i, in LDS): the same steps as sov_lane_sum64, with ln T_lower
// = H(tau) + a ln(K R^2) from the CDF rows (K R^2 = tau (2 - tau)) and the
// quantile from tab64_quantile_l.  The lattice residues k z_j mod N advance by
// 64 z_j mod N per lane step (the same integers as point64's product).
__device__ __forceinline__ double quantile_step64_tab(double x, double xb, double e, double eb, double lne,
                                                      bool lowt, double a, double lb, const double *tab,
                                                      double &Q) {
    const double p = x * e;
    const double pb = xb * e + eb;
    const bool lower = lowt || p <= 0.5;
    const double lnq = lowt ? log(x) + lne : log(lower ? p : pb);
    const double tq = exp(tab64_quantile_l(tab, lnq, a, lb));
    const double sabs = 1.0 - tq;
    Q *= 1.0 / sqrt(tq * (2.0 - tq));
    return (lower ? -sabs : sabs) * Q;
}

__device__ __forceinline__ void point64_r(const Lattice &Lt, int s, int j, uint32_t r, double &x, double &xb) {
    double t = (double)r / (double)Lt.N + Lt.shifts[s * LATD + j];
    if (t >= 1.0) t -= 1.0;
    double xbv = fabs(2.0 * t - 1.0);
    double xv = 1.0 - xbv;
    const double lo = 1.0 / 16777216.0;
    if (xv < lo) { xv = lo; xbv = 1.0 - lo; }
    if (xv > 1.0 - lo) { xv = 1.0 - lo; xbv = lo; }
    x = xv;
    xb = xbv;
}

template <int M>
__device__ double sov_lane_sum64_tab(const double *b, const double *L, double nu, const Lattice &Lt, int s,
                                     const double *tab, double e0, double eb0, double lne0, bool low0, int lane) {
    constexpr int MQ = M > 1 ? M - 1 : 1;       // coordinates that draw a quantile
    double a[M], lb[M];
#pragma unroll
    for (int i = 0; i < M; ++i) { a[i] = 0.5 * (nu + i); lb[i] = dm_lbeta_half(a[i]); }
    const uint32_t N = (uint32_t)Lt.N;
    uint32_t r[MQ], st[MQ];
#pragma unroll
    for (int j = 0; j < MQ; ++j) {
        const uint32_t z = (uint32_t)Lt.z[j];
        r[j] = (uint32_t)(((uint64_t)lane * z) % N);
        st[j] = (uint32_t)((64ull * z) % N);
    }
    double acc = 0.0;
    for (int k = lane; k < Lt.N; k += 64) {
        double y[M];
        double Q = sqrt(nu);
        double x, xb;
        point64_r(Lt, s, 0, r[0], x, xb);
        y[0] = quantile_step64_tab(x, xb, e0, eb0, lne0, low0, a[0], lb[0], tab, Q);
        double f = 1.0;
#pragma unroll
        for (int i = 1; i < M; ++i) {
            double num = b[i];
#pragma unroll
            for (int j = 0; j < i; ++j) num -= L[i * M + j] * y[j];
            const double LQ = L[i * M + i] * Q;
            const double K = LQ * LQ;
            const double R = 1.0 / sqrt(K + num * num);
            const double lt = tab64_H(tab + i * TAB64_DOUBLES, 1.0 - fabs(num) * R) + a[i] * log(K * R * R);
            const double small = exp(lt);
            const bool lowt = num <= 0.0;
            const double e = lowt ? small : 1.0 - small;
            const double eb = lowt ? 1.0 - small : small;
            f *= e;
            if (f == 0.0) break;
            if (i < M - 1) {
                point64_r(Lt, s, i, r[i], x, xb);
                y[i] = quantile_step64_tab(x, xb, e, eb, lt, lowt, a[i], lb[i], tab + i * TAB64_DOUBLES, Q);
            }
        }
        acc += f;
#pragma unroll
        for (int j = 0; j < MQ; ++j) {
            r[j] += st[j];
            r[j] = r[j] >= N ? r[j] - N : r[j];
        }
    }
    return acc;
}

// Normal limit (dof infinite), FP64: the conditional laws are normal with
// fixed scale, so y_i = Phi^-1(x_i e_i) and no scale is carried.
__device__ __forceinline__ double nquantile_step64(double x, double xb, double e, double eb, double lne,
                                                   bool lowt) {
    const double p = x * e;
    const double pb = xb * e + eb;
    const bool lower = lowt || p <= 0.5;
    const double lnq = lowt ? log(x) + lne : log(lower ? p : pb);
    const double z = dm_ninv_lower(lnq);
    return lower ? z : -z;
}

template <int M>
__device__ double sov_lane_sum64_normal(const double *b, const double *L, const Lattice &Lt, int s, double e0,
                                        double eb0, double lne0, bool low0, int lane) {
    double acc = 0.0;
    for (int k = lane; k < Lt.N; k += 64) {
        double y[M];
        double x, xb;
        point64(Lt, s, k, 0, x, xb);
        y[0] = nquantile_step64(x, xb, e0, eb0, lne0, low0);
        double f = 1.0;
#pragma unroll
        for (int i = 1; i < M; ++i) {
            double num = b[i];
#pragma unroll
            for (int j = 0; j < i; ++j) num -= L[i * M + j] * y[j];
            const double lt = dm_lnPhi_lower(-fabs(num) / L[i * M + i]);
            const double small = exp(lt);
            const bool lowt = num <= 0.0;
            const double e = lowt ? small : 1.0 - small;
            const double eb = lowt ? 1.0 - small : small;
            f *= e;
            if (f == 0.0) break;
            if (i < M - 1) {
                point64(Lt, s, k, i, x, xb);
                y[i] = nquantile_step64(x, xb, e, eb, lt, lowt);
            }
        }
        acc += f;
    }
    return acc;
}

// ------------------------------------------------------------- FP32 path ---

// Lattice coordinate (FP32): t in 32-bit fixed point, t = 2^32 frac(k z_j / N
// + shift) (needs N a power of two): ((k z_j) << (32 - log2 N)) + shift (the
// shift drops the bits of k z_j above log2 N, so no reduction mod N is
// needed), carried from point to point by adding ((64 z_j) << (32 - log2 N)).
// As a signed integer, |t| = 2^31 min(t, 1-t) = 2^31 x (the tent transform),
// and with the top bit flipped (t - 1/2 mod 1), |t ^ 2^31| = 2^31 |2t - 1| =
// 2^31 (1 - x): both come straight from the integers, so x keeps full
// relative accuracy near 0 (it enters log2 x in the lower tail) and so does
// 1 - x near 0 (it enters the upper-tail complement p_b = (1 - x) e + e_b,
// whose relative accuracy sets the quantile where the conditional law is
// sampled far in its upper tail).  The clamp to [2^-24, 1 - 2^-24] is
// [128, 2^31 - 128] in these units (exact floats); both values are returned
// in units of 2^-31 (unscaled) or scaled.
__device__ __forceinline__ float tent_units(uint32_t t) {
    return __builtin_amdgcn_fmed3f(fabsf((float)(int32_t)t), 128.0f, 2147483520.0f);
}

__device__ __forceinline__ void point32(uint32_t t, float &x, float &xb) {
    x = tent_units(t) * 4.656612873077393e-10f;                  // 2^-31
    xb = tent_units(t ^ 0x80000000u) * 4.656612873077393e-10f;
}

// The quantile steps below carry the conditional scale sqrt(nu + sum y^2) in
// units of sqrt(nu), Q = sqrt(1 + sum y^2 / nu) (the draws y and the limits
// are in the same units: the setup divides b_i by L_ii sqrt(nu)), and cap Q
// at 1e15: a point whose tau = 2^G underflows (G below about -100, where
// 1/sqrt(tau (2 - tau)) and so Q, at least 1, exceed 1e15) draws its quantile
// at the cap, with no clamp on G.  What follows such a draw depends on the
// cap only through limits of order b / 1e15.
//
// Quantile step of coordinate 0 (the truncation probability e_0 is the same
// for every point).  LOW0: e_0 is a lower-tail probability that may be far
// below the FP32 range, so p = x e_0 <= 1/2 is taken in the log domain,
// log2 p = log2(2^31 x) + (log2 e_0 - 31); otherwise e_0 >= 1/2 and
// p = (2^31 x)(2^-31 e_0), p_b = (2^31 (1-x))(2^-31 e_0) + e_b0.
struct Sov32Setup {
    float b[MAXQ];
    float L[MAXQ * MAXQ];      // row-major, stride M
    float a[MAXQ];             // nu + i (mixed t path); 1 / L_ii (normal limit)
    float e0s, eb0, l2e0m31;           // 2^-31 e_0, 1 - e_0, log2 e_0 - 31
    float e0, l2e0;                     // e_0, log2 e_0 (normal limit)
    bool low0;
};

// The FP32 t-law lookups of the fine-layout slots (TABF_FLOATS per dof):
// log2 tau of the quantile, and log2 T_lower less a log2(tau (2 - tau)) at
// tau = 1 - |s|, given s = num R (1 + tau = 2 - |num| R, one FMA).
__device__ __forceinline__ float tab_G(const float *tab, float l2p) { return tabf_inv_G(tab, l2p); }
// The same for l2p = log2 p of an FP32 p in [0, 1/2] (no clamp needed).
__device__ __forceinline__ float tab_G_p(const float *tab, float l2p) { return tabf_inv_G<false>(tab, l2p); }
__device__ __forceinline__ float tab_H_num_R(const float *tab, float num, float R) {
    return tabf_cdf_H_1p(tab, fmaf(-fabsf(num), R, 2.0f));
}

// xu, xbu: the coordinate and its complement in units of 2^-31 (xbu unused
// when LOW0); with L2X (LOW0 only), xu is already log2 of the coordinate.
template <bool LOW0, bool L2X = false>
__device__ __forceinline__ float quantile_step32_first_u(const Sov32Setup &P, float xu, float xbu, const float *tab,
                                                         float &Q) {
    bool lower;
    float l2q;
    if (LOW0) {
        lower = true;
        l2q = (L2X ? xu : flog2(xu)) + P.l2e0m31;
    } else {
        const float p = xu * P.e0s;
        const float pb = fmaf(xbu, P.e0s, P.eb0);
        lower = p <= 0.5f;
        l2q = flog2(lower ? p : pb);
    }
    // LOW0: log2 e_0 may be far below the FP32 range, so l2q is clamped
    // below (above, l2q <= log2 e_0 <= -1 already)
    const float tq = fexp2(tab_G_p(tab, LOW0 ? fmaxf(l2q, -511.999969f) : l2q));
    const float sabs = 1.0f - tq;
    Q = fminf(Q * frsq(fmaf(tq, sabs, tq)), 1e15f);      // tau (2 - tau) = tau + tau (1 - tau)
    return (lower ? -sabs : sabs) * Q;
}

template <bool LOW0>
__device__ __forceinline__ float quantile_step32_first(const Sov32Setup &P, uint32_t t, const float *tab, float &Q) {
    return quantile_step32_first_u<LOW0>(P, tent_units(t), LOW0 ? 0.0f : tent_units(t ^ 0x80000000u), tab, Q);
}

// Quantile step of coordinate i >= 1, given the lower-tail value small =
// T_lower of the coordinate's conditional law and lowt (its limit is in the
// lower half, e = small; otherwise e = 1 - small).  p = x e is formed
// directly: a point whose factor e is below the FP32 range contributes 0 to
// the product, whatever it draws.  When !lowt the complement is
// 1 - x e = (1 - x) e + small.
__device__ __forceinline__ float quantile_step32(float x, float xb, float e, float small, const float *tab,
                                                 float &Q) {
    const float p = x * e;
    const float pb = fmaf(xb, e, small);
    const bool lower = p <= 0.5f;
    const float tq = fexp2(tab_G_p(tab, flog2(lower ? p : pb)));
    const float sabs = 1.0f - tq;
    Q = fminf(Q * frsq(fmaf(tq, sabs, tq)), 1e15f);      // tau (2 - tau) = tau + tau (1 - tau)
    return (lower ? -sabs : sabs) * Q;
}

// Integrand value of lattice point k (FP32), the product e_1 ... e_{M-1},
// added to acc with weight w, its last factor in the same FMA.
template <int M, bool LOW0>
__device__ __forceinline__ void sov_point32(const Sov32Setup &P, const float *tabs, const uint32_t *t, float w,
                                            float &acc) {
    float y[M];
    float Q = 1.0f;
    y[0] = quantile_step32_first<LOW0>(P, t[0], tabs, Q);
    float f = 1.0f;
#pragma unroll
    for (int i = 1; i < M; ++i) {
        float num = P.b[i];
#pragma unroll
        for (int j = 0; j < i; ++j) num = fmaf(-P.L[i * M + j], y[j], num);
        // lower-tail probability of the conditional t (row i of b and L divided by
        // L_ii): with R = 1 / sqrt(num^2 + Q^2) and s = num R, log2 T_lower =
        // ((nu + i)/2) log2(1 - s^2) + H(1 - |s|), and 1 - s^2 = (Q R)^2, so the
        // power law is (nu + i) log2(Q R): no division
        const float R = frsq(fmaf(num, num, Q * Q));
        const float *tab = tabs + i * TABF_FLOATS;
        const float l2 = fmaf(P.a[i], flog2(Q * R), tab_H_num_R(tab, num, R));
        const float small = fexp2(l2);
        const float e = num <= 0.0f ? small : 1.0f - small;
        if (i < M - 1) {
            f *= e;
            float x, xb;
            point32(t[i], x, xb);
            y[i] = quantile_step32(x, xb, e, small, tab, Q);
        } else {
            acc = fmaf(f, e * w, acc);      // w = 0 or 1: the same sum as the coordinate-table form
        }
    }
}

// The same point (E-step tables, fine layout), with its coordinates read from
// the E-step's coordinate table instead of formed from the lattice: c[2i] is coordinate i and
// c[2i + 1] its complement, coordinate 0 in units of 2^-31 and the others
// scaled -- the values point32 / tent_units form, bit for bit.  Under LOW0,
// c[0] is log2 of coordinate 0 (in those units), the value the first quantile
// step would take of it.  The point's product is added to acc, its last
// factor in the same FMA.
template <int M, bool LOW0>
__device__ __forceinline__ void sov_point32_c(const Sov32Setup &P, const float *tabs, const float *c, float &acc) {
    float y[M];
    float Q = 1.0f;
    y[0] = quantile_step32_first_u<LOW0, LOW0>(P, c[0], c[1], tabs, Q);
    float f = 1.0f;
#pragma unroll
    for (int i = 1; i < M; ++i) {
        float num = P.b[i];
#pragma unroll
        for (int j = 0; j < i; ++j) num = fmaf(-P.L[i * M + j], y[j], num);
        const float R = frsq(fmaf(num, num, Q * Q));
        const float *tab = tabs + i * TABF_FLOATS;
        const float l2 = fmaf(P.a[i], flog2(Q * R), tab_H_num_R(tab, num, R));
        const float small = fexp2(l2);
        const float e = num <= 0.0f ? small : 1.0f - small;
        if (i < M - 1) {
            f *= e;
            y[i] = quantile_step32(c[2 * i], c[2 * i + 1], e, small, tab, Q);
        } else {
            acc = fmaf(f, e, acc);
        }
    }
}

// Loads of one trip's coordinates through a buffer resource over the shift's
// table (rows of N floats: row 0 log2 of coordinate 0, row 1 + 2i coordinate
// i, row 2 + 2i its complement): the lane offset is the vector offset and
// the row and trip go in the scalar offset, so no vector instruction forms an
// address.  Under LOW0 the first quantile needs only log2 of coordinate 0, so
// c[0] is that logarithm and coordinate 0 itself and its complement are not
// read.
constexpr int BUF_RSRC_WORD3 = 0x00020000;     // raw buffer, 32-bit elements (gfx9 family)

template <int M, bool LOW0>
__device__ __forceinline__ void load_coords(__amdgpu_buffer_rsrc_t r, int vo, int so, int row_bytes, float *c) {
#pragma unroll
    for (int i = 0; i < M - 1; ++i) {
        const int row = (i == 0 && LOW0) ? 0 : 1 + 2 * i;
        c[2 * i] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so + row * row_bytes, 0));
        c[2 * i + 1] = (i == 0 && LOW0) ? 0.0f
                     : __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so + (2 + 2 * i) * row_bytes, 0));
    }
}

// Per-lane FP32 sum over the shift's points from the coordinate table
// `cshift` (N a multiple of 64; lane l takes points l, l + 64, ...).  At
// m = 2 a point is short (about 40 VALU), so its coordinates are loaded one
// trip ahead into an alternating pair of register sets (the load after the
// last even trip re-reads that trip's own coordinates, so every load stays
// inside the table); at larger m the loads of a trip are waited for where
// the point first needs them and the other resident waves cover their
// latency (loading ahead there only cost registers).  Each point's product
// enters the sum with its last factor in one FMA, as in the loop that forms
// the coordinates itself, so both give the same sums bit for bit.
template <int M, bool LOW0>
__device__ __forceinline__ float sov_lane_sum32_c(const Sov32Setup &P, const float *tabs, const float *cshift, int N,
                                                  int lane) {
#pragma clang fp contract(off)
    constexpr int R = 2 * (M - 1);              // coordinates and complements per point
    const int row_bytes = N * 4;
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void *)cshift, (short)0, (R + 1) * row_bytes, BUF_RSRC_WORD3);
    const int vo = lane * 4;
    const int trips = N / 64;
    float acc = 0.0f;
    if constexpr (M == 2) {
        float c0[R], c1[R];
        load_coords<M, LOW0>(rs, vo, 0, row_bytes, c0);
        int it = 0;
        for (; it + 2 <= trips; it += 2) {
            load_coords<M, LOW0>(rs, vo, (it + 1) * 256, row_bytes, c1);
            sov_point32_c<M, LOW0>(P, tabs, c0, acc);
            load_coords<M, LOW0>(rs, vo, min(it + 2, trips - 1) * 256, row_bytes, c0);
            sov_point32_c<M, LOW0>(P, tabs, c1, acc);
        }
        if (it < trips) sov_point32_c<M, LOW0>(P, tabs, c0, acc);
    } else {
        float c[R];
        for (int it = 0; it < trips; ++it) {
            load_coords<M, LOW0>(rs, vo, it * 256, row_bytes, c);
            sov_point32_c<M, LOW0>(P, tabs, c, acc);
        }
    }
    return acc;
}

// Normal limit, FP32, from the dof-free normal table (`tab`): the CDF rows
// give log2 Phi(-v), the quantile rows Phi^-1 directly, in the same
// log-domain form as the t path (so the first coordinate, whose e_0 comes
// from FP64 and may be far below the FP32 range, keeps its accuracy).
__device__ __forceinline__ float nquantile_step32(float x, float xb, float e, float eb, float l2e, bool lowt,
                                                  const float *tab) {
    const float p = x * e;
    const float pb = fmaf(xb, e, eb);
    const bool lower = lowt || p <= 0.5f;
    const float arg = lowt ? x : (lower ? p : pb);
    const float l2q = flog2(arg) + (lowt ? l2e : 0.0f);
    const float z = tab_inv_G(tab, l2q);             // Phi^-1(2^l2q) <= 0
    return lower ? z : -z;
}

template <int M>
__device__ __forceinline__ float sov_point32_normal(const Sov32Setup &P, const float *tab, const uint32_t *t) {
    float y[M];
    float x, xb;
    point32(t[0], x, xb);
    y[0] = nquantile_step32(x, xb, P.e0, P.eb0, P.l2e0, P.low0, tab);
    float f = 1.0f;
#pragma unroll
    for (int i = 1; i < M; ++i) {
        float num = P.b[i];
#pragma unroll
        for (int j = 0; j < i; ++j) num = fmaf(-P.L[i * M + j], y[j], num);
        const float l2 = tab_ncdf_l2(tab, fabsf(num) * P.a[i]);      // a[i] = 1 / L_ii
        const float small = fexp2(l2);
        const bool lowt = num <= 0.0f;
        const float e = lowt ? small : 1.0f - small;
        const float eb = lowt ? 1.0f - small : small;
        f *= e;
        if (i < M - 1) {
            point32(t[i], x, xb);
            y[i] = nquantile_step32(x, xb, e, eb, l2, lowt, tab);
        }
    }
    return f;
}

// Per-lane FP32 sum over this lane's points of one shift: lane l takes points
// l, l + 64, ...  PPL independent points are evaluated per loop trip
// (instruction-level parallelism across the dependency chains).  With N a
// multiple of 64 PPL the trip count is the same for every lane, so the loop
// is counted in scalar registers; N < 64 (PPL 1) is one weighted trip.  NORMAL
// selects the normal-limit integrand; LOW0 (t integrand) the form of the
// first coordinate.
template <int M, int PPL, bool NORMAL, bool LOW0>
__device__ __forceinline__ float sov_lane_sum32_f(const Sov32Setup &P, const float *tabs, const uint32_t *zz, int sh,
                                  const uint32_t *shfix, int N, int lane) {
    uint32_t t[PPL][M], step[M];
#pragma unroll
    for (int i = 0; i < M - 1; ++i) {
        step[i] = ((uint32_t)(64 * PPL) * zz[i]) << sh;
#pragma unroll
        for (int u = 0; u < PPL; ++u) t[u][i] = (((uint32_t)(lane + 64 * u) * zz[i]) << sh) + shfix[i];
    }
    // a point's product into acc, weighted by w (0 or 1)
    auto point = [&](const uint32_t *tt, float w, float &a) {
        if constexpr (NORMAL) a = fmaf(sov_point32_normal<M>(P, tabs, tt), w, a);
        else sov_point32<M, LOW0>(P, tabs, tt, w, a);
    };
    // N < 64 (PPL 1): one trip in which the lanes at or past N weigh 0
    const float wl = (N >= 64 * PPL || lane < N) ? 1.0f : 0.0f;
    const int trips = max(N / (64 * PPL), 1);
    float acc = 0.0f;
    for (int it = 0; it < trips; ++it) {
#pragma unroll
        for (int u = 0; u < PPL; ++u) point(t[u], wl, acc);
#pragma unroll
        for (int u = 0; u < PPL; ++u)
#pragma unroll
            for (int i = 0; i < M - 1; ++i) t[u][i] += step[i];
    }
    return acc;
}

// The first coordinate's form is the same for every point of an item, so the
// choice between the two loops is uniform across the wave.
template <int M, int PPL, bool NORMAL>
__device__ __forceinline__ float sov_lane_sum32(const Sov32Setup &P, const float *tabs, const uint32_t *zz, int sh,
                                const uint32_t *shfix, int N, int lane) {
    if (NORMAL) return sov_lane_sum32_f<M, PPL, true, false>(P, tabs, zz, sh, shfix, N, lane);
    if (P.low0) return sov_lane_sum32_f<M, PPL, false, true>(P, tabs, zz, sh, shfix, N, lane);
    return sov_lane_sum32_f<M, PPL, false, false>(P, tabs, zz, sh, shfix, N, lane);
}

// ------------------------------------------------------------- driver -------

// The first factor e_0 = T_nu(b_0 / L_00) of the SOV product, FP64, with its
// complement and logarithm (finite even when e_0 underflows).
struct SovHead {
    double e0, eb0, lne0;
    bool low0;
};

__device__ inline SovHead sov_head(const double *b, const double *L, double nu) {
    if (isinf(nu)) {                                  // normal limit: Phi(b_0 / L_00)
        const double u = b[0] / L[0];
        const double lt0 = dm_lnPhi_lower(-fabs(u));
        const double small0 = exp(lt0);
        SovHead H;
        H.low0 = u <= 0.0;
        H.e0 = H.low0 ? small0 : 1.0 - small0;
        H.eb0 = H.low0 ? 1.0 - small0 : small0;
        H.lne0 = H.low0 ? lt0 : log1p(-small0);
        return H;
    }
    const double a0 = 0.5 * nu, lb0 = dm_lbeta_half(a0);
    const double u = b[0] / L[0];
    const double au = fabs(u);
    double z0, zc0;
    if (au > 1.0) { const double r = (nu / au) / au; z0 = r / (1.0 + r); zc0 = 1.0 / (1.0 + r); }
    else { const double den = nu + u * u; z0 = nu / den; zc0 = u * u / den; }
    const double lt0 = dm_lnT_lower(z0, zc0, a0, lb0);
    const double small0 = exp(lt0);
    SovHead H;
    H.low0 = u <= 0.0;
    H.e0 = H.low0 ? small0 : 1.0 - small0;
    H.eb0 = H.low0 ? 1.0 - small0 : small0;
    H.lne0 = H.low0 ? lt0 : log(H.e0);
    return H;
}

// The same first factor from the E-step's FP32 table of dof nu (fine layout): the
// table gives H(tau) = log2 T_lower - (nu/2) log2(tau (2 - tau)) with
// tau = 1 - |s|, s = u / sqrt(nu + u^2), u = b_0 / L_00.  tau and the log are
// formed in FP64, so no range is lost; only H carries the table's FP32 accuracy.
__device__ inline SovHead sov_head_tab(const double *b, const double *L, double nu, const float *tab) {
    const double u = b[0] / L[0];
    const double au = fabs(u);
    const double r = au > 1.0 ? au * sqrt(1.0 + (nu / au) / au) : sqrt(nu + u * u);
    const double tau = nu / (r * (r + au));
    const double l2 = 0.5 * nu * log2(tau * (2.0 - tau)) + (double)tabf_cdf_H(tab, (float)(64.0 * tau));
    const double lt0 = l2 * LN2;
    const double small0 = exp(lt0);
    SovHead H;
    H.low0 = u <= 0.0;
    H.e0 = H.low0 ? small0 : 1.0 - small0;
    H.eb0 = H.low0 ? 1.0 - small0 : small0;
    H.lne0 = H.low0 ? lt0 : log1p(-small0);
    return H;
}

// Mean over shifts, its standard error and ln(e_0 * mean) from the per-shift
// means in this wave's LDS slice (written by lane 0).
__device__ inline void sov_finish(const SovHead &H, const double *smean, int S,
                                  double *est, double *se, double *lnest) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double mean = 0.0;
    for (int s = 0; s < S; ++s) mean += smean[s];
    mean /= S;
    double var = 0.0;
    for (int s = 0; s < S; ++s) var += (smean[s] - mean) * (smean[s] - mean);
    const double sem = S > 1 ? sqrt(var / ((double)S * (S - 1))) : 0.0;
    *est = H.e0 * mean;
    *se = H.e0 * sem;
    *lnest = mean > 0.0 ? H.lne0 + log(mean) : -INFINITY;
}

// FP32 lattice sums (mixed precision).  Returns false when the FP32 product
// underflowed for the whole item (mean below 1e-30): the caller then redoes
// the item in FP64.  tabs: LDS tables of dofs nu .. nu+M-1.
// COORDS: the lattice coordinates come from the E-step's coordinate table
// `coords` (C coordinates per point; N a multiple of 64, one point per lane
// per trip) instead of being formed in the loop.  `tabs`: fine-layout slots.
template <int M, int PPL, bool COORDS = false>
__device__ __forceinline__ bool sov_mixed(const SovHead &H, const double *b, const double *L, double nu, const Lattice &Lt,
                          const float *tabs, double *smean, int lane, const float *coords = nullptr, int C = 0) {
    Sov32Setup P;
    // rows 1.. of b and L divided by their diagonal, b also by sqrt(nu) (FP64,
    // then rounded): the conditional limit of coordinate i is then num / Q,
    // with no product by L_ii or sqrt(nu) in the loop
    const double rnu = sqrt(nu);
#pragma unroll
    for (int i = 0; i < M; ++i) {
        const double d = i > 0 ? L[i * M + i] : 1.0;
        P.b[i] = (float)(i > 0 ? b[i] / (d * rnu) : b[i]);
        P.a[i] = (float)(nu + i);
#pragma unroll
        for (int j = 0; j < M; ++j) P.L[i * M + j] = (float)(L[i * M + j] / d);
    }
    P.e0s = (float)(H.e0 * 4.656612873077393e-10); P.eb0 = (float)H.eb0;
    P.l2e0m31 = (float)(H.lne0 / LN2 - 31.0); P.low0 = H.low0;
    uint32_t zz[M], shfix[M];
    const int sh = 32 - Lt.log2N;
#pragma unroll
    for (int i = 0; i < M - 1; ++i) zz[i] = (uint32_t)Lt.z[i];
    double tot = 0.0;
    for (int s = 0; s < Lt.S; ++s) {
#pragma unroll
        for (int i = 0; i < M - 1; ++i) shfix[i] = (uint32_t)(Lt.shifts[s * LATD + i] * 4294967296.0);
        float ls;
        if (COORDS) {
            const float *cshift = coords + (size_t)s * (2 * C + 1) * Lt.N;
            ls = P.low0 ? sov_lane_sum32_c<M, true>(P, tabs, cshift, Lt.N, lane)
                        : sov_lane_sum32_c<M, false>(P, tabs, cshift, Lt.N, lane);
        } else {
            ls = sov_lane_sum32<M, PPL, false>(P, tabs, zz, sh, shfix, Lt.N, lane);
        }
        const double ms = wave_sum((double)ls) / (double)Lt.N;
        if (lane == 0) smean[s] = ms;
        tot += ms;
    }
    return tot / Lt.S > 1e-30;
}

// The same for the normal limit (dof infinite), with the dof-free normal
// table `tab` (every coordinate uses it).  An item whose first factor is
// below 2^-480 (past the quantile table's range) is left to the FP64
// integrand (returns false).
template <int M, int PPL>
__device__ __forceinline__ bool sov_mixed_normal(const SovHead &H, const double *b, const double *L, const Lattice &Lt,
                                 const float *tab, double *smean, int lane) {
    if (H.low0 && H.lne0 < -480.0 * LN2) return false;
    Sov32Setup P;
#pragma unroll
    for (int i = 0; i < M; ++i) { P.b[i] = (float)b[i]; P.a[i] = (float)(1.0 / L[i * M + i]); }
#pragma unroll
    for (int i = 0; i < M * M; ++i) P.L[i] = (float)L[i];
    P.e0s = (float)(H.e0 * 4.656612873077393e-10); P.eb0 = (float)H.eb0;
    P.l2e0m31 = (float)(H.lne0 / LN2 - 31.0); P.low0 = H.low0;
    P.e0 = (float)H.e0; P.l2e0 = (float)(H.lne0 / LN2);
    uint32_t zz[M], shfix[M];
    const int sh = 32 - Lt.log2N;
#pragma unroll
    for (int i = 0; i < M - 1; ++i) zz[i] = (uint32_t)Lt.z[i];
    double tot = 0.0;
    for (int s = 0; s < Lt.S; ++s) {
#pragma unroll
        for (int i = 0; i < M - 1; ++i) shfix[i] = (uint32_t)(Lt.shifts[s * LATD + i] * 4294967296.0);
        const float ls = sov_lane_sum32<M, PPL, true>(P, tab, zz, sh, shfix, Lt.N, lane);
        const double ms = wave_sum((double)ls) / (double)Lt.N;
        if (lane == 0) smean[s] = ms;
        tot += ms;
    }
    return tot / Lt.S > 1e-30;
}

// FP64 integrand from the dof tables (the normal limit has its own
// dof-free transforms).
template <int M>
__device__ __forceinline__ void sov_fp64_tab(const SovHead &H, const double *b, const double *L, double nu,
                                             const Lattice &Lt, const double *tab, double *smean, int lane) {
    for (int s = 0; s < Lt.S; ++s) {
        const double ls = isinf(nu) ? sov_lane_sum64_normal<M>(b, L, Lt, s, H.e0, H.eb0, H.lne0, H.low0, lane)
                                    : sov_lane_sum64_tab<M>(b, L, nu, Lt, s, tab, H.e0, H.eb0, H.lne0, H.low0, lane);
        const double ms = wave_sum(ls) / (double)Lt.N;
        if (lane == 0) smean[s] = ms;
    }
}

template <int M>
__device__ __forceinline__ void sov_fp64(const SovHead &H, const double *b, const double *L, double nu, const Lattice &Lt,
                         double *smean, int lane) {
    for (int s = 0; s < Lt.S; ++s) {
        const double ls = isinf(nu) ? sov_lane_sum64_normal<M>(b, L, Lt, s, H.e0, H.eb0, H.lne0, H.low0, lane)
                                    : sov_lane_sum64<M>(b, L, nu, Lt, s, H.e0, H.eb0, H.lne0, H.low0, lane);
        const double ms = wave_sum(ls) / (double)Lt.N;
        if (lane == 0) smean[s] = ms;
    }
}

}  // namespace cfust
