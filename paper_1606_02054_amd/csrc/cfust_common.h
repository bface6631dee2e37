// cfust_common.h -- layouts shared by the HIP kernels and the host side of the
// library (private; the public boundary is include/cfust.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/cfust.h"

namespace cfust {

constexpr int MAXP = CFUST_MAX_P;
constexpr int MAXQ = CFUST_MAX_Q;
constexpr int MAXG = CFUST_MAX_G;
constexpr int LATD = CFUST_LATTICE_DIM;
constexpr int MAXS = CFUST_MAX_SHIFTS;
constexpr int MAXPAIR = MAXQ * (MAXQ - 1) / 2;
constexpr int MAXJ = 2 + MAXQ + MAXPAIR;          // integrals per (obs, comp)
constexpr int NDOF = MAXQ + 2;                    // dofs nu+p .. nu+p+q+1 per component

// The dof-free FP32 table of the normal limit (compact layout: rows of 7
// monomial coefficients plus one pad float):
//   rows 0..7  : log2 Phi(-v) on the 8 intervals [c(2^k - 1), c(2^{k+1} - 1)]
//                of v, c = 1/4;
//   rows 8..18 : Phi^-1(2^-(lam+1)) on the 11 intervals of lambda of the same
//                form, lambda = -log2(2p);
// each row a polynomial in the float mantissa in [1/2, 1) of v + 1/4 (resp.
// lambda + 1/4).
constexpr int TAB_CDF_ROWS = 8;
constexpr int TAB_INV_ROWS = 11;
constexpr int TAB_ROWS = 20;                      // 8 + 11 + 1 pad row
constexpr int TAB_FLOATS = TAB_ROWS * 8;          // 160 floats per dof
constexpr float INV_LAMBDA_MAX = 511.0f;

// The FP32 tables of the t law ("fine" layout, one slot per dof; the E-step and
// the batched T_m kernels), the
// same two functions on narrower intervals, degree 3, so a lookup reads one
// 16-byte row and takes three FMAs:
//   rows 0..63   : H(tau) on 64 equal intervals of tau, a cubic in the
//                  position inside the interval (fraction of 64 tau);
//   rows 64..191 : log2 tau against lambda on the 9 octaves of lambda + 1 =
//                  -log2 p in [1, 512), each cut into 8 equal parts, a cubic
//                  in the position inside the part (the low 20 mantissa bits
//                  of log2 p).  The part's row is the low 4 bits of the
//                  exponent of log2 p and its top 3 mantissa bits, so no
//                  offset is subtracted in the lookup: octaves 2^1 .. 2^8
//                  (exponents 128..135) are rows 64 + 0..63, octave 2^0
//                  (exponent 127) rows 64 + 120..127, and rows 64 + 64..119
//                  are unused (zero).
// A normal-limit slot (dof infinite) holds the dof-free table above in its
// first TAB_FLOATS floats.
constexpr int TABF_CDF_ROWS = 64;
constexpr int TABF_INV_OCTAVES = 9;
constexpr int TABF_INV_PARTS = 8;
constexpr int TABF_INV_ROWS = TABF_INV_OCTAVES * TABF_INV_PARTS;  // 72 rows with values
constexpr int TABF_INV_SLOTS = 128;                               // rows they span
constexpr int TABF_FLOATS = 4 * (TABF_CDF_ROWS + TABF_INV_SLOTS); // 768 floats per dof
static_assert(TABF_INV_OCTAVES <= 16 && TABF_INV_PARTS == 8, "octave rows are indexed by 4 exponent bits");
// Slot of quantile row r (r = 8 octave + part, octave 0 the one of lambda + 1 in [1, 2)).
__host__ __device__ constexpr int tabf_inv_slot(int r) { return (r + 15 * TABF_INV_PARTS) & (TABF_INV_SLOTS - 1); }
static_assert(TABF_FLOATS >= TAB_FLOATS, "a fine slot holds a normal-limit table");

// FP64 tables of the univariate t law for one dof (FP64 integrand), the same
// variables in natural logs, as Chebyshev series of degree TAB64_NC - 1:
//   rows 0..15  : H(tau) = ln T_lower(tau) - a ln(tau (2 - tau)) on 16 equal
//                 intervals of tau in [0,1];
//   rows 16..30 : ln tau as a function of lambda = -log2(2p) on the 15
//                 intervals [c(2^k - 1), c(2^{k+1} - 1)], c = 1/4 (lambda < 8191.75).
// Degree 11 on these intervals keeps H within about 1e-14 of its value for
// every dof from 1 to 210; the quantile rows only start a Newton step.
constexpr int TAB64_NC = 12;
constexpr int TAB64_CDF_ROWS = 16;
constexpr int TAB64_INV_ROWS = 15;
constexpr int TAB64_ROWS = TAB64_CDF_ROWS + TAB64_INV_ROWS;
constexpr int TAB64_DOUBLES = TAB64_ROWS * TAB64_NC;            // 372 doubles per dof
constexpr double TAB64_ZZ_END = 8192.0;                          // 2^(TAB64_INV_ROWS - 2)
// Largest dof the FP64 tables serve (H within ~4e-12 at 1000; the intervals
// cannot follow the boundary layer near tau ~ 1/nu beyond): integrals with a
// larger dof take the exact transforms.
constexpr double TAB64_NU_MAX = 1000.0;

// Per-component quantities that every observation shares (Sec. 2 eq. 4 and the
// conditional pieces of the truncated-t moments).  FP64 unless noted.
struct CompPre {
    double nu;          // nu_h
    double ltp_const;   // lgamma((nu+p)/2) - lgamma(nu/2) - p/2 log(pi nu) - 1/2 log|Omega|
    double digam;       // psi((nu+p)/2)
    double lt1_s;       // log of t_1 normaliser for dof nu+p+2: lgamma((v+1)/2)-lgamma(v/2)-1/2 log(pi v)
    double lt1_s1;      // same for dof nu+p+1
    double LO[MAXP * MAXP];          // chol Omega (lower)
    double B[MAXP * MAXQ];           // Omega^{-1} Delta, [p][q]
    double Lam[MAXQ * MAXQ];         // Lambda
    double LL[MAXQ * MAXQ];          // chol Lambda
    double LC[MAXQ][(MAXQ - 1) * (MAXQ - 1)];   // chol Lambda_{-i|i}
    double LD[MAXPAIR][(MAXQ - 2) * (MAXQ - 2)];// chol Lambda_{-ik|ik}
    double RD[MAXPAIR][(MAXQ - 2) * 2];         // Lambda_{-ik,ik} Lambda_{ik,ik}^{-1}
    double ID[MAXPAIR][3];                      // Lambda_{ik,ik}^{-1}: (00, 01, 11)
    float LLf[MAXQ * MAXQ];                     // FP32 copies for the lattice kernel
    float LCf[MAXQ][(MAXQ - 1) * (MAXQ - 1)];
    float LDf[MAXPAIR][(MAXQ - 2) * (MAXQ - 2)];
    int32_t status;
    int32_t pad;
};

// Integral list of one (observation, component) pair: 0 = A (density CDF,
// dim q, dof nu+p), 1 = B (w numerator, dim q, dof nu+p+2), 2..q+1 = C_i
// (dim q-1, dof nu+p+1), then D_ik for i<k (dim q-2, dof nu+p).
enum IntType : int { INT_A = 0, INT_B = 1, INT_C = 2, INT_D = 3 };

struct IntDesc {
    int type, i, k, pair, m, dofoff;
};

__host__ __device__ inline int npairs(int q) { return q * (q - 1) / 2; }
__host__ __device__ inline int nint_all(int q) { return 2 + q + npairs(q); }

__host__ __device__ inline IntDesc int_desc(int q, int idx) {
    IntDesc d{0, 0, 0, 0, 0, 0};
    if (idx == 0) { d.type = INT_A; d.m = q; d.dofoff = 0; return d; }
    if (idx == 1) { d.type = INT_B; d.m = q; d.dofoff = 2; return d; }
    if (idx < 2 + q) { d.type = INT_C; d.i = idx - 2; d.m = q - 1; d.dofoff = 1; return d; }
    int pr = idx - 2 - q;
    d.type = INT_D; d.pair = pr; d.m = q - 2; d.dofoff = 0;
    int i = 0, r = pr;
    while (r >= q - 1 - i) { r -= q - 1 - i; ++i; }
    d.i = i; d.k = i + 1 + r;
    return d;
}

// Integrals estimated on the lattice are those of dimension >= 2; they are the
// first nint_qmc(q) entries of the list above restricted to m >= 2, which is
// a prefix in the order A, B, C, D because m decreases along the list.
__host__ __device__ inline int nint_qmc(int q) {
    int J = 0;
    if (q >= 2) J += 2;
    if (q >= 3) J += q;
    if (q >= 4) J += npairs(q);
    return J;
}

// Number of M-step sufficient statistics per component.
__host__ __device__ inline int nstat(int p, int q) {
    return 3 + p + q + p * (p + 1) / 2 + p * q + q * (q + 1) / 2;
}

}  // namespace cfust
