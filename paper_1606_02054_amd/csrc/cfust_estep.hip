// cfust_estep.hip -- E-step kernels of the CFUST mixture (Sec. 3.1) and the
// batched multivariate t probabilities.
//
//   k_precompute   per component: Omega = Sigma + Delta Delta^T, chol Omega,
//                  Omega^{-1} Delta, Lambda = I - Delta^T Omega^{-1} Delta
//                  (Sec. 2 eq. 4), chol Lambda and the Cholesky factors of the
//                  conditional matrices Lambda_{-i|i}, Lambda_{-ik|ik} that
//                  the truncated-t moments need; log-density constants.
//   k_tables       per (component, dof): FP32 tables of the t law (mixed mode,
//                  fine layout).
//   k_lattice_coords  the lattice coordinates of every point (mixed mode).
//   k_estep_qmc    one wave per (observation, component, integral): the
//                  lattice estimate of one T_m (the hot loop).
//   k_assemble     one thread per (observation, component): log f_h (eq. 4),
//                  w (eq. 13), e1 (eq. 15), e2, e3 (eqs. 16-17).
//   k_lse          one thread per observation: tau (eq. 12), log f(y_j) and
//                  per-block partial sums of the log-likelihood (eq. 27).
//   k_mvt          one wave per item of mvt_cdf_batch.
#include "cfust_kernels.h"
#include "cfust_sov.h"

namespace cfust {

// ------------------------------------------------------------------ helpers

// Lower Cholesky of an n x n matrix (row-major, stride n), in place on L.
__device__ inline bool chol_inplace(double *A, int n) {
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j <= i; ++j) {
            double s = A[i * n + j];
            for (int k = 0; k < j; ++k) s -= A[i * n + k] * A[j * n + k];
            if (i == j) {
                if (!(s > 0.0)) return false;
                A[i * n + i] = sqrt(s);
            } else {
                A[i * n + j] = s / A[j * n + j];
            }
        }
        for (int j = i + 1; j < n; ++j) A[i * n + j] = 0.0;
    }
    return true;
}

__device__ inline void pair_of(int q, int pr, int &i, int &k) {
    i = 0;
    int r = pr;
    while (r >= q - 1 - i) { r -= q - 1 - i; ++i; }
    k = i + 1 + r;
}

__device__ inline int pair_index(int q, int i, int k) {  // i < k
    return i * (2 * q - i - 1) / 2 + (k - i - 1);
}

// ------------------------------------------------------------ precompute ---

// Component h of one parameter set; a block of 64 threads.
__device__ inline void precompute_body(const double *__restrict__ pi, const double *__restrict__ Sigma,
                                       const double *__restrict__ Delta, const double *__restrict__ nu, int p,
                                       int q, CompPre *__restrict__ pre, int h) {
    CompPre &P = pre[h];
    __shared__ double Lam[MAXQ * MAXQ];
    __shared__ int st;
    if (threadIdx.x == 0) {
        int status = 0;
        const double v = nu[h];
        // nu = +infinity is the normal limit of the family (CFUSN)
        if (!(v > 0.0) || !(pi[h] >= 0.0) || !isfinite(pi[h])) status |= CFUST_DEV_BADPARAM;
        double Om[MAXP * MAXP];
        const double *Sg = Sigma + (size_t)h * p * p;
        const double *Dl = Delta + (size_t)h * p * q;
        for (int i = 0; i < p; ++i)
            for (int k = 0; k < p; ++k) {
                double s = Sg[i * p + k];
                for (int l = 0; l < q; ++l) s += Dl[i * q + l] * Dl[k * q + l];
                Om[i * p + k] = s;
            }
        // symmetrise (Sigma is symmetric in exact arithmetic)
        for (int i = 0; i < p; ++i)
            for (int k = 0; k < i; ++k) Om[i * p + k] = Om[k * p + i] = 0.5 * (Om[i * p + k] + Om[k * p + i]);
        double Lo[MAXP * MAXP];
        for (int i = 0; i < p * p; ++i) Lo[i] = Om[i];
        if (!chol_inplace(Lo, p)) { status |= CFUST_DEV_NOTSPD_OMEGA; for (int i = 0; i < p; ++i) Lo[i * p + i] = 1.0; }
        double logdet = 0.0;
        for (int i = 0; i < p; ++i) logdet += 2.0 * log(Lo[i * p + i]);
        for (int i = 0; i < p * p; ++i) P.LO[i] = Lo[i];
        // B = Omega^{-1} Delta: forward then backward substitution per column
        double Bm[MAXP * MAXQ];
        for (int c = 0; c < q; ++c) {
            for (int i = 0; i < p; ++i) {
                double s = Dl[i * q + c];
                for (int k = 0; k < i; ++k) s -= Lo[i * p + k] * Bm[k * q + c];
                Bm[i * q + c] = s / Lo[i * p + i];
            }
            for (int i = p - 1; i >= 0; --i) {
                double s = Bm[i * q + c];
                for (int k = i + 1; k < p; ++k) s -= Lo[k * p + i] * Bm[k * q + c];
                Bm[i * q + c] = s / Lo[i * p + i];
            }
        }
        for (int i = 0; i < p * q; ++i) P.B[i] = Bm[i];
        for (int i = 0; i < q; ++i)
            for (int k = 0; k < q; ++k) {
                double s = (i == k) ? 1.0 : 0.0;
                for (int l = 0; l < p; ++l) s -= Dl[l * q + i] * Bm[l * q + k];
                Lam[i * q + k] = s;
            }
        for (int i = 0; i < q; ++i)
            for (int k = 0; k < i; ++k) Lam[i * q + k] = Lam[k * q + i] = 0.5 * (Lam[i * q + k] + Lam[k * q + i]);
        double LL[MAXQ * MAXQ];
        for (int i = 0; i < q * q; ++i) { LL[i] = Lam[i]; P.Lam[i] = Lam[i]; }
        if (!chol_inplace(LL, q)) { status |= CFUST_DEV_NOTSPD_LAMBDA; for (int i = 0; i < q; ++i) LL[i * q + i] = 1.0; }
        for (int i = 0; i < q * q; ++i) { P.LL[i] = LL[i]; P.LLf[i] = (float)LL[i]; }
        P.nu = v;
        P.ltp_const = isinf(v) ? -0.5 * p * log(2.0 * M_PI) - 0.5 * logdet
                               : lgamma(0.5 * (v + p)) - lgamma(0.5 * v) - 0.5 * p * log(M_PI * v) - 0.5 * logdet;
        P.digam = isinf(v) ? 0.0 : dm_digamma(0.5 * (v + p));
        P.lt1_s = dm_lt1_const(v + p + 2.0);
        P.lt1_s1 = dm_lt1_const(v + p + 1.0);
        st = status;
    }
    __syncthreads();
    const int t = threadIdx.x;
    int mystat = 0;
    if (t < q && q >= 2) {   // Lambda_{-i|i}
        const int i = t, m = q - 1;
        double A[(MAXQ - 1) * (MAXQ - 1)];
        int r = 0;
        for (int k = 0; k < q; ++k) {
            if (k == i) continue;
            int c = 0;
            for (int l = 0; l < q; ++l) {
                if (l == i) continue;
                A[r * m + c] = Lam[k * q + l] - Lam[k * q + i] * Lam[i * q + l] / Lam[i * q + i];
                ++c;
            }
            ++r;
        }
        if (!chol_inplace(A, m)) { mystat |= CFUST_DEV_NOTSPD_LAMBDA; for (int d = 0; d < m; ++d) A[d * m + d] = 1.0; }
        for (int e = 0; e < m * m; ++e) { P.LC[i][e] = A[e]; P.LCf[i][e] = (float)A[e]; }
    }
    if (t < npairs(q)) {     // Lambda_{-ik|ik}
        int i, k;
        pair_of(q, t, i, k);
        const double a00 = Lam[i * q + i], a01 = Lam[i * q + k], a11 = Lam[k * q + k];
        const double det = a00 * a11 - a01 * a01;
        const double i00 = a11 / det, i01 = -a01 / det, i11 = a00 / det;
        P.ID[t][0] = i00; P.ID[t][1] = i01; P.ID[t][2] = i11;
        const int m = q - 2;
        double Rg[(MAXQ - 2) * 2];
        int r = 0;
        for (int l = 0; l < q; ++l) {
            if (l == i || l == k) continue;
            Rg[r * 2 + 0] = Lam[l * q + i] * i00 + Lam[l * q + k] * i01;
            Rg[r * 2 + 1] = Lam[l * q + i] * i01 + Lam[l * q + k] * i11;
            ++r;
        }
        double A[(MAXQ - 2) * (MAXQ - 2)];
        r = 0;
        for (int l = 0; l < q; ++l) {
            if (l == i || l == k) continue;
            int c = 0;
            for (int u = 0; u < q; ++u) {
                if (u == i || u == k) continue;
                A[r * m + c] = Lam[l * q + u] - Rg[r * 2 + 0] * Lam[i * q + u] - Rg[r * 2 + 1] * Lam[k * q + u];
                ++c;
            }
            ++r;
        }
        // symmetrise before factorising
        for (int a = 0; a < m; ++a)
            for (int b = 0; b < a; ++b) A[a * m + b] = A[b * m + a] = 0.5 * (A[a * m + b] + A[b * m + a]);
        for (int e = 0; e < 2 * m; ++e) P.RD[t][e] = Rg[e];
        if (m > 0 && !chol_inplace(A, m)) { mystat |= CFUST_DEV_NOTSPD_LAMBDA; for (int d = 0; d < m; ++d) A[d * m + d] = 1.0; }
        for (int e = 0; e < m * m; ++e) { P.LD[t][e] = A[e]; P.LDf[t][e] = (float)A[e]; }
    }
    // fold the per-thread status bits (no atomics: a shared-memory tree)
    __shared__ int sst[64];
    sst[t] = mystat;
    __syncthreads();
    if (t == 0) {
        int s = st;
        for (int u = 0; u < 64; ++u) s |= sst[u];
        P.status = s;
    }
}

__global__ __launch_bounds__(64) void k_precompute(const double *__restrict__ pi, const double *__restrict__ Sigma,
                                                   const double *__restrict__ Delta,
                                                   const double *__restrict__ nu, int p, int q,
                                                   CompPre *__restrict__ pre) {
    precompute_body(pi, Sigma, Delta, nu, p, q, pre, blockIdx.x);
}

// Fold the per-component status words into the caller's status word.
__global__ void k_status_fold(const CompPre *__restrict__ pre, int g, int32_t *__restrict__ status) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        int s = status[0];
        for (int h = 0; h < g; ++h) s |= pre[h].status;
        status[0] = s;
    }
}

// --------------------------------------------------------------- tables ----

// Node n of row `row` of the dof-free normal table (compact layout, 7 nodes
// per row): CDF rows hold log2 Phi(-v) on geometric intervals of v + 1/4,
// quantile rows Phi^-1(2^-(lam+1)) on those of lam + 1/4.
__device__ inline double normal_node_value(int row, int n) {
    const double x = cos(M_PI * (n + 0.5) / 7.0);
    const int k = row < TAB_CDF_ROWS ? row : row - TAB_CDF_ROWS;
    const double w = 0.25 * (double)(1 << k);
    const double v = w - 0.25 + w * 0.5 * (x + 1.0);
    return row < TAB_CDF_ROWS ? dm_lnPhi_lower(-v) / LN2 : dm_ninv_lower(-(v + 1.0) * LN2);
}

// Row of the compact normal table: the Chebyshev fit of the 7 node values on
// x in [-1, 1], stored as monomial coefficients in the lookup's own variable
// v, x = alpha v + beta (v = the float mantissa in [1/2, 1) of the geometric
// rows, alpha = 4, beta = -3), so a lookup evaluates the polynomial at v
// directly.
// cos7: the 7 x 7 cosines cos(pi j (n + 1/2) / 7) at [j][n], or null to compute them here.
__device__ inline void table_fit_row(const double *f, float *dst, double alpha, double beta,
                                     const double *cos7 = nullptr) {
    double c[7];
    for (int j = 0; j < 7; ++j) {
        double sacc = 0.0;
        for (int n = 0; n < 7; ++n) sacc += f[n] * (cos7 ? cos7[7 * j + n] : cos(M_PI * j * (n + 0.5) / 7.0));
        c[j] = sacc * (2.0 / 7.0);
    }
    c[0] *= 0.5;
    double mono[7] = {0, 0, 0, 0, 0, 0, 0};
    double Tm2[7] = {1, 0, 0, 0, 0, 0, 0}, Tm1[7] = {0, 1, 0, 0, 0, 0, 0}, Tj[7];
    for (int i = 0; i < 7; ++i) mono[i] = c[0] * Tm2[i] + c[1] * Tm1[i];
    for (int j = 2; j < 7; ++j) {
        for (int i = 0; i < 7; ++i) Tj[i] = (i > 0 ? 2.0 * Tm1[i - 1] : 0.0) - Tm2[i];
        for (int i = 0; i < 7; ++i) { mono[i] += c[j] * Tj[i]; Tm2[i] = Tm1[i]; Tm1[i] = Tj[i]; }
    }
    double r[7] = {0, 0, 0, 0, 0, 0, 0};             // r(v) = sum_i mono_i (alpha v + beta)^i, Horner in x
    for (int i = 6; i >= 0; --i) {
        for (int k = 6; k >= 1; --k) r[k] = alpha * r[k - 1] + beta * r[k];
        r[0] = beta * r[0] + mono[i];
    }
    for (int i = 0; i < 7; ++i) dst[i] = (float)r[i];
    dst[7] = 0.0f;
}

constexpr int TAB_NODES = (TAB_CDF_ROWS + TAB_INV_ROWS) * 7;   // 133
constexpr int TABF_NODES = (TABF_CDF_ROWS + TABF_INV_ROWS) * 4; // 544 node values per finite-dof slot

// Row of a fine-layout table (cubic): the Chebyshev fit of the 4 node values
// at x_n = cos(pi (n + 1/2) / 4) on [-1, 1], stored as monomial coefficients
// in the row's position v = (x + 1) / 2 in [0, 1).  cos4[j][n] = cos(pi j (n + 1/2) / 4).
__device__ inline void table_fit_row4(const double *f, float *dst, const double *cos4) {
    double c[4];
    for (int j = 0; j < 4; ++j) {
        double acc = 0.0;
        for (int n = 0; n < 4; ++n) acc += f[n] * cos4[4 * j + n];
        c[j] = 0.5 * acc;
    }
    c[0] *= 0.5;
    // c0 T0 + c1 T1 + c2 T2 + c3 T3 in powers of x, then x = 2v - 1
    const double m0 = c[0] - c[2], m1 = c[1] - 3.0 * c[3], m2 = 2.0 * c[2], m3 = 4.0 * c[3];
    dst[0] = (float)(m0 - m1 + m2 - m3);
    dst[1] = (float)(2.0 * m1 - 4.0 * m2 + 6.0 * m3);
    dst[2] = (float)(4.0 * m2 - 12.0 * m3);
    dst[3] = (float)(8.0 * m3);
}

// The cosines of the Chebyshev fits, computed once per block into LDS:
// cos64[j][n] = cos(pi j (n + 1/2) / TAB64_NC), cos7[j][n] and cos4[j][n]
// likewise for 7 and 4 nodes.  Every thread of the block takes part; a
// barrier follows.
__device__ inline void fit_cosines(double *cos64, double *cos7, double *cos4 = nullptr) {
    for (int t = threadIdx.x; t < TAB64_NC * TAB64_NC; t += blockDim.x)
        cos64[t] = cos(M_PI * (t / TAB64_NC) * ((t % TAB64_NC) + 0.5) / (double)TAB64_NC);
    if (cos7)
        for (int t = threadIdx.x; t < 49; t += blockDim.x) cos7[t] = cos(M_PI * (t / 7) * ((t % 7) + 0.5) / 7.0);
    if (cos4)
        for (int t = threadIdx.x; t < 16; t += blockDim.x) cos4[t] = cos(M_PI * (t / 4) * ((t % 4) + 0.5) / 4.0);
    __syncthreads();
}

// Chebyshev coefficients of rows [row0, row0 + nrows) from their TAB64_NC
// node values in fv (same row layout), one thread per coefficient.
__device__ inline void cheb_fit64_rows(const double *fv, double *c, int row0, int nrows, const double *cos64) {
    for (int u = threadIdx.x; u < nrows * TAB64_NC; u += blockDim.x) {
        const int row = row0 + u / TAB64_NC, j = u % TAB64_NC;
        const double *f = fv + row * TAB64_NC;
        double acc = 0.0;
        for (int n = 0; n < TAB64_NC; ++n) acc += f[n] * cos64[j * TAB64_NC + n];
        c[row * TAB64_NC + j] = acc * (j == 0 ? 1.0 : 2.0) / (double)TAB64_NC;
    }
}

// First step of both table builds (finite dof): the FP64 CDF rows of dof nu
// into h64 (LDS), one continued fraction per node and thread; fv is LDS
// scratch for the node values.  Every thread of the block takes part.
__device__ inline void build_cdf64(double nu, double *fv, double *h64, const double *cos64) {
    const double a = 0.5 * nu, lb = dm_lbeta_half(a);
    for (int t = threadIdx.x; t < TAB64_CDF_ROWS * TAB64_NC; t += blockDim.x) {
        const int row = t / TAB64_NC, n = t % TAB64_NC;
        const double x = cos(M_PI * (n + 0.5) / (double)TAB64_NC);
        const double tau = (row + 0.5 * (x + 1.0)) / (double)TAB64_CDF_ROWS;
        const double s = 1.0 - tau;
        fv[t] = dm_H_lower(tau * (2.0 - tau), s * s, a, lb);
    }
    __syncthreads();
    cheb_fit64_rows(fv, h64, 0, TAB64_CDF_ROWS, cos64);
    __syncthreads();
}

// Node n of row `row` of a fine-layout table (finite dof) from the FP64 CDF
// rows: H in log2 units on 64 equal intervals of tau, and log2 tau of the
// quantile solved on those rows at lambda + 1 = 2^k (1 + (part + v)/8) in
// part `part` of octave k.
__device__ inline double tablef_node_from64(double nu, const double *h64, int row, int n) {
    const double v = 0.5 * (cos(M_PI * (n + 0.5) / 4.0) + 1.0);
    if (row < TABF_CDF_ROWS) return tab64_H(h64, (row + v) / (double)TABF_CDF_ROWS) / LN2;
    const int r = row - TABF_CDF_ROWS, k = r / TABF_INV_PARTS, part = r % TABF_INV_PARTS;
    const double lam = ldexp(1.0 + (part + v) / (double)TABF_INV_PARTS, k) - 1.0;
    const double a = 0.5 * nu;
    return tab64_l_solve(h64, -(lam + 1.0) * LN2, a, dm_lbeta_half(a)) / LN2;
}

// One table slot (fine layout) of dof nu, written by a block of 192 threads.
// Finite dof: the FP64 CDF rows first, then the 136 x 4 nodes from them, one
// thread per row fitting it into its slot row (the quantile rows at
// tabf_inv_slot, the unused slot rows zero); infinite dof (normal limit): the
// dof-free closed forms, in the compact layout at the start of the slot, the
// rest of the slot zero.  Every thread of the block takes part.
__device__ inline void table_slot_body(double nu, float *__restrict__ dst) {
    __shared__ double fv[TABF_NODES];
    __shared__ double fv64[TAB64_CDF_ROWS * TAB64_NC], h64[TAB64_CDF_ROWS * TAB64_NC];
    __shared__ double cos64[TAB64_NC * TAB64_NC], cos7[49], cos4[16];
    const int t = threadIdx.x;
    fit_cosines(cos64, cos7, cos4);
    if (isinf(nu)) {
        if (t < TAB_NODES) fv[t] = normal_node_value(t / 7, t % 7);
        __syncthreads();
        if (t < TAB_CDF_ROWS + TAB_INV_ROWS) table_fit_row(fv + 7 * t, dst + 8 * t, 4.0, -3.0, cos7);
        for (int u = 8 * (TAB_CDF_ROWS + TAB_INV_ROWS) + t; u < TABF_FLOATS; u += blockDim.x) dst[u] = 0.0f;
    } else {
        build_cdf64(nu, fv64, h64, cos64);
        for (int u = t; u < TABF_NODES; u += blockDim.x) fv[u] = tablef_node_from64(nu, h64, u / 4, u % 4);
        __syncthreads();
        if (t < TABF_CDF_ROWS + TABF_INV_ROWS) {
            const int row = t < TABF_CDF_ROWS ? t : TABF_CDF_ROWS + tabf_inv_slot(t - TABF_CDF_ROWS);
            table_fit_row4(fv + 4 * t, dst + 4 * row, cos4);
        }
        for (int u = 4 * (TABF_CDF_ROWS + tabf_inv_slot(TABF_INV_ROWS)) + t;
             u < 4 * (TABF_CDF_ROWS + tabf_inv_slot(0)); u += blockDim.x)
            dst[u] = 0.0f;
    }
}

// Block `bid` = (component, dof offset) of one parameter set.
__device__ inline void tables_body(const CompPre *__restrict__ pre, int p, int ndof, float *__restrict__ tabs,
                                   int bid) {
    const int h = bid / ndof, off = bid % ndof;
    table_slot_body(pre[h].nu + p + off, tabs + ((size_t)h * NDOF + off) * TABF_FLOATS);
}

__global__ __launch_bounds__(192) void k_tables(const CompPre *__restrict__ pre, int p, int ndof,
                                                float *__restrict__ tabs) {
    tables_body(pre, p, ndof, tabs, blockIdx.x);
}

// Block `bid` = (component, dof offset): the FP64 CDF rows, then every
// quantile node solved on them, one per thread, and one thread per row for
// the fits.  A component with infinite dof (normal limit) has no t tables:
// zeros.
__device__ inline void table64_slot_body(double nu, double *__restrict__ dst) {
    __shared__ double fv64[TAB64_DOUBLES], t64[TAB64_DOUBLES], cos64[TAB64_NC * TAB64_NC];
    if (isinf(nu)) {
        for (int t = threadIdx.x; t < TAB64_DOUBLES; t += blockDim.x) dst[t] = 0.0;
        return;
    }
    fit_cosines(cos64, nullptr);
    build_cdf64(nu, fv64, t64, cos64);
    const double a = 0.5 * nu, lb = dm_lbeta_half(a);
    constexpr int Q0 = TAB64_CDF_ROWS * TAB64_NC;
    for (int t = threadIdx.x; t < TAB64_INV_ROWS * TAB64_NC; t += blockDim.x) {
        const int row = t / TAB64_NC, n = t % TAB64_NC;
        const double x = cos(M_PI * (n + 0.5) / (double)TAB64_NC);
        const double w = 0.25 * (double)(1 << row);
        const double lam = w - 0.25 + w * 0.5 * (x + 1.0);
        fv64[Q0 + t] = tab64_l_solve(t64, -(lam + 1.0) * LN2, a, lb);
    }
    __syncthreads();
    cheb_fit64_rows(fv64, t64, TAB64_CDF_ROWS, TAB64_INV_ROWS, cos64);
    __syncthreads();
    for (int t = threadIdx.x; t < TAB64_DOUBLES; t += blockDim.x) dst[t] = t64[t];
}

__device__ inline void tables64_body(const CompPre *__restrict__ pre, int p, int ndof, double *__restrict__ tabs,
                                     int bid) {
    const int h = bid / ndof, off = bid % ndof;
    table64_slot_body(pre[h].nu + p + off, tabs + ((size_t)h * NDOF + off) * TAB64_DOUBLES);
}

__global__ __launch_bounds__(192) void k_tables64(const CompPre *__restrict__ pre, int p, int ndof,
                                                  double *__restrict__ tabs) {
    tables64_body(pre, p, ndof, tabs, blockIdx.x);
}

// ------------------------------------------------------------- geometry ----

// r = y_j - mu_h, d = r^T Omega^{-1} r, c = Delta^T Omega^{-1} r (Sec. 2 eq. 4).
__device__ inline void pair_geometry(const double *__restrict__ y, int n, int p, int q, int j,
                                     const double *__restrict__ mu, const CompPre &P, double *c, double &d) {
    double r[MAXP], v[MAXP];
    for (int i = 0; i < p; ++i) r[i] = y[(size_t)i * n + j] - mu[i];
    d = 0.0;
    for (int i = 0; i < p; ++i) {
        double s = r[i];
        for (int k = 0; k < i; ++k) s -= P.LO[i * p + k] * v[k];
        v[i] = s / P.LO[i * p + i];
        d += v[i] * v[i];
    }
    for (int l = 0; l < q; ++l) {
        double s = 0.0;
        for (int k = 0; k < p; ++k) s += P.B[k * q + l] * r[k];
        c[l] = s;
    }
}

// The same with caller-provided storage v[p] (the forward-substitution
// vector) and r recomputed where needed: no private arrays, so an
// out-of-line caller keeps no stack frame (v and c may live in LDS).
__device__ inline void pair_geometry_ws(const double *__restrict__ y, int n, int p, int q, int j,
                                        const double *__restrict__ mu, const CompPre &P, double *c, double &d,
                                        double *v) {
    d = 0.0;
    for (int i = 0; i < p; ++i) {
        double s = y[(size_t)i * n + j] - mu[i];
        for (int k = 0; k < i; ++k) s -= P.LO[i * p + k] * v[k];
        v[i] = s / P.LO[i * p + i];
        d += v[i] * v[i];
    }
    for (int l = 0; l < q; ++l) {
        double s = 0.0;
        for (int k = 0; k < p; ++k) s += P.B[k * q + l] * (y[(size_t)k * n + j] - mu[k]);
        c[l] = s;
    }
}

// Standardised limits of integral D of the pair: T_m(b; 0, L L^T, nu0) with L
// a per-component Cholesky factor (stride m) and the per-observation scale
// folded into b.  Returns L (FP64).
__device__ inline const double *integral_limits(const IntDesc &D, const CompPre &P, int p, int q,
                                                const double *c, double d, double *b) {
    const double v = P.nu;                       // infinite: the normal limit, every ratio below is 1
    const double nus = v + p + 2.0;
    const double sc = dm_ratio(v, d, p + 2.0);   // (v + d) / nus
    if (D.type == INT_A || D.type == INT_B) {
        const double f = sqrt(dm_ratio(v, D.type == INT_A ? p : p + 2.0, d));
        for (int l = 0; l < q; ++l) b[l] = c[l] * f;
        return P.LL;
    }
    if (D.type == INT_C) {
        const int i = D.i;
        const double Lii = P.Lam[i * q + i];
        const double kap = dm_ratio(nus, c[i] * c[i] / (sc * Lii), -1.0);
        const double f = 1.0 / sqrt(kap * sc);
        int r = 0;
        for (int k = 0; k < q; ++k) {
            if (k == i) continue;
            b[r++] = (c[k] - P.Lam[k * q + i] / Lii * c[i]) * f;
        }
        return P.LC[i];
    }
    const int i = D.i, k = D.k, t = D.pair;
    const double Qf = (c[i] * c[i] * P.ID[t][0] + 2.0 * c[i] * c[k] * P.ID[t][1] + c[k] * c[k] * P.ID[t][2]) / sc;
    const double kk = dm_ratio(nus, Qf, -2.0);
    const double f = 1.0 / sqrt(kk * sc);
    int r = 0;
    for (int l = 0; l < q; ++l) {
        if (l == i || l == k) continue;
        b[r] = (c[l] - P.RD[t][2 * r] * c[i] - P.RD[t][2 * r + 1] * c[k]) * f;
        ++r;
    }
    return P.LD[t];
}

// --------------------------------------------------------------- lattice ---

// FP64 prologue and epilogue of one integral.  They are kept out of line:
// inlined into a loop over items (the persistent kernel), their FP64
// constants would be hoisted out of the loop and stay live in vector
// registers through the lattice loop, halving the occupancy.  Their work
// arrays are a per-wave LDS slot (the values are the same in every lane of
// the wave) and their arguments are scalars, so they need no stack frame.
struct WaveItem {
    double v[MAXP];      // forward-substitution vector of the pair's geometry
    double c[MAXQ];      // Delta^T Omega^-1 (y - mu)
    double b[MAXQ];      // standardised limits of the integral
    SovHead H;           // first SOV factor
    const double *L;     // Cholesky factor of the integral (FP64, stride m)
    double nu0;          // dof of the integral
};

// Limits of integral idx of pair (j, h); with fp64_head also the first SOV
// factor in FP64 (otherwise the caller takes it from the FP32 tables).
__device__ __attribute__((noinline)) void item_head(const double *y, const double *mu, const CompPre *pre, int n,
                                                    int p, int q, int h, int idx, int j, WaveItem *w,
                                                    bool fp64_head) {
    const IntDesc D = int_desc(q, idx);
    const CompPre &P = pre[h];
    double d;
    pair_geometry_ws(y, n, p, q, j, mu + (size_t)h * p, P, w->c, d, w->v);
    w->L = integral_limits(D, P, p, q, w->c, d, w->b);
    w->nu0 = P.nu + p + D.dofoff;
    if (fp64_head || isinf(w->nu0)) w->H = sov_head(w->b, w->L, w->nu0);   // normal limit: no tables
}

__device__ __attribute__((noinline)) void item_head_tab(WaveItem *w, const float *tab) {
    w->H = sov_head_tab(w->b, w->L, w->nu0, tab);
}

struct ItemResult {
    double est, se, lnest;
};

__device__ __attribute__((noinline)) ItemResult item_finish(const WaveItem *w, const double *smean, int S) {
    ItemResult r;
    sov_finish(w->H, smean, S, &r.est, &r.se, &r.lnest);
    return r;
}

// Integral idx of pair (observation j, component h), evaluated by one wave.
// MIXED: FP32 integrand with the dof tables in `tab` (LDS), the first factor
// included (log domain, from the table); returns false, writing nothing,
// when the FP32 product underflowed (the item then needs the FP64 integrand).
// w: this wave's LDS work slot.  Lane 0 writes the estimate (and, for idx 0,
// ln A and its standard error).
// !MIXED: with T64 the FP64 integrand reads the FP64 dof tables of the
// integral in tab64 (LDS); without, it uses the exact transforms (the redo
// pass of mixed mode, whose FP32 tables do not serve it).
template <int M, bool MIXED, int PPL, bool T64 = false, bool COORDS = false>
__device__ inline bool qmc_item(const EstepQmcArgs &a, int h, int idx, int j, const float *tab,
                                const double *tab64, double *smean, WaveItem *w, int lane) {
    item_head(a.y, a.mu, a.pre, a.n, a.p, a.q, h, idx, j, w, !MIXED);
    const bool normal = isinf(w->nu0);          // the normal limit of the family (dof infinite)
    if (MIXED && !normal) item_head_tab(w, tab);
    ItemResult r{0.0, 0.0, -INFINITY};
    if (w->H.e0 > 0.0 || w->H.lne0 > -INFINITY) {
        if (MIXED) {
            const bool ok = normal ? sov_mixed_normal<M, PPL>(w->H, w->b, w->L, a.lat, tab, smean, lane)
                                   : sov_mixed<M, PPL, COORDS>(w->H, w->b, w->L, w->nu0, a.lat, tab, smean, lane,
                                                               a.coords, a.coordC);
            if (!ok) return false;
        } else if (T64) {
            sov_fp64_tab<M>(w->H, w->b, w->L, w->nu0, a.lat, tab64, smean, lane);
        } else {
            sov_fp64<M>(w->H, w->b, w->L, w->nu0, a.lat, smean, lane);
        }
        r = item_finish(w, smean, a.lat.S);
    }
    if (lane == 0) {
        const size_t o = ((size_t)h * a.J + idx) * a.n + j;
        a.est[o] = r.est;
        if (idx == 0) {
            a.lnA[(size_t)h * a.n + j] = r.lnest;
            if (a.se) a.se[(size_t)h * a.n + j] = r.se;
        }
    }
    return true;
}

// Stage the FP32 tables (fine layout) of the dofs an integral of dimension M uses.
template <int M>
__device__ inline void load_tables(const float *__restrict__ tabs, int h, int dofoff, float *tab) {
    const float4 *src = reinterpret_cast<const float4 *>(tabs + ((size_t)h * NDOF + dofoff) * TABF_FLOATS);
    float4 *d = reinterpret_cast<float4 *>(tab);
    for (int t = threadIdx.x; t < M * TABF_FLOATS / 4; t += blockDim.x) d[t] = src[t];
}

// True when integral idx of component h (dimension M) uses a finite dof past
// the FP64 tables' range: its items take the exact FP64 transforms.
template <int M>
__device__ inline bool beyond_tab64(const CompPre *__restrict__ pre, int p, int q, int h, int idx) {
    const double nu_hi = pre[h].nu + p + int_desc(q, idx).dofoff + (M - 1);
    return isfinite(nu_hi) && nu_hi > TAB64_NU_MAX;
}

// Stage the FP64 tables of the dofs an integral of dimension M uses.
template <int M>
__device__ inline void load_tables64(const double *__restrict__ tabs64, int h, int dofoff, double *tab64) {
    const double *src = tabs64 + ((size_t)h * NDOF + dofoff) * TAB64_DOUBLES;
    for (int t = threadIdx.x; t < M * TAB64_DOUBLES; t += blockDim.x) tab64[t] = src[t];
}

// Blocks per CU (= waves per SIMD) the FP32 lattice kernels are held to
// (m = 5, 6; no bound elsewhere).  Held to 8 waves, the m = 4 kernel was 1.5%
// faster but spilled its prologue to memory (8 -> 46 MiB of HBM traffic per
// launch of the bench workload), so it keeps 69 VGPRs and 7 waves.
constexpr int fp32_min_blocks(int m) { return m == 5 ? 6 : m == 6 ? 5 : 1; }

// One wave per (observation j, integral idx, component h); 4 observations per
// block share the integral's tables.  MIXED: FP32 integrand, items whose FP32
// product underflows are flagged for the FP64 pass (k_estep_flagged).
// !MIXED: FP64 integrand on the FP64 tables, items whose dof is past the
// tables flagged for the same pass.  The FP32 kernels are held to
// fp32_min_blocks(m) waves per SIMD.
template <int M, bool MIXED, int PPL, bool COORDS = false>
__global__ __launch_bounds__(256, MIXED && PPL == 1 ? fp32_min_blocks(M) : 1) void k_estep_qmc(EstepQmcArgs a) {
    constexpr bool TAB64 = !MIXED;
    __shared__ __align__(16) float tab[MIXED ? M * TABF_FLOATS : 4];
    __shared__ double tab64[TAB64 ? M * TAB64_DOUBLES : 1];
    __shared__ double smean[4][MAXS];
    __shared__ WaveItem witem[4];
    const int h = blockIdx.z, idx = a.idx0 + blockIdx.y;
    if (MIXED) {
        load_tables<M>(a.tabs, h, int_desc(a.q, idx).dofoff, tab);
        __syncthreads();
    }
    if (TAB64 && a.tabs64) {
        load_tables64<M>(a.tabs64, h, int_desc(a.q, idx).dofoff, tab64);
        __syncthreads();
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int j = blockIdx.x * 4 + wave;
    if (j >= a.n) return;
    const size_t o = ((size_t)h * a.J + idx) * a.n + j;
    if (a.need && a.need[o] == 0) {   // answered by the surrogate
        if (lane == 0) a.flag[o] = 0;
        return;
    }
    if (TAB64 && beyond_tab64<M>(a.pre, a.p, a.q, h, idx)) {   // left to the exact pass
        if (lane == 0) a.flag[o] = 1;
        return;
    }
    const bool ok = qmc_item<M, MIXED, PPL, TAB64, COORDS>(a, h, idx, j, tab, tab64, smean[wave], &witem[wave], lane);
    if (lane == 0) a.flag[o] = ok ? 0 : 1;
}

// The flagged items of a launch's integrals (mixed: FP32 underflow; FP64
// mode: a dof past the FP64 tables), evaluated with the exact FP64
// transforms.  Each wave scans 64 consecutive items u of [g][nidx][n] (one
// flag per lane) and evaluates the flagged ones in turn, so a pass with
// nothing flagged costs one coalesced read per 64 items instead of a wave
// per item.
template <int M>
__global__ __launch_bounds__(256) void k_estep_flagged(EstepQmcArgs a, int nidx) {
    __shared__ double smean[4][MAXS];
    __shared__ WaveItem witem[4];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const long long total = (long long)a.g * nidx * a.n;
    const long long u = ((long long)blockIdx.x * 4 + wave) * 64 + lane;
    int flagged = 0;
    size_t o = 0;
    int h = 0, idx = 0, j = 0;
    if (u < total) {
        j = (int)(u % a.n);
        const long long r = u / a.n;
        idx = a.idx0 + (int)(r % nidx);
        h = (int)(r / nidx);
        o = ((size_t)h * a.J + idx) * a.n + j;
        flagged = a.flag[o] != 0;
    }
    uint64_t mask = __ballot(flagged);
    while (mask) {
        const int src = __ffsll((unsigned long long)mask) - 1;
        mask &= mask - 1;
        const int hs = __shfl(h, src), is = __shfl(idx, src), js = __shfl(j, src);
        qmc_item<M, false, 1>(a, hs, is, js, nullptr, nullptr, smean[wave], &witem[wave], lane);
        if (lane == src) a.flag[o] = 0;
    }
}

// Mixed mode, before k_estep_flagged: the flagged items whose dofs are within
// the FP64 tables' range, on the components' FP64 tables (a.tabs64), one
// wave per block scanning 64 items; clears their flags.
template <int M>
__global__ __launch_bounds__(64) void k_estep_flagged64(EstepQmcArgs a, int nidx) {
    __shared__ double tab64[M * TAB64_DOUBLES];
    __shared__ double smean[MAXS];
    __shared__ WaveItem witem;
    const int lane = threadIdx.x;
    const long long total = (long long)a.g * nidx * a.n;
    const long long u = (long long)blockIdx.x * 64 + lane;
    int flagged = 0;
    size_t o = 0;
    int h = 0, idx = 0, j = 0;
    if (u < total) {
        j = (int)(u % a.n);
        const long long r = u / a.n;
        idx = a.idx0 + (int)(r % nidx);
        h = (int)(r / nidx);
        o = ((size_t)h * a.J + idx) * a.n + j;
        flagged = a.flag[o] != 0 && !beyond_tab64<M>(a.pre, a.p, a.q, h, idx);
    }
    uint64_t mask = __ballot(flagged);
    int cur_h = -1, cur_idx = -1;
    while (mask) {
        const int src = __ffsll((unsigned long long)mask) - 1;
        mask &= mask - 1;
        const int hs = __shfl(h, src), is = __shfl(idx, src), js = __shfl(j, src);
        if (hs != cur_h || is != cur_idx) {
            __syncthreads();
            load_tables64<M>(a.tabs64, hs, int_desc(a.q, is).dofoff, tab64);
            __syncthreads();
            cur_h = hs;
            cur_idx = is;
        }
        qmc_item<M, false, 1, true>(a, hs, is, js, nullptr, tab64, smean, &witem, lane);
        if (lane == src) a.flag[o] = 0;
    }
}

// ------------------------------------------------------------- assembly ----

// Value of integral idx of the pair: lattice estimate (m >= 2) or closed form.
__device__ inline double integral_value(const EstepAsmArgs &a, const CompPre &P, int h, int j, int idx,
                                        const double *c, double d) {
    const IntDesc D = int_desc(a.q, idx);
    if (D.m >= 2) return a.est[((size_t)h * a.J + idx) * a.n + j];
    if (D.m == 0) return 1.0;
    double b[MAXQ];
    const double *L = integral_limits(D, P, a.p, a.q, c, d, b);
    return dm_tcdf(b[0] / L[0], P.nu + a.p + D.dofoff);
}

// Pair gid = h * n + j of one parameter set.
__device__ inline void assemble_body(const EstepAsmArgs &a, int gid) {
    if (gid >= a.n * a.g) return;
    const int h = gid / a.n, j = gid % a.n;
    const CompPre &P = a.pre[h];
    const int p = a.p, q = a.q;
    double c[MAXQ], d;
    pair_geometry(a.y, a.n, p, q, j, a.mu + (size_t)h * p, P, c, d);
    const double v = P.nu;
    // ln A: lattice (finite even when A underflows) or closed form
    double lnA;
    if (q >= 2) lnA = a.lnA[(size_t)h * a.n + j];
    else lnA = log(integral_value(a, P, h, j, 0, c, d));
    const double logf = q * LN2 + P.ltp_const + (isinf(v) ? -0.5 * d : -0.5 * (v + p) * log1p(d / v)) + lnA;
    a.logf_comp[(size_t)h * a.n + j] = logf;
    if (a.density_only) return;
    const size_t o = (size_t)h * a.n + j;
    const int nq2 = q * (q + 1) / 2;
    double w = 0.0, e1 = 0.0, e2[MAXQ], e3[MAXQ * (MAXQ + 1) / 2];
    for (int i = 0; i < q; ++i) e2[i] = 0.0;
    for (int i = 0; i < nq2; ++i) e3[i] = 0.0;
    const double A = (q >= 2) ? integral_value(a, P, h, j, 0, c, d) : exp(lnA);
    const double Bv = integral_value(a, P, h, j, 1, c, d);
    // Normal limit: W = 1 for every observation, so w = 1 and e1 = E[log W] = 0
    // whenever the pair has a density, even where A and B are below the FP64
    // range (the lattice keeps ln A finite); the moments below need B.
    if (isinf(v) && isfinite(logf)) w = 1.0;
    if (A > 0.0 && Bv > 0.0 && isfinite(logf)) {
        const double nus = v + p + 2.0, sc = dm_ratio(v, d, p + 2.0);
        if (isinf(v)) {                          // normal limit: W = 1
            w = 1.0;
            e1 = 0.0;
        } else {
            w = (v + p) / (v + d) * Bv / A;                               // eq. (13)
            e1 = w - log(0.5 * (v + d)) - (v + p) / (v + d) + P.digam;    // eq. (15)
        }
        // xi_i and the conditional pieces of each i
        double xi[MAXQ], t1k[MAXQ];
        for (int i = 0; i < q; ++i) {
            const double Rii = sc * P.Lam[i * q + i];
            const double kap = dm_ratio(nus, c[i] * c[i] / Rii, -1.0);
            const double t1 = exp(dm_lt1pdf(c[i], Rii, nus, P.lt1_s));
            t1k[i] = t1 * kap;
            xi[i] = t1k[i] * integral_value(a, P, h, j, 2 + i, c, d);
        }
        // G, column by column
        double G[MAXQ * MAXQ];
        for (int i = 0; i < q; ++i) {
            const double Lii = P.Lam[i * q + i];
            const double kap = dm_ratio(nus, c[i] * c[i] / (sc * Lii), -1.0);
            double bb[MAXQ], xs[MAXQ];
            for (int k = 0; k < q; ++k) bb[k] = c[k] - P.Lam[k * q + i] / Lii * c[i];
            for (int k = 0; k < q; ++k) {
                if (k == i) { xs[k] = 0.0; continue; }
                const double Vkk = kap * sc * (P.Lam[k * q + k] - P.Lam[k * q + i] * P.Lam[i * q + k] / Lii);
                const double kp = dm_ratio(nus - 1.0, bb[k] * bb[k] / Vkk, -1.0);
                const double t1 = exp(dm_lt1pdf(bb[k], Vkk, nus - 1.0, P.lt1_s1));
                const int pr = i < k ? pair_index(q, i, k) : pair_index(q, k, i);
                xs[k] = t1 * kp * integral_value(a, P, h, j, 2 + q + pr, c, d);
            }
            for (int k = 0; k < q; ++k) {
                double g = P.Lam[k * q + i] / Lii * c[i] * xi[i];
                if (k != i) {
                    double vx = 0.0;
                    for (int l = 0; l < q; ++l) {
                        if (l == i) continue;
                        vx += kap * sc * (P.Lam[k * q + l] - P.Lam[k * q + i] * P.Lam[i * q + l] / Lii) * xs[l];
                    }
                    g -= t1k[i] * vx;
                }
                G[k * q + i] = g;
            }
        }
        double M1[MAXQ], M2[MAXQ * MAXQ];
        for (int i = 0; i < q; ++i) {
            double s = 0.0;
            for (int k = 0; k < q; ++k) s += sc * P.Lam[i * q + k] * xi[k];
            M1[i] = -s;
        }
        for (int i = 0; i < q; ++i)
            for (int k = 0; k < q; ++k) {
                double s = 0.0;
                for (int l = 0; l < q; ++l) s += G[i * q + l] * sc * P.Lam[l * q + k];
                M2[i * q + k] = dm_ratio(nus, 0.0, -2.0) * A * sc * P.Lam[i * q + k] - s;
            }
        for (int i = 0; i < q; ++i) e2[i] = w * (c[i] - M1[i] / Bv);
        int t = 0;
        for (int i = 0; i < q; ++i)
            for (int k = i; k < q; ++k, ++t) {
                const double euu = c[i] * c[k] - (c[i] * M1[k] + M1[i] * c[k]) / Bv
                                   + 0.5 * (M2[i * q + k] + M2[k * q + i]) / Bv;
                e3[t] = w * euu;
            }
    }
    if (a.mixed) {
        float *W = (float *)a.w, *E1 = (float *)a.e1, *E2 = (float *)a.e2, *E3 = (float *)a.e3;
        W[o] = (float)w; E1[o] = (float)e1;
        for (int i = 0; i < q; ++i) E2[((size_t)h * q + i) * a.n + j] = (float)e2[i];
        for (int i = 0; i < nq2; ++i) E3[((size_t)h * nq2 + i) * a.n + j] = (float)e3[i];
    } else {
        double *W = (double *)a.w, *E1 = (double *)a.e1, *E2 = (double *)a.e2, *E3 = (double *)a.e3;
        W[o] = w; E1[o] = e1;
        for (int i = 0; i < q; ++i) E2[((size_t)h * q + i) * a.n + j] = e2[i];
        for (int i = 0; i < nq2; ++i) E3[((size_t)h * nq2 + i) * a.n + j] = e3[i];
    }
}

__global__ __launch_bounds__(128) void k_assemble(EstepAsmArgs a) {
    assemble_body(a, blockIdx.x * blockDim.x + threadIdx.x);
}

// ------------------------------------------------------------------ LSE ----

// Block bid (256 observations) of one parameter set; writes partial[bid].
__device__ inline void lse_body(const EstepLseArgs &a, int bid) {
    __shared__ double red[256];
    const int j = bid * 256 + threadIdx.x;
    double lj = 0.0;
    if (j < a.n) {
        double mx = -INFINITY;
        for (int h = 0; h < a.g; ++h) {
            const double v = log(a.pi[h]) + a.logf_comp[(size_t)h * a.n + j];
            mx = fmax(mx, v);
        }
        double l = -INFINITY;
        if (mx > -INFINITY && isfinite(mx)) {
            double s = 0.0;
            for (int h = 0; h < a.g; ++h) s += exp(log(a.pi[h]) + a.logf_comp[(size_t)h * a.n + j] - mx);
            l = mx + log(s);
        }
        if (a.logf_obs) a.logf_obs[j] = l;
        lj = l;
        if (a.tau) {
            const int nq2 = a.q * (a.q + 1) / 2;
            for (int h = 0; h < a.g; ++h) {
                const double t = isfinite(l) ? exp(log(a.pi[h]) + a.logf_comp[(size_t)h * a.n + j] - l) : 0.0;
                a.tau[(size_t)h * a.n + j] = t;
                if (!(t > 0.0) && a.w) {   // no weight: zero the e-terms
                    const size_t o = (size_t)h * a.n + j;
                    if (a.mixed) {
                        ((float *)a.w)[o] = 0.0f; ((float *)a.e1)[o] = 0.0f;
                        for (int i = 0; i < a.q; ++i) ((float *)a.e2)[((size_t)h * a.q + i) * a.n + j] = 0.0f;
                        for (int i = 0; i < nq2; ++i) ((float *)a.e3)[((size_t)h * nq2 + i) * a.n + j] = 0.0f;
                    } else {
                        ((double *)a.w)[o] = 0.0; ((double *)a.e1)[o] = 0.0;
                        for (int i = 0; i < a.q; ++i) ((double *)a.e2)[((size_t)h * a.q + i) * a.n + j] = 0.0;
                        for (int i = 0; i < nq2; ++i) ((double *)a.e3)[((size_t)h * nq2 + i) * a.n + j] = 0.0;
                    }
                }
            }
        }
    }
    red[threadIdx.x] = lj;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) a.partial[bid] = red[0];
}

__global__ __launch_bounds__(256) void k_lse(EstepLseArgs a) {
    lse_body(a, blockIdx.x);
}

// Sum of per-block partials in a fixed order (deterministic).
__device__ inline void sum_partials_body(const double *__restrict__ part, int np, double *__restrict__ out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < np; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

__global__ __launch_bounds__(256) void k_sum_partials(const double *__restrict__ part, int np,
                                                      double *__restrict__ out) {
    sum_partials_body(part, np, out);
}

// ------------------------------------------------------------ mvt batch ----

// Mixed precision, in two kernels: the FP32 tables of every item of a chunk
// (k_mvt_tables, one block per item and dof, into global memory; the
// dof-free normal table once per call), then the lattice sums (k_mvt_qmc,
// one wave per item, reading its tables from LDS) -- the table build and
// its FP64 registers stay out of the integrand's kernel.

// Block (local item, dof offset d) of the chunk starting at item it0.  Items
// with an infinite dof use the shared normal slot and build nothing.
__global__ __launch_bounds__(192) void k_mvt_tables(MvtArgs a, int it0, int M, float *__restrict__ tabs) {
    const int local = blockIdx.x / M, d = blockIdx.x % M;
    const double nu = a.nu[it0 + local];
    if (isinf(nu)) return;
    table_slot_body(nu + d, tabs + ((size_t)local * M + d) * TABF_FLOATS);
}

// The dof-free normal table (one block).
__global__ __launch_bounds__(192) void k_mvt_normal_table(float *__restrict__ slot) {
    table_slot_body(INFINITY, slot);
}

// The item's limits and Cholesky factor, staged in the wave's LDS slot; the
// first SOV factor from the FP32 table (finite dof, tab given) or in FP64
// (normal limit, or tab null).  Out of line for the same reason as item_head.
__device__ __attribute__((noinline)) void mvt_item_head(const MvtArgs &a, int it, int mi, int M, double *b, double *L,
                                                        double nu, const float *tab, SovHead *H) {
    for (int i = 0; i < M; ++i) b[i] = a.b[(size_t)it * M + i];
    for (int i = 0; i < M * M; ++i) L[i] = a.L[(size_t)mi * M * M + i];
    *H = (isinf(nu) || !tab) ? sov_head(b, L, nu) : sov_head_tab(b, L, nu, tab);
}

// FP64 with per-item FP64 tables: FP64 mode, and the items whose FP32 product
// underflowed in mixed mode -- every item with flag 1 whose dofs are within
// the tables' range (infinite dof included: the normal integrand needs no
// table); the others keep their flag for the exact transforms (k_mvt).
__device__ inline bool mvt_tab64_item(double nu, int M) { return isinf(nu) || nu + (M - 1) <= TAB64_NU_MAX; }

// Block (local item, dof offset d) of the chunk at it0: the FP64 table of
// dof nu + d of a flagged item.
__global__ __launch_bounds__(192) void k_mvt_tables64(MvtArgs a, int it0, int M, double *__restrict__ tabs64) {
    const int local = blockIdx.x / M, d = blockIdx.x % M;
    const int it = it0 + local;
    if (a.flag[it] == 0) return;
    const double nu = a.nu[it];
    if (isinf(nu) || !mvt_tab64_item(nu, M)) return;
    table64_slot_body(nu + d, tabs64 + ((size_t)local * M + d) * TAB64_DOUBLES);
}

// One flagged item per wave (blocks of 64 threads): the FP64 integrand on the
// item's FP64 tables in LDS; clears the flag.
template <int M>
__global__ __launch_bounds__(64) void k_mvt_fp64tab(MvtArgs a, int it0, const double *__restrict__ tabs64) {
    __shared__ double tab64[M * TAB64_DOUBLES];
    __shared__ double smean[MAXS];
    __shared__ double bs[M], Ls[M * M];
    __shared__ SovHead Hs;
    const int lane = threadIdx.x;
    const int it = it0 + blockIdx.x;
    if (a.flag[it] == 0) return;
    const double nu = a.nu[it];
    if (!mvt_tab64_item(nu, M)) return;
    const int mi = a.mat_idx[it];
    if (mi < 0 || mi >= a.nmat) {   // invalid matrix index: NaN result, no access
        if (lane == 0) {
            a.p[it] = NAN; if (a.logp) a.logp[it] = NAN; if (a.se) a.se[it] = NAN;
            a.flag[it] = 0;
        }
        return;
    }
    if (!isinf(nu)) {
        const double *src = tabs64 + (size_t)blockIdx.x * M * TAB64_DOUBLES;
        for (int t = lane; t < M * TAB64_DOUBLES; t += 64) tab64[t] = src[t];
    }
    if (lane == 0) mvt_item_head(a, it, mi, M, bs, Ls, nu, nullptr, &Hs);
    __syncthreads();
    const SovHead H = Hs;
    double est = 0.0, se = 0.0, lnest = -INFINITY;
    if (H.e0 > 0.0 || H.lne0 > -INFINITY) {
        sov_fp64_tab<M>(H, bs, Ls, nu, a.lat, tab64, smean, lane);
        sov_finish(H, smean, a.lat.S, &est, &se, &lnest);
    }
    if (lane == 0) {
        a.p[it] = est;
        if (a.logp) a.logp[it] = lnest;
        if (a.se) a.se[it] = se;
        a.flag[it] = 0;
    }
}

// One wave per item of the chunk (blocks of 64 threads).  Writes the item's
// flag: 1 when the FP32 product underflowed (the FP64 pass redoes it), else 0.
template <int M>
__global__ __launch_bounds__(64) void k_mvt_qmc(MvtArgs a, int it0, const float *__restrict__ tabs,
                                                const float *__restrict__ ntab, const float *__restrict__ coords, int C) {
    __shared__ __align__(16) float tab[M * TABF_FLOATS];
    __shared__ double smean[MAXS];
    __shared__ double bs[M], Ls[M * M];
    __shared__ SovHead Hs;
    const int lane = threadIdx.x;
    const int it = it0 + blockIdx.x;
    const int mi = a.mat_idx[it];
    if (mi < 0 || mi >= a.nmat) {   // invalid matrix index: NaN result, no access
        if (lane == 0) {
            a.p[it] = NAN; if (a.logp) a.logp[it] = NAN; if (a.se) a.se[it] = NAN;
            a.flag[it] = 0;
        }
        return;
    }
    const double nu = a.nu[it];
    const bool normal = isinf(nu);
    const float4 *src = reinterpret_cast<const float4 *>(normal ? ntab : tabs + (size_t)blockIdx.x * M * TABF_FLOATS);
    float4 *dst = reinterpret_cast<float4 *>(tab);
    for (int t = lane; t < (normal ? TABF_FLOATS : M * TABF_FLOATS) / 4; t += 64) dst[t] = src[t];
    __syncthreads();
    if (lane == 0) mvt_item_head(a, it, mi, M, bs, Ls, nu, tab, &Hs);
    __syncthreads();
    const SovHead H = Hs;
    double est = 0.0, se = 0.0, lnest = -INFINITY;
    if (H.e0 > 0.0 || H.lne0 > -INFINITY) {
        bool ok;
        if (normal) ok = sov_mixed_normal<M, 1>(H, bs, Ls, a.lat, tab, smean, lane);
        else if (coords) ok = sov_mixed<M, 1, true>(H, bs, Ls, nu, a.lat, tab, smean, lane, coords, C);
        else ok = sov_mixed<M, 1, false>(H, bs, Ls, nu, a.lat, tab, smean, lane);
        if (!ok) {
            if (lane == 0) a.flag[it] = 1;
            return;
        }
        sov_finish(H, smean, a.lat.S, &est, &se, &lnest);
    }
    if (lane == 0) {
        a.p[it] = est;
        if (a.logp) a.logp[it] = lnest;
        if (a.se) a.se[it] = se;
        a.flag[it] = 0;
    }
}

// FP64 integrand with the exact transforms, one wave per item: the items still
// flagged after k_mvt_fp64tab (a dof past the FP64 tables' range).
template <int M>
__global__ __launch_bounds__(256) void k_mvt(MvtArgs a) {
    __shared__ double smean[4][MAXS];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int it = blockIdx.x * 4 + wave;
    if (it >= a.batch) return;
    if (a.flag[it] == 0) return;
    const double nu = a.nu[it];
    double b[M], L[M * M];
    const int mi = a.mat_idx[it];
    if (mi < 0 || mi >= a.nmat) {   // invalid matrix index: NaN result, no access
        if (lane == 0) { a.p[it] = NAN; if (a.logp) a.logp[it] = NAN; if (a.se) a.se[it] = NAN; }
        return;
    }
#pragma unroll
    for (int i = 0; i < M; ++i) b[i] = a.b[(size_t)it * M + i];
#pragma unroll
    for (int i = 0; i < M * M; ++i) L[i] = a.L[(size_t)mi * M * M + i];
    const SovHead H = sov_head(b, L, nu);
    double est = 0.0, se = 0.0, lnest = -INFINITY;
    if (H.e0 > 0.0 || H.lne0 > -INFINITY) {
        sov_fp64<M>(H, b, L, nu, a.lat, smean[wave], lane);
        sov_finish(H, smean[wave], a.lat.S, &est, &se, &lnest);
    }
    if (lane == 0) {
        a.p[it] = est;
        if (a.logp) a.logp[it] = lnest;
        if (a.se) a.se[it] = se;
    }
}

// m = 1: the univariate t CDF in closed form, one thread per item.
__global__ __launch_bounds__(256) void k_mvt1(MvtArgs a) {
    const int it = blockIdx.x * blockDim.x + threadIdx.x;
    if (it >= a.batch) return;
    const double nu = a.nu[it];
    const int mi = a.mat_idx[it];
    if (mi < 0 || mi >= a.nmat) {
        a.p[it] = NAN; if (a.logp) a.logp[it] = NAN; if (a.se) a.se[it] = NAN;
        return;
    }
    const double b = a.b[it], L = a.L[mi];
    const SovHead H = sov_head(&b, &L, nu);
    a.p[it] = H.e0;
    if (a.logp) a.logp[it] = H.lne0;
    if (a.se) a.se[it] = 0.0;
}

// ------------------------------------------------------------- surrogate ---

// Features of T_m(b; 0, L L^T, nu) for the network: standardised limits
// z_i = b_i / sqrt(R_ii), as z_i / 6; correlations R_ij / sqrt(R_ii R_jj)
// (i < j, row order); (ln nu - ln 2) / (ln 30 - ln 2); the marginal log-CDFs
// ln T_nu(z_i) / 10; zero padding; R = L L^T.  *base receives
// sum_i ln T_nu(z_i) (the log-probability under independence), which the
// network corrects.  Returns whether the problem lies in the training domain
// (|z_i| <= 6, 2 <= nu <= 30).
__device__ inline bool sur_features(int m, const double *b, const double *L, double nu, float *x, double *base) {
    double R[MAXQ * MAXQ], sd[MAXQ];
    for (int i = 0; i < m; ++i)
        for (int k = 0; k <= i; ++k) {
            double s = 0.0;
            for (int l = 0; l <= k; ++l) s += L[i * m + l] * L[k * m + l];
            R[i * m + k] = R[k * m + i] = s;
        }
    bool ok = nu >= 2.0 && nu <= 30.0;
    const double nuc = fmin(fmax(nu, 0.5), 1e4);
    const double a = 0.5 * nuc, lb = dm_lbeta_half(a);
    for (int i = 0; i < m; ++i) sd[i] = sqrt(R[i * m + i]);
    int c = 0;
    double lm[MAXQ], sum = 0.0;
    for (int i = 0; i < m; ++i) {
        const double z = b[i] / sd[i];
        ok = ok && fabs(z) <= 6.0;
        const double zc = fmax(-6.0, fmin(6.0, z));
        x[c++] = (float)(zc / 6.0);
        // ln T_nu(z): lower-tail form, complement for z > 0
        const double az = fabs(z);
        double zz, zzc;
        if (az > 1.0) { const double r = (nuc / az) / az; zz = r / (1.0 + r); zzc = 1.0 / (1.0 + r); }
        else { const double den = nuc + z * z; zz = nuc / den; zzc = z * z / den; }
        const double lt = dm_lnT_lower(zz, zzc, a, lb);
        lm[i] = z <= 0.0 ? lt : log1p(-exp(lt));
        sum += lm[i];
    }
    for (int i = 0; i < m; ++i)
        for (int k = i + 1; k < m; ++k) x[c++] = (float)(R[i * m + k] / (sd[i] * sd[k]));
    x[c++] = (float)((log(nuc) - 0.69314718055994531) / (3.4011973816621555 - 0.69314718055994531));
    for (int i = 0; i < m; ++i) x[c++] = (float)fmax(lm[i] / 10.0, -10.0);
    while (c < CFUST_MLP_IN) x[c++] = 0.0f;
    *base = sum;
    return ok;
}

constexpr double SUR_RESID_SCALE = 5.0;   // network output 0 = (ln T - base) / 5

__device__ __forceinline__ uint16_t sur_f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__global__ __launch_bounds__(128) void k_sur_features(SurFeatArgs a) {
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long rows = (long)a.g * a.cnt * a.n;
    if (gid >= rows) return;
    const int j = (int)(gid % a.n);
    const int t = (int)((gid / a.n) % a.cnt);
    const int h = (int)(gid / ((long)a.n * a.cnt));
    const IntDesc D = int_desc(a.q, a.idx0 + t);
    const CompPre &P = a.pre[h];
    double c[MAXQ], d, b[MAXQ];
    pair_geometry(a.y, a.n, a.p, a.q, j, a.mu + (size_t)h * a.p, P, c, d);
    const double *L = integral_limits(D, P, a.p, a.q, c, d, b);
    float x[CFUST_MLP_IN];
    double base;
    const bool ok = sur_features(D.m, b, L, P.nu + a.p + D.dofoff, x, &base);
    for (int i = 0; i < CFUST_MLP_IN; ++i) a.X0[gid * CFUST_MLP_IN + i] = sur_f2bf(x[i]);
    a.inrange[gid] = ok ? 1 : 0;
    a.base[gid] = base;
}

__global__ __launch_bounds__(256) void k_sur_select(SurSelArgs a) {
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long rows = (long)a.g * a.cnt * a.n;
    if (gid >= rows) return;
    const int j = (int)(gid % a.n);
    const int t = (int)((gid / a.n) % a.cnt);
    const int h = (int)(gid / ((long)a.n * a.cnt));
    const int idx = a.idx0 + t;
    const size_t o = ((size_t)h * a.J + idx) * a.n + j;
    const float o0 = a.out[gid * CFUST_MLP_OUT], o1 = a.out[gid * CFUST_MLP_OUT + 1];
    const double lnT = fmin(a.base[gid] + SUR_RESID_SCALE * (double)o0, 0.0);
    const double err = SUR_RESID_SCALE * pow(10.0, (double)o1);   // predicted |error| of ln T
    const bool use = a.inrange[gid] && isfinite(lnT) && err <= a.tol;
    a.need[o] = use ? 0 : 1;
    if (use) {
        a.est[o] = exp(lnT);
        if (idx == 0) a.lnA[(size_t)h * a.n + j] = lnT;
    }
}

__global__ void k_fill_i32(int32_t *p, size_t count, int32_t v) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

__global__ __launch_bounds__(256) void k_count_i32(const int32_t *__restrict__ p, size_t count, int32_t *out) {
    __shared__ int red[256];
    int s = 0;
    for (size_t i = threadIdx.x; i < count; i += 256) s += p[i] != 0;
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

__global__ __launch_bounds__(128) void k_mvt_features(int m, int batch, const double *__restrict__ bb,
                                                      const double *__restrict__ LL,
                                                      const int32_t *__restrict__ mat_idx,
                                                      const double *__restrict__ nu, uint16_t *__restrict__ X0,
                                                      int32_t *__restrict__ inrange, int rows_pad, int nmat,
                                                      double *__restrict__ basev) {
    const int it = blockIdx.x * blockDim.x + threadIdx.x;
    if (it >= rows_pad) return;
    float x[CFUST_MLP_IN];
    bool ok = false;
    const int mi = it < batch ? mat_idx[it] : -1;
    if (mi >= 0 && mi < nmat) {
        double b[MAXQ], L[MAXQ * MAXQ];
        for (int i = 0; i < m; ++i) b[i] = bb[(size_t)it * m + i];
        for (int i = 0; i < m * m; ++i) L[i] = LL[(size_t)mi * m * m + i];
        double base;
        ok = sur_features(m, b, L, nu[it], x, &base);
        if (basev) basev[it] = base;
    } else {
        for (int i = 0; i < CFUST_MLP_IN; ++i) x[i] = 0.0f;
        if (basev && it < batch) basev[it] = 0.0;
    }
    for (int i = 0; i < CFUST_MLP_IN; ++i) X0[(size_t)it * CFUST_MLP_IN + i] = sur_f2bf(x[i]);
    if (inrange && it < batch) inrange[it] = ok ? 1 : 0;
}

hipError_t launch_sur_features(const SurFeatArgs &a, hipStream_t s) {
    const long rows = (long)a.g * a.cnt * a.n;
    if (rows == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sur_features, dim3((unsigned)((rows + 127) / 128)), dim3(128), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_sur_select(const SurSelArgs &a, hipStream_t s) {
    const long rows = (long)a.g * a.cnt * a.n;
    if (rows == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sur_select, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, size_t count, int32_t v, hipStream_t s) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, count, v);
    return hipGetLastError();
}

hipError_t launch_count_i32(const int32_t *p, size_t count, int32_t *out, hipStream_t s) {
    hipLaunchKernelGGL(k_count_i32, dim3(1), dim3(256), 0, s, p, count, out);
    return hipGetLastError();
}

hipError_t launch_mvt_features(int m, int batch, int rows_pad, const double *b, const double *L,
                               const int32_t *mat_idx, int nmat, const double *nu, uint16_t *X0, int32_t *inrange,
                               double *base, hipStream_t s) {
    if (rows_pad == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mvt_features, dim3((rows_pad + 127) / 128), dim3(128), 0, s, m, batch, b, L, mat_idx,
                       nu, X0, inrange, rows_pad, nmat, base);
    return hipGetLastError();
}

// --------------------------------------------------------------- launch ----

hipError_t launch_precompute(const cfust_params &P, int p, int q, int g, CompPre *pre, hipStream_t s) {
    hipLaunchKernelGGL(k_precompute, dim3(g), dim3(64), 0, s, P.pi, P.Sigma, P.Delta, P.nu, p, q, pre);
    return hipGetLastError();
}

hipError_t launch_status_fold(const CompPre *pre, int g, int32_t *status, hipStream_t s) {
    hipLaunchKernelGGL(k_status_fold, dim3(1), dim3(64), 0, s, pre, g, status);
    return hipGetLastError();
}

hipError_t launch_tables(const CompPre *pre, int p, int g, int ndof, float *tabs, hipStream_t s) {
    hipLaunchKernelGGL(k_tables, dim3(g * ndof), dim3(192), 0, s, pre, p, ndof, tabs);
    return hipGetLastError();
}

hipError_t launch_tables64(const CompPre *pre, int p, int g, int ndof, double *tabs, hipStream_t s) {
    hipLaunchKernelGGL(k_tables64, dim3(g * ndof), dim3(192), 0, s, pre, p, ndof, tabs);
    return hipGetLastError();
}

template <int M>
static void launch_qmc_m(const EstepQmcArgs &a, int nidx, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, int ppl) {
    dim3 grid((a.n + 3) / 4, nidx, a.g);
    if (ev0) (void)hipEventRecord(ev0, s);
    if (a.mixed) {
        if (ppl == 2) hipLaunchKernelGGL((k_estep_qmc<M, true, 2>), grid, dim3(256), 0, s, a);
        else if (a.coords) hipLaunchKernelGGL((k_estep_qmc<M, true, 1, true>), grid, dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_estep_qmc<M, true, 1>), grid, dim3(256), 0, s, a);
    } else {
        hipLaunchKernelGGL((k_estep_qmc<M, false, 1>), grid, dim3(256), 0, s, a);
    }
    if (ev1) (void)hipEventRecord(ev1, s);
    // flagged items (mixed: FP32 underflow; FP64: a dof past the FP64 tables):
    // in mixed mode on the FP64 tables where they reach, the rest exact
    const long long total = (long long)a.g * nidx * a.n;
    if (a.mixed && a.tabs64)
        hipLaunchKernelGGL((k_estep_flagged64<M>), dim3((unsigned)((total + 63) / 64)), dim3(64), 0, s, a, nidx);
    const long long blocks = (total + 255) / 256;
    hipLaunchKernelGGL((k_estep_flagged<M>), dim3((unsigned)blocks), dim3(256), 0, s, a, nidx);
}

hipError_t launch_estep_qmc(const EstepQmcArgs &a, int m, int nidx, hipStream_t s, hipEvent_t ev0,
                            hipEvent_t ev1, int ppl) {
    if (a.n == 0 || nidx == 0) return hipSuccess;
    if (a.lat.N % 128 != 0) ppl = 1;
    switch (m) {
    case 2: launch_qmc_m<2>(a, nidx, s, ev0, ev1, ppl); break;
    case 3: launch_qmc_m<3>(a, nidx, s, ev0, ev1, ppl); break;
    case 4: launch_qmc_m<4>(a, nidx, s, ev0, ev1, ppl); break;
    case 5: launch_qmc_m<5>(a, nidx, s, ev0, ev1, ppl); break;
    case 6: launch_qmc_m<6>(a, nidx, s, ev0, ev1, ppl); break;
    case 7: launch_qmc_m<7>(a, nidx, s, ev0, ev1, ppl); break;
    case 8: launch_qmc_m<8>(a, nidx, s, ev0, ev1, ppl); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// The lattice coordinates of every point, coordinate and shift, formed as the
// FP32 integrand forms them (one thread per point; grid (N/256, C, S)), and
// log2 of coordinate 0, all the first quantile step takes of it when the
// item's first limit is in the lower half.  Per shift 2C + 1 rows of N
// floats: row 0 that logarithm, row 1 + 2i coordinate i, row 2 + 2i its
// complement.
__global__ __launch_bounds__(256) void k_lattice_coords(LatticeArgs L, int C, float *__restrict__ coords) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y, s = blockIdx.z;
    if (k >= (uint32_t)L.N) return;
    const int sh = 32 - L.log2N;
    const uint32_t t = ((k * (uint32_t)L.z[i]) << sh) + (uint32_t)(L.shifts[s * LATD + i] * 4294967296.0);
    const float scale = i == 0 ? 1.0f : 4.656612873077393e-10f;      // 2^-31 past coordinate 0
    float *shift = coords + (size_t)s * (2 * C + 1) * L.N;
    float *row = shift + (size_t)(1 + 2 * i) * L.N;
    const float v = tent_units(t) * scale;
    row[k] = v;
    row[L.N + k] = tent_units(t ^ 0x80000000u) * scale;
    if (i == 0) shift[k] = flog2(v);
}

hipError_t launch_lattice_coords(const LatticeArgs &L, int C, float *coords, hipStream_t s) {
    if (C <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_lattice_coords, dim3((L.N + 255) / 256, C, L.S), dim3(256), 0, s, L, C, coords);
    return hipGetLastError();
}

hipError_t launch_assemble(const EstepAsmArgs &a, hipStream_t s) {
    const long tot = (long)a.n * a.g;
    if (tot == 0) return hipSuccess;
    hipLaunchKernelGGL(k_assemble, dim3((unsigned)((tot + 127) / 128)), dim3(128), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_lse(const EstepLseArgs &a, double *loglik, hipStream_t s) {
    const int nb = (a.n + 255) / 256;
    if (nb > 0) hipLaunchKernelGGL(k_lse, dim3(nb), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, a.partial, nb, loglik);
    return hipGetLastError();
}

// Mixed: per chunk the FP32 tables and integrand (flagging underflows), then
// the FP64 tables and integrand of the flagged items; FP64 mode: every item
// flagged, the FP64 passes only.  Last, the exact transforms for what is left.
template <int M>
static hipError_t launch_mvt_m(const MvtArgs &a, const MvtWork &w, hipStream_t s) {
    hipError_t e = hipSuccess;
    if (a.mixed) {
        if (w.C > 0) e = launch_lattice_coords(a.lat, w.C, w.coords, s);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_mvt_normal_table, dim3(1), dim3(192), 0, s, w.ntab);
            e = hipGetLastError();
        }
    } else {
        e = launch_fill_i32(a.flag, (size_t)a.batch, 1, s);
    }
    for (int it0 = 0; it0 < a.batch && e == hipSuccess; it0 += w.chunk) {
        const int cnt = a.batch - it0 < w.chunk ? a.batch - it0 : w.chunk;
        if (a.mixed) {
            hipLaunchKernelGGL(k_mvt_tables, dim3(cnt * M), dim3(192), 0, s, a, it0, M, w.tabs);
            hipLaunchKernelGGL((k_mvt_qmc<M>), dim3(cnt), dim3(64), 0, s, a, it0, (const float *)w.tabs,
                               (const float *)w.ntab, (const float *)(w.C > 0 ? w.coords : nullptr), w.C);
        }
        hipLaunchKernelGGL(k_mvt_tables64, dim3(cnt * M), dim3(192), 0, s, a, it0, M, w.tabs64);
        hipLaunchKernelGGL((k_mvt_fp64tab<M>), dim3(cnt), dim3(64), 0, s, a, it0, (const double *)w.tabs64);
        e = hipGetLastError();
    }
    if (e == hipSuccess) hipLaunchKernelGGL((k_mvt<M>), dim3((a.batch + 3) / 4), dim3(256), 0, s, a);
    return e == hipSuccess ? hipGetLastError() : e;
}

hipError_t launch_mvt(const MvtArgs &a, const MvtWork &w, hipStream_t s) {
    if (a.batch == 0) return hipSuccess;
    switch (a.m) {
    case 1: hipLaunchKernelGGL(k_mvt1, dim3((a.batch + 255) / 256), dim3(256), 0, s, a); return hipGetLastError();
    case 2: return launch_mvt_m<2>(a, w, s);
    case 3: return launch_mvt_m<3>(a, w, s);
    case 4: return launch_mvt_m<4>(a, w, s);
    case 5: return launch_mvt_m<5>(a, w, s);
    case 6: return launch_mvt_m<6>(a, w, s);
    case 7: return launch_mvt_m<7>(a, w, s);
    case 8: return launch_mvt_m<8>(a, w, s);
    default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------ batches ----

// Fit owning block b: the largest f with prefix[f] <= b.
__device__ inline int batch_fit(const int *__restrict__ prefix, int nfits, int b) {
    int lo = 0, hi = nfits - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(64) void k_batch_precompute(BatchArgs B) {
    const int *pf = B.prefix + BK_PRE * (B.nfits + 1);
    const int f = batch_fit(pf, B.nfits, blockIdx.x);
    if (!B.active[f]) return;
    const PrecompArgs &a = B.fits[f].pc;
    precompute_body(a.pi, a.Sigma, a.Delta, a.nu, a.p, a.q, a.pre, blockIdx.x - pf[f]);
}

__global__ __launch_bounds__(192) void k_batch_tables(BatchArgs B) {
    const int *pf = B.prefix + BK_TAB * (B.nfits + 1);
    const int f = batch_fit(pf, B.nfits, blockIdx.x);
    if (!B.active[f]) return;
    const FitDesc &F = B.fits[f];
    // mixed: the FP32 tables, and the FP64 ones for the redo list; FP64: FP64 tables
    if (F.qa.mixed) tables_body(F.pc.pre, F.pc.p, F.ndof, F.tabs, blockIdx.x - pf[f]);
    if (F.tabs64) tables64_body(F.pc.pre, F.pc.p, F.ndof, F.tabs64, blockIdx.x - pf[f]);
}

__global__ __launch_bounds__(128) void k_batch_assemble(BatchArgs B) {
    const int *pf = B.prefix + BK_ASM * (B.nfits + 1);
    const int f = batch_fit(pf, B.nfits, blockIdx.x);
    if (!B.active[f]) return;
    const EstepAsmArgs a = B.fits[f].aa;
    assemble_body(a, (blockIdx.x - pf[f]) * 128 + threadIdx.x);
}

__global__ __launch_bounds__(256) void k_batch_lse(BatchArgs B) {
    const int *pf = B.prefix + BK_LSE * (B.nfits + 1);
    const int f = batch_fit(pf, B.nfits, blockIdx.x);
    if (!B.active[f]) return;
    const EstepLseArgs a = B.fits[f].la;
    lse_body(a, blockIdx.x - pf[f]);
}

// One block per fit: log-likelihood from the LSE partials, status fold.
__global__ __launch_bounds__(256) void k_batch_sum(BatchArgs B) {
    const int f = blockIdx.x;
    if (!B.active[f]) return;
    const FitDesc &F = B.fits[f];
    sum_partials_body(F.la.partial, F.nlse, F.loglik);
    if (threadIdx.x == 0 && F.status) {
        int s = F.status[0];
        for (int h = 0; h < F.g; ++h) s |= F.pc.pre[h].status;
        F.status[0] = s;
    }
}

// Persistent lattice kernel: each block draws tiles from the queue until it
// is empty; the 4 waves of a block share the tile's component and integral,
// hence its LDS tables, and take its observations in turn.
template <int M, bool MIXED, int PPL, bool COORDS = false>
__global__ __launch_bounds__(256, MIXED && PPL == 1 ? fp32_min_blocks(M) : 1) void k_queue_qmc(QueueArgs Q) {
    __shared__ __align__(16) float tab[MIXED ? M * TABF_FLOATS : 4];
    __shared__ double tab64[MIXED ? 1 : M * TAB64_DOUBLES];
    __shared__ double smean[4][MAXS];
    __shared__ WaveItem witem[4];
    __shared__ long long s_tile;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int cur_f = -1, cur_h = -1, cur_dof = -1;
    EstepQmcArgs acopy;
    for (;;) {
        if (threadIdx.x == 0) s_tile = (long long)atomicAdd(Q.counter, 1ULL);
        __syncthreads();              // also: every wave is done with the previous tile
        // the tile number is block-uniform: keep it (and all that derives from
        // it, including the fit's argument block) in scalar registers
        const unsigned long long tv = (unsigned long long)s_tile;
        const long long t = (long long)(((unsigned long long)__builtin_amdgcn_readfirstlane((unsigned)(tv >> 32)) << 32) |
                                        (unsigned)__builtin_amdgcn_readfirstlane((unsigned)tv));
        __syncthreads();
        if (t >= Q.ntiles) break;
        int lo = 0, hi = Q.nseg - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (Q.seg[mid].t0 <= t) lo = mid;
            else hi = mid - 1;
        }
        const QSeg S = Q.seg[lo];
        if (!Q.active[S.fit]) continue;
        const long long local = t - S.t0;
        const int rt = (int)(local % S.rtiles);
        const long long rest = local / S.rtiles;
        const int idx = S.idx0 + (int)(rest % S.nidx);
        const int h = (int)(rest / S.nidx);
        // FP64: a copy, not a reference into device memory (read through the
        // reference its fields were kept in VGPRs and the kernel spilled); the
        // FP32 form keeps the reference (a copy held across the tile loop costs
        // it registers instead)
        if (!MIXED) acopy = Q.fits[S.fit].qa;
        const EstepQmcArgs &a = MIXED ? Q.fits[S.fit].qa : acopy;
        const int dof = int_desc(a.q, idx).dofoff;
        if (S.fit != cur_f || h != cur_h || dof != cur_dof) {
            if (MIXED) load_tables<M>(a.tabs, h, dof, tab);
            else if (a.tabs64) load_tables64<M>(a.tabs64, h, dof, tab64);
            __syncthreads();
            cur_f = S.fit; cur_h = h; cur_dof = dof;
        }
        const int jb = S.j0 + rt * S.rows;
        const bool exact = !MIXED && beyond_tab64<M>(a.pre, a.p, a.q, h, idx);
        for (int r = wave; r < S.rows; r += 4) {
            const int j = jb + r;
            const bool ok = !exact && qmc_item<M, MIXED, PPL, !MIXED, COORDS>(a, h, idx, j, tab, tab64, smean[wave],
                                                                      &witem[wave], lane);
            if (!ok && lane == 0) {
                const unsigned slot = atomicAdd(Q.redo_count, 1u);
                Q.redo[slot] = ((unsigned long long)S.fit << 43) | ((unsigned long long)h << 37) |
                               ((unsigned long long)idx << 31) | (unsigned long long)j;
            }
        }
    }
}

// The same queue with one block per tile, in queue order (blocks are handed
// out in increasing index, so the longest-first order of the queue holds):
// tiles of at most 4 observations, one per wave.  With no loop around the
// item its registers are not held across items, which the persistent form
// pays for; the autotuner picks between the two.  Block t = y * gridDim.x + x.
template <int M, bool MIXED, int PPL, bool COORDS = false>
__global__ __launch_bounds__(256, MIXED && PPL == 1 ? fp32_min_blocks(M) : 1) void k_queue_grid(QueueArgs Q) {
    __shared__ __align__(16) float tab[MIXED ? M * TABF_FLOATS : 4];
    __shared__ double tab64[MIXED ? 1 : M * TAB64_DOUBLES];
    __shared__ double smean[4][MAXS];
    __shared__ WaveItem witem[4];
    const long long t = (long long)blockIdx.y * gridDim.x + blockIdx.x;
    if (t >= Q.ntiles) return;
    int lo = 0, hi = Q.nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (Q.seg[mid].t0 <= t) lo = mid;
        else hi = mid - 1;
    }
    const QSeg S = Q.seg[lo];
    if (!Q.active[S.fit]) return;
    const long long local = t - S.t0;
    const int rt = (int)(local % S.rtiles);
    const long long rest = local / S.rtiles;
    const int idx = S.idx0 + (int)(rest % S.nidx);
    const int h = (int)(rest / S.nidx);
    const EstepQmcArgs a = Q.fits[S.fit].qa;       // a copy: through a reference its fields took VGPRs
    if (MIXED) {
        load_tables<M>(a.tabs, h, int_desc(a.q, idx).dofoff, tab);
        __syncthreads();
    } else if (a.tabs64) {
        load_tables64<M>(a.tabs64, h, int_desc(a.q, idx).dofoff, tab64);
        __syncthreads();
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (wave >= S.rows) return;
    const int j = S.j0 + rt * S.rows + wave;
    const bool exact = !MIXED && beyond_tab64<M>(a.pre, a.p, a.q, h, idx);
    const bool ok = !exact && qmc_item<M, MIXED, PPL, !MIXED, COORDS>(a, h, idx, j, tab, tab64, smean[wave],
                                                              &witem[wave], lane);
    if (!ok && lane == 0) {
        const unsigned slot = atomicAdd(Q.redo_count, 1u);
        Q.redo[slot] = ((unsigned long long)S.fit << 43) | ((unsigned long long)h << 37) |
                       ((unsigned long long)idx << 31) | (unsigned long long)j;
    }
}

// FP64 integrand for the items of the redo list, one wave per entry, in two
// passes: TABLES, the entries whose fit has FP64 tables (mixed: every fit)
// and whose dofs they reach, on those tables (one wave per block, the
// entry's tables in its LDS), each marked done (~0) afterwards; then the
// rest with the exact transforms.
constexpr unsigned long long REDO_DONE = ~0ULL;

template <int M, bool TABLES>
__global__ __launch_bounds__(TABLES ? 64 : 256) void k_queue_redo(QueueArgs Q) {
    constexpr int W = TABLES ? 1 : 4;
    __shared__ double tab64[TABLES ? M * TAB64_DOUBLES : 1];
    __shared__ double smean[W][MAXS];
    __shared__ WaveItem witem[W];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const unsigned cnt = Q.redo_count[0];
    for (unsigned e = blockIdx.x * W + wave; e < cnt; e += gridDim.x * W) {
        const unsigned long long v0 = Q.redo[e];
        const unsigned long long v = ((unsigned long long)__builtin_amdgcn_readfirstlane((unsigned)(v0 >> 32)) << 32) |
                                     (unsigned)__builtin_amdgcn_readfirstlane((unsigned)v0);
        if (v == REDO_DONE) continue;
        const int f = (int)(v >> 43), h = (int)((v >> 37) & 63), idx = (int)((v >> 31) & 63);
        const int j = (int)(v & 0x7fffffffULL);
        const EstepQmcArgs a = Q.fits[f].qa;
        if (TABLES) {
            if (!a.tabs64 || beyond_tab64<M>(a.pre, a.p, a.q, h, idx)) continue;
            __syncthreads();
            load_tables64<M>(a.tabs64, h, int_desc(a.q, idx).dofoff, tab64);
            __syncthreads();
            qmc_item<M, false, 1, true>(a, h, idx, j, nullptr, tab64, smean[wave], &witem[wave], lane);
            if (lane == 0) Q.redo[e] = REDO_DONE;
        } else {
            qmc_item<M, false, 1>(a, h, idx, j, nullptr, nullptr, smean[wave], &witem[wave], lane);
        }
    }
}

// Between the E-step and the M-step of a batched EM iteration: records the
// log-likelihood of every active fit in trace[iter][fit] and retires a fit by
// Aitken's criterion (Sec. 3.4, eqs. 24-26) with tolerance tol, or when its
// log-likelihood is unchanged or not finite.  A retired fit's M-step and
// later E-steps are skipped, so its parameters stay those of its last E-step.
// hist[f] = (l^(k-1), l^(k)) of the fit's two previous iterations.  One block.
__global__ __launch_bounds__(256) void k_batch_check(const FitDesc *__restrict__ fits, int nfits,
                                                     int32_t *__restrict__ active, int32_t *__restrict__ iter,
                                                     double *__restrict__ hist, const BatchCtl *__restrict__ ctl) {
    const int it = iter[0];
    const double tol = ctl->tol;
    double *trace = ctl->trace;
    int32_t *iters_done = ctl->iters_done;
    const int max_trace = ctl->max_trace;
    for (int f = threadIdx.x; f < nfits; f += blockDim.x) {
        if (!active[f]) continue;
        const double l1 = fits[f].loglik[0];            // l^(k+1), this iteration
        if (trace && it < max_trace) trace[(size_t)it * nfits + f] = l1;
        if (iters_done) iters_done[f] = it + 1;
        const double lm = hist[2 * f], l0 = hist[2 * f + 1];   // l^(k-1), l^(k)
        bool stop = !isfinite(l1);
        if (!stop && it >= 1 && l1 == l0) stop = true;
        if (!stop && it >= 2 && tol > 0.0) {
            const double d1 = l1 - l0, d0 = l0 - lm;
            double gap;                                   // |l_inf^(k+1) - l^(k+1)|
            if (d0 == 0.0) {
                gap = fabs(d1);                           // a = +-inf: l_inf = l^(k)
            } else {
                const double a = d1 / d0;                 // eq. (26)
                const double linf = l0 + d1 / (1.0 - a);  // eq. (25)
                gap = fabs(linf - l1);
            }
            stop = gap < tol;                             // eq. (24)
        }
        hist[2 * f] = l0;
        hist[2 * f + 1] = l1;
        if (stop) active[f] = 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) iter[0] = it + 1;
}

hipError_t launch_batch_precompute(const BatchArgs &b, int nblocks, hipStream_t s) {
    if (nblocks > 0) hipLaunchKernelGGL(k_batch_precompute, dim3(nblocks), dim3(64), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_batch_tables(const BatchArgs &b, int nblocks, hipStream_t s) {
    if (nblocks > 0) hipLaunchKernelGGL(k_batch_tables, dim3(nblocks), dim3(192), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_batch_assemble(const BatchArgs &b, int nblocks, hipStream_t s) {
    if (nblocks > 0) hipLaunchKernelGGL(k_batch_assemble, dim3(nblocks), dim3(128), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_batch_lse(const BatchArgs &b, int nblocks, hipStream_t s) {
    if (nblocks > 0) hipLaunchKernelGGL(k_batch_lse, dim3(nblocks), dim3(256), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_batch_sum(const BatchArgs &b, hipStream_t s) {
    if (b.nfits > 0) hipLaunchKernelGGL(k_batch_sum, dim3(b.nfits), dim3(256), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_batch_check(const FitDesc *fits, int nfits, int32_t *active, int32_t *iter, double *hist,
                              const BatchCtl *ctl, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_check, dim3(1), dim3(256), 0, s, fits, nfits, active, iter, hist, ctl);
    return hipGetLastError();
}

// coords: the fits' argument blocks carry the coordinate table (mixed, one
// point per lane per trip only)
template <int M>
static const void *queue_kernel(bool mixed, int ppl, bool persist, bool coords) {
    if (persist) {
        if (!mixed) return (const void *)k_queue_qmc<M, false, 1>;
        if (ppl == 2) return (const void *)k_queue_qmc<M, true, 2>;
        return coords ? (const void *)k_queue_qmc<M, true, 1, true> : (const void *)k_queue_qmc<M, true, 1>;
    }
    if (!mixed) return (const void *)k_queue_grid<M, false, 1>;
    if (ppl == 2) return (const void *)k_queue_grid<M, true, 2>;
    return coords ? (const void *)k_queue_grid<M, true, 1, true> : (const void *)k_queue_grid<M, true, 1>;
}

static const void *queue_kernel_m(int m, bool mixed, int ppl, bool persist, bool coords) {
    switch (m) {
    case 2: return queue_kernel<2>(mixed, ppl, persist, coords);
    case 3: return queue_kernel<3>(mixed, ppl, persist, coords);
    case 4: return queue_kernel<4>(mixed, ppl, persist, coords);
    case 5: return queue_kernel<5>(mixed, ppl, persist, coords);
    case 6: return queue_kernel<6>(mixed, ppl, persist, coords);
    case 7: return queue_kernel<7>(mixed, ppl, persist, coords);
    case 8: return queue_kernel<8>(mixed, ppl, persist, coords);
    default: return nullptr;
    }
}

template <bool TABLES>
static const void *redo_kernel_m(int m) {
    switch (m) {
    case 2: return (const void *)k_queue_redo<2, TABLES>;
    case 3: return (const void *)k_queue_redo<3, TABLES>;
    case 4: return (const void *)k_queue_redo<4, TABLES>;
    case 5: return (const void *)k_queue_redo<5, TABLES>;
    case 6: return (const void *)k_queue_redo<6, TABLES>;
    case 7: return (const void *)k_queue_redo<7, TABLES>;
    case 8: return (const void *)k_queue_redo<8, TABLES>;
    default: return nullptr;
    }
}

hipError_t launch_queue_qmc(const QueueArgs &q, int m, bool mixed, int ppl, int grid, hipStream_t s, bool coords) {
    const bool persist = grid > 0;
    const void *k = queue_kernel_m(m, mixed, ppl, persist, coords);
    if (!k) return hipErrorInvalidValue;
    void *args[] = {(void *)&q};
    if (persist) return hipLaunchKernel(k, dim3(grid), dim3(256), args, 0, s);
    if (q.ntiles <= 0) return hipSuccess;
    const long long gx = q.ntiles < 32768 ? q.ntiles : 32768;
    const long long gy = (q.ntiles + gx - 1) / gx;
    if (gy > 0x7fffffffLL) return hipErrorInvalidValue;
    return hipLaunchKernel(k, dim3((unsigned)gx, (unsigned)gy), dim3(256), args, 0, s);
}

hipError_t launch_queue_redo(const QueueArgs &q, int m, int grid, int grid64, hipStream_t s) {
    const void *k64 = redo_kernel_m<true>(m), *k = redo_kernel_m<false>(m);
    if (!k || !k64 || grid < 1 || grid64 < 1) return hipErrorInvalidValue;
    void *args[] = {(void *)&q};
    hipError_t e = hipLaunchKernel(k64, dim3(grid64), dim3(64), args, 0, s);
    if (e == hipSuccess) e = hipLaunchKernel(k, dim3(grid), dim3(256), args, 0, s);
    return e;
}

int queue_qmc_occupancy(int m, bool mixed, int ppl, bool coords) {
    const void *k = queue_kernel_m(m, mixed, ppl, true, coords);
    int nb = 0;
    if (!k || hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, 256, 0) != hipSuccess) return 1;
    return nb > 0 ? nb : 1;
}

int queue_redo_occupancy(int m, bool tables) {
    const void *k = tables ? redo_kernel_m<true>(m) : redo_kernel_m<false>(m);
    int nb = 0;
    if (!k || hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, tables ? 64 : 256, 0) != hipSuccess) return 1;
    return nb > 0 ? nb : 1;
}

}  // namespace cfust
