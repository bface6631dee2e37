/*
 * cfust_oracle.c -- plain FP64 CPU oracle for the CFUST mixture E-step and M-step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links or calls this
 * file; it exists so that tests, the smoke check and the CPU baseline of the
 * bench can compare the HIP path against an independent, slow, obviously
 * correct implementation.  It shares no source with the HIP library.
 *
 * What it follows (Lee, Leemaqz & McLachlan, "A simple multithreaded
 * implementation of the EM algorithm for mixture models"):
 *   - Sec. 2 eq. (3)  multivariate t density, read with (pi*nu)^(-p/2) and the
 *                     exponent -(nu+p)/2 (the printed form is garbled);
 *   - Sec. 2 eq. (4)  CFUST density with Omega, c(y), Lambda, d(y);
 *   - Sec. 3.1 eqs. (12), (13), (15)-(17)  tau, w, e1, e2, e3, with "nu d" in
 *                     (13) read as "nu + d";
 *   - Sec. 3.2 eqs. (18)-(22)  M-step, in the order pi, mu, Delta, Sigma, nu,
 *                     with the sign of the last sum in (22) read as "+";
 *   - Sec. 4.3 eq. (27)  log-likelihood.
 * The paper does not say how the q-variate t CDF T_q or the truncated-t
 * moments in (16)-(17) are computed.  Here:
 *   - T_m is Genz's separation-of-variables (SOV) integrand for the
 *     multivariate t (sequential conditional univariate t's with dof nu+i)
 *     averaged over a randomly shifted rank-1 lattice with the tent transform;
 *     lattice vector and shifts are inputs;
 *   - the truncated-t moments use the first/second moment identities obtained
 *     by integrating the gradient of the t kernel (they need T_{m-1} with dof
 *     nu-1 and T_{m-2} with dof nu-2), written recursively on dense matrices.
 * The normal limit of Table 1 (CFUSN: nu -> infinity) is nu = +INFINITY for a
 * component: every t law becomes the normal one (CDF 0.5 erfc(-x/sqrt 2) from
 * the C library, its quantile by the same safeguarded Newton iteration), each
 * dof ratio (nu+a)/(nu+b) becomes 1, W is 1 (w = 1, e1 = E[log W] = 0), and
 * the M-step keeps nu.
 * Special functions come from published mathematics: the continued fraction
 * for the regularised incomplete beta (DLMF 8.17.22, modified Lentz), the
 * asymptotic series of the digamma function (DLMF 5.11.2) with upward
 * recurrence, and a safeguarded Newton iteration for the t quantile.  lgamma
 * is the C library's.
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXM 8

/* ------------------------------------------------------------------------- */
/* special functions                                                          */
/* ------------------------------------------------------------------------- */

/* Digamma: recurrence psi(x) = psi(x+1) - 1/x until x >= 10, then
 * psi(x) ~ ln x - 1/(2x) - sum_k B_2k / (2k x^2k)  (DLMF 5.11.2). */
double or_digamma(double x)
{
    if (!(x > 0.0) || isinf(x)) return NAN;   /* only positive arguments occur */
    double acc = 0.0;
    while (x < 10.0) { acc -= 1.0 / x; x += 1.0; }
    double r = 1.0 / (x * x);
    double s = r * (1.0 / 12 - r * (1.0 / 120 - r * (1.0 / 252 - r * (1.0 / 240
               - r * (1.0 / 132 - r * (691.0 / 32760 - r / 12.0))))));
    return acc + log(x) - 0.5 / x - s;
}

/* Continued fraction 1 + d1/(1 + d2/(1 + ...)) of DLMF 8.17.22 for I_x(a,b):
 * d_{2k+1} = -(a+k)(a+b+k) x / ((a+2k)(a+2k+1)),  d_{2k} = k(b-k) x / ((a+2k-1)(a+2k)).
 * Evaluated by the modified Lentz method. */
static double or_betacf(double a, double b, double x)
{
    const double tiny = 1e-300;
    double f = 1.0, C = 1.0, D = 0.0;
    for (int j = 1; j <= 20000; ++j) {
        int k = j / 2;
        double d;
        if (j & 1) d = -(a + k) * (a + b + k) * x / ((a + 2 * k) * (a + 2 * k + 1));
        else       d = k * (b - k) * x / ((a + 2 * k - 1) * (a + 2 * k));
        D = 1.0 + d * D; if (fabs(D) < tiny) D = tiny; D = 1.0 / D;
        C = 1.0 + d / C; if (fabs(C) < tiny) C = tiny;
        double del = C * D;
        f *= del;
        if (fabs(del - 1.0) < 1e-16) break;
    }
    return f;
}

/* Regularised incomplete beta I_x(a,b) and its complement; x, xc = 1-x and
 * their logarithms are all supplied so that none loses accuracy (x may be far
 * below the double range's reach through x itself).  Uses
 * I_x(a,b) = 1 - I_{1-x}(b,a) to stay where the continued fraction converges fast. */
static void or_betai2l(double a, double b, double x, double xc, double lx, double lxc,
                       double *I, double *Ic)
{
    if (lx == -INFINITY) { *I = 0.0; *Ic = 1.0; return; }
    if (lxc == -INFINITY) { *I = 1.0; *Ic = 0.0; return; }
    double lbeta = lgamma(a) + lgamma(b) - lgamma(a + b);
    if (x < (a + 1.0) / (a + b + 2.0)) {
        double v = exp(a * lx + b * lxc - log(a) - lbeta) / or_betacf(a, b, x);
        *I = v; *Ic = 1.0 - v;
    } else {
        double v = exp(b * lxc + a * lx - log(b) - lbeta) / or_betacf(b, a, xc);
        *Ic = v; *I = 1.0 - v;
    }
}

void or_betai2(double a, double b, double x, double xc, double *I, double *Ic)
{
    or_betai2l(a, b, x, xc, x > 0 ? log(x) : -INFINITY, xc > 0 ? log(xc) : -INFINITY, I, Ic);
}

double or_betai(double a, double b, double x)
{
    double I, Ic;
    or_betai2(a, b, x, 1.0 - x, &I, &Ic);
    return I;
}

/* Student t CDF with real dof nu: P(T <= t) = I_{nu/(nu+t^2)}(nu/2, 1/2) / 2 for t < 0. */
double or_tcdf(double t, double nu)
{
    if (isnan(t)) return t;
    if (isinf(t)) return t > 0 ? 1.0 : 0.0;
    if (isinf(nu)) return 0.5 * erfc(-t / M_SQRT2);   /* normal limit */
    double z, zc, lz, lzc;            /* z = nu/(nu+t^2), zc = t^2/(nu+t^2) */
    double at = fabs(t);
    if (at > 1.0) {
        double r = (nu / at) / at;
        z = r / (1.0 + r); zc = 1.0 / (1.0 + r);
        lz = log(nu) - 2.0 * log(at) - log1p(r); lzc = -log1p(r);
    } else {
        double den = nu + t * t;
        z = nu / den; zc = t * t / den;
        lz = log(z); lzc = zc > 0 ? log(zc) : -INFINITY;
    }
    double I, Ic;                     /* I = P(|T| > |t|) */
    or_betai2l(0.5 * nu, 0.5, z, zc, lz, lzc, &I, &Ic);
    return t < 0 ? 0.5 * I : 1.0 - 0.5 * I;
}

/* Univariate t density with scale parameter s (variance-like) and dof nu. */
double or_t1pdf(double x, double s, double nu)
{
    if (isinf(nu)) return exp(-0.5 * x * x / s) / sqrt(2.0 * M_PI * s);   /* normal limit */
    return exp(lgamma(0.5 * (nu + 1.0)) - lgamma(0.5 * nu) - 0.5 * log(M_PI * nu * s)
               - 0.5 * (nu + 1.0) * log1p(x * x / (nu * s)));
}

/* (nu + a) / (nu + b), with its limit 1 at nu = infinity. */
static double or_ratio(double nu, double a, double b)
{
    return isinf(nu) ? 1.0 : (nu + a) / (nu + b);
}

/* t quantile: solve T_nu(y) = p.  Works on the lower half (p <= 1/2) and
 * reflects.  Newton on log T_nu (quadratic in the far tail) inside a bracket
 * that is kept by bisection whenever a Newton step would leave it. */
double or_tinv(double p, double nu)
{
    if (!(p > 0.0)) return -INFINITY;
    if (!(p < 1.0)) return INFINITY;
    if (p == 0.5) return 0.0;
    double q = p < 0.5 ? p : 1.0 - p;        /* exact for p >= 1/2 */
    double lo = -1.0, hi = 0.0;
    while (or_tcdf(lo, nu) > q && lo > -1e300) { hi = lo; lo *= 2.0; }
    double lq = log(q);
    double y = 0.5 * (lo + hi);
    for (int it = 0; it < 500; ++it) {
        double F = or_tcdf(y, nu);
        if (F > q) hi = y; else lo = y;
        double dens = or_t1pdf(y, 1.0, nu);
        double yn = y - (log(F) - lq) * F / dens;
        if (!(yn > lo && yn < hi)) yn = 0.5 * (lo + hi);
        double step = fabs(yn - y);
        y = yn;
        if (step <= 1e-15 * fabs(y) || hi - lo <= 1e-15 * fabs(lo)) break;
    }
    return p < 0.5 ? y : -y;
}

/* ------------------------------------------------------------------------- */
/* small dense linear algebra (row-major)                                     */
/* ------------------------------------------------------------------------- */

/* Lower Cholesky A = L L^T.  Returns 0 on success, -1 if A is not SPD. */
static int or_chol(int n, const double *A, double *L)
{
    memset(L, 0, sizeof(double) * n * n);
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j <= i; ++j) {
            double s = A[i * n + j];
            for (int k = 0; k < j; ++k) s -= L[i * n + k] * L[j * n + k];
            if (i == j) {
                if (!(s > 0.0)) return -1;
                L[i * n + i] = sqrt(s);
            } else {
                L[i * n + j] = s / L[j * n + j];
            }
        }
    }
    return 0;
}

/* Solve A X = B for SPD A (n x n) and B (n x r), via Cholesky.  X overwrites B. */
static int or_spd_solve(int n, int r, const double *A, double *B)
{
    double L[16 * 16];
    if (or_chol(n, A, L)) return -1;
    for (int c = 0; c < r; ++c) {
        for (int i = 0; i < n; ++i) {
            double s = B[i * r + c];
            for (int k = 0; k < i; ++k) s -= L[i * n + k] * B[k * r + c];
            B[i * r + c] = s / L[i * n + i];
        }
        for (int i = n - 1; i >= 0; --i) {
            double s = B[i * r + c];
            for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * B[k * r + c];
            B[i * r + c] = s / L[i * n + i];
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* multivariate t CDF by separation of variables on a shifted lattice          */
/* ------------------------------------------------------------------------- */

typedef struct {
    int N, S;
    const int32_t *z;        /* [8] */
    const double *shifts;    /* [S][8] */
} or_qmc;

#define OR_LATDIM 8
#define OR_XCLAMP (1.0 / 16777216.0)   /* 2^-24 */

/* Lattice coordinate j of point k under shift s, after the tent transform. */
static double or_point(const or_qmc *Q, int s, long k, int j)
{
    long r = (k * (long)Q->z[j]) % Q->N;
    double t = (double)r / (double)Q->N + Q->shifts[s * OR_LATDIM + j];
    if (t >= 1.0) t -= 1.0;
    double x = 1.0 - fabs(2.0 * t - 1.0);
    if (x < OR_XCLAMP) x = OR_XCLAMP;
    if (x > 1.0 - OR_XCLAMP) x = 1.0 - OR_XCLAMP;
    return x;
}

/* T_m(b; 0, L L^T, nu).  m = 0 gives 1, m = 1 the univariate CDF, m >= 2 the
 * SOV lattice estimate (mean over shifts of the per-shift means); *se gets
 * the standard error over shifts (0 for the closed forms). */
double or_mvt(int m, const double *b, const double *L, double nu, const or_qmc *Q, double *se)
{
    if (se) *se = 0.0;
    if (m == 0) return 1.0;
    double e0 = or_tcdf(b[0] / L[0], nu);
    if (m == 1) return e0;
    double mean_s[64];
    int S = Q->S;
    double tot = 0.0;
    for (int s = 0; s < S; ++s) {
        double acc = 0.0;
        for (long k = 0; k < Q->N; ++k) {
            if (e0 == 0.0) break;
            double y[OR_MAXM];
            double f = e0;
            y[0] = or_tinv(or_point(Q, s, k, 0) * e0, nu);
            double s2 = y[0] * y[0];
            for (int i = 1; i < m; ++i) {
                double sc = sqrt(or_ratio(nu, s2, i));
                double num = b[i];
                for (int j = 0; j < i; ++j) num -= L[i * m + j] * y[j];
                double e = or_tcdf(num / (L[i * m + i] * sc), nu + i);
                f *= e;
                if (f == 0.0) break;
                if (i < m - 1) {
                    y[i] = sc * or_tinv(or_point(Q, s, k, i) * e, nu + i);
                    s2 += y[i] * y[i];
                }
            }
            acc += f;
        }
        mean_s[s] = acc / Q->N;
        tot += mean_s[s];
    }
    double est = tot / S;
    if (se && S > 1) {
        double v = 0.0;
        for (int s = 0; s < S; ++s) v += (mean_s[s] - est) * (mean_s[s] - est);
        *se = sqrt(v / ((double)S * (S - 1)));
    }
    return est;
}

/* Direct SOV moments: the same points and weights f = e_0 e_1 ... e_{m-1} as
 * or_mvt, but every coordinate of the point is drawn (the last one with
 * lattice coordinate m-1), z = L y, and
 *     P = E[1{Z<=b}],  M1 = E[Z 1{Z<=b}],  M2 = E[Z Z^T 1{Z<=b}]
 * (Z ~ t_m(0, L L^T, nu)) are the lattice means of f, f z, f z z^T.
 * M2 is dense m x m.  m >= 1. */
void or_mvt_mom(int m, const double *b, const double *L, double nu, const or_qmc *Q,
                double *P, double *M1, double *M2)
{
    double e0 = or_tcdf(b[0] / L[0], nu);
    double sP = 0.0, s1[OR_MAXM], s2m[OR_MAXM * OR_MAXM];
    for (int i = 0; i < m; ++i) s1[i] = 0.0;
    for (int i = 0; i < m * m; ++i) s2m[i] = 0.0;
    for (int s = 0; s < Q->S; ++s) {
        double a0 = 0.0, a1[OR_MAXM], a2[OR_MAXM * OR_MAXM];
        for (int i = 0; i < m; ++i) a1[i] = 0.0;
        for (int i = 0; i < m * m; ++i) a2[i] = 0.0;
        for (long k = 0; k < Q->N; ++k) {
            if (e0 == 0.0) break;
            double y[OR_MAXM], zz[OR_MAXM];
            double f = e0;
            y[0] = or_tinv(or_point(Q, s, k, 0) * e0, nu);
            double s2 = y[0] * y[0];
            for (int i = 1; i < m && f > 0.0; ++i) {
                double sc = sqrt(or_ratio(nu, s2, i));
                double num = b[i];
                for (int j = 0; j < i; ++j) num -= L[i * m + j] * y[j];
                double e = or_tcdf(num / (L[i * m + i] * sc), nu + i);
                f *= e;
                if (f == 0.0) break;
                y[i] = sc * or_tinv(or_point(Q, s, k, i) * e, nu + i);
                s2 += y[i] * y[i];
            }
            if (f == 0.0) continue;
            for (int i = 0; i < m; ++i) {
                double v = 0.0;
                for (int j = 0; j <= i; ++j) v += L[i * m + j] * y[j];
                zz[i] = v;
            }
            a0 += f;
            for (int i = 0; i < m; ++i) {
                a1[i] += f * zz[i];
                for (int k2 = 0; k2 < m; ++k2) a2[i * m + k2] += f * zz[i] * zz[k2];
            }
        }
        sP += a0 / Q->N;
        for (int i = 0; i < m; ++i) s1[i] += a1[i] / Q->N;
        for (int i = 0; i < m * m; ++i) s2m[i] += a2[i] / Q->N;
    }
    *P = sP / Q->S;
    for (int i = 0; i < m; ++i) M1[i] = s1[i] / Q->S;
    for (int i = 0; i < m * m; ++i) M2[i] = s2m[i] / Q->S;
}

/* T_m(b; 0, R, nu) for a dense SPD R. */
static double or_mvt_dense(int m, const double *b, const double *R, double nu, const or_qmc *Q)
{
    if (m == 0) return 1.0;
    double L[OR_MAXM * OR_MAXM];
    if (or_chol(m, R, L)) return NAN;
    return or_mvt(m, b, L, nu, Q, NULL);
}

/* ------------------------------------------------------------------------- */
/* truncated multivariate t moments                                           */
/* ------------------------------------------------------------------------- */
/* Z ~ t_m(0, R, nu).  For each i the conditional piece obtained by fixing
 * z_i = a_i in the gradient identity is
 *     kappa_i = (nu + a_i^2/R_ii)/(nu-1),  mvec = R_{-i,i} a_i / R_ii,
 *     V_i = kappa_i (R_{-i,-i} - R_{-i,i} R_{i,-i} / R_ii),  b_i = a_{-i} - mvec,
 *     xi_i = t1(a_i; R_ii, nu) kappa_i T_{m-1}(b_i; V_i, nu-1).
 * Then E[Z 1{Z<=a}] = -R xi and
 *     E[Z Z^T 1{Z<=a}] = nu/(nu-2) T_m(a; nu/(nu-2) R, nu-2) R - G R,
 *     G[:,i] = R[:,i]/R_ii a_i xi_i - t1(a_i;R_ii,nu) kappa_i embed_i(V_i xi^(i)),
 * with xi^(i) the xi vector of the (m-1)-variate problem (b_i, V_i, nu-1). */

typedef struct {
    double kappa, t1;
    double b[OR_MAXM];              /* b_i (m-1) */
    double V[OR_MAXM * OR_MAXM];    /* V_i (m-1)x(m-1) */
} or_cond;

static void or_condition(int m, const double *a, const double *R, double nu, int i, or_cond *c)
{
    double Rii = R[i * m + i];
    c->kappa = or_ratio(nu, a[i] * a[i] / Rii, -1.0);
    c->t1 = or_t1pdf(a[i], Rii, nu);
    int r = 0;
    for (int k = 0; k < m; ++k) {
        if (k == i) continue;
        c->b[r] = a[k] - R[k * m + i] * a[i] / Rii;
        int cc = 0;
        for (int l = 0; l < m; ++l) {
            if (l == i) continue;
            c->V[r * (m - 1) + cc] = c->kappa * (R[k * m + l] - R[k * m + i] * R[i * m + l] / Rii);
            ++cc;
        }
        ++r;
    }
}

/* xi vector of the problem (a, R, nu) of dimension m. */
static void or_xi(int m, const double *a, const double *R, double nu, const or_qmc *Q, double *xi)
{
    for (int i = 0; i < m; ++i) {
        or_cond c;
        or_condition(m, a, R, nu, i, &c);
        xi[i] = c.t1 * c.kappa * or_mvt_dense(m - 1, c.b, c.V, nu - 1.0, Q);
    }
}

/* M0 = T_m(a;R,nu), M1 = E[Z 1{Z<=a}], M2 = E[Z Z^T 1{Z<=a}];
 * T2 receives T_m(a; nu/(nu-2) R, nu-2). */
void or_tmoments(int m, const double *a, const double *R, double nu, const or_qmc *Q,
                 double *M0, double *M1, double *M2, double *T2)
{
    double xi[OR_MAXM], G[OR_MAXM * OR_MAXM], R2[OR_MAXM * OR_MAXM];
    *M0 = or_mvt_dense(m, a, R, nu, Q);
    or_xi(m, a, R, nu, Q, xi);
    for (int i = 0; i < m; ++i) {
        double s = 0.0;
        for (int k = 0; k < m; ++k) s += R[i * m + k] * xi[k];
        M1[i] = -s;
    }
    const double r2 = or_ratio(nu, 0.0, -2.0);
    for (int k = 0; k < m * m; ++k) R2[k] = R[k] * r2;
    double t2 = or_mvt_dense(m, a, R2, nu - 2.0, Q);
    if (T2) *T2 = t2;
    for (int i = 0; i < m; ++i) {
        or_cond c;
        or_condition(m, a, R, nu, i, &c);
        double xs[OR_MAXM], Vx[OR_MAXM];
        or_xi(m - 1, c.b, c.V, nu - 1.0, Q, xs);
        for (int r = 0; r < m - 1; ++r) {
            double s = 0.0;
            for (int l = 0; l < m - 1; ++l) s += c.V[r * (m - 1) + l] * xs[l];
            Vx[r] = s;
        }
        int r = 0;
        for (int k = 0; k < m; ++k) {
            double gk = R[k * m + i] / R[i * m + i] * a[i] * xi[i];
            if (k != i) { gk -= c.t1 * c.kappa * Vx[r]; ++r; }
            G[k * m + i] = gk;
        }
    }
    for (int i = 0; i < m; ++i)
        for (int k = 0; k < m; ++k) {
            double s = 0.0;
            for (int l = 0; l < m; ++l) s += G[i * m + l] * R[l * m + k];
            M2[i * m + k] = r2 * t2 * R[i * m + k] - s;
        }
}

/* ------------------------------------------------------------------------- */
/* E-step                                                                     */
/* ------------------------------------------------------------------------- */

/* Outputs use the [g][.][rows] layout; e3 holds the packed upper triangle
 * (row-major, (i,k) with i <= k).  logf_comp[h][r] = log f_h(y_j) (eq. 4),
 * logf_obs[r] = log sum_h pi_h f_h(y_j).  intA/intB (optional) receive the
 * density CDF T_q(c sqrt((nu+p)/(nu+d)); Lambda, nu+p) and the w-numerator CDF.
 * rows: observation indices to evaluate (NULL = all n).  Returns 0 or -(h+1)
 * if Omega_h or Lambda_h is not SPD. */
int or_estep(int n, int p, int q, int g, const double *y,
             const double *pi, const double *mu, const double *Sigma, const double *Delta,
             const double *nu, int N, int S, const int32_t *z, const double *shifts,
             const int32_t *rows, int nrows, int direct,
             double *tau, double *logf_obs, double *logf_comp,
             double *w, double *e1, double *e2, double *e3, double *intA, double *intB)
{
    or_qmc Q = {N, S, z, shifts};
    int nr = rows ? nrows : n;
    int nq2 = q * (q + 1) / 2;
    double *LO = malloc(sizeof(double) * g * p * p);     /* chol Omega */
    double *BB = malloc(sizeof(double) * g * p * q);     /* Omega^{-1} Delta */
    double *LAM = malloc(sizeof(double) * g * q * q);
    double *LLAM = malloc(sizeof(double) * g * q * q);
    double *logdet = malloc(sizeof(double) * g);
    int status = 0;
    for (int h = 0; h < g && !status; ++h) {
        double Om[16 * 16];
        const double *Sg = Sigma + (size_t)h * p * p, *Dl = Delta + (size_t)h * p * q;
        for (int i = 0; i < p; ++i)
            for (int k = 0; k < p; ++k) {
                double s = Sg[i * p + k];
                for (int l = 0; l < q; ++l) s += Dl[i * q + l] * Dl[k * q + l];
                Om[i * p + k] = s;
            }
        if (or_chol(p, Om, LO + (size_t)h * p * p)) { status = -(h + 1); break; }
        double ld = 0.0;
        for (int i = 0; i < p; ++i) ld += 2.0 * log(LO[(size_t)h * p * p + i * p + i]);
        logdet[h] = ld;
        double *Bh = BB + (size_t)h * p * q;
        memcpy(Bh, Dl, sizeof(double) * p * q);
        or_spd_solve(p, q, Om, Bh);
        for (int i = 0; i < q; ++i)
            for (int k = 0; k < q; ++k) {
                double s = (i == k) ? 1.0 : 0.0;
                for (int l = 0; l < p; ++l) s -= Dl[l * q + i] * Bh[l * q + k];
                LAM[(size_t)h * q * q + i * q + k] = s;
            }
        for (int i = 0; i < q; ++i)      /* symmetrise */
            for (int k = 0; k < i; ++k) {
                double v = 0.5 * (LAM[(size_t)h * q * q + i * q + k] + LAM[(size_t)h * q * q + k * q + i]);
                LAM[(size_t)h * q * q + i * q + k] = LAM[(size_t)h * q * q + k * q + i] = v;
            }
        if (or_chol(q, LAM + (size_t)h * q * q, LLAM + (size_t)h * q * q)) status = -(h + 1);
    }
    if (status) { free(LO); free(BB); free(LAM); free(LLAM); free(logdet); return status; }

    double *LF = malloc(sizeof(double) * (size_t)g * (nr > 0 ? nr : 1));
    /* every (observation, component) pair is independent (Sec. 4.1) */
    #pragma omp parallel for schedule(dynamic, 1) collapse(2)
    for (int r = 0; r < nr; ++r) {
        for (int h = 0; h < g; ++h) {
            int j = rows ? rows[r] : r;
            const double *Lo = LO + (size_t)h * p * p;
            const double *Bh = BB + (size_t)h * p * q;
            const double *Lam = LAM + (size_t)h * q * q;
            double nuh = nu[h];
            double res[16], v[16], c[OR_MAXM];
            for (int i = 0; i < p; ++i) res[i] = y[(size_t)j * p + i] - mu[(size_t)h * p + i];
            double d = 0.0;                         /* d = r^T Omega^{-1} r = |L^{-1} r|^2 */
            for (int i = 0; i < p; ++i) {
                double s = res[i];
                for (int k = 0; k < i; ++k) s -= Lo[i * p + k] * v[k];
                v[i] = s / Lo[i * p + i];
                d += v[i] * v[i];
            }
            for (int i = 0; i < q; ++i) {           /* c = Delta^T Omega^{-1} r = B^T r */
                double s = 0.0;
                for (int k = 0; k < p; ++k) s += Bh[k * q + i] * res[k];
                c[i] = s;
            }
            double logt = isinf(nuh)                /* normal limit: log phi_p(y; mu, Omega) */
                          ? -0.5 * p * log(2.0 * M_PI) - 0.5 * logdet[h] - 0.5 * d
                          : lgamma(0.5 * (nuh + p)) - lgamma(0.5 * nuh) - 0.5 * p * log(M_PI * nuh)
                            - 0.5 * logdet[h] - 0.5 * (nuh + p) * log1p(d / nuh);
            /* A = T_q(c sqrt((nu+p)/(nu+d)); 0, Lambda, nu+p) */
            double ca[OR_MAXM];
            double fa = sqrt(or_ratio(nuh, p, d));
            for (int i = 0; i < q; ++i) ca[i] = c[i] * fa;
            double A = or_mvt(q, ca, LLAM + (size_t)h * q * q, nuh + p, &Q, NULL);
            /* U | y ~ tt_q(c, s Lambda, nu*; R+) with s = (nu+d)/nu*, nu* = nu+p+2 */
            double nus = nuh + p + 2.0, sc = or_ratio(nuh, d, p + 2.0);
            double Rm[OR_MAXM * OR_MAXM], M0, M1[OR_MAXM], M2[OR_MAXM * OR_MAXM], T2;
            if (direct && q >= 2) {
                /* Z = sqrt(sc) Zs, Zs ~ t_q(0, Lambda, nu*) truncated to Zs <= c / sqrt(sc) */
                double cb[OR_MAXM], Ms1[OR_MAXM], Ms2[OR_MAXM * OR_MAXM];
                double rs = sqrt(sc);
                for (int i = 0; i < q; ++i) cb[i] = c[i] / rs;
                or_mvt_mom(q, cb, LLAM + (size_t)h * q * q, nus, &Q, &M0, Ms1, Ms2);
                for (int i = 0; i < q; ++i) M1[i] = rs * Ms1[i];
                for (int k = 0; k < q * q; ++k) M2[k] = sc * Ms2[k];
            } else {
                for (int k = 0; k < q * q; ++k) Rm[k] = sc * Lam[k];
                or_tmoments(q, c, Rm, nus, &Q, &M0, M1, M2, &T2);
            }
            double Bv = M0;          /* T_q(c sqrt(nu_s/(nu+d)); Lambda, nu_s), nu_s = nu+p+2 */
            double lfh = q * M_LN2 + logt + log(A);
            LF[(size_t)h * nr + r] = lfh;
            size_t o = (size_t)h * nr + r;
            if (logf_comp) logf_comp[o] = lfh;
            if (intA) intA[o] = A;
            if (intB) intB[o] = Bv;
            double wv = 0.0, e1v = 0.0, EU[OR_MAXM], EUU[OR_MAXM * OR_MAXM];
            if (A > 0.0 && Bv > 0.0) {
                if (isinf(nuh)) {                 /* normal limit: W = 1 */
                    wv = 1.0;
                    e1v = 0.0;
                } else {
                    wv = (nuh + p) / (nuh + d) * Bv / A;
                    e1v = wv - log(0.5 * (nuh + d)) - (nuh + p) / (nuh + d) + or_digamma(0.5 * (nuh + p));
                }
                for (int i = 0; i < q; ++i) EU[i] = c[i] - M1[i] / Bv;
                for (int i = 0; i < q; ++i)
                    for (int k = 0; k < q; ++k)
                        EUU[i * q + k] = c[i] * c[k] - (c[i] * M1[k] + M1[i] * c[k]) / Bv
                                         + 0.5 * (M2[i * q + k] + M2[k * q + i]) / Bv;
            } else {
                for (int i = 0; i < q; ++i) EU[i] = 0.0;
                for (int k = 0; k < q * q; ++k) EUU[k] = 0.0;
            }
            w[o] = wv;
            e1[o] = e1v;
            for (int i = 0; i < q; ++i) e2[((size_t)h * q + i) * nr + r] = wv * EU[i];
            int t = 0;
            for (int i = 0; i < q; ++i)
                for (int k = i; k < q; ++k, ++t)
                    e3[((size_t)h * nq2 + t) * nr + r] = wv * EUU[i * q + k];
        }
    }
    #pragma omp parallel for schedule(static)
    for (int r = 0; r < nr; ++r) {
        double lf[64];
        for (int h = 0; h < g; ++h) lf[h] = LF[(size_t)h * nr + r];
        /* eq. (12) and (27): tau_hj = pi_h f_h / sum_l pi_l f_l, via log-sum-exp */
        double mx = -INFINITY;
        for (int h = 0; h < g; ++h) {
            double v = log(pi[h]) + lf[h];
            if (v > mx) mx = v;
        }
        double s = 0.0;
        for (int h = 0; h < g; ++h) s += exp(log(pi[h]) + lf[h] - mx);
        double l = mx + log(s);
        logf_obs[r] = l;
        for (int h = 0; h < g; ++h) {
            double t = exp(log(pi[h]) + lf[h] - l);
            tau[(size_t)h * nr + r] = isfinite(l) ? t : 0.0;
            if (!(t > 0.0)) {      /* underflowed component: e-terms carry no weight */
                size_t o = (size_t)h * nr + r;
                w[o] = e1[o] = 0.0;
                for (int i = 0; i < q; ++i) e2[((size_t)h * q + i) * nr + r] = 0.0;
                for (int k = 0; k < nq2; ++k) e3[((size_t)h * nq2 + k) * nr + r] = 0.0;
            }
        }
    }
    free(LO); free(BB); free(LAM); free(LLAM); free(logdet); free(LF);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* M-step, eqs. (18)-(22)                                                     */
/* ------------------------------------------------------------------------- */

static double or_nu_eq(double nu, double mean_e1w)
{
    return log(0.5 * nu) - or_digamma(0.5 * nu) + 1.0 + mean_e1w;
}

/* Inputs in the E-step layout.  Outputs Psi^(k+1).  A component with
 * n_h < p + 1 keeps its mu, Sigma, Delta, nu (pi_h is still n_h / n); its bit
 * is set in *frozen.  Returns 0, or -(h+1) if sum tau e3 or Sigma is not SPD. */
int or_mstep(int n, int p, int q, int g, const double *y,
             const double *tau, const double *w, const double *e1, const double *e2,
             const double *e3, const double *pi0, const double *mu0, const double *Sigma0,
             const double *Delta0, const double *nu0,
             double *pi1, double *mu1, double *Sigma1, double *Delta1, double *nu1,
             int32_t *frozen)
{
    int nq2 = q * (q + 1) / 2;
    int status = 0;
    if (frozen) *frozen = 0;
    for (int h = 0; h < g; ++h) {
        double nh = 0.0, sw = 0.0, sew = 0.0, swy[16] = {0}, se2[OR_MAXM] = {0};
        for (int j = 0; j < n; ++j) {
            size_t o = (size_t)h * n + j;
            double t = tau[o];
            nh += t;
            sw += t * w[o];
            sew += t * (e1[o] - w[o]);
            for (int i = 0; i < p; ++i) swy[i] += t * w[o] * y[(size_t)j * p + i];
            for (int i = 0; i < q; ++i) se2[i] += t * e2[((size_t)h * q + i) * n + j];
        }
        pi1[h] = nh / n;                                        /* (18) */
        const double *Dk = Delta0 + (size_t)h * p * q;
        double *mu = mu1 + (size_t)h * p, *Dn = Delta1 + (size_t)h * p * q, *Sg = Sigma1 + (size_t)h * p * p;
        if (nh < p + 1.0) {
            memcpy(mu, mu0 + (size_t)h * p, sizeof(double) * p);
            memcpy(Dn, Dk, sizeof(double) * p * q);
            memcpy(Sg, Sigma0 + (size_t)h * p * p, sizeof(double) * p * p);
            nu1[h] = nu0[h];
            if (frozen) *frozen |= 1 << h;
            continue;
        }
        for (int i = 0; i < p; ++i) {                           /* (19), uses Delta^(k) */
            double s = swy[i];
            for (int l = 0; l < q; ++l) s -= Dk[i * q + l] * se2[l];
            mu[i] = s / sw;
        }
        double X[16 * OR_MAXM] = {0}, E3[OR_MAXM * OR_MAXM] = {0};
        for (int j = 0; j < n; ++j) {
            double t = tau[(size_t)h * n + j];
            for (int i = 0; i < p; ++i) {
                double r = y[(size_t)j * p + i] - mu[i];
                for (int l = 0; l < q; ++l) X[i * q + l] += t * r * e2[((size_t)h * q + l) * n + j];
            }
            int k = 0;
            for (int a = 0; a < q; ++a)
                for (int b = a; b < q; ++b, ++k) {
                    double v = t * e3[((size_t)h * nq2 + k) * n + j];
                    E3[a * q + b] += v;
                    if (b != a) E3[b * q + a] += v;
                }
        }
        /* (20): Delta = X E3^{-1}, i.e. Delta^T = E3^{-1} X^T */
        double XT[OR_MAXM * 16];
        for (int i = 0; i < p; ++i)
            for (int l = 0; l < q; ++l) XT[l * p + i] = X[i * q + l];
        if (or_spd_solve(q, p, E3, XT)) { status = -(h + 1); continue; }
        for (int i = 0; i < p; ++i)
            for (int l = 0; l < q; ++l) Dn[i * q + l] = XT[l * p + i];
        /* (21) with mu^(k+1), Delta^(k+1) */
        double A[16 * 16] = {0};
        for (int j = 0; j < n; ++j) {
            size_t o = (size_t)h * n + j;
            double t = tau[o];
            if (t == 0.0) continue;
            double r[16], De2[16], e3f[OR_MAXM * OR_MAXM];
            for (int i = 0; i < p; ++i) r[i] = y[(size_t)j * p + i] - mu[i];
            for (int i = 0; i < p; ++i) {
                double s = 0.0;
                for (int l = 0; l < q; ++l) s += Dn[i * q + l] * e2[((size_t)h * q + l) * n + j];
                De2[i] = s;
            }
            int k = 0;
            for (int a = 0; a < q; ++a)
                for (int b = a; b < q; ++b, ++k)
                    e3f[a * q + b] = e3f[b * q + a] = e3[((size_t)h * nq2 + k) * n + j];
            for (int a = 0; a < p; ++a)
                for (int b = 0; b < p; ++b) {
                    double dd = 0.0;
                    for (int l = 0; l < q; ++l)
                        for (int m = 0; m < q; ++m) dd += Dn[a * q + l] * e3f[l * q + m] * Dn[b * q + m];
                    A[a * p + b] += t * (w[o] * r[a] * r[b] - De2[a] * r[b] - r[a] * De2[b] + dd);
                }
        }
        for (int a = 0; a < p; ++a)
            for (int b = 0; b < p; ++b) Sg[a * p + b] = 0.5 * (A[a * p + b] + A[b * p + a]) / nh;
        double Lt[16 * 16];
        if (or_chol(p, Sg, Lt)) status = -(h + 1);
        /* (22), last sum with "+": log(nu/2) - psi(nu/2) + 1 + (1/n_h) sum tau (e1 - w) = 0 */
        double m = sew / nh;
        double lo = 1.0, hi = 200.0;
        if (isinf(nu0[h])) nu1[h] = nu0[h];      /* normal limit: nu stays infinite */
        else if (or_nu_eq(lo, m) <= 0.0) nu1[h] = lo;
        else if (or_nu_eq(hi, m) >= 0.0) nu1[h] = hi;
        else {
            for (int it = 0; it < 100; ++it) {
                double mid = 0.5 * (lo + hi);
                if (or_nu_eq(mid, m) > 0.0) lo = mid; else hi = mid;
            }
            nu1[h] = 0.5 * (lo + hi);
        }
    }
    return status;
}

/* ------------------------------------------------------------------------- */
/* flat entry points for the Python wrapper                                   */
/* ------------------------------------------------------------------------- */
#ifdef _OPENMP
#include <omp.h>
#endif

void or_set_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

int or_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

double or_mvt_c(int m, const double *b, const double *L, double nu, int N, int S,
                const int32_t *z, const double *shifts, double *se)
{
    or_qmc Q = {N, S, z, shifts};
    return or_mvt(m, b, L, nu, &Q, se);
}

void or_mvt_mom_c(int m, const double *b, const double *L, double nu, int N, int S,
                  const int32_t *z, const double *shifts, double *P, double *M1, double *M2)
{
    or_qmc Q = {N, S, z, shifts};
    or_mvt_mom(m, b, L, nu, &Q, P, M1, M2);
}

void or_tmoments_c(int m, const double *a, const double *R, double nu, int N, int S,
                   const int32_t *z, const double *shifts,
                   double *M0, double *M1, double *M2, double *T2)
{
    or_qmc Q = {N, S, z, shifts};
    or_tmoments(m, a, R, nu, &Q, M0, M1, M2, T2);
}
