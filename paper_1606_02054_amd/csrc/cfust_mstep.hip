// cfust_mstep.hip -- M-step of the CFUST mixture (Sec. 3.2, eqs. 18-22).
//
//   k_mstep_reduce  grid (blocks, component): FP64 weighted sums over the
//                   observations of a component, in coordinates shifted by
//                   mu_h^(k) for conditioning.  A tile of 64 observations is
//                   staged in LDS (coalesced SoA reads, each input read once);
//                   every thread then owns one or two statistics.  Partials
//                   per block are written out and summed in a fixed order, so
//                   results are reproducible run to run.
//   k_mstep_solve   one block per component: sums the partials, then the
//                   closed-form updates pi, mu, Delta, Sigma and the nu root.
#include "cfust_devmath.h"
#include "cfust_kernels.h"

namespace cfust {

constexpr int MS_TILE = 64;
constexpr int MS_STRIDE = MS_TILE + 1;           // pad: rows land in different banks
constexpr int MS_MAXROWS = MAXP + 4 + MAXQ + MAXQ * (MAXQ + 1) / 2;

// Row layout of the staged tile: r_0..r_{p-1}, tau, w, e1 - w, e2_0.., e3_0.., one.
struct MsRows {
    int r0, tau, w, e1w, e20, e30, one, nrows;
};

__device__ inline MsRows ms_rows(int p, int q) {
    MsRows R;
    R.r0 = 0; R.tau = p; R.w = p + 1; R.e1w = p + 2; R.e20 = p + 3; R.e30 = p + 3 + q;
    R.one = R.e30 + q * (q + 1) / 2;
    R.nrows = R.one + 1;
    return R;
}

// Statistic s as a product of up to four staged rows.
//   0 n_h            tau
//   1 sum tau w      tau w
//   2 sum tau (e1-w) tau (e1-w)
//   3.. p            tau w r_i
//   q                tau e2_l
//   p(p+1)/2         tau w r_i r_k   (i <= k)
//   p q              tau r_i e2_l
//   q(q+1)/2         tau e3_t
__device__ inline void ms_stat_rows(int s, int p, int q, const MsRows &R, int *f) {
    f[0] = R.tau; f[1] = R.one; f[2] = R.one; f[3] = R.one;
    if (s == 0) return;
    if (s == 1) { f[1] = R.w; return; }
    if (s == 2) { f[1] = R.e1w; return; }
    s -= 3;
    if (s < p) { f[1] = R.w; f[2] = R.r0 + s; return; }
    s -= p;
    if (s < q) { f[1] = R.e20 + s; return; }
    s -= q;
    if (s < p * (p + 1) / 2) {
        int i = 0;
        while (s >= p - i) { s -= p - i; ++i; }
        f[1] = R.w; f[2] = R.r0 + i; f[3] = R.r0 + i + s;
        return;
    }
    s -= p * (p + 1) / 2;
    if (s < p * q) { f[1] = R.r0 + s / q; f[2] = R.e20 + s % q; return; }
    s -= p * q;
    f[1] = R.e30 + s;
}

// Block bx of component h of one fit.
__device__ inline void mstep_reduce_body(const MstepArgs &a, int bx, int h) {
    __shared__ double tile[MS_MAXROWS * MS_STRIDE];
    const int p = a.p, q = a.q, n = a.n;
    const int nq2 = q * (q + 1) / 2;
    const MsRows R = ms_rows(p, q);
    const int NS = nstat(p, q);
    int fa[4], fb[4];
    const int s0 = threadIdx.x, s1 = threadIdx.x + 256;
    if (s0 < NS) ms_stat_rows(s0, p, q, R, fa);
    if (s1 < NS) ms_stat_rows(s1, p, q, R, fb);
    double acc0 = 0.0, acc1 = 0.0;
    const double *mu0 = a.mu0 + (size_t)h * p;
    const int ntiles = (n + MS_TILE - 1) / MS_TILE;
    for (int tl = bx; tl < ntiles; tl += a.nblk) {
        const int base = tl * MS_TILE;
        // stage: each (row, obs) element once, coalesced along observations
        for (int e = threadIdx.x; e < R.nrows * MS_TILE; e += blockDim.x) {
            const int row = e / MS_TILE, o = e % MS_TILE, j = base + o;
            double v = 0.0;
            if (j < n) {
                const size_t hj = (size_t)h * n + j;
                if (row < p) v = a.y[(size_t)row * n + j] - mu0[row];
                else if (row == R.tau) v = a.tau[hj];
                else if (row == R.w) v = a.mixed ? (double)((const float *)a.w)[hj] : ((const double *)a.w)[hj];
                else if (row == R.e1w) {
                    const double e1 = a.mixed ? (double)((const float *)a.e1)[hj] : ((const double *)a.e1)[hj];
                    const double w = a.mixed ? (double)((const float *)a.w)[hj] : ((const double *)a.w)[hj];
                    v = e1 - w;
                } else if (row < R.e30) {
                    const size_t ix = ((size_t)h * q + (row - R.e20)) * n + j;
                    v = a.mixed ? (double)((const float *)a.e2)[ix] : ((const double *)a.e2)[ix];
                } else if (row < R.one) {
                    const size_t ix = ((size_t)h * nq2 + (row - R.e30)) * n + j;
                    v = a.mixed ? (double)((const float *)a.e3)[ix] : ((const double *)a.e3)[ix];
                } else v = 1.0;
            }
            tile[row * MS_STRIDE + o] = v;
        }
        __syncthreads();
        if (s0 < NS) {
            const double *t0 = tile + fa[0] * MS_STRIDE, *t1 = tile + fa[1] * MS_STRIDE;
            const double *t2 = tile + fa[2] * MS_STRIDE, *t3 = tile + fa[3] * MS_STRIDE;
            double s = 0.0;
            for (int o = 0; o < MS_TILE; ++o) s += t0[o] * t1[o] * t2[o] * t3[o];
            acc0 += s;
        }
        if (s1 < NS) {
            const double *t0 = tile + fb[0] * MS_STRIDE, *t1 = tile + fb[1] * MS_STRIDE;
            const double *t2 = tile + fb[2] * MS_STRIDE, *t3 = tile + fb[3] * MS_STRIDE;
            double s = 0.0;
            for (int o = 0; o < MS_TILE; ++o) s += t0[o] * t1[o] * t2[o] * t3[o];
            acc1 += s;
        }
        __syncthreads();
    }
    double *out = a.partial + ((size_t)h * a.nblk + bx) * NS;
    if (s0 < NS) out[s0] = acc0;
    if (s1 < NS) out[s1] = acc1;
}

__global__ __launch_bounds__(256) void k_mstep_reduce(MstepArgs a) {
    mstep_reduce_body(a, blockIdx.x, blockIdx.y);
}

__device__ inline bool ms_chol(double *A, int n) {
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j <= i; ++j) {
            double s = A[i * n + j];
            for (int k = 0; k < j; ++k) s -= A[i * n + k] * A[j * n + k];
            if (i == j) {
                if (!(s > 0.0) || !isfinite(s)) return false;
                A[i * n + i] = sqrt(s);
            } else {
                A[i * n + j] = s / A[j * n + j];
            }
        }
    }
    return true;
}

// eq. (22) with "+": log(nu/2) - psi(nu/2) + 1 + mean(e1 - w)
__device__ inline double ms_nu_eq(double v, double m) {
    return log(0.5 * v) - dm_digamma(0.5 * v) + 1.0 + m;
}

// Component h of one fit.
__device__ inline void mstep_solve_body(const MsolveArgs &a, int32_t *cstat, int h) {
    __shared__ double st[512];
    const int p = a.p, q = a.q;
    const int NS = nstat(p, q);
    for (int s = threadIdx.x; s < NS; s += blockDim.x) {
        double v = 0.0;
        for (int b = 0; b < a.nblk; ++b) v += a.partial[((size_t)h * a.nblk + b) * NS + s];
        st[s] = v;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    int status = 0;
    const double nh = st[0], Sw = st[1], Sew = st[2];
    const double *Swr = st + 3, *Se2 = st + 3 + p, *Swrr = st + 3 + p + q;
    const double *Sre2 = Swrr + p * (p + 1) / 2, *Se3 = Sre2 + p * q;
    const double *mu0 = a.mu0 + (size_t)h * p, *S0 = a.Sigma0 + (size_t)h * p * p;
    const double *D0 = a.Delta0 + (size_t)h * p * q;
    double mu[MAXP], Sg[MAXP * MAXP], Dn[MAXP * MAXQ], nu = a.nu0[h];
    for (int i = 0; i < p; ++i) mu[i] = mu0[i];
    for (int i = 0; i < p * p; ++i) Sg[i] = S0[i];
    for (int i = 0; i < p * q; ++i) Dn[i] = D0[i];
    a.pi1[h] = a.n > 0 ? nh / a.n : 0.0;                               // (18)
    bool keep = false;
    if (!(nh >= p + 1.0)) { status |= CFUST_DEV_FROZEN; keep = true; }
    double dl[MAXP], X[MAXP * MAXQ], E3[MAXQ * MAXQ], Lc[MAXQ * MAXQ], Dnew[MAXP * MAXQ], Snew[MAXP * MAXP];
    if (!keep) {
        for (int i = 0; i < p; ++i) {                                  // (19), Delta^(k)
            double s = Swr[i];
            for (int l = 0; l < q; ++l) s -= D0[i * q + l] * Se2[l];
            dl[i] = s / Sw;
        }
        for (int i = 0; i < p; ++i)                                    // sum tau (y - mu1) e2^T
            for (int l = 0; l < q; ++l) X[i * q + l] = Sre2[i * q + l] - dl[i] * Se2[l];
        int t = 0;
        for (int i = 0; i < q; ++i)
            for (int k = i; k < q; ++k, ++t) E3[i * q + k] = E3[k * q + i] = Se3[t];
        for (int i = 0; i < q * q; ++i) Lc[i] = E3[i];
        if (!ms_chol(Lc, q)) { status |= CFUST_DEV_NOTSPD_E3; keep = true; }
        if (!keep) {
            for (int i = 0; i < p; ++i) {                              // (20): Delta E3 = X
                double z[MAXQ];
                for (int l = 0; l < q; ++l) {
                    double s = X[i * q + l];
                    for (int k = 0; k < l; ++k) s -= Lc[l * q + k] * z[k];
                    z[l] = s / Lc[l * q + l];
                }
                for (int l = q - 1; l >= 0; --l) {
                    double s = z[l];
                    for (int k = l + 1; k < q; ++k) s -= Lc[k * q + l] * z[k];
                    z[l] = s / Lc[l * q + l];
                }
                for (int l = 0; l < q; ++l) Dnew[i * q + l] = z[l];
            }
            // (21) with mu^(k+1), Delta^(k+1)
            double DE3[MAXP * MAXQ];
            for (int i = 0; i < p; ++i)
                for (int l = 0; l < q; ++l) {
                    double s = 0.0;
                    for (int k = 0; k < q; ++k) s += Dnew[i * q + k] * E3[k * q + l];
                    DE3[i * q + l] = s;
                }
            for (int i = 0; i < p; ++i)
                for (int k = i; k < p; ++k) {
                    const int ik = i * p - i * (i - 1) / 2 + (k - i);
                    double Wik = Swrr[ik] - dl[i] * Swr[k] - Swr[i] * dl[k] + Sw * dl[i] * dl[k];
                    double cross = 0.0, quad = 0.0;
                    for (int l = 0; l < q; ++l) {
                        cross += Dnew[i * q + l] * X[k * q + l] + X[i * q + l] * Dnew[k * q + l];
                        quad += DE3[i * q + l] * Dnew[k * q + l];
                    }
                    const double v = (Wik - cross + quad) / nh;
                    Snew[i * p + k] = v;
                    Snew[k * p + i] = v;
                }
            double Ls[MAXP * MAXP];
            for (int i = 0; i < p * p; ++i) Ls[i] = Snew[i];
            if (!ms_chol(Ls, p)) { status |= CFUST_DEV_NOTSPD_SIGMA; keep = true; }
        }
    }
    if (!keep) {
        for (int i = 0; i < p; ++i) mu[i] = mu0[i] + dl[i];
        for (int i = 0; i < p * q; ++i) Dn[i] = Dnew[i];
        for (int i = 0; i < p * p; ++i) Sg[i] = Snew[i];
        const double m = Sew / nh;                                     // (22)
        double lo = 1.0, hi = 200.0;
        if (ms_nu_eq(lo, m) <= 0.0) { nu = lo; status |= CFUST_DEV_NU_CLAMPED; }
        else if (ms_nu_eq(hi, m) >= 0.0) { nu = hi; status |= CFUST_DEV_NU_CLAMPED; }
        else {
            for (int it = 0; it < 100; ++it) {
                const double mid = 0.5 * (lo + hi);
                if (ms_nu_eq(mid, m) > 0.0) lo = mid; else hi = mid;
            }
            nu = 0.5 * (lo + hi);
        }
    }
    for (int i = 0; i < p; ++i) a.mu1[(size_t)h * p + i] = mu[i];
    for (int i = 0; i < p * q; ++i) a.Delta1[(size_t)h * p * q + i] = Dn[i];
    for (int i = 0; i < p * p; ++i) a.Sigma1[(size_t)h * p * p + i] = Sg[i];
    a.nu1[h] = nu;
    cstat[h] = status;
}

__global__ __launch_bounds__(256) void k_mstep_solve(MsolveArgs a, int32_t *cstat) {
    mstep_solve_body(a, cstat, blockIdx.x);
}

__global__ void k_mstep_status(const int32_t *__restrict__ cstat, int g, int32_t *__restrict__ status) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        int s = status[0];
        for (int h = 0; h < g; ++h) s |= cstat[h];
        status[0] = s;
    }
}

hipError_t launch_mstep(const MstepArgs &r, const MsolveArgs &s, hipStream_t st) {
    // always launched: with n = 0 it writes zero partials
    hipLaunchKernelGGL(k_mstep_reduce, dim3(r.nblk, r.g), dim3(256), 0, st, r);
    int32_t *cstat = (int32_t *)(r.partial + (size_t)r.g * r.nblk * nstat(r.p, r.q));
    hipLaunchKernelGGL(k_mstep_solve, dim3(s.g), dim3(256), 0, st, s, cstat);
    if (s.status) hipLaunchKernelGGL(k_mstep_status, dim3(1), dim3(64), 0, st, cstat, s.g, s.status);
    return hipGetLastError();
}

// ------------------------------------------------------------ batches ----

__device__ inline int mbatch_fit(const int *__restrict__ prefix, int nfits, int b) {
    int lo = 0, hi = nfits - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_batch_mreduce(BatchArgs B) {
    const int *pf = B.prefix + BK_MRED * (B.nfits + 1);
    const int f = mbatch_fit(pf, B.nfits, blockIdx.x);
    if (!B.active[f]) return;
    const MstepArgs a = B.fits[f].ma;
    const int local = blockIdx.x - pf[f];
    mstep_reduce_body(a, local % a.nblk, local / a.nblk);
}

__global__ __launch_bounds__(256) void k_batch_msolve(BatchArgs B) {
    const int *pf = B.prefix + BK_MSOL * (B.nfits + 1);
    const int f = mbatch_fit(pf, B.nfits, blockIdx.x);
    if (!B.active[f]) return;
    const FitDesc &F = B.fits[f];
    const MsolveArgs a = F.sa;
    mstep_solve_body(a, F.cstat, blockIdx.x - pf[f]);
}

__global__ void k_batch_mstatus(BatchArgs B) {
    const int f = blockIdx.x;
    if (threadIdx.x != 0 || !B.active[f]) return;
    const FitDesc &F = B.fits[f];
    if (!F.status) return;
    int s = F.status[0];
    for (int h = 0; h < F.g; ++h) s |= F.cstat[h];
    F.status[0] = s;
}

hipError_t launch_batch_mstep(const BatchArgs &b, int nred, int nsol, hipStream_t s) {
    if (nred > 0) hipLaunchKernelGGL(k_batch_mreduce, dim3(nred), dim3(256), 0, s, b);
    if (nsol > 0) hipLaunchKernelGGL(k_batch_msolve, dim3(nsol), dim3(256), 0, s, b);
    if (b.nfits > 0) hipLaunchKernelGGL(k_batch_mstatus, dim3(b.nfits), dim3(64), 0, s, b);
    return hipGetLastError();
}

}  // namespace cfust
