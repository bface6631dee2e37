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
#include <type_traits>

#include "cfust_devmath.h"
#include "cfust_kernels.h"

namespace cfust {

constexpr int MS_TILE = 64;
constexpr int MS_STRIDE = MS_TILE + 1;           // pad: rows land in different banks
constexpr int MS_ROWS64_PER_WAVE = (MAXP + 1 + 3) / 4;                       // y rows + tau, 4 waves
constexpr int MS_EROWS_PER_WAVE = (2 + MAXQ + MAXQ * (MAXQ + 1) / 2 + 3) / 4;  // w, e1, e2, e3

// Row layout of the staged tile.  Raw rows r_i = y_i - mu_i, tau, w, e1;
// rows weighted in place tau e2_l, tau e3_t; rows added by the weighting
// pass tau w, tau (e1 - w), tau w r_i; and a row of ones.  Every statistic is
// then the sum over the tile of the product of two rows.
struct MsRows {
    int r0, tau, w, e1, e20, e30, tw, te1w, twr0, one, nrows;
};

__host__ __device__ inline MsRows ms_rows(int p, int q) {
    MsRows R;
    R.r0 = 0; R.tau = p; R.w = p + 1; R.e1 = p + 2; R.e20 = p + 3; R.e30 = p + 3 + q;
    R.tw = R.e30 + q * (q + 1) / 2; R.te1w = R.tw + 1; R.twr0 = R.tw + 2;
    R.one = R.twr0 + p;
    R.nrows = R.one + 1;
    return R;
}

// LDS bytes of the staged tile.
__host__ __device__ inline size_t ms_lds_bytes(int p, int q) {
    return (size_t)ms_rows(p, q).nrows * MS_STRIDE * sizeof(double);
}

// Statistic s as the product of two staged rows:
//   0 n_h            tau . 1
//   1 sum tau w      tau w . 1
//   2 sum tau (e1-w) tau (e1-w) . 1
//   3.. p            tau w r_i . 1
//   q                tau e2_l . 1
//   p(p+1)/2         tau w r_i . r_k   (i <= k)
//   p q              r_i . tau e2_l
//   q(q+1)/2         tau e3_t . 1
__device__ inline void ms_stat_rows(int s, int p, int q, const MsRows &R, int *f) {
    f[1] = R.one;
    if (s == 0) { f[0] = R.tau; return; }
    if (s == 1) { f[0] = R.tw; return; }
    if (s == 2) { f[0] = R.te1w; return; }
    s -= 3;
    if (s < p) { f[0] = R.twr0 + s; return; }
    s -= p;
    if (s < q) { f[0] = R.e20 + s; return; }
    s -= q;
    if (s < p * (p + 1) / 2) {
        int i = 0;
        while (s >= p - i) { s -= p - i; ++i; }
        f[0] = R.twr0 + i; f[1] = R.r0 + i + s;
        return;
    }
    s -= p * (p + 1) / 2;
    if (s < p * q) { f[0] = R.r0 + s / q; f[1] = R.e20 + s % q; return; }
    s -= p * q;
    f[0] = R.e30 + s;
}

// Block bx of component h of one fit; `tile` is the block's dynamic LDS
// (ms_lds_bytes).
template <bool MIXED>
__device__ inline void mstep_reduce_prec(const MstepArgs &a, int bx, int h, double *tile) {
    using E = typename std::conditional<MIXED, float, double>::type;   // storage of w, e1, e2, e3
    const int p = a.p, q = a.q, n = a.n;
    const int nq2 = q * (q + 1) / 2;
    const MsRows R = ms_rows(p, q);
    const int NS = nstat(p, q);
    int fa[2], fb[2];
    const int s0 = threadIdx.x, s1 = threadIdx.x + 256;
    if (s0 < NS) ms_stat_rows(s0, p, q, R, fa);
    if (s1 < NS) ms_stat_rows(s1, p, q, R, fb);
    double acc0 = 0.0, acc1 = 0.0;
    const double *mu0 = a.mu0 + (size_t)h * p;
    const int ntiles = (n + MS_TILE - 1) / MS_TILE;
    // Raw rows of one tile, held in registers: wave w takes rows w, w+4, ...,
    // one observation per lane (coalesced).  A wave's rows are fixed, so their
    // base pointers are wave-uniform values set up once; the loads carry no
    // branches (indices clamped into range; rows past the last one re-read
    // the last row and are dropped at the store), so all of a wave's loads
    // are in flight together, and the next tile's loads are issued before the
    // current tile is weighted and reduced.
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int ne = 2 + q + nq2;                  // rows w, e1, e2_l, e3_t
    const size_t hn = (size_t)h * n;
    const double *src64[MS_ROWS64_PER_WAVE];
    double off64[MS_ROWS64_PER_WAVE];
#pragma unroll
    for (int k = 0; k < MS_ROWS64_PER_WAVE; ++k) {
        const int row = min(wave + 4 * k, p);    // rows 0..p-1: y_i - mu_i; row p: tau
        src64[k] = row < p ? a.y + (size_t)row * n : a.tau + hn;
        off64[k] = row < p ? mu0[row] : 0.0;
    }
    const E *srce[MS_EROWS_PER_WAVE];
#pragma unroll
    for (int k = 0; k < MS_EROWS_PER_WAVE; ++k) {
        const int e = min(wave + 4 * k, ne - 1);
        srce[k] = e == 0 ? (const E *)a.w + hn
                : e == 1 ? (const E *)a.e1 + hn
                : e < 2 + q ? (const E *)a.e2 + ((size_t)h * q + (e - 2)) * n
                            : (const E *)a.e3 + ((size_t)h * nq2 + (e - 2 - q)) * n;
    }
    double v64[MS_ROWS64_PER_WAVE];
    E ve[MS_EROWS_PER_WAVE];
    auto load_tile = [&](int tl) {
        if (tl >= ntiles) return;                // uniform: nothing past the last tile
        const int jc = min(tl * MS_TILE + lane, n - 1);
#pragma unroll
        for (int k = 0; k < MS_ROWS64_PER_WAVE; ++k) v64[k] = src64[k][jc];
#pragma unroll
        for (int k = 0; k < MS_EROWS_PER_WAVE; ++k) ve[k] = srce[k][jc];
    };
    load_tile(bx);
    for (int tl = bx; tl < ntiles; tl += a.nblk) {
        const bool in = tl * MS_TILE + lane < n;
#pragma unroll
        for (int k = 0; k < MS_ROWS64_PER_WAVE; ++k) {
            const int row = wave + 4 * k;
            if (row <= p) tile[row * MS_STRIDE + lane] = in ? v64[k] - off64[k] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < MS_EROWS_PER_WAVE; ++k) {
            const int e = wave + 4 * k;
            if (e < ne) tile[(R.w + e) * MS_STRIDE + lane] = in ? (double)ve[k] : 0.0;
        }
        __syncthreads();
        load_tile(tl + a.nblk);
        // weight by tau: e2, e3 in place; tau w, tau (e1 - w), tau w r_i, ones as new rows
        for (int e = threadIdx.x; e < (R.nrows - R.e20) * MS_TILE; e += blockDim.x) {
            const int row = R.e20 + e / MS_TILE, o = e % MS_TILE;
            const double t = tile[R.tau * MS_STRIDE + o], w = tile[R.w * MS_STRIDE + o];
            double v;
            if (row < R.tw) v = t * tile[row * MS_STRIDE + o];
            else if (row == R.tw) v = t * w;
            else if (row == R.te1w) v = t * (tile[R.e1 * MS_STRIDE + o] - w);
            else if (row < R.one) v = t * w * tile[(R.r0 + row - R.twr0) * MS_STRIDE + o];
            else v = 1.0;
            tile[row * MS_STRIDE + o] = v;
        }
        __syncthreads();
        if (s0 < NS) {
            const double *t0 = tile + fa[0] * MS_STRIDE, *t1 = tile + fa[1] * MS_STRIDE;
            double s = 0.0;
            for (int o = 0; o < MS_TILE; ++o) s += t0[o] * t1[o];
            acc0 += s;
        }
        if (s1 < NS) {
            const double *t0 = tile + fb[0] * MS_STRIDE, *t1 = tile + fb[1] * MS_STRIDE;
            double s = 0.0;
            for (int o = 0; o < MS_TILE; ++o) s += t0[o] * t1[o];
            acc1 += s;
        }
        __syncthreads();
    }
    double *out = a.partial + ((size_t)h * a.nblk + bx) * NS;
    if (s0 < NS) out[s0] = acc0;
    if (s1 < NS) out[s1] = acc1;
}

__device__ inline void mstep_reduce_body(const MstepArgs &a, int bx, int h, double *tile) {
    if (a.mixed) mstep_reduce_prec<true>(a, bx, h, tile);
    else mstep_reduce_prec<false>(a, bx, h, tile);
}

__global__ __launch_bounds__(256) void k_mstep_reduce(MstepArgs a) {
    extern __shared__ double ms_tile[];
    mstep_reduce_body(a, blockIdx.x, blockIdx.y, ms_tile);
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
    __shared__ int s_mode;                       // 0 keep theta, 1 clamp, 2 root search
    __shared__ double s_m, s_lo, s_hi;
    __shared__ unsigned long long s_mask[4];
    int status = 0;
    double mu[MAXP], Sg[MAXP * MAXP], Dn[MAXP * MAXQ], nu = a.nu0[h];
    if (threadIdx.x == 0) {
    const double nh = st[0], Sw = st[1], Sew = st[2];
    const double *Swr = st + 3, *Se2 = st + 3 + p, *Swrr = st + 3 + p + q;
    const double *Sre2 = Swrr + p * (p + 1) / 2, *Se3 = Sre2 + p * q;
    const double *mu0 = a.mu0 + (size_t)h * p, *S0 = a.Sigma0 + (size_t)h * p * p;
    const double *D0 = a.Delta0 + (size_t)h * p * q;
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
    s_mode = 0;
    if (!keep) {
        for (int i = 0; i < p; ++i) mu[i] = mu0[i] + dl[i];
        for (int i = 0; i < p * q; ++i) Dn[i] = Dnew[i];
        for (int i = 0; i < p * p; ++i) Sg[i] = Snew[i];
        const double m = Sew / nh;                                     // (22)
        s_m = m;
        s_lo = 1.0; s_hi = 200.0;
        s_mode = 2;
        if (ms_nu_eq(1.0, m) <= 0.0) { nu = 1.0; s_mode = 1; status |= CFUST_DEV_NU_CLAMPED; }
        else if (ms_nu_eq(200.0, m) >= 0.0) { nu = 200.0; s_mode = 1; status |= CFUST_DEV_NU_CLAMPED; }
    }
    }
    __syncthreads();
    if (s_mode == 2) {
        // eq. (22) decreases in nu: multisection of [lo, hi] by the block, each
        // round evaluating it at blockDim.x interior points and keeping the
        // interval of the first sign change (257-fold shrink per round)
        const double m = s_m, np1 = blockDim.x + 1.0;
        for (int round = 0; round < 8; ++round) {
            const double lo = s_lo, hi = s_hi;
            const double x = lo + (hi - lo) * (threadIdx.x + 1) / np1;
            const unsigned long long bal = __ballot(ms_nu_eq(x, m) <= 0.0);
            if ((threadIdx.x & 63) == 0) s_mask[threadIdx.x >> 6] = bal;
            __syncthreads();
            if (threadIdx.x == 0) {
                int first = blockDim.x;
                for (int w = 0; w < (int)(blockDim.x >> 6); ++w)
                    if (s_mask[w]) { first = w * 64 + __ffsll(s_mask[w]) - 1; break; }
                s_lo = lo + (hi - lo) * first / np1;
                s_hi = first == (int)blockDim.x ? hi : lo + (hi - lo) * (first + 1) / np1;
            }
            __syncthreads();
        }
        nu = 0.5 * (s_lo + s_hi);
    }
    if (threadIdx.x != 0) return;
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
    hipLaunchKernelGGL(k_mstep_reduce, dim3(r.nblk, r.g), dim3(256), ms_lds_bytes(r.p, r.q), st, r);
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
    extern __shared__ double ms_tile[];
    mstep_reduce_body(a, local % a.nblk, local / a.nblk, ms_tile);
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

size_t mstep_lds_bytes(int p, int q) { return ms_lds_bytes(p, q); }

hipError_t launch_batch_mstep(const BatchArgs &b, int nred, int nsol, size_t lds, hipStream_t s) {
    if (nred > 0) hipLaunchKernelGGL(k_batch_mreduce, dim3(nred), dim3(256), lds, s, b);
    if (nsol > 0) hipLaunchKernelGGL(k_batch_msolve, dim3(nsol), dim3(256), 0, s, b);
    if (b.nfits > 0) hipLaunchKernelGGL(k_batch_mstatus, dim3(b.nfits), dim3(64), 0, s, b);
    return hipGetLastError();
}

}  // namespace cfust
