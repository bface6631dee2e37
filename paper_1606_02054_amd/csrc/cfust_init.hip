// cfust_init.hip -- starting values of the EM algorithm (Sec. 3.3, eq. 23,
// Algorithm 1): cluster statistics of every starting partition, the
// candidate parameter sets for every value of alpha, and the choice of the
// candidate with the largest log-likelihood (evaluated by a density-only
// batch, cfust_batch.hip).
//
//   k_init_reduce<0>  per (start, component): count and sum of y       (tile in LDS,
//   k_init_reduce<1>  per (start, component): centred cross products and  one statistic
//                     third powers about the cluster mean                 per thread)
//   k_init_stats      partial sums in a fixed order -> n_h, mean, S (divisor n_h - 1), m3
//   k_init_candidates per (candidate, component): eq. (23) and the validity checks
//   k_init_select     the first candidate with the largest log-likelihood
#include "cfust_kernels.h"

namespace cfust {

constexpr int IN_TILE = 64;
constexpr int IN_STRIDE = IN_TILE + 1;

__device__ inline int init_nstat(int pass, int p) { return pass == 0 ? 1 + p : p * (p + 1) / 2 + p; }

// Statistic s of a pass as the rows of the staged tile it multiplies
// (row p is the cluster indicator): pass 0: 1, y_i; pass 1: r_i r_k (i <= k), r_i^3.
template <int PASS>
__global__ __launch_bounds__(256) void k_init_reduce(InitArgs a) {
    __shared__ double tile[(MAXP + 1) * IN_STRIDE];
    const int bx = blockIdx.x, h = blockIdx.y, s = blockIdx.z;
    const int p = a.p, n = a.n;
    const int NS = init_nstat(PASS, p);
    const int st = threadIdx.x;
    int r0 = p, r1 = p, pow3 = 0;
    if (st < NS) {
        if (PASS == 0) {
            if (st > 0) r1 = st - 1;
        } else if (st < p * (p + 1) / 2) {
            int i = 0, t = st;
            while (t >= p - i) { t -= p - i; ++i; }
            r0 = i; r1 = i + t;
        } else {
            r0 = r1 = st - p * (p + 1) / 2;
            pow3 = 1;
        }
    }
    const double *mu = a.mean + ((size_t)s * a.g + h) * p;
    const int32_t *lab = a.labels + (size_t)s * n;
    double acc = 0.0;
    const int ntiles = (n + IN_TILE - 1) / IN_TILE;
    for (int tl = bx; tl < ntiles; tl += a.nblk) {
        const int base = tl * IN_TILE;
        for (int t = threadIdx.x; t < (p + 1) * IN_TILE; t += blockDim.x) {
            const int row = t / IN_TILE, o = t % IN_TILE, j = base + o;
            double v = 0.0;
            if (j < n) {
                if (row == p) v = lab[j] == h ? 1.0 : 0.0;
                else v = PASS == 0 ? a.y[(size_t)row * n + j] : a.y[(size_t)row * n + j] - mu[row];
            }
            tile[row * IN_STRIDE + o] = v;
        }
        __syncthreads();
        if (st < NS) {
            const double *m = tile + p * IN_STRIDE, *x0 = tile + r0 * IN_STRIDE, *x1 = tile + r1 * IN_STRIDE;
            double sum = 0.0;
            for (int o = 0; o < IN_TILE; ++o) {
                const double v = m[o] * x0[o] * x1[o];
                sum += pow3 ? v * x1[o] : v;
            }
            acc += sum;
        }
        __syncthreads();
    }
    double *out = (PASS == 0 ? a.part0 : a.part1) + (((size_t)s * a.g + h) * a.nblk + bx) * NS;
    if (st < NS) out[st] = acc;
}

// One thread per (start, component): block partials in order.  PASS 0 gives
// n_h and the mean; PASS 1 the covariance (divisor n_h - 1) and m3.
template <int PASS>
__global__ void k_init_stats(InitArgs a) {
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= a.nstarts * a.g) return;
    const int p = a.p;
    const int NS = init_nstat(PASS, p);
    const double *part = (PASS == 0 ? a.part0 : a.part1) + (size_t)id * a.nblk * NS;
    double tot[1 + MAXP * (MAXP + 1) / 2 + MAXP];
    for (int k = 0; k < NS; ++k) tot[k] = 0.0;
    for (int b = 0; b < a.nblk; ++b)
        for (int k = 0; k < NS; ++k) tot[k] += part[(size_t)b * NS + k];
    if (PASS == 0) {
        const double nh = tot[0];
        a.cnt[id] = nh;
        for (int i = 0; i < p; ++i) a.mean[(size_t)id * p + i] = nh > 0.0 ? tot[1 + i] / nh : 0.0;
        return;
    }
    const double nh = a.cnt[id];
    double *S = a.S + (size_t)id * p * p;
    int t = 0;
    for (int i = 0; i < p; ++i)
        for (int k = i; k < p; ++k, ++t) {
            const double v = nh > 1.0 ? tot[t] / (nh - 1.0) : 0.0;
            S[i * p + k] = S[k * p + i] = v;
        }
    for (int i = 0; i < p; ++i) a.m3[(size_t)id * p + i] = nh > 0.0 ? tot[t + i] / nh : 0.0;
}

// One thread per (candidate c = start * nalpha + a, component h): eq. (23).
__global__ void k_init_candidates(InitArgs a) {
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    const int C = a.nstarts * a.nalpha;
    if (id >= C * a.g) return;
    const int c = id / a.g, h = id % a.g, s = c / a.nalpha;
    const int p = a.p, q = a.q, g = a.g;
    const double alpha = a.alpha[c % a.nalpha];
    const int sh = s * g + h;
    const double nh = a.cnt[sh];
    const double *ybar = a.mean + (size_t)sh * p, *Sm = a.S + (size_t)sh * p * p, *m3 = a.m3 + (size_t)sh * p;
    double *pi = a.pi + (size_t)c * g, *mu = a.mu + ((size_t)c * g + h) * p;
    double *Sg = a.Sigma + ((size_t)c * g + h) * p * p, *Dl = a.Delta + ((size_t)c * g + h) * p * q;
    pi[h] = nh / a.n;
    a.nu[(size_t)c * g + h] = a.nu0;
    for (int i = 0; i < p * p; ++i) Sg[i] = Sm[i];
    for (int i = 0; i < p * q; ++i) Dl[i] = 0.0;
    const double kd = M_PI * (1.0 - alpha) / (M_PI - 2.0), km = sqrt(2.0 / M_PI);
    for (int i = 0; i < p; ++i) {
        double delta = 0.0;
        if (i < q) {
            const double sstar = Sm[i * p + i];
            delta = (m3[i] < 0.0 ? -1.0 : 1.0) * sqrt(kd * sstar);
            Sg[i * p + i] = sstar - (1.0 - alpha) * sstar;
            Dl[i * q + i] = delta;
        }
        mu[i] = ybar[i] - km * delta;
    }
    // valid: enough points for S, and Sigma positive definite (Cholesky)
    int ok = nh >= p + 1.0;
    double L[MAXP * MAXP];
    for (int i = 0; i < p && ok; ++i)
        for (int j = 0; j <= i && ok; ++j) {
            double v = Sg[i * p + j];
            for (int k = 0; k < j; ++k) v -= L[i * p + k] * L[j * p + k];
            if (i == j) {
                if (!(v > 0.0)) ok = 0;
                else L[i * p + i] = sqrt(v);
            } else {
                L[i * p + j] = v / L[j * p + j];
            }
        }
    a.valid_ch[id] = ok;
}

// One thread per candidate: valid when every component is.
__global__ void k_init_valid(InitArgs a, int32_t *active) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.nstarts * a.nalpha) return;
    int ok = 1;
    for (int h = 0; h < a.g; ++h) ok &= a.valid_ch[(size_t)c * a.g + h];
    active[c] = ok;
}

// One thread: the first candidate with the largest log-likelihood; its
// parameters are copied to the output by the whole block.
__global__ __launch_bounds__(256) void k_init_select(InitArgs a, const int32_t *active, const double *llc,
                                                     double *ll_out, int32_t *best_index, cfust_params_out best) {
    __shared__ int sbest;
    const int C = a.nstarts * a.nalpha;
    if (threadIdx.x == 0) {
        int bi = -1;
        double bl = -INFINITY;
        for (int c = 0; c < C; ++c) {
            const double l = active[c] ? llc[c] : -INFINITY;
            if (ll_out) ll_out[c] = l;
            if (l > bl) { bl = l; bi = c; }
        }
        if (best_index) best_index[0] = bi;
        sbest = bi;
    }
    __syncthreads();
    const int c = sbest;
    if (c < 0) return;
    const int g = a.g, p = a.p, q = a.q;
    for (int i = threadIdx.x; i < g; i += blockDim.x) {
        best.pi[i] = a.pi[(size_t)c * g + i];
        best.nu[i] = a.nu[(size_t)c * g + i];
    }
    for (int i = threadIdx.x; i < g * p; i += blockDim.x) best.mu[i] = a.mu[(size_t)c * g * p + i];
    for (int i = threadIdx.x; i < g * p * p; i += blockDim.x) best.Sigma[i] = a.Sigma[(size_t)c * g * p * p + i];
    for (int i = threadIdx.x; i < g * p * q; i += blockDim.x) best.Delta[i] = a.Delta[(size_t)c * g * p * q + i];
}

hipError_t launch_init_stats(const InitArgs &a, hipStream_t s) {
    const dim3 grid(a.nblk, a.g, a.nstarts);
    const int nsh = a.nstarts * a.g;
    hipLaunchKernelGGL(k_init_reduce<0>, grid, dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_init_stats<0>, dim3((nsh + 63) / 64), dim3(64), 0, s, a);
    hipLaunchKernelGGL(k_init_reduce<1>, grid, dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_init_stats<1>, dim3((nsh + 63) / 64), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_init_candidates(const InitArgs &a, int32_t *active, hipStream_t s) {
    const int C = a.nstarts * a.nalpha;
    hipLaunchKernelGGL(k_init_candidates, dim3((C * a.g + 63) / 64), dim3(64), 0, s, a);
    hipLaunchKernelGGL(k_init_valid, dim3((C + 63) / 64), dim3(64), 0, s, a, active);
    return hipGetLastError();
}

hipError_t launch_init_select(const InitArgs &a, const int32_t *active, const double *llc, double *ll_out,
                              int32_t *best_index, const cfust_params_out &best, hipStream_t s) {
    hipLaunchKernelGGL(k_init_select, dim3(1), dim3(256), 0, s, a, active, llc, ll_out, best_index, best);
    return hipGetLastError();
}

}  // namespace cfust
