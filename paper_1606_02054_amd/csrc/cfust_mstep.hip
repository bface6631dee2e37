// cfust_mstep.hip -- M-step of the CFUST mixture (Sec. 3.2, eqs. 18-22).
//
//   k_mstep_reduce  grid (blocks, component): FP64 weighted sums over the
//                   observations of a component, in coordinates shifted by
//                   mu_h^(k) for conditioning.  Tiles of 64 observations:
//                   coalesced SoA reads into registers (each input read once),
//                   plain sums kept per lane, the two product blocks from LDS
//                   in 4x4 register blocks.  Partials per block are written
//                   out and summed in a fixed order, so results are
//                   reproducible run to run.
//   k_mstep_solve   one block per component: sums the partials, then the
//                   closed-form updates pi, mu, Delta, Sigma and the nu root.
#include <type_traits>

#include "cfust_devmath.h"
#include "cfust_kernels.h"

namespace cfust {

constexpr int MS_TILE = 64;                      // observations per block iteration
constexpr int MS_STRIDE = MS_TILE + 1;           // LDS row pitch (doubles)
constexpr int MS_E_PER_WAVE = (1 + MAXQ + MAXQ * (MAXQ + 1) / 2 + 3) / 4;      // rows e1, e2_l, e3_t
static_assert(MAXP <= 16 && MAXQ <= 8, "product blocks are sized for p <= 16, q <= 8");

// Two sizes of the reduction: NR rows r_i per wave (4 waves), so p <= 4 NR.
//   NR = 2: p <= 8,  at most 3 + 4 = 7 product blocks: 8 groups of 32 lanes, one each
//   NR = 4: p <= 16, at most 10 + 8 = 18 blocks: 16 groups of 16 lanes, two each
// LDS rows of one buffer: A_i = r_i (i < 4 NR), then B_c = tau w r_c
// (c < 4 NR) and B_{4 NR + l} = tau e2_l (l < MAXQ).  Two buffers: the rows of
// the next tile are written while other waves still read the current one.
template <int NR> struct MsShape {
    static constexpr int AROWS = 4 * NR, BROWS = 4 * NR + MAXQ;
    static constexpr int BUF = (AROWS + BROWS) * MS_STRIDE;
    static constexpr int OGW = NR == 2 ? 32 : 16;        // lanes sharing a block (observation groups)
    static constexpr int NGRP = 256 / OGW;               // thread groups
    static constexpr int NBT = NR == 2 ? 1 : 2;          // product blocks per thread group
    static_assert(NGRP * NBT >= (NR * (NR + 1) / 2 + NR * ((MAXQ + 3) / 4)), "too few block slots");
};

__host__ __device__ inline int ms_nr(int p) { return p <= 8 ? 2 : 4; }

// LDS bytes of the reduction for p.
__host__ __device__ inline size_t ms_lds_bytes(int p, int) {
    return 2 * (size_t)(ms_nr(p) == 2 ? MsShape<2>::BUF : MsShape<4>::BUF) * sizeof(double);
}

// Statistic indices (the order mstep_solve_body reads):
//   0 n_h = sum tau             1 sum tau w            2 sum tau (e1 - w)
//   3 + i          sum tau w r_i                      (p)
//   3 + p + l      sum tau e2_l                        (q)
//   O1(i, k)       sum tau w r_i r_k, i <= k, i-major  (p(p+1)/2)
//   O2(i, l)       sum r_i tau e2_l                    (p q)
//   last q(q+1)/2  sum tau e3_t
__device__ inline int ms_idx_o1(int p, int q, int i, int k) { return 3 + p + q + i * p - i * (i - 1) / 2 + (k - i); }
__device__ inline int ms_idx_o2(int p, int q, int i, int l) { return 3 + p + q + p * (p + 1) / 2 + i * q + l; }
__device__ inline int ms_idx_e3(int p, int q, int t) { return 3 + p + q + p * (p + 1) / 2 + p * q + t; }

// Sum over `width` adjacent lanes (fixed butterfly: reproducible).
__device__ inline double ms_lane_sum(double v, int width) {
    for (int m = width >> 1; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// Product block b of 4x4 entries: A rows ab*4.., B rows bbase..  The blocks
// are the lower triangle (cb <= ab) of r_i . tau w r_c, then r_i . tau e2_l.
__device__ inline void ms_block(int b, int na, int nq, int arows, int &ab, int &bbase) {
    const int ntri = na * (na + 1) / 2;
    if (b < ntri) {
        ab = 0;
        while ((ab + 1) * (ab + 2) / 2 <= b) ++ab;
        bbase = 4 * (b - ab * (ab + 1) / 2);
    } else {
        ab = (b - ntri) / nq;
        bbase = arows + 4 * ((b - ntri) % nq);
    }
}

// Block bx of component h of one fit; `lds` is the block's dynamic LDS
// (ms_lds_bytes).  Work split:
//   * loads: wave w loads rows r_i (i = w, w+4, ...) and e1 / e2_l / e3_t
//     rows w, w+4, ..., one observation per lane; every wave also loads tau
//     and w of its lanes.  Row base pointers are wave-uniform and set up once;
//     the loads carry no per-lane branches (indices clamped into range,
//     values of observations past n zeroed afterwards) and the next tile's
//     loads are issued before the current tile's products, so their latency
//     is hidden.
//   * weighting in registers: tau w r_i, tau (e1 - w), tau e2_l, tau e3_t;
//     every statistic that is a plain sum over observations accumulates in a
//     per-lane register and is summed over lanes once, at the end.
//   * the product blocks r_i . [tau w r_c | tau e2_l] from LDS: thread =
//     (block group, observation group), 16 accumulators per 4x4 block,
//     summed over the lanes of the group at the end.
template <bool MIXED, int NR>
__device__ inline void mstep_reduce_prec(const MstepArgs &a, int bx, int h, double *lds) {
    using E = typename std::conditional<MIXED, float, double>::type;   // storage of w, e1, e2, e3
    using S = MsShape<NR>;
    const int p = a.p, q = a.q, n = a.n;
    const int nq2 = q * (q + 1) / 2;
    const int ne = 1 + q + nq2;                  // rows e1, e2_l, e3_t
    const int ntiles = (n + MS_TILE - 1) / MS_TILE;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const size_t hn = (size_t)h * n;
    const double *mu0 = a.mu0 + (size_t)h * p;

    // both LDS buffers start at zero: rows past p and q are never written
    for (int t = threadIdx.x; t < 2 * S::BUF; t += blockDim.x) lds[t] = 0.0;

    const double *srcr[NR];
    double offr[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        const int i = min(wave + 4 * k, p - 1);
        srcr[k] = a.y + (size_t)i * n;
        offr[k] = mu0[i];
    }
    const E *srce[MS_E_PER_WAVE];
#pragma unroll
    for (int k = 0; k < MS_E_PER_WAVE; ++k) {
        const int e = min(wave + 4 * k, ne - 1);
        srce[k] = e == 0 ? (const E *)a.e1 + hn
                : e <= q ? (const E *)a.e2 + ((size_t)h * q + (e - 1)) * n
                         : (const E *)a.e3 + ((size_t)h * nq2 + (e - 1 - q)) * n;
    }
    const double *srct = a.tau + hn;
    const E *srcw = (const E *)a.w + hn;

    double vt = 0.0, vr[NR] = {};
    E vw = 0, ve[MS_E_PER_WAVE] = {};
    auto load_tile = [&](int tl) {
        if (tl >= ntiles) return;                // uniform: nothing past the last tile
        const int jc = min(tl * MS_TILE + lane, n - 1);
        vt = srct[jc];
        vw = srcw[jc];
#pragma unroll
        for (int k = 0; k < NR; ++k)
            if (wave + 4 * k < p) vr[k] = srcr[k][jc];
#pragma unroll
        for (int k = 0; k < MS_E_PER_WAVE; ++k)
            if (wave + 4 * k < ne) ve[k] = srce[k][jc];
    };

    double sr[NR] = {}, se[MS_E_PER_WAVE] = {}, s_tau = 0.0, s_tw = 0.0;
    // product blocks of this thread group: blk, blk + NGRP; observations og, og + OGW, ...
    const int blk = threadIdx.x / S::OGW, og = threadIdx.x % S::OGW;
    const int na = (p + 3) / 4, nq = (q + 3) / 4, nb = na * (na + 1) / 2 + na * nq;
    int aoff[S::NBT], boff[S::NBT];
#pragma unroll
    for (int u = 0; u < S::NBT; ++u) {
        int ab = 0, bbase = 0;
        if (blk + S::NGRP * u < nb) ms_block(blk + S::NGRP * u, na, nq, S::AROWS, ab, bbase);
        aoff[u] = ab * 4 * MS_STRIDE;
        boff[u] = bbase * MS_STRIDE;
    }
    double acc[S::NBT][4][4] = {};

    __syncthreads();
    load_tile(bx);
    int buf = 0;
    for (int tl = bx; tl < ntiles; tl += a.nblk, buf ^= 1) {
        double *A = lds + buf * S::BUF, *B = A + S::AROWS * MS_STRIDE;
        const bool in = tl * MS_TILE + lane < n;
        const double t = in ? vt : 0.0, w = in ? (double)vw : 0.0, tw = t * w;
        if (wave == 0) { s_tau += t; s_tw += tw; }
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const int i = wave + 4 * k;
            if (i < p) {
                const double r = in ? vr[k] - offr[k] : 0.0, x = tw * r;
                A[i * MS_STRIDE + lane] = r;
                B[i * MS_STRIDE + lane] = x;
                sr[k] += x;
            }
        }
#pragma unroll
        for (int k = 0; k < MS_E_PER_WAVE; ++k) {
            const int e = wave + 4 * k;
            const double v = in ? (double)ve[k] : 0.0;
            if (e == 0) {
                se[k] += t * (v - w);
            } else if (e <= q) {
                const double x = t * v;
                B[(S::AROWS + e - 1) * MS_STRIDE + lane] = x;
                se[k] += x;
            } else if (e < ne) {
                se[k] += t * v;
            }
        }
        __syncthreads();
        load_tile(tl + a.nblk);
#pragma unroll
        for (int u = 0; u < S::NBT; ++u) {
            if (blk + S::NGRP * u >= nb) continue;
            const double *Ab = A + aoff[u], *Bb = B + boff[u];
#pragma unroll
            for (int oo = 0; oo < MS_TILE / S::OGW; ++oo) {
                const int o = og + S::OGW * oo;
                double x[4], y[4];
#pragma unroll
                for (int ii = 0; ii < 4; ++ii) x[ii] = Ab[ii * MS_STRIDE + o];
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) y[jj] = Bb[jj * MS_STRIDE + o];
#pragma unroll
                for (int ii = 0; ii < 4; ++ii)
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) acc[u][ii][jj] += x[ii] * y[jj];
            }
        }
    }

    // lane sums, then the block's partials
    // partials are stat-major, [g][nstat][nblk], so the solve sums them coalesced
    double *out = a.partial + (size_t)h * nstat(p, q) * a.nblk + bx;
    const size_t ld = a.nblk;
    s_tau = ms_lane_sum(s_tau, 64);
    s_tw = ms_lane_sum(s_tw, 64);
    if (wave == 0 && lane == 0) { out[0] = s_tau; out[ld] = s_tw; }
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        const double v = ms_lane_sum(sr[k], 64);
        const int i = wave + 4 * k;
        if (lane == 0 && i < p) out[(3 + i) * ld] = v;
    }
#pragma unroll
    for (int k = 0; k < MS_E_PER_WAVE; ++k) {
        const double v = ms_lane_sum(se[k], 64);
        const int e = wave + 4 * k;
        if (lane == 0 && e < ne) out[(e == 0 ? 2 : e <= q ? 3 + p + (e - 1) : ms_idx_e3(p, q, e - 1 - q)) * ld] = v;
    }
#pragma unroll
    for (int u = 0; u < S::NBT; ++u)
#pragma unroll
        for (int ii = 0; ii < 4; ++ii)
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                const double v = ms_lane_sum(acc[u][ii][jj], S::OGW);   // over og
                if (og != 0 || blk + S::NGRP * u >= nb) continue;
                const int i = aoff[u] / MS_STRIDE + ii, c = boff[u] / MS_STRIDE + jj;
                if (i >= p) continue;
                if (c < S::AROWS) {
                    // r_i . tau w r_c = statistic O1(c, i) when c <= i
                    if (c <= i) out[ms_idx_o1(p, q, c, i) * ld] = v;
                } else if (c - S::AROWS < q) {
                    out[ms_idx_o2(p, q, i, c - S::AROWS) * ld] = v;
                }
            }
}

template <int NR>
__device__ inline void mstep_reduce_body(const MstepArgs &a, int bx, int h, double *tile) {
    if (a.mixed) mstep_reduce_prec<true, NR>(a, bx, h, tile);
    else mstep_reduce_prec<false, NR>(a, bx, h, tile);
}

template <int NR>
__global__ __launch_bounds__(256) void k_mstep_reduce(MstepArgs a) {
    extern __shared__ double ms_tile[];
    mstep_reduce_body<NR>(a, blockIdx.x, blockIdx.y, ms_tile);
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

// Component h of one fit, by one block: the sums of the block partials, then
// eqs. (18)-(22).  The matrices live in LDS; each step runs one thread per
// output entry, the two small Cholesky factorisations (q x q and the p x p
// positivity check) on one thread.
__device__ inline void mstep_solve_body(const MsolveArgs &a, int32_t *cstat, int h) {
    __shared__ double st[512];
    __shared__ double dl[MAXP], X[MAXP * MAXQ], E3[MAXQ * MAXQ], Lc[MAXQ * MAXQ], Dnew[MAXP * MAXQ];
    __shared__ double DE3[MAXP * MAXQ], Snew[MAXP * MAXP], Ls[MAXP * MAXP];
    __shared__ int s_keep, s_status, s_mode;     // s_mode: 0 keep theta, 1 clamp, 2 root search
    __shared__ double s_m, s_lo, s_hi, s_nu;
    __shared__ unsigned long long s_mask[4];
    const int p = a.p, q = a.q, tid = threadIdx.x, nt = blockDim.x;
    const int NS = nstat(p, q);
    // block partials of statistic s: lanes over blocks (coalesced), then a
    // fixed butterfly, so the sum is reproducible; each wave takes 4
    // statistics per pass so that their loads are in flight together
    {
        const int wave = tid >> 6, lane = tid & 63, nw = nt >> 6;
        for (int s0 = 4 * wave; s0 < NS; s0 += 4 * nw) {
            double v[4] = {0.0, 0.0, 0.0, 0.0};
            const double *src = a.partial + ((size_t)h * NS + s0) * a.nblk;
            for (int b = lane; b < a.nblk; b += 64)
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (s0 + u < NS) v[u] += src[(size_t)u * a.nblk + b];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                v[u] = ms_lane_sum(v[u], 64);
                if (lane == 0 && s0 + u < NS) st[s0 + u] = v[u];
            }
        }
    }
    __syncthreads();
    const double nh = st[0], Sw = st[1], Sew = st[2];
    const double *Swr = st + 3, *Se2 = st + 3 + p, *Swrr = st + 3 + p + q;
    const double *Sre2 = Swrr + p * (p + 1) / 2, *Se3 = Sre2 + p * q;
    const double *mu0 = a.mu0 + (size_t)h * p, *S0 = a.Sigma0 + (size_t)h * p * p;
    const double *D0 = a.Delta0 + (size_t)h * p * q;
    if (tid == 0) {
        a.pi1[h] = a.n > 0 ? nh / a.n : 0.0;                           // (18)
        const bool frozen = !(nh >= p + 1.0);
        s_keep = frozen;
        s_status = frozen ? CFUST_DEV_FROZEN : 0;
        s_mode = 0;
    }
    for (int i = tid; i < p; i += nt) {                                // (19), Delta^(k)
        double v = Swr[i];
        for (int l = 0; l < q; ++l) v -= D0[i * q + l] * Se2[l];
        dl[i] = v / Sw;
    }
    for (int t = tid; t < q * q; t += nt) {                            // E3 from its upper triangle
        const int i = min(t / q, t % q), k = max(t / q, t % q);
        const double v = Se3[i * q - i * (i - 1) / 2 + (k - i)];
        E3[t] = v;
        Lc[t] = v;
    }
    __syncthreads();
    for (int t = tid; t < p * q; t += nt) {                            // sum tau (y - mu1) e2^T
        const int i = t / q, l = t % q;
        X[t] = Sre2[t] - dl[i] * Se2[l];
    }
    if (tid == 0 && !s_keep && !ms_chol(Lc, q)) { s_status |= CFUST_DEV_NOTSPD_E3; s_keep = 1; }
    __syncthreads();
    if (!s_keep) {
        for (int i = tid; i < p; i += nt) {                            // (20): Delta E3 = X, row i
            double z[MAXQ];                      // unrolled to MAXQ: z stays in registers
#pragma unroll
            for (int l = 0; l < MAXQ; ++l) {
                if (l >= q) break;
                double v = X[i * q + l];
#pragma unroll
                for (int k = 0; k < l; ++k) v -= Lc[l * q + k] * z[k];
                z[l] = v / Lc[l * q + l];
            }
#pragma unroll
            for (int l = MAXQ - 1; l >= 0; --l) {
                if (l >= q) continue;
                double v = z[l];
#pragma unroll
                for (int k = l + 1; k < MAXQ; ++k)
                    if (k < q) v -= Lc[k * q + l] * z[k];
                z[l] = v / Lc[l * q + l];
            }
#pragma unroll
            for (int l = 0; l < MAXQ; ++l)
                if (l < q) Dnew[i * q + l] = z[l];
        }
        __syncthreads();
        for (int t = tid; t < p * q; t += nt) {                        // Delta^(k+1) E3
            const int i = t / q, l = t % q;
            double v = 0.0;
            for (int k = 0; k < q; ++k) v += Dnew[i * q + k] * E3[k * q + l];
            DE3[t] = v;
        }
        __syncthreads();
        for (int t = tid; t < p * p; t += nt) {                        // (21) with mu^(k+1), Delta^(k+1)
            const int i = min(t / p, t % p), k = max(t / p, t % p);
            const int ik = i * p - i * (i - 1) / 2 + (k - i);
            const double Wik = Swrr[ik] - dl[i] * Swr[k] - Swr[i] * dl[k] + Sw * dl[i] * dl[k];
            double cross = 0.0, quad = 0.0;
            for (int l = 0; l < q; ++l) {
                cross += Dnew[i * q + l] * X[k * q + l] + X[i * q + l] * Dnew[k * q + l];
                quad += DE3[i * q + l] * Dnew[k * q + l];
            }
            Snew[t] = (Wik - cross + quad) / nh;
        }
        __syncthreads();
        for (int t = tid; t < p * p; t += nt) Ls[t] = Snew[t];
        __syncthreads();
        if (tid == 0 && !ms_chol(Ls, p)) { s_status |= CFUST_DEV_NOTSPD_SIGMA; s_keep = 1; }
        __syncthreads();
    }
    if (tid == 0 && !s_keep && !isinf(a.nu0[h])) {                    // an infinite nu (normal limit) stays
        const double m = Sew / nh;                                     // (22)
        s_m = m;
        s_lo = 1.0; s_hi = 200.0;
        s_mode = 2;
        if (ms_nu_eq(1.0, m) <= 0.0) { s_nu = 1.0; s_mode = 1; s_status |= CFUST_DEV_NU_CLAMPED; }
        else if (ms_nu_eq(200.0, m) >= 0.0) { s_nu = 200.0; s_mode = 1; s_status |= CFUST_DEV_NU_CLAMPED; }
    }
    __syncthreads();
    if (s_mode == 2) {
        // eq. (22) decreases in nu: multisection of [lo, hi] by the block, each
        // round evaluating it at blockDim.x interior points and keeping the
        // interval of the first sign change (257-fold shrink per round)
        const double m = s_m, np1 = nt + 1.0;
        for (int round = 0; round < 8; ++round) {
            const double lo = s_lo, hi = s_hi;
            const double x = lo + (hi - lo) * (tid + 1) / np1;
            const unsigned long long bal = __ballot(ms_nu_eq(x, m) <= 0.0);
            if ((tid & 63) == 0) s_mask[tid >> 6] = bal;
            __syncthreads();
            if (tid == 0) {
                int first = nt;
                for (int w = 0; w < (nt >> 6); ++w)
                    if (s_mask[w]) { first = w * 64 + __ffsll(s_mask[w]) - 1; break; }
                s_lo = lo + (hi - lo) * first / np1;
                s_hi = first == nt ? hi : lo + (hi - lo) * (first + 1) / np1;
            }
            __syncthreads();
        }
        if (tid == 0) s_nu = 0.5 * (s_lo + s_hi);
        __syncthreads();
    }
    // outputs: the updates, or theta^(k) where the update was refused
    const bool keep = s_keep;
    for (int i = tid; i < p; i += nt) a.mu1[(size_t)h * p + i] = keep ? mu0[i] : mu0[i] + dl[i];
    for (int i = tid; i < p * q; i += nt) a.Delta1[(size_t)h * p * q + i] = keep ? D0[i] : Dnew[i];
    for (int i = tid; i < p * p; i += nt) a.Sigma1[(size_t)h * p * p + i] = keep ? S0[i] : Snew[i];
    if (tid == 0) {
        a.nu1[h] = s_mode == 0 ? a.nu0[h] : s_nu;
        cstat[h] = s_status;
    }
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
    if (ms_nr(r.p) == 2) hipLaunchKernelGGL(k_mstep_reduce<2>, dim3(r.nblk, r.g), dim3(256), ms_lds_bytes(r.p, r.q), st, r);
    else hipLaunchKernelGGL(k_mstep_reduce<4>, dim3(r.nblk, r.g), dim3(256), ms_lds_bytes(r.p, r.q), st, r);
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

template <int NR>
__global__ __launch_bounds__(256) void k_batch_mreduce(BatchArgs B) {
    const int *pf = B.prefix + BK_MRED * (B.nfits + 1);
    const int f = mbatch_fit(pf, B.nfits, blockIdx.x);
    if (!B.active[f]) return;
    const MstepArgs a = B.fits[f].ma;
    const int local = blockIdx.x - pf[f];
    extern __shared__ double ms_tile[];
    mstep_reduce_body<NR>(a, local % a.nblk, local / a.nblk, ms_tile);
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
    // the larger reduction when any fit needs it (lds is the largest of the fits')
    if (nred > 0 && lds <= ms_lds_bytes(8, 0)) hipLaunchKernelGGL(k_batch_mreduce<2>, dim3(nred), dim3(256), lds, s, b);
    else if (nred > 0) hipLaunchKernelGGL(k_batch_mreduce<4>, dim3(nred), dim3(256), lds, s, b);
    if (nsol > 0) hipLaunchKernelGGL(k_batch_msolve, dim3(nsol), dim3(256), 0, s, b);
    if (b.nfits > 0) hipLaunchKernelGGL(k_batch_mstatus, dim3(b.nfits), dim3(64), 0, s, b);
    return hipGetLastError();
}

}  // namespace cfust
