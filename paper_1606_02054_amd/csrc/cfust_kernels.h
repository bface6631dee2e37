// cfust_kernels.h -- kernel argument blocks and launchers (private).
#pragma once
#include "cfust_common.h"

namespace cfust {

struct LatticeArgs {
    int N, S, log2N;            // log2N < 0 when N is not a power of two
    const int32_t *z;           // [LATD]
    const double *shifts;       // [S][LATD]
};

struct EstepQmcArgs {
    const double *y;            // [p][n]
    const double *mu;           // [g][p]
    const CompPre *pre;         // [g]
    const float *tabs;          // [g][NDOF][TABF_FLOATS] (mixed; fine layout)
    const double *tabs64 = nullptr;   // [g][NDOF][TAB64_DOUBLES] (FP64 mode), or null: exact transforms
    LatticeArgs lat;
    int n, p, q, g;
    int J;                      // integrals stored per pair in est
    int idx0;                   // first integral index of this launch
    int mixed;
    double *est;                // [g][J][n]
    double *lnA;                // [g][n]  ln of integral 0 (A)
    double *se;                 // [g][n]  optional stderr of A
    int32_t *flag;              // [g][J][n] mixed: 1 where the FP32 estimate underflowed
    const int32_t *need;        // [g][J][n] or null: only items with need != 0 are evaluated
    const float *coords = nullptr;   // mixed: lattice coordinate table [S][coordC][2][N] (see
    int coordC = 0;                  // launch_lattice_coords), or null: formed in the loop
};

// Surrogate features of the lattice integrals of one dimension m: rows
// ((h * cnt) + (idx - idx0)) * n + j of X0 [rows][16] BF16.
struct SurFeatArgs {
    const double *y, *mu;
    const CompPre *pre;
    int n, p, q, g, J;
    int m, idx0, cnt;           // integrals idx0 .. idx0+cnt-1 have dimension m
    uint16_t *X0;               // [rows_pad][CFUST_MLP_IN]
    int32_t *inrange;           // [rows]
    double *base;               // [rows] sum of marginal log-CDFs
};

struct SurSelArgs {
    int n, g, J, m, idx0, cnt;
    const float *out;           // [rows_pad][CFUST_MLP_OUT]
    const int32_t *inrange;
    const double *base;
    float tol;                  // fallback when the predicted |error| of ln T exceeds tol
    double *est, *lnA;
    int32_t *need;              // [g][J][n]
};

struct EstepAsmArgs {
    const double *y, *mu;
    const CompPre *pre;
    int n, p, q, g, J;
    int mixed, density_only;
    const double *est, *lnA;
    double *logf_comp;
    void *w, *e1, *e2, *e3;
};

struct EstepLseArgs {
    const double *pi;
    const double *logf_comp;
    int n, g, q, mixed;
    double *tau, *logf_obs;
    void *w, *e1, *e2, *e3;
    double *partial;            // [ceil(n/256)]
};

struct MvtArgs {
    int m, batch, mixed, nmat;
    const double *b, *L, *nu;
    const int32_t *mat_idx;
    LatticeArgs lat;
    double *p, *logp, *se;
    int32_t *flag;              // [batch] mixed: FP32 underflow -> redo in FP64
};

struct MstepArgs {
    const double *y;            // [p][n]
    const double *tau;          // [g][n]
    const void *w, *e1, *e2, *e3;
    const double *mu0;          // [g][p] shift (Psi^(k) means)
    int n, p, q, g, mixed;
    int nblk;                   // blocks per component
    double *partial;            // [g][nblk][nstat]
};

struct MsolveArgs {
    const double *partial;
    int n, p, q, g, nblk;
    const double *mu0, *Sigma0, *Delta0, *nu0;
    double *pi1, *mu1, *Sigma1, *Delta1, *nu1;
    int32_t *status;            // optional
};

// ------------------------------------------------------------ batches ----
// Many independent fits share one launch per kernel kind: each fit keeps the
// argument blocks of its single-fit kernels in a FitDesc (device memory), and a
// block finds its fit from a per-kind prefix table of block counts.

struct PrecompArgs {
    const double *pi, *Sigma, *Delta, *nu;
    int p, q;
    CompPre *pre;               // [g]
};

struct FitDesc {
    int g;
    PrecompArgs pc;
    int ndof;                   // dof tables per component (mixed)
    float *tabs;                // [g][NDOF][TABF_FLOATS]
    double *tabs64;             // [g][NDOF][TAB64_DOUBLES] (FP64 batches) or null
    EstepQmcArgs qa;
    EstepAsmArgs aa;
    EstepLseArgs la;
    int nlse;                   // LSE blocks = partials
    double *loglik;             // [1]
    int32_t *status;            // optional [1]
    MstepArgs ma;
    MsolveArgs sa;
    int32_t *cstat;             // [g] per-component M-step status
};

enum BatchKind { BK_PRE = 0, BK_TAB, BK_ASM, BK_LSE, BK_MRED, BK_MSOL, BK_NKIND };

struct BatchArgs {
    const FitDesc *fits;
    int nfits;
    const int32_t *active;      // [nfits]: 0 = fit skipped
    const int *prefix;          // [BK_NKIND][nfits + 1] block prefix per kernel kind
};

// A run of tiles of one fit in a lattice work queue: tiles of `rows`
// observations starting at j0 + rt * rows (rt < rtiles), for every component
// h < g and integral idx0 .. idx0 + nidx - 1 (all of one dimension m).
// Tile number t0 + (h * nidx + (idx - idx0)) * rtiles + rt.
struct QSeg {
    int fit, idx0, nidx, j0, rows, rtiles;
    long long t0;
};

struct QueueArgs {
    const FitDesc *fits;
    const int32_t *active;
    const QSeg *seg;            // [nseg], t0 ascending
    int nseg;
    long long ntiles;           // tiles handed out (all of them, or a prefix while tuning)
    unsigned long long *counter;        // next tile
    unsigned long long *redo;           // mixed: packed (fit, h, idx, j) of underflowed items
    unsigned int *redo_count;
    LatticeArgs lat;            // the batch's lattice (also in every fit's argument block)
};

constexpr int BATCH_MAX_FITS = 1024;   // fit index packs into 10 bits of a redo entry

hipError_t launch_batch_precompute(const BatchArgs &b, int nblocks, hipStream_t s);
hipError_t launch_batch_tables(const BatchArgs &b, int nblocks, hipStream_t s);
hipError_t launch_batch_assemble(const BatchArgs &b, int nblocks, hipStream_t s);
hipError_t launch_batch_lse(const BatchArgs &b, int nblocks, hipStream_t s);
hipError_t launch_batch_sum(const BatchArgs &b, hipStream_t s);
// lds: dynamic LDS of the reduction, the largest mstep_lds_bytes of the fits.
hipError_t launch_batch_mstep(const BatchArgs &b, int nred, int nsol, size_t lds, hipStream_t s);
size_t mstep_lds_bytes(int p, int q);
// Lattice kernel of dimension m over a queue.  grid > 0: persistent, `grid`
// blocks draw tiles until the queue is empty; grid == 0: one block per tile
// in queue order (tiles of at most 4 observations).  Mixed mode appends
// underflowed items to the redo list and launch_queue_redo evaluates them
// with the FP64 integrand.  coords: the fits' argument blocks point at a
// lattice coordinate table (used in mixed mode at one point per lane).
hipError_t launch_queue_qmc(const QueueArgs &q, int m, bool mixed, int ppl, int grid, hipStream_t s,
                            bool coords = false);
// The FP64 pass over the redo list: the entries the fits' FP64 tables reach
// first (grid64 blocks of one wave), then the rest exact (grid blocks).
hipError_t launch_queue_redo(const QueueArgs &q, int m, int grid, int grid64, hipStream_t s);
// Resident blocks per compute unit of the queue kernels.
int queue_qmc_occupancy(int m, bool mixed, int ppl, bool coords = false);
int queue_redo_occupancy(int m, bool tables);
// Arguments of a batched EM run that the captured iteration reads from
// device memory, so that one graph serves every call.
struct BatchCtl {
    double tol;                 // Aitken tolerance (<= 0: no stop on it)
    double *trace;              // optional [max_trace][nfits]
    int32_t *iters_done;        // optional [nfits]
    int max_trace;
};

// Convergence check between the E-step and the M-step of a batched EM
// iteration (see k_batch_check).
hipError_t launch_batch_check(const FitDesc *fits, int nfits, int32_t *active, int32_t *iter, double *hist,
                              const BatchCtl *ctl, hipStream_t s);

// ------------------------------------------------------ initialisation ----
struct InitArgs {
    const double *y;            // [p][n]
    int n, p, q, g;
    int nstarts, nalpha;
    const int32_t *labels;      // [nstarts][n]
    const double *alpha;        // [nalpha]
    double nu0;
    int nblk;                   // reduction blocks per (start, component)
    double *part0, *part1;      // block partials of the two passes
    double *cnt, *mean, *S, *m3;                // [nstarts][g] (x p, x p x p, x p)
    double *pi, *mu, *Sigma, *Delta, *nu;       // candidates [C][g] ...
    int32_t *valid_ch;          // [C][g]
};

hipError_t launch_init_stats(const InitArgs &a, hipStream_t s);
hipError_t launch_init_candidates(const InitArgs &a, int32_t *active, hipStream_t s);
hipError_t launch_init_select(const InitArgs &a, const int32_t *active, const double *llc, double *ll_out,
                              int32_t *best_index, const cfust_params_out &best, hipStream_t s);

hipError_t launch_precompute(const cfust_params &P, int p, int q, int g, CompPre *pre, hipStream_t s);
hipError_t launch_status_fold(const CompPre *pre, int g, int32_t *status, hipStream_t s);
hipError_t launch_tables(const CompPre *pre, int p, int g, int ndof, float *tabs, hipStream_t s);
hipError_t launch_tables64(const CompPre *pre, int p, int g, int ndof, double *tabs, hipStream_t s);
// Lattice integrals idx0 .. idx0+nidx-1 of every pair; all must share the
// same dimension m >= 2.  In mixed mode the FP32 kernel runs first and an
// FP64 pass then redoes only the flagged (underflowed) items.
// ev0/ev1 (optional) bracket the main kernel of the launch; ppl = lattice
// points per lane per loop trip of the FP32 kernel (1 or 2).
hipError_t launch_estep_qmc(const EstepQmcArgs &a, int m, int nidx, hipStream_t s,
                            hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr, int ppl = 1);
hipError_t launch_assemble(const EstepAsmArgs &a, hipStream_t s);
// Table of the tent-transformed lattice coordinates 0 .. C-1 of every point
// and shift (N a power of two >= 64): coords[((s C + i) 2 + r) N + k], r = 0
// the coordinate, r = 1 its complement; coordinate 0 in units of 2^-31, the
// others scaled (the values the FP32 integrand forms in its loop).
hipError_t launch_lattice_coords(const LatticeArgs &L, int C, float *coords, hipStream_t s);
// Floats of that table.
inline size_t lattice_coords_floats(int N, int S, int C) { return (size_t)(2 * C + 1) * N * S; }
hipError_t launch_lse(const EstepLseArgs &a, double *loglik, hipStream_t s);
// Work areas of mvt_cdf_batch (m >= 2): per chunk of items the FP64 tables
// ([chunk][m][TAB64_DOUBLES]) and, in mixed precision, the FP32 tables
// ([chunk][m][TABF_FLOATS]); mixed: the dof-free normal table ([TABF_FLOATS])
// and the lattice coordinate table (C > 0, see launch_lattice_coords).
struct MvtWork {
    int chunk = 0;
    float *tabs = nullptr, *ntab = nullptr, *coords = nullptr;
    double *tabs64 = nullptr;
    int C = 0;
};
hipError_t launch_mvt(const MvtArgs &a, const MvtWork &w, hipStream_t s);
hipError_t launch_mstep(const MstepArgs &r, const MsolveArgs &s, hipStream_t st);

hipError_t launch_sur_features(const SurFeatArgs &a, hipStream_t s);
hipError_t launch_sur_select(const SurSelArgs &a, hipStream_t s);
hipError_t launch_fill_i32(int32_t *p, size_t count, int32_t v, hipStream_t s);
hipError_t launch_count_i32(const int32_t *p, size_t count, int32_t *out, hipStream_t s);
// Features of batched T_m problems (training inputs of the surrogate).
hipError_t launch_mvt_features(int m, int batch, int rows_pad, const double *b, const double *L,
                               const int32_t *mat_idx, int nmat, const double *nu, uint16_t *X0, int32_t *inrange,
                               double *base, hipStream_t s);

int mlp_layer_k(int l);
int mlp_layer_n(int l);
// BF16 elements of the weights in the fused pass's fragment order; without
// acts, launch_mlp_forward packs the weights into scratch_a (at least this
// many elements) and runs the fused inference kernel.
size_t mlp_packed_elems();
hipError_t launch_mlp_forward(const cfust_mlp_weights &W, const uint16_t *X0, int B, float *out,
                              const cfust_mlp_acts *acts, uint16_t *scratch_a, uint16_t *scratch_b,
                              hipStream_t s);
hipError_t launch_mlp_backward(const cfust_mlp_weights &W, const cfust_mlp_acts &A, const float *dout, int B,
                               const cfust_mlp_grads &G, float *part, float *dY, uint16_t *dZb, uint16_t *dZbT,
                               hipStream_t s);
hipError_t launch_mlp_adam(const cfust_mlp_master &Mst, const cfust_mlp_grads &G, const cfust_mlp_weights &W,
                           float lr, float b1, float b2, float eps, int step, hipStream_t s);
hipError_t launch_mlp_loss(const float *out, const float *label, int B, int nvalid, float lam, float *dout,
                           float *part, float *loss, hipStream_t s);
hipError_t launch_transpose_in(const uint16_t *X0, int B, uint16_t *X, uint16_t *XT, hipStream_t s);

}  // namespace cfust
