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
    const float *tabs;          // [g][NDOF][TAB_FLOATS] (mixed)
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

hipError_t launch_precompute(const cfust_params &P, int p, int q, int g, CompPre *pre, hipStream_t s);
hipError_t launch_status_fold(const CompPre *pre, int g, int32_t *status, hipStream_t s);
hipError_t launch_tables(const CompPre *pre, int p, int g, int ndof, float *tabs, hipStream_t s);
// Lattice integrals idx0 .. idx0+nidx-1 of every pair; all must share the
// same dimension m >= 2.  In mixed mode the FP32 kernel runs first and an
// FP64 pass then redoes only the flagged (underflowed) items.
// ev0/ev1 (optional) bracket the main kernel of the launch; ppl = lattice
// points per lane per loop trip of the FP32 kernel (1 or 2).
hipError_t launch_estep_qmc(const EstepQmcArgs &a, int m, int nidx, hipStream_t s,
                            hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr, int ppl = 1);
hipError_t launch_assemble(const EstepAsmArgs &a, hipStream_t s);
hipError_t launch_lse(const EstepLseArgs &a, double *loglik, hipStream_t s);
hipError_t launch_mvt(const MvtArgs &a, hipStream_t s);
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
