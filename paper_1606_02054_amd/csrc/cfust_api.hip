// cfust_api.hip -- host side of the C ABI declared in include/cfust.h:
// argument checks, workspace, and the launch sequence of each call.
#include <string.h>

#include <mutex>
#include <new>

#include "cfust_host.h"

namespace {

using namespace cfust;
using namespace cfust_host;

cfust_status check_mlp_b(cfust_handle h, int32_t B) {
    if (B <= 0 || B % 64) return fail(h, CFUST_EINVAL, "B = %d is not a positive multiple of 64", B);
    return CFUST_OK;
}

bool weights_ok(const cfust_mlp_weights *w) {
    if (!w) return false;
    for (int l = 0; l < CFUST_MLP_LAYERS; ++l)
        if (!w->W[l] || !w->Wt[l] || !w->b[l]) return false;
    return true;
}

// Workspace layout of an E-step (or log-likelihood) call.
struct EstepWs {
    size_t pre, tabs, tabs64, est, lnA, flag, logf, partial, coords, total;
    int coordC;
};

// Items of mvt_cdf_batch whose tables are built and used per launch pair:
// 16384 items hold at most 16384 x 8 x (2176 + 2976) B = 675 MB.
constexpr int MVT_CHUNK = 16384;

int coord_count(const cfust_dims &d, const cfust_qmc *Q) {
    return d.n == 0 ? 0 : lattice_coord_count(d.q, Q);
}

EstepWs estep_layout(const cfust_dims &d, int J, bool own_logf, int coordC = 0, const cfust_qmc *Q = nullptr) {
    Carve c;
    EstepWs w;
    w.pre = c.take<CompPre>(d.g);
    w.tabs = c.take<float>((size_t)d.g * NDOF * TABF_FLOATS);
    w.tabs64 = c.take<double>((size_t)d.g * NDOF * TAB64_DOUBLES);
    w.est = c.take<double>((size_t)d.g * (J > 0 ? J : 1) * (d.n > 0 ? d.n : 1));
    w.lnA = c.take<double>((size_t)d.g * (d.n > 0 ? d.n : 1));
    w.flag = c.take<int32_t>((size_t)d.g * (J > 0 ? J : 1) * (d.n > 0 ? d.n : 1));
    w.logf = c.take<double>(own_logf ? (size_t)d.g * (d.n > 0 ? d.n : 1) : 1);
    w.partial = c.take<double>((size_t)(d.n + 255) / 256 + 1);
    w.coordC = coordC;
    w.coords = c.take<float>(coordC > 0 ? lattice_coords_floats(Q->N, Q->S, coordC) : 1);
    w.total = c.off;
    return w;
}

hipError_t timed_qmc(cfust_handle h, const EstepQmcArgs &a, bool may_time, int m, int nidx, hipStream_t s) {
    const int ppl = tuned_ppl(h, m, a.lat, a.mixed != 0);
    if (!may_time || !h->prof || a.n == 0 || nidx == 0) return launch_estep_qmc(a, m, nidx, s, nullptr, nullptr, ppl);
    ProfRec r{m, pool_event(h), pool_event(h)};
    const hipError_t e = launch_estep_qmc(a, m, nidx, s, r.e0, r.e1, ppl);
    if (r.e0 && r.e1) h->rec.push_back(r);
    return e;
}

// Shared launch sequence of cfust_estep / cfust_loglik.
constexpr int SUR_CHUNK = 65536;   // network rows per forward launch

cfust_status run_estep(cfust_handle h, const double *y, const cfust_dims &d, const cfust_params *P,
                       const cfust_qmc *Q, bool density_only, double *tau, double *logf_obs, double *loglik,
                       void *w, void *e1, void *e2, void *e3, double *logf_comp, double *se,
                       int32_t *status, hipStream_t s, const cfust_surrogate *sur = nullptr,
                       char *fixed_ws = nullptr, size_t fixed_cap = 0) {
    cfust_status st;
    if ((st = check_dims(h, d)) != CFUST_OK) return st;
    if ((st = check_params(h, P)) != CFUST_OK) return st;
    const bool lattice = d.q >= 2;
    if ((st = check_qmc(h, Q, lattice)) != CFUST_OK) return st;
    if (d.n > 0 && !y) return fail(h, CFUST_EINVAL, "y is NULL");
    if (!loglik) return fail(h, CFUST_EINVAL, "loglik is NULL");
    if (!density_only && d.n > 0 && (!tau || !w || !e1 || !e2 || !e3))
        return fail(h, CFUST_EINVAL, "an E-step output array is NULL");
    const bool mixed = Q->precision == CFUST_MIXED;
    const int J = density_only ? (lattice ? 1 : 0) : nint_qmc(d.q);
    const EstepWs L = estep_layout(d, J, logf_comp == nullptr, J > 0 ? coord_count(d, Q) : 0, Q);
    // surrogate workspace: need flags, and per dimension group features/outputs
    struct SurGroup { int m, idx0, cnt; long rows, rows_pad; size_t x0, out, inr, base; };
    SurGroup sg[3];
    int nsg = 0;
    size_t need_off = 0, sa_off = 0, sb_off = 0, total = L.total;
    if (sur && J > 0) {
        Carve c;
        c.off = L.total;
        need_off = c.take<int32_t>((size_t)d.g * J * (d.n > 0 ? d.n : 1));
        const int gm[3][3] = {{d.q, 0, 2}, {d.q - 1, 2, d.q}, {d.q - 2, 2 + d.q, npairs(d.q)}};
        for (int k = 0; k < 3; ++k) {
            const int m = gm[k][0];
            if (m < 2 || m > MAXQ || !sur->model[m] || gm[k][1] + gm[k][2] > J) continue;
            if (!weights_ok(sur->model[m])) return fail(h, CFUST_EINVAL, "surrogate model for m = %d is incomplete", m);
            SurGroup G;
            G.m = m; G.idx0 = gm[k][1]; G.cnt = gm[k][2];
            G.rows = (long)d.g * G.cnt * d.n;
            G.rows_pad = (G.rows + 63) / 64 * 64;
            G.x0 = c.take<uint16_t>((size_t)(G.rows_pad > 0 ? G.rows_pad : 64) * CFUST_MLP_IN);
            G.out = c.take<float>((size_t)(G.rows_pad > 0 ? G.rows_pad : 64) * CFUST_MLP_OUT);
            G.inr = c.take<int32_t>((size_t)(G.rows > 0 ? G.rows : 1));
            G.base = c.take<double>((size_t)(G.rows > 0 ? G.rows : 1));
            sg[nsg++] = G;
        }
        sa_off = c.take<uint16_t>(std::max((size_t)SUR_CHUNK * CFUST_MLP_HIDDEN, mlp_packed_elems()));
        sb_off = c.take<uint16_t>((size_t)SUR_CHUNK * CFUST_MLP_HIDDEN);
        total = c.off;
    }
    char *base;
    if (fixed_ws) {                  // caller-independent fixed array: no allocation
        if (total > fixed_cap)
            return fail(h, CFUST_EINVAL, "E-step workspace of %zu bytes exceeds the fixed %zu-byte array "
                        "(n = %d, q = %d, g = %d)", total, fixed_cap, d.n, d.q, d.g);
        base = fixed_ws;
    } else {
        if ((st = ensure_ws(h, total)) != CFUST_OK) return st;
        base = (char *)h->ws;
    }
    auto W = [base](size_t off) { return (void *)(base + off); };
    if ((st = hip_check(h, hipSetDevice(h->device), "hipSetDevice")) != CFUST_OK) return st;
    CompPre *pre = (CompPre *)W(L.pre);
    double *lfc = logf_comp ? logf_comp : (double *)W(L.logf);
    hipError_t e = launch_precompute(*P, d.p, d.q, d.g, pre, s);
    if (e == hipSuccess && mixed && J > 0) e = launch_tables(pre, d.p, d.g, d.q + 2, (float *)W(L.tabs), s);
    // FP64 tables: the FP64 integrand (FP64 mode) and, in mixed mode, the
    // items whose FP32 product underflows
    if (e == hipSuccess && J > 0) e = launch_tables64(pre, d.p, d.g, d.q + 2, (double *)W(L.tabs64), s);
    int32_t *need = nullptr;
    if (e == hipSuccess && sur && J > 0) {
        need = (int32_t *)W(need_off);
        e = launch_fill_i32(need, (size_t)d.g * J * d.n, 1, s);
        for (int k = 0; k < nsg && e == hipSuccess; ++k) {
            const SurGroup &G = sg[k];
            if (G.rows == 0) continue;
            SurFeatArgs fa;
            fa.y = y; fa.mu = P->mu; fa.pre = pre;
            fa.n = d.n; fa.p = d.p; fa.q = d.q; fa.g = d.g; fa.J = J;
            fa.m = G.m; fa.idx0 = G.idx0; fa.cnt = G.cnt;
            fa.X0 = (uint16_t *)W(G.x0); fa.inrange = (int32_t *)W(G.inr); fa.base = (double *)W(G.base);
            e = launch_sur_features(fa, s);
            if (e == hipSuccess && G.rows_pad > G.rows)
                e = launch_fill_i32((int32_t *)(fa.X0 + (size_t)G.rows * CFUST_MLP_IN),
                                    (size_t)(G.rows_pad - G.rows) * CFUST_MLP_IN / 2, 0, s);
            for (long r = 0; r < G.rows_pad && e == hipSuccess; r += SUR_CHUNK) {
                const int B = (int)(G.rows_pad - r < SUR_CHUNK ? G.rows_pad - r : SUR_CHUNK);
                e = launch_mlp_forward(*sur->model[G.m], fa.X0 + (size_t)r * CFUST_MLP_IN, B,
                                       (float *)W(G.out) + (size_t)r * CFUST_MLP_OUT, nullptr,
                                       (uint16_t *)W(sa_off), (uint16_t *)W(sb_off), s);
            }
            if (e != hipSuccess) break;
            SurSelArgs sa;
            sa.n = d.n; sa.g = d.g; sa.J = J; sa.m = G.m; sa.idx0 = G.idx0; sa.cnt = G.cnt;
            sa.out = (float *)W(G.out); sa.inrange = (int32_t *)W(G.inr); sa.tol = sur->tol;
            sa.base = (double *)W(G.base);
            sa.est = (double *)W(L.est); sa.lnA = (double *)W(L.lnA); sa.need = need;
            e = launch_sur_select(sa, s);
        }
    }
    if (e == hipSuccess && J > 0) {
        EstepQmcArgs a;
        a.need = need;
        a.y = y; a.mu = P->mu; a.pre = pre; a.tabs = (float *)W(L.tabs);
        a.tabs64 = (double *)W(L.tabs64);
        a.lat = lattice_of(Q);
        a.n = d.n; a.p = d.p; a.q = d.q; a.g = d.g; a.J = J; a.mixed = mixed ? 1 : 0;
        a.est = (double *)W(L.est); a.lnA = (double *)W(L.lnA); a.se = se;
        a.flag = (int32_t *)W(L.flag);
        if (L.coordC > 0) {
            a.coords = (const float *)W(L.coords);
            a.coordC = L.coordC;
            e = launch_lattice_coords(a.lat, L.coordC, (float *)W(L.coords), s);
        }
        // integrals of equal dimension share a launch: (A, B) m = q, C_i m = q-1, D_ik m = q-2
        a.idx0 = 0;
        if (e == hipSuccess) e = timed_qmc(h, a, fixed_ws == nullptr, d.q, density_only ? 1 : 2, s);
        if (e == hipSuccess && !density_only && d.q - 1 >= 2) {
            a.idx0 = 2;
            e = timed_qmc(h, a, fixed_ws == nullptr, d.q - 1, d.q, s);
        }
        if (e == hipSuccess && !density_only && d.q - 2 >= 2) {
            a.idx0 = 2 + d.q;
            e = timed_qmc(h, a, fixed_ws == nullptr, d.q - 2, npairs(d.q), s);
        }
    }
    if (e == hipSuccess) {
        EstepAsmArgs a;
        a.y = y; a.mu = P->mu; a.pre = pre;
        a.n = d.n; a.p = d.p; a.q = d.q; a.g = d.g; a.J = J > 0 ? J : 1;
        a.mixed = mixed ? 1 : 0; a.density_only = density_only ? 1 : 0;
        a.est = (double *)W(L.est); a.lnA = (double *)W(L.lnA);
        a.logf_comp = lfc;
        a.w = w; a.e1 = e1; a.e2 = e2; a.e3 = e3;
        e = launch_assemble(a, s);
    }
    if (e == hipSuccess) {
        EstepLseArgs a;
        a.pi = P->pi; a.logf_comp = lfc;
        a.n = d.n; a.g = d.g; a.q = d.q; a.mixed = mixed ? 1 : 0;
        a.tau = density_only ? nullptr : tau;
        a.logf_obs = logf_obs;
        a.w = density_only ? nullptr : w; a.e1 = e1; a.e2 = e2; a.e3 = e3;
        a.partial = (double *)W(L.partial);
        e = launch_lse(a, loglik, s);
    }
    if (e == hipSuccess && status) e = launch_status_fold(pre, d.g, status, s);
    if (e == hipSuccess && sur && sur->n_fallback) {
        if (need) e = launch_count_i32(need, (size_t)d.g * J * d.n, sur->n_fallback, s);
        else e = launch_fill_i32(sur->n_fallback, 1, 0, s);
    }
    return hip_check(h, e, density_only ? "cfust_loglik launch" : "cfust_estep launch");
}

// Fixed device workspace of the allocation-free E-step.  In host code the
// name `scratch` is only a stand-in for the array: its device address comes
// from hipGetSymbolAddress, once per device (with that device current), and
// only that address is ever handed to kernels.  Each device that loads the
// library holds its own copy until the process ends.  Every call on a device
// shares that device's array; nothing in it needs to start at zero (an E-step
// writes every workspace element before reading it).
static __device__ __align__(256) unsigned char scratch[CFUST_NOALLOC_WS_BYTES];

constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};
hipError_t g_scratch_err[SCRATCH_MAX_DEVICES] = {};
bool g_scratch_done[SCRATCH_MAX_DEVICES] = {};

// Looks up (once per device) the address of this device's copy of `scratch`
// with the device current, restoring the caller's current device afterwards.
void scratch_setup(cfust_ctx *c) {
    if (c->device < 0 || c->device >= SCRATCH_MAX_DEVICES) {
        c->scratch_err = (int)hipErrorInvalidDevice;
        return;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_done[c->device]) {
        int prev = 0;
        hipError_t e = hipGetDevice(&prev);
        if (e == hipSuccess) e = hipSetDevice(c->device);
        void *ptr = nullptr;
        if (e == hipSuccess) {
            e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            const hipError_t r = hipSetDevice(prev);
            if (e == hipSuccess) e = r;
        }
        g_scratch_ptr[c->device] = e == hipSuccess ? ptr : nullptr;
        g_scratch_err[c->device] = e;
        g_scratch_done[c->device] = true;
    }
    c->scratch = g_scratch_ptr[c->device];
    c->scratch_err = (int)g_scratch_err[c->device];
}

}  // namespace

extern "C" {

cfust_status cfust_create(cfust_handle *handle, int device) {
    if (!handle) return CFUST_EINVAL;
    *handle = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return CFUST_EDEVICE;
    if (device < 0 || device >= ndev) return CFUST_EINVAL;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return CFUST_EDEVICE;
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return CFUST_EUNSUPPORTED;
    cfust_ctx *c = new (std::nothrow) cfust_ctx;
    if (!c) return CFUST_ENOMEM;
    c->device = device;
    c->ncu = prop.multiProcessorCount;
    c->arch = prop.gcnArchName;
    scratch_setup(c);
    *handle = c;
    return CFUST_OK;
}

cfust_status cfust_destroy(cfust_handle h) {
    if (!h) return CFUST_EINVAL;
    // teardown: errors here have no caller left to act on them
    (void)hipSetDevice(h->device);
    for (auto &r : h->rec) { (void)hipEventSynchronize(r.e1); (void)hipEventDestroy(r.e0); (void)hipEventDestroy(r.e1); }
    for (auto e : h->pool) (void)hipEventDestroy(e);
    if (h->ws) (void)hipFree(h->ws);
    delete h;
    return CFUST_OK;
}

const char *cfust_last_error(cfust_handle h) {
    return h ? h->err.c_str() : "null handle";
}

cfust_status cfust_estep(cfust_handle h, const double *y, cfust_dims dims, const cfust_params *params,
                         const cfust_qmc *qmc, const cfust_estep_out *out, void *stream) {
    if (!h) return CFUST_EINVAL;
    if (!out) return fail(h, CFUST_EINVAL, "out is NULL");
    return run_estep(h, y, dims, params, qmc, false, out->tau, out->logf_obs, out->loglik, out->w, out->e1,
                     out->e2, out->e3, out->logf_comp, out->cdf_stderr, out->status, (hipStream_t)stream);
}

cfust_status cfust_estep_noalloc(cfust_handle h, const double *y, cfust_dims dims, const cfust_params *params,
                                 const cfust_qmc *qmc, const cfust_estep_out *out, void *stream) {
    if (!h) return CFUST_EINVAL;
    if (!out) return fail(h, CFUST_EINVAL, "out is NULL");
    if (!h->scratch)
        return fail(h, CFUST_EDEVICE, "fixed workspace of device %d unavailable: hipGetSymbolAddress: %s", h->device,
                    hipGetErrorString((hipError_t)h->scratch_err));
    return run_estep(h, y, dims, params, qmc, false, out->tau, out->logf_obs, out->loglik, out->w, out->e1,
                     out->e2, out->e3, out->logf_comp, out->cdf_stderr, out->status, (hipStream_t)stream, nullptr,
                     (char *)h->scratch, (size_t)CFUST_NOALLOC_WS_BYTES);
}

cfust_status cfust_estep_surrogate(cfust_handle h, const double *y, cfust_dims dims, const cfust_params *params,
                                   const cfust_qmc *qmc, const cfust_surrogate *sur, const cfust_estep_out *out,
                                   void *stream) {
    if (!h) return CFUST_EINVAL;
    if (!out) return fail(h, CFUST_EINVAL, "out is NULL");
    if (!sur) return fail(h, CFUST_EINVAL, "sur is NULL");
    return run_estep(h, y, dims, params, qmc, false, out->tau, out->logf_obs, out->loglik, out->w, out->e1,
                     out->e2, out->e3, out->logf_comp, out->cdf_stderr, out->status, (hipStream_t)stream, sur);
}

cfust_status cfust_mlp_features(cfust_handle h, int32_t m, int32_t batch, int32_t rows_pad, const double *b,
                                const double *L, const int32_t *mat_idx, int32_t nmat, const double *nu,
                                uint16_t *X0, int32_t *inrange, double *base, void *stream) {
    if (!h) return CFUST_EINVAL;
    if (m < 2 || m > MAXQ) return fail(h, CFUST_EINVAL, "m = %d outside [2, %d]", m, MAXQ);
    if (batch < 0 || rows_pad < batch) return fail(h, CFUST_EINVAL, "rows_pad < batch");
    if (nmat < 1) return fail(h, CFUST_EINVAL, "nmat < 1");
    if (!X0 || (batch > 0 && (!b || !L || !mat_idx || !nu))) return fail(h, CFUST_EINVAL, "a buffer is NULL");
    cfust_status st;
    if ((st = hip_check(h, hipSetDevice(h->device), "hipSetDevice")) != CFUST_OK) return st;
    return hip_check(h, launch_mvt_features(m, batch, rows_pad, b, L, mat_idx, nmat, nu, X0, inrange, base,
                                            (hipStream_t)stream),
                     "cfust_mlp_features");
}

cfust_status cfust_loglik(cfust_handle h, const double *y, cfust_dims dims, const cfust_params *params,
                          const cfust_qmc *qmc, double *loglik, double *logf_obs, int32_t *status,
                          void *stream) {
    if (!h) return CFUST_EINVAL;
    return run_estep(h, y, dims, params, qmc, true, nullptr, logf_obs, loglik, nullptr, nullptr, nullptr,
                     nullptr, nullptr, nullptr, status, (hipStream_t)stream);
}

cfust_status cfust_mstep(cfust_handle h, const double *y, cfust_dims d, const cfust_estep_out *es,
                         int32_t precision, const cfust_params *in, const cfust_params_out *out,
                         int32_t *status, void *stream) {
    if (!h) return CFUST_EINVAL;
    cfust_status st;
    if ((st = check_dims(h, d)) != CFUST_OK) return st;
    if ((st = check_params(h, in)) != CFUST_OK) return st;
    if (!out || !out->pi || !out->mu || !out->Sigma || !out->Delta || !out->nu)
        return fail(h, CFUST_EINVAL, "an output parameter array is NULL");
    if (precision != CFUST_FP64 && precision != CFUST_MIXED)
        return fail(h, CFUST_EINVAL, "precision %d is neither CFUST_FP64 nor CFUST_MIXED", precision);
    if (d.n > 0 && (!y || !es || !es->tau || !es->w || !es->e1 || !es->e2 || !es->e3))
        return fail(h, CFUST_EINVAL, "y or an E-step array is NULL");
    const int nblk = mstep_nblk(d, h->ncu);
    if ((st = ensure_ws(h, mstep_bytes(d, h->ncu))) != CFUST_OK) return st;
    if ((st = hip_check(h, hipSetDevice(h->device), "hipSetDevice")) != CFUST_OK) return st;
    MstepArgs r;
    r.y = y; r.tau = es ? es->tau : nullptr;
    r.w = es ? es->w : nullptr; r.e1 = es ? es->e1 : nullptr;
    r.e2 = es ? es->e2 : nullptr; r.e3 = es ? es->e3 : nullptr;
    r.mu0 = in->mu;
    r.n = d.n; r.p = d.p; r.q = d.q; r.g = d.g; r.mixed = precision == CFUST_MIXED;
    r.nblk = nblk;
    r.partial = at<double>(h, 0);
    MsolveArgs sv;
    sv.partial = r.partial;
    sv.n = d.n; sv.p = d.p; sv.q = d.q; sv.g = d.g; sv.nblk = nblk;
    sv.mu0 = in->mu; sv.Sigma0 = in->Sigma; sv.Delta0 = in->Delta; sv.nu0 = in->nu;
    sv.pi1 = out->pi; sv.mu1 = out->mu; sv.Sigma1 = out->Sigma; sv.Delta1 = out->Delta; sv.nu1 = out->nu;
    sv.status = status;
    return hip_check(h, launch_mstep(r, sv, (hipStream_t)stream), "cfust_mstep launch");
}

cfust_status mvt_cdf_batch(cfust_handle h, int32_t m, int32_t batch, const double *b, const double *L,
                           const int32_t *mat_idx, int32_t nmat, const double *nu, const cfust_qmc *qmc,
                           double *p, double *logp, double *stderr_, void *stream) {
    if (!h) return CFUST_EINVAL;
    if (m < 1 || m > MAXQ) return fail(h, CFUST_EINVAL, "m = %d outside [1, %d]", m, MAXQ);
    if (batch < 0) return fail(h, CFUST_EINVAL, "batch = %d < 0", batch);
    if (nmat < 1) return fail(h, CFUST_EINVAL, "nmat = %d < 1", nmat);
    cfust_status st;
    if ((st = check_qmc(h, qmc, m >= 2)) != CFUST_OK) return st;
    if (batch > 0 && (!b || !L || !mat_idx || !nu || !p))
        return fail(h, CFUST_EINVAL, "an mvt_cdf_batch array is NULL");
    const bool mixed = qmc->precision == CFUST_MIXED;
    // workspace: flags [batch]; m >= 2: the FP64 tables of a chunk of items,
    // and in mixed precision their FP32 tables, the normal table and the
    // lattice coordinates
    Carve c;
    const size_t o_flag = c.take<int32_t>(batch > 0 ? batch : 1);
    MvtWork w;
    size_t o_tabs = 0, o_ntab = 0, o_coords = 0, o_tabs64 = 0;
    if (m >= 2) {
        w.chunk = batch < MVT_CHUNK ? (batch > 0 ? batch : 1) : MVT_CHUNK;
        o_tabs64 = c.take<double>((size_t)w.chunk * m * TAB64_DOUBLES);
    }
    if (mixed && m >= 2) {
        w.C = lattice_coord_count(m, qmc);
        o_tabs = c.take<float>((size_t)w.chunk * m * TABF_FLOATS);
        o_ntab = c.take<float>(TABF_FLOATS);
        o_coords = c.take<float>(w.C > 0 ? lattice_coords_floats(qmc->N, qmc->S, w.C) : 1);
    }
    if ((st = ensure_ws(h, c.off)) != CFUST_OK) return st;
    if ((st = hip_check(h, hipSetDevice(h->device), "hipSetDevice")) != CFUST_OK) return st;
    if (m >= 2) w.tabs64 = at<double>(h, o_tabs64);
    if (mixed && m >= 2) {
        w.tabs = at<float>(h, o_tabs);
        w.ntab = at<float>(h, o_ntab);
        w.coords = at<float>(h, o_coords);
    }
    MvtArgs a;
    a.m = m; a.batch = batch; a.mixed = mixed ? 1 : 0; a.nmat = nmat;
    a.b = b; a.L = L; a.nu = nu; a.mat_idx = mat_idx;
    a.lat = lattice_of(qmc);
    a.p = p; a.logp = logp; a.se = stderr_;
    a.flag = at<int32_t>(h, o_flag);
    return hip_check(h, launch_mvt(a, w, (hipStream_t)stream), "mvt_cdf_batch launch");
}

cfust_status cfust_autotune(cfust_handle h, const double *y, cfust_dims d, const cfust_params *P,
                            const cfust_qmc *Q, int32_t *chosen, void *stream) {
    if (!h) return CFUST_EINVAL;
    cfust_status st;
    if ((st = check_dims(h, d)) != CFUST_OK) return st;
    if ((st = check_params(h, P)) != CFUST_OK) return st;
    if ((st = check_qmc(h, Q, d.q >= 2)) != CFUST_OK) return st;
    if (chosen) for (int m = 0; m <= MAXQ; ++m) chosen[m] = 0;
    if (d.q < 2 || d.n == 0) return CFUST_OK;
    if (!y) return fail(h, CFUST_EINVAL, "y is NULL");
    hipStream_t s = (hipStream_t)stream;
    const bool mixed = Q->precision == CFUST_MIXED;
    const int J = nint_qmc(d.q);
    const EstepWs L = estep_layout(d, J, true, coord_count(d, Q), Q);
    if ((st = ensure_ws(h, L.total)) != CFUST_OK) return st;
    if ((st = hip_check(h, hipSetDevice(h->device), "hipSetDevice")) != CFUST_OK) return st;
    CompPre *pre = at<CompPre>(h, L.pre);
    hipError_t e = launch_precompute(*P, d.p, d.q, d.g, pre, s);
    if (e == hipSuccess && mixed) e = launch_tables(pre, d.p, d.g, d.q + 2, at<float>(h, L.tabs), s);
    if (e == hipSuccess && !mixed) e = launch_tables64(pre, d.p, d.g, d.q + 2, at<double>(h, L.tabs64), s);
    if (e != hipSuccess) return hip_check(h, e, "cfust_autotune");
    EstepQmcArgs a;
    a.y = y; a.mu = P->mu; a.pre = pre; a.tabs = at<float>(h, L.tabs);
    a.tabs64 = mixed ? nullptr : at<double>(h, L.tabs64);
    a.lat = lattice_of(Q);
    a.n = d.n; a.p = d.p; a.q = d.q; a.g = d.g; a.J = J; a.mixed = mixed ? 1 : 0;
    a.est = at<double>(h, L.est); a.lnA = at<double>(h, L.lnA); a.se = nullptr;
    a.flag = at<int32_t>(h, L.flag);
    a.need = nullptr;
    if (L.coordC > 0) {
        a.coords = at<float>(h, L.coords);
        a.coordC = L.coordC;
        if ((e = launch_lattice_coords(a.lat, L.coordC, at<float>(h, L.coords), s)) != hipSuccess)
            return hip_check(h, e, "cfust_autotune");
    }
    struct Group { int idx0, m, nidx; };
    Group groups[3] = {{0, d.q, 2}, {2, d.q - 1, d.q}, {2 + d.q, d.q - 2, npairs(d.q)}};
    hipEvent_t e0 = pool_event(h), e1 = pool_event(h);
    if (!e0 || !e1) return fail(h, CFUST_EDEVICE, "cfust_autotune: event creation failed");
    for (const Group &gr : groups) {
        if (gr.m < 2) continue;
        a.idx0 = gr.idx0;
        int best = 1;
        float best_ms = 1e30f;
        const int maxp = (mixed && a.lat.N % 128 == 0) ? 2 : 1;
        for (int ppl = 1; ppl <= maxp; ++ppl) {
            float t = 0.0f;
            e = launch_estep_qmc(a, gr.m, gr.nidx, s, nullptr, nullptr, ppl);          // warm
            if (e == hipSuccess) e = launch_estep_qmc(a, gr.m, gr.nidx, s, e0, e1, ppl);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
            if (e != hipSuccess) break;
            if (t < best_ms) { best_ms = t; best = ppl; }
        }
        if (e != hipSuccess) break;
        h->tuned[std::make_tuple(gr.m, a.lat.N, a.lat.S, mixed ? 1 : 0)] = best;
        if (chosen) chosen[gr.m] = best;
    }
    h->pool.push_back(e0);
    h->pool.push_back(e1);
    return hip_check(h, e, "cfust_autotune");
}

// ------------------------------------------------------------- surrogate MLP


cfust_status cfust_mlp_forward(cfust_handle h, const cfust_mlp_weights *w, const uint16_t *X0, int32_t B,
                               float *out, const cfust_mlp_acts *acts, void *stream) {
    if (!h) return CFUST_EINVAL;
    cfust_status st;
    if ((st = check_mlp_b(h, B)) != CFUST_OK) return st;
    if (!weights_ok(w) || !X0 || !out) return fail(h, CFUST_EINVAL, "a network buffer is NULL");
    if (acts) {
        for (int l = 0; l < CFUST_MLP_LAYERS; ++l)
            if (!acts->X[l] || !acts->XT[l] || (l < CFUST_MLP_LAYERS - 1 && !acts->Z[l]))
                return fail(h, CFUST_EINVAL, "an activation buffer is NULL");
    }
    Carve c;
    const size_t sa = c.take<uint16_t>(std::max((size_t)B * CFUST_MLP_HIDDEN, mlp_packed_elems()));
    const size_t sb = c.take<uint16_t>((size_t)B * CFUST_MLP_HIDDEN);
    if (!acts && (st = ensure_ws(h, c.off)) != CFUST_OK) return st;
    if ((st = hip_check(h, hipSetDevice(h->device), "hipSetDevice")) != CFUST_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    const uint16_t *x0 = X0;
    if (acts) {
        e = launch_transpose_in(X0, B, acts->X[0], acts->XT[0], s);
        x0 = acts->X[0];
    }
    if (e == hipSuccess)
        e = launch_mlp_forward(*w, x0, B, out, acts, acts ? nullptr : at<uint16_t>(h, sa),
                               acts ? nullptr : at<uint16_t>(h, sb), s);
    return hip_check(h, e, "cfust_mlp_forward");
}

cfust_status cfust_mlp_backward(cfust_handle h, const cfust_mlp_weights *w, const cfust_mlp_acts *acts,
                                const float *dout, int32_t B, const cfust_mlp_grads *grads, void *stream) {
    if (!h) return CFUST_EINVAL;
    cfust_status st;
    if ((st = check_mlp_b(h, B)) != CFUST_OK) return st;
    if (!weights_ok(w) || !acts || !dout || !grads) return fail(h, CFUST_EINVAL, "a network buffer is NULL");
    for (int l = 0; l < CFUST_MLP_LAYERS; ++l)
        if (!grads->dW[l] || !grads->db[l]) return fail(h, CFUST_EINVAL, "a gradient buffer is NULL");
    Carve c;
    const size_t part = c.take<float>((size_t)16 * CFUST_MLP_HIDDEN * CFUST_MLP_HIDDEN);
    const size_t dy = c.take<float>((size_t)B * CFUST_MLP_HIDDEN);
    const size_t dzb = c.take<uint16_t>((size_t)B * CFUST_MLP_HIDDEN);
    const size_t dzt = c.take<uint16_t>((size_t)B * CFUST_MLP_HIDDEN);
    if ((st = ensure_ws(h, c.off)) != CFUST_OK) return st;
    if ((st = hip_check(h, hipSetDevice(h->device), "hipSetDevice")) != CFUST_OK) return st;
    return hip_check(h, launch_mlp_backward(*w, *acts, dout, B, *grads, at<float>(h, part), at<float>(h, dy),
                                            at<uint16_t>(h, dzb), at<uint16_t>(h, dzt), (hipStream_t)stream),
                     "cfust_mlp_backward");
}

cfust_status cfust_mlp_adam(cfust_handle h, const cfust_mlp_master *m, const cfust_mlp_grads *g,
                            const cfust_mlp_weights *w, float lr, float b1, float b2, float eps, int32_t step,
                            void *stream) {
    if (!h) return CFUST_EINVAL;
    if (!m || !g || !weights_ok(w) || step < 1) return fail(h, CFUST_EINVAL, "bad Adam arguments");
    cfust_status st;
    if ((st = hip_check(h, hipSetDevice(h->device), "hipSetDevice")) != CFUST_OK) return st;
    return hip_check(h, launch_mlp_adam(*m, *g, *w, lr, b1, b2, eps, step, (hipStream_t)stream), "cfust_mlp_adam");
}

cfust_status cfust_mlp_loss(cfust_handle h, const float *out, const float *label, int32_t B, int32_t nvalid,
                            float lam, float *dout, float *loss_sum, void *stream) {
    if (!h) return CFUST_EINVAL;
    cfust_status st;
    if ((st = check_mlp_b(h, B)) != CFUST_OK) return st;
    if (nvalid < 1 || nvalid > B) return fail(h, CFUST_EINVAL, "nvalid = %d outside [1, B]", nvalid);
    if (!out || !label || !dout || !loss_sum) return fail(h, CFUST_EINVAL, "a loss buffer is NULL");
    if ((st = ensure_ws(h, align256((size_t)(B / 256 + 2) * sizeof(float)))) != CFUST_OK) return st;
    if ((st = hip_check(h, hipSetDevice(h->device), "hipSetDevice")) != CFUST_OK) return st;
    return hip_check(h, launch_mlp_loss(out, label, B, nvalid, lam, dout, at<float>(h, 0), loss_sum,
                                        (hipStream_t)stream), "cfust_mlp_loss");
}

cfust_status cfust_profile_enable(cfust_handle h, int enable) {
    if (!h) return CFUST_EINVAL;
    h->prof = enable != 0;
    return CFUST_OK;
}

cfust_status cfust_profile_read(cfust_handle h, double *ms, int32_t *launches) {
    if (!h || !ms || !launches) return CFUST_EINVAL;
    for (int m = 0; m <= MAXQ; ++m) { ms[m] = 0.0; launches[m] = 0; }
    cfust_status st = CFUST_OK;
    for (auto &r : h->rec) {
        float t = 0.0f;
        hipError_t e = hipEventSynchronize(r.e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&t, r.e0, r.e1);
        if (e != hipSuccess) st = hip_check(h, e, "cfust_profile_read");
        else if (r.m >= 0 && r.m <= MAXQ) { ms[r.m] += t; launches[r.m] += 1; }
        h->pool.push_back(r.e0);
        h->pool.push_back(r.e1);
    }
    h->rec.clear();
    return st;
}

cfust_status cfust_reserve(cfust_handle h, cfust_dims d, const cfust_qmc *qmc) {
    if (!h) return CFUST_EINVAL;
    cfust_status st;
    if ((st = check_dims(h, d)) != CFUST_OK) return st;
    size_t need = estep_layout(d, nint_qmc(d.q), true, coord_count(d, qmc), qmc).total;
    const size_t ms = mstep_bytes(d, h->ncu);
    if (ms > need) need = ms;
    if ((st = hip_check(h, hipSetDevice(h->device), "hipSetDevice")) != CFUST_OK) return st;
    return ensure_ws(h, need);
}

}  // extern "C"
