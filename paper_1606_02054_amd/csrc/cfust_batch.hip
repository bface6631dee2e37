// cfust_batch.hip -- host side of batched fits: plan (workspace, per-fit
// argument blocks, lattice work queues), the launch sequence of one E-step,
// M-step and EM iteration over all fits, its capture in a HIP graph, and the
// autotuner of the queues.
//
// Work queues.  The lattice integrals of every fit are grouped by dimension m
// (A and B: m = q; C_i: q - 1; D_ik: q - 2; only m >= 2 use the lattice).
// Queue m holds tiles (fit, component h, integral idx, `rows` consecutive
// observations); one persistent kernel per m draws them with an atomic
// counter.  Every full tile of a queue costs the same (same m, same lattice),
// and a fit's last, partial tile costs less, so longest-processing-time order
// is: all full tiles, then the partial ones; queues run from the largest m
// down.  Mixed precision appends the items whose FP32 product underflowed to a
// per-queue list that an FP64 kernel then evaluates.
#include <string.h>

#include <algorithm>
#include <new>

#include "cfust_host.h"

using namespace cfust;
using namespace cfust_host;

namespace {

struct Queue {
    int m = 0;
    std::vector<QSeg> seg;
    QSeg *dseg = nullptr;
    int seg_cap = 0;
    long long ntiles = 0;
    long long items = 0;                    // (pair, integral) items
    unsigned long long *counter = nullptr;
    unsigned long long *redo = nullptr;     // [items]
    unsigned int *redo_count = nullptr;
    int rows = 4, mult = 1, ppl = 1;
    bool persist = false;                   // persistent blocks, or one block per tile (default)
    int grid = 0, redo_grid = 0, redo_grid64 = 0;
};

struct Group {
    int m, idx0, nidx;
};

// Lattice integrals of a fit by dimension; a density-only fit needs A only.
int fit_groups(int q, bool density, Group *gr) {
    int ng = 0;
    if (q >= 2) gr[ng++] = {q, 0, density ? 1 : 2};
    if (density) return ng;
    if (q - 1 >= 2) gr[ng++] = {q - 1, 2, q};
    if (q - 2 >= 2) gr[ng++] = {q - 2, 2 + q, npairs(q)};
    return ng;
}

// A fit with observations and no E-step output arrays asks for its
// log-likelihood only (an empty fit's arrays may be NULL either way).
bool density_only(const cfust_fit &F) {
    return F.dims.n > 0 && !F.out.tau && !F.out.w && !F.out.e1 && !F.out.e2 && !F.out.e3;
}

}  // namespace

struct cfust_batch_ctx {
    cfust_handle h = nullptr;
    int nfits = 0;
    bool mixed = false;
    LatticeArgs lat{};
    float *coords = nullptr;         // lattice coordinate table (see lattice_coord_count), or null
    int coordC = 0;
    std::vector<cfust_fit> fits;
    std::vector<char> dens;          // per fit: log-likelihood only
    bool any_density = false;
    void *ws = nullptr;
    size_t ws_size = 0;
    FitDesc *dfits = nullptr;
    int *dprefix = nullptr;
    int nblocks[BK_NKIND] = {};
    size_t mred_lds = 0;             // dynamic LDS of the batched M-step reduction
    int32_t *active = nullptr;       // [nfits]
    int32_t *iter = nullptr;         // [1]
    double *hist = nullptr;          // [nfits][2]
    int32_t *counters = nullptr;     // 4 words per queue: tile counter (u64), redo count (u32), pad
    std::vector<Queue> queues;       // largest m first
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    BatchCtl *ctl = nullptr;         // device copy of the run's arguments
    BatchCtl hctl{};                 // host staging of *ctl
};

namespace {

template <class T> T *bat(cfust_batch b, size_t off) { return (T *)((char *)b->ws + off); }

BatchArgs batch_args(cfust_batch b) {
    BatchArgs a;
    a.fits = b->dfits;
    a.nfits = b->nfits;
    a.active = b->active;
    a.prefix = b->dprefix;
    return a;
}

// Segments of queue Q for tiles of `rows` observations: full tiles of every
// fit first, then the partial tiles.
void build_segments(cfust_batch b, Queue &Q, int rows) {
    Q.seg.clear();
    Q.rows = rows;
    long long t = 0;
    for (int pass = 0; pass < 2; ++pass) {
        for (int f = 0; f < b->nfits; ++f) {
            const cfust_dims &d = b->fits[f].dims;
            Group gr[3];
            const int ng = fit_groups(d.q, b->dens[f] != 0, gr);
            for (int k = 0; k < ng; ++k) {
                if (gr[k].m != Q.m || d.n == 0) continue;
                QSeg s;
                s.fit = f; s.idx0 = gr[k].idx0; s.nidx = gr[k].nidx;
                if (pass == 0) {
                    s.j0 = 0; s.rows = rows; s.rtiles = d.n / rows;
                } else {
                    s.rows = d.n % rows; s.j0 = d.n - s.rows; s.rtiles = s.rows > 0 ? 1 : 0;
                }
                if (s.rtiles == 0) continue;
                s.t0 = t;
                t += (long long)d.g * s.nidx * s.rtiles;
                Q.seg.push_back(s);
            }
        }
    }
    Q.ntiles = t;
}

cfust_status upload_segments(cfust_batch b, Queue &Q) {
    if (Q.seg.empty()) return CFUST_OK;
    return hip_check(b->h, hipMemcpy(Q.dseg, Q.seg.data(), Q.seg.size() * sizeof(QSeg), hipMemcpyHostToDevice),
                     "batch segments upload");
}

// grid = 0 selects one block per tile (launch_queue_qmc).
void set_grid(cfust_batch b, Queue &Q) {
    const int ncu = b->h->ncu > 0 ? b->h->ncu : 256;
    Q.grid = Q.persist ? ncu * queue_qmc_occupancy(Q.m, b->mixed, Q.ppl, b->coordC > 0) * Q.mult : 0;
    Q.redo_grid = ncu * queue_redo_occupancy(Q.m, false);
    Q.redo_grid64 = ncu * queue_redo_occupancy(Q.m, true);
}

QueueArgs queue_args(cfust_batch b, const Queue &Q, long long ntiles) {
    QueueArgs a;
    a.fits = b->dfits;
    a.active = b->active;
    a.seg = Q.dseg;
    a.nseg = (int)Q.seg.size();
    a.ntiles = ntiles;
    a.counter = Q.counter;
    a.redo = Q.redo;
    a.redo_count = Q.redo_count;
    a.lat = b->lat;
    return a;
}

void drop_graph(cfust_batch b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

hipError_t enqueue_estep(cfust_batch b, hipStream_t s) {
    const BatchArgs A = batch_args(b);
    hipError_t e = launch_fill_i32(b->counters, 4 * b->queues.size(), 0, s);
    if (e == hipSuccess) e = launch_batch_precompute(A, b->nblocks[BK_PRE], s);
    if (e == hipSuccess) e = launch_batch_tables(A, b->nblocks[BK_TAB], s);
    if (e == hipSuccess && b->coordC > 0) e = launch_lattice_coords(b->lat, b->coordC, b->coords, s);
    // timing events (cfust_profile_enable) only outside stream capture
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    const bool prof = b->h->prof && hipStreamIsCapturing(s, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone;
    for (const Queue &Q : b->queues) {
        if (e != hipSuccess || Q.ntiles == 0) continue;
        const QueueArgs qa = queue_args(b, Q, Q.ntiles);
        ProfRec r{Q.m, prof ? pool_event(b->h) : nullptr, prof ? pool_event(b->h) : nullptr};
        if (r.e0) e = hipEventRecord(r.e0, s);
        if (e == hipSuccess) e = launch_queue_qmc(qa, Q.m, b->mixed, Q.ppl, Q.grid, s, b->coordC > 0);
        if (e == hipSuccess && r.e1) e = hipEventRecord(r.e1, s);
        if (r.e0 && r.e1) b->h->rec.push_back(r);
        // mixed: items whose FP32 product underflowed; FP64: items of integrals
        // whose dof is past the FP64 tables
        if (e == hipSuccess) e = launch_queue_redo(qa, Q.m, Q.redo_grid, Q.redo_grid64, s);
    }
    if (e == hipSuccess) e = launch_batch_assemble(A, b->nblocks[BK_ASM], s);
    if (e == hipSuccess) e = launch_batch_lse(A, b->nblocks[BK_LSE], s);
    if (e == hipSuccess) e = launch_batch_sum(A, s);
    return e;
}

hipError_t enqueue_mstep(cfust_batch b, hipStream_t s) {
    return launch_batch_mstep(batch_args(b), b->nblocks[BK_MRED], b->nblocks[BK_MSOL], b->mred_lds, s);
}

hipError_t enqueue_iteration(cfust_batch b, hipStream_t s) {
    hipError_t e = enqueue_estep(b, s);
    if (e == hipSuccess) e = launch_batch_check(b->dfits, b->nfits, b->active, b->iter, b->hist, b->ctl, s);
    if (e == hipSuccess) e = enqueue_mstep(b, s);
    return e;
}

cfust_status check_fit(cfust_handle h, int f, const cfust_fit &F) {
    cfust_status st;
    if ((st = check_dims(h, F.dims)) != CFUST_OK) return fail(h, st, "fit %d: %s", f, h->err.c_str());
    const cfust_params_out &P = F.params;
    if (!P.pi || !P.mu || !P.Sigma || !P.Delta || !P.nu) return fail(h, CFUST_EINVAL, "fit %d: a parameter array is NULL", f);
    const cfust_estep_out &O = F.out;
    if (!O.loglik) return fail(h, CFUST_EINVAL, "fit %d: loglik is NULL", f);
    if (F.dims.n > 0 && !F.y) return fail(h, CFUST_EINVAL, "fit %d: y is NULL", f);
    if (F.dims.n > 0 && !density_only(F) && (!O.tau || !O.logf_obs || !O.w || !O.e1 || !O.e2 || !O.e3))
        return fail(h, CFUST_EINVAL, "fit %d: an E-step output array is NULL", f);
    return CFUST_OK;
}

}  // namespace

extern "C" {

cfust_status cfust_batch_create(cfust_handle h, int32_t nfits, const cfust_fit *fits, const cfust_qmc *qmc,
                                cfust_batch *out) {
    if (!h) return CFUST_EINVAL;
    if (!out) return fail(h, CFUST_EINVAL, "batch is NULL");
    *out = nullptr;
    if (nfits < 1 || nfits > BATCH_MAX_FITS)
        return fail(h, CFUST_EINVAL, "nfits = %d outside [1, %d]", nfits, BATCH_MAX_FITS);
    if (!fits) return fail(h, CFUST_EINVAL, "fits is NULL");
    cfust_status st;
    bool lattice = false;
    int maxq = 0;
    for (int f = 0; f < nfits; ++f) {
        if ((st = check_fit(h, f, fits[f])) != CFUST_OK) return st;
        lattice = lattice || fits[f].dims.q >= 2;
        if (fits[f].dims.n > 0) maxq = std::max(maxq, fits[f].dims.q);
    }
    if ((st = check_qmc(h, qmc, lattice)) != CFUST_OK) return st;
    if ((st = hip_check(h, hipSetDevice(h->device), "hipSetDevice")) != CFUST_OK) return st;

    cfust_batch b = new (std::nothrow) cfust_batch_ctx;
    if (!b) return fail(h, CFUST_ENOMEM, "batch allocation failed");
    b->h = h;
    b->nfits = nfits;
    b->mixed = qmc->precision == CFUST_MIXED;
    b->lat = lattice ? lattice_of(qmc) : LatticeArgs{};
    b->coordC = lattice ? lattice_coord_count(maxq, qmc) : 0;
    b->fits.assign(fits, fits + nfits);
    b->dens.resize(nfits);
    for (int f = 0; f < nfits; ++f) {
        b->dens[f] = density_only(fits[f]) ? 1 : 0;
        b->any_density = b->any_density || b->dens[f];
    }

    // queues: one per lattice dimension present, largest first
    for (int m = MAXQ; m >= 2; --m) {
        Queue Q;
        Q.m = m;
        for (int f = 0; f < nfits; ++f) {
            const cfust_dims &d = fits[f].dims;
            Group gr[3];
            const int ng = fit_groups(d.q, b->dens[f] != 0, gr);
            for (int k = 0; k < ng; ++k)
                if (gr[k].m == m) {
                    Q.items += (long long)d.g * gr[k].nidx * d.n;
                    Q.seg_cap += 2;
                }
        }
        if (Q.items > 0) b->queues.push_back(Q);
    }

    // workspace layout
    Carve c;
    struct FitOff { size_t pre, tabs, tabs64, est, lnA, logf, lse, mpart, cstat; };
    std::vector<FitOff> fo(nfits);
    for (int f = 0; f < nfits; ++f) {
        const cfust_dims &d = fits[f].dims;
        const size_t n1 = d.n > 0 ? d.n : 1;
        const bool dn = b->dens[f] != 0;
        const int J = dn ? (d.q >= 2 ? 1 : 0) : nint_qmc(d.q);
        fo[f].pre = c.take<CompPre>(d.g);
        fo[f].tabs = c.take<float>(b->mixed && J > 0 ? (size_t)d.g * NDOF * TABF_FLOATS : 1);
        fo[f].tabs64 = c.take<double>(J > 0 ? (size_t)d.g * NDOF * TAB64_DOUBLES : 1);
        fo[f].est = c.take<double>((size_t)d.g * (J > 0 ? J : 1) * n1);
        fo[f].lnA = c.take<double>((size_t)d.g * n1);
        fo[f].logf = c.take<double>(fits[f].out.logf_comp ? 1 : (size_t)d.g * n1);
        fo[f].lse = c.take<double>((size_t)(d.n + 255) / 256 + 1);
        fo[f].mpart = c.take<double>(dn ? 1 : (size_t)d.g * mstep_nblk(d, h->ncu) * nstat(d.p, d.q));
        fo[f].cstat = c.take<int32_t>(d.g);
    }
    const size_t o_fits = c.take<FitDesc>(nfits);
    const size_t o_prefix = c.take<int>((size_t)BK_NKIND * (nfits + 1));
    const size_t o_active = c.take<int32_t>(nfits);
    const size_t o_iter = c.take<int32_t>(1);
    const size_t o_hist = c.take<double>((size_t)2 * nfits);
    const size_t o_counters = c.take<int32_t>(4 * (b->queues.size() > 0 ? b->queues.size() : 1));
    const size_t o_ctl = c.take<BatchCtl>(1);
    const size_t o_coords = c.take<float>(b->coordC > 0 ? lattice_coords_floats(b->lat.N, b->lat.S, b->coordC) : 1);
    std::vector<size_t> o_seg(b->queues.size()), o_redo(b->queues.size());
    for (size_t k = 0; k < b->queues.size(); ++k) {
        o_seg[k] = c.take<QSeg>(b->queues[k].seg_cap);
        o_redo[k] = c.take<unsigned long long>((size_t)b->queues[k].items);
    }
    b->ws_size = c.off;
    if (hipMalloc(&b->ws, b->ws_size) != hipSuccess) {
        b->ws = nullptr;
        delete b;
        return fail(h, CFUST_ENOMEM, "batch workspace of %zu bytes failed", c.off);
    }
    b->dfits = bat<FitDesc>(b, o_fits);
    b->dprefix = bat<int>(b, o_prefix);
    b->active = bat<int32_t>(b, o_active);
    b->iter = bat<int32_t>(b, o_iter);
    b->hist = bat<double>(b, o_hist);
    b->counters = bat<int32_t>(b, o_counters);
    b->ctl = bat<BatchCtl>(b, o_ctl);
    if (b->coordC > 0) b->coords = bat<float>(b, o_coords);
    for (size_t k = 0; k < b->queues.size(); ++k) {
        Queue &Q = b->queues[k];
        Q.counter = (unsigned long long *)(b->counters + 4 * k);
        Q.redo_count = (unsigned int *)(b->counters + 4 * k + 2);
        Q.dseg = bat<QSeg>(b, o_seg[k]);
        Q.redo = bat<unsigned long long>(b, o_redo[k]);
    }

    // per-fit argument blocks and block prefixes
    std::vector<FitDesc> hd(nfits);
    std::vector<int> pref((size_t)BK_NKIND * (nfits + 1), 0);
    for (int f = 0; f < nfits; ++f) {
        const cfust_fit &F = fits[f];
        const cfust_dims &d = F.dims;
        const bool dn = b->dens[f] != 0;
        const int J = dn ? (d.q >= 2 ? 1 : 0) : nint_qmc(d.q);
        FitDesc &D = hd[f];
        memset(&D, 0, sizeof D);
        CompPre *pre = bat<CompPre>(b, fo[f].pre);
        float *tabs = bat<float>(b, fo[f].tabs);
        double *est = bat<double>(b, fo[f].est), *lnA = bat<double>(b, fo[f].lnA);
        double *lfc = F.out.logf_comp ? F.out.logf_comp : bat<double>(b, fo[f].logf);
        const int nblk = mstep_nblk(d, b->h->ncu);
        if (!dn) b->mred_lds = std::max(b->mred_lds, mstep_lds_bytes(d.p, d.q));
        D.g = d.g;
        D.pc.pi = F.params.pi; D.pc.Sigma = F.params.Sigma; D.pc.Delta = F.params.Delta; D.pc.nu = F.params.nu;
        D.pc.p = d.p; D.pc.q = d.q; D.pc.pre = pre;
        D.ndof = d.q + 2;
        D.tabs = tabs;
        D.tabs64 = J > 0 ? bat<double>(b, fo[f].tabs64) : nullptr;   // mixed: for the redo list
        EstepQmcArgs &q = D.qa;
        q.y = F.y; q.mu = F.params.mu; q.pre = pre; q.tabs = tabs; q.tabs64 = D.tabs64; q.lat = b->lat;
        q.n = d.n; q.p = d.p; q.q = d.q; q.g = d.g; q.J = J > 0 ? J : 1; q.idx0 = 0; q.mixed = b->mixed;
        q.est = est; q.lnA = lnA; q.se = F.out.cdf_stderr; q.flag = nullptr; q.need = nullptr;
        q.coords = b->coords; q.coordC = b->coordC;
        EstepAsmArgs &a = D.aa;
        a.y = F.y; a.mu = F.params.mu; a.pre = pre;
        a.n = d.n; a.p = d.p; a.q = d.q; a.g = d.g; a.J = J > 0 ? J : 1;
        a.mixed = b->mixed; a.density_only = dn ? 1 : 0;
        a.est = est; a.lnA = lnA; a.logf_comp = lfc;
        a.w = F.out.w; a.e1 = F.out.e1; a.e2 = F.out.e2; a.e3 = F.out.e3;
        EstepLseArgs &l = D.la;
        l.pi = F.params.pi; l.logf_comp = lfc;
        l.n = d.n; l.g = d.g; l.q = d.q; l.mixed = b->mixed;
        l.tau = dn ? nullptr : F.out.tau; l.logf_obs = F.out.logf_obs;
        l.w = F.out.w; l.e1 = F.out.e1; l.e2 = F.out.e2; l.e3 = F.out.e3;
        l.partial = bat<double>(b, fo[f].lse);
        D.nlse = (d.n + 255) / 256;
        D.loglik = F.out.loglik;
        D.status = F.status;
        MstepArgs &r = D.ma;
        r.y = F.y; r.tau = F.out.tau; r.w = F.out.w; r.e1 = F.out.e1; r.e2 = F.out.e2; r.e3 = F.out.e3;
        r.mu0 = F.params.mu;
        r.n = d.n; r.p = d.p; r.q = d.q; r.g = d.g; r.mixed = b->mixed; r.nblk = nblk;
        r.partial = bat<double>(b, fo[f].mpart);
        MsolveArgs &sv = D.sa;
        sv.partial = r.partial;
        sv.n = d.n; sv.p = d.p; sv.q = d.q; sv.g = d.g; sv.nblk = nblk;
        sv.mu0 = F.params.mu; sv.Sigma0 = F.params.Sigma; sv.Delta0 = F.params.Delta; sv.nu0 = F.params.nu;
        sv.pi1 = F.params.pi; sv.mu1 = F.params.mu; sv.Sigma1 = F.params.Sigma; sv.Delta1 = F.params.Delta;
        sv.nu1 = F.params.nu;
        sv.status = nullptr;
        D.cstat = bat<int32_t>(b, fo[f].cstat);
        const int cnt[BK_NKIND] = {d.g,
                                   J > 0 ? d.g * D.ndof : 0,
                                   (d.n * d.g + 127) / 128,
                                   (d.n + 255) / 256,
                                   dn ? 0 : nblk * d.g,
                                   dn ? 0 : d.g};
        for (int k = 0; k < BK_NKIND; ++k) pref[(size_t)k * (nfits + 1) + f + 1] = pref[(size_t)k * (nfits + 1) + f] + cnt[k];
    }
    for (int k = 0; k < BK_NKIND; ++k) b->nblocks[k] = pref[(size_t)k * (nfits + 1) + nfits];
    hipError_t e = hipMemcpy(b->dfits, hd.data(), nfits * sizeof(FitDesc), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->dprefix, pref.data(), pref.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if ((st = hip_check(h, e, "batch setup")) != CFUST_OK) {
        cfust_batch_destroy(b);
        return st;
    }
    for (Queue &Q : b->queues) {
        Q.ppl = (b->mixed && b->lat.N % 128 == 0) ? tuned_ppl(h, Q.m, b->lat, true) : 1;
        set_grid(b, Q);
        build_segments(b, Q, Q.rows);
        if ((st = upload_segments(b, Q)) != CFUST_OK) {
            cfust_batch_destroy(b);
            return st;
        }
    }
    *out = b;
    return CFUST_OK;
}

cfust_status cfust_batch_destroy(cfust_batch b) {
    if (!b) return CFUST_EINVAL;
    // teardown: errors here have no caller left to act on them
    (void)hipSetDevice(b->h->device);
    drop_graph(b);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->ws) {
        (void)hipDeviceSynchronize();
        (void)hipFree(b->ws);
    }
    delete b;
    return CFUST_OK;
}

cfust_status cfust_batch_estep(cfust_batch b, void *stream) {
    if (!b) return CFUST_EINVAL;
    cfust_status st;
    if ((st = hip_check(b->h, hipSetDevice(b->h->device), "hipSetDevice")) != CFUST_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_fill_i32(b->active, b->nfits, 1, s);
    if (e == hipSuccess) e = enqueue_estep(b, s);
    return hip_check(b->h, e, "cfust_batch_estep launch");
}

cfust_status cfust_batch_mstep(cfust_batch b, void *stream) {
    if (!b) return CFUST_EINVAL;
    if (b->any_density) return fail(b->h, CFUST_EINVAL, "the batch has log-likelihood-only fits");
    cfust_status st;
    if ((st = hip_check(b->h, hipSetDevice(b->h->device), "hipSetDevice")) != CFUST_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_fill_i32(b->active, b->nfits, 1, s);
    if (e == hipSuccess) e = enqueue_mstep(b, s);
    return hip_check(b->h, e, "cfust_batch_mstep launch");
}

cfust_status cfust_fit_batch(cfust_batch b, int32_t iters, double tol, int32_t use_graph, double *trace,
                             int32_t *iters_done, void *stream) {
    if (!b) return CFUST_EINVAL;
    cfust_handle h = b->h;
    if (iters < 0) return fail(h, CFUST_EINVAL, "iters = %d < 0", iters);
    if (b->any_density) return fail(h, CFUST_EINVAL, "the batch has log-likelihood-only fits");
    cfust_status st;
    if ((st = hip_check(h, hipSetDevice(h->device), "hipSetDevice")) != CFUST_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    // the run's arguments go to device memory: the captured iteration reads them there
    b->hctl.tol = tol;
    b->hctl.trace = trace;
    b->hctl.iters_done = iters_done;
    b->hctl.max_trace = iters;
    hipError_t e = hipMemcpyAsync(b->ctl, &b->hctl, sizeof(BatchCtl), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_fill_i32(b->active, b->nfits, 1, s);
    if (e == hipSuccess) e = launch_fill_i32(b->iter, 1, 0, s);
    if (e == hipSuccess) e = launch_fill_i32((int32_t *)b->hist, (size_t)4 * b->nfits, 0, s);
    if (e == hipSuccess && iters_done) e = launch_fill_i32(iters_done, b->nfits, 0, s);
    if (e != hipSuccess || iters == 0) return hip_check(h, e, "cfust_fit_batch launch");
    if (!use_graph) {
        for (int it = 0; it < iters && e == hipSuccess; ++it) e = enqueue_iteration(b, s);
        return hip_check(h, e, "cfust_fit_batch launch");
    }
    if (!b->exec) {
        e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            const hipError_t el = enqueue_iteration(b, b->cap);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(b->cap, &g);
            if (el != hipSuccess) e = el;
            if (e == hipSuccess) b->graph = g;
            else if (g) (void)hipGraphDestroy(g);
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            drop_graph(b);
            return hip_check(h, e, "cfust_fit_batch graph capture");
        }
    }
    for (int it = 0; it < iters && e == hipSuccess; ++it) e = hipGraphLaunch(b->exec, s);
    return hip_check(h, e, "cfust_fit_batch graph launch");
}

cfust_status cfust_batch_tune(cfust_batch b, int32_t *chosen, void *stream) {
    if (!b) return CFUST_EINVAL;
    cfust_handle h = b->h;
    cfust_status st;
    if ((st = hip_check(h, hipSetDevice(h->device), "hipSetDevice")) != CFUST_OK) return st;
    if (chosen) for (int i = 0; i < (MAXQ + 1) * 3; ++i) chosen[i] = 0;
    hipStream_t s = (hipStream_t)stream;
    const BatchArgs A = batch_args(b);
    hipError_t e = launch_fill_i32(b->active, b->nfits, 1, s);
    if (e == hipSuccess) e = launch_batch_precompute(A, b->nblocks[BK_PRE], s);
    if (e == hipSuccess) e = launch_batch_tables(A, b->nblocks[BK_TAB], s);
    if (e == hipSuccess && b->coordC > 0) e = launch_lattice_coords(b->lat, b->coordC, b->coords, s);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    const bool ppl2 = b->mixed && b->lat.N % 128 == 0;
    // candidates: persistent (rows per tile, blocks per resident slot) or one
    // block per tile (rows 4, written as 0 blocks per slot), each with 1 or 2
    // lattice points per lane per trip
    struct Cand { bool persist; int rows, mult; };
    const Cand cands[7] = {{true, 4, 1}, {true, 4, 2}, {true, 8, 1}, {true, 8, 2},
                           {true, 16, 1}, {true, 16, 2}, {false, 4, 0}};
    const int ncu = h->ncu > 0 ? h->ncu : 256;
    for (Queue &Q : b->queues) {
        if (e != hipSuccess) break;
        double best = 1e300, best_grid = 1e300;
        Cand bc{Q.persist, Q.rows, Q.mult};
        int bppl = Q.ppl, grid_ppl = 1;
        // the same prefix of the queue for every candidate: about 16 items
        // per wave the chip holds at 8 waves per SIMD
        const long long want = std::min(Q.items, (long long)ncu * 4 * 8 * 16);
        for (int ci = 0; ci < 7 && e == hipSuccess; ++ci)
            for (int ppl = 1; ppl <= (ppl2 ? 2 : 1) && e == hipSuccess; ++ppl) {
                const Cand &C = cands[ci];
                Q.persist = C.persist; Q.mult = C.mult; Q.ppl = ppl;
                set_grid(b, Q);
                build_segments(b, Q, C.rows);
                if ((st = upload_segments(b, Q)) != CFUST_OK) { e = hipErrorUnknown; break; }
                const long long tiles = std::min(Q.ntiles, (want + Q.rows - 1) / Q.rows);
                if (tiles == 0) continue;
                const QueueArgs qa = queue_args(b, Q, tiles);
                float ms = 0.0f;
                for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
                    e = launch_fill_i32(b->counters, 4 * b->queues.size(), 0, s);
                    if (e == hipSuccess) e = hipEventRecord(e0, s);
                    if (e == hipSuccess) e = launch_queue_qmc(qa, Q.m, b->mixed, Q.ppl, Q.grid, s, b->coordC > 0);
                    if (e == hipSuccess) e = hipEventRecord(e1, s);
                    if (e == hipSuccess) e = hipEventSynchronize(e1);
                    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                }
                const double per_item = ms / (double)std::min(tiles * Q.rows, Q.items);
                if (e == hipSuccess && per_item < best) {
                    best = per_item; bc = C; bppl = ppl;
                }
                if (e == hipSuccess && !C.persist && per_item < best_grid) {
                    best_grid = per_item; grid_ppl = ppl;
                }
            }
        // a persistent form must win clearly on the prefix: its timing there
        // has been seen to overstate it on the whole queue
        if (bc.persist && best_grid < 1e300 && best > 0.95 * best_grid) {
            bc = cands[6]; bppl = grid_ppl;
        }
        Q.persist = bc.persist; Q.mult = bc.mult; Q.ppl = bppl;
        set_grid(b, Q);
        build_segments(b, Q, bc.rows);
        if (e == hipSuccess && (st = upload_segments(b, Q)) != CFUST_OK) e = hipErrorUnknown;
        if (chosen) {
            chosen[Q.m * 3 + 0] = Q.rows;
            chosen[Q.m * 3 + 1] = Q.persist ? Q.mult : 0;
            chosen[Q.m * 3 + 2] = Q.ppl;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    drop_graph(b);
    if (e == hipSuccess) e = launch_fill_i32(b->counters, 4 * b->queues.size(), 0, s);
    return hip_check(h, e, "cfust_batch_tune");
}

cfust_status cfust_init(cfust_handle h, const double *y, cfust_dims d, int32_t nstarts, const int32_t *labels,
                        int32_t nalpha, const double *alpha, double nu0, const cfust_qmc *qmc,
                        const cfust_params_out *best, double *loglik, int32_t *best_index, void *stream) {
    if (!h) return CFUST_EINVAL;
    cfust_status st;
    if ((st = check_dims(h, d)) != CFUST_OK) return st;
    if (d.q > d.p) return fail(h, CFUST_EINVAL, "q = %d > p = %d", d.q, d.p);
    if (d.n < 1 || !y || !labels) return fail(h, CFUST_EINVAL, "y or labels is NULL, or n = 0");
    if (nstarts < 1 || nalpha < 1 || (long)nstarts * nalpha > BATCH_MAX_FITS)
        return fail(h, CFUST_EINVAL, "nstarts * nalpha outside [1, %d]", BATCH_MAX_FITS);
    if (!alpha) return fail(h, CFUST_EINVAL, "alpha is NULL");
    for (int a = 0; a < nalpha; ++a)
        if (!(alpha[a] > 0.0 && alpha[a] < 1.0)) return fail(h, CFUST_EINVAL, "alpha[%d] outside (0, 1)", a);
    if (!(nu0 > 0.0)) return fail(h, CFUST_EINVAL, "nu0 must be positive (+infinity: the normal limit)");
    if (!best || !best->pi || !best->mu || !best->Sigma || !best->Delta || !best->nu)
        return fail(h, CFUST_EINVAL, "an output parameter array is NULL");
    if ((st = check_qmc(h, qmc, d.q >= 2)) != CFUST_OK) return st;
    if ((st = hip_check(h, hipSetDevice(h->device), "hipSetDevice")) != CFUST_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const int C = nstarts * nalpha, g = d.g, p = d.p, q = d.q;
    const int ntiles = (d.n + 63) / 64;
    int nblk = (ntiles + 3) / 4;
    nblk = nblk < 1 ? 1 : (nblk > 256 ? 256 : nblk);
    const int ns0 = 1 + p, ns1 = p * (p + 1) / 2 + p;
    Carve c;
    const size_t o_p0 = c.take<double>((size_t)nstarts * g * nblk * ns0);
    const size_t o_p1 = c.take<double>((size_t)nstarts * g * nblk * ns1);
    const size_t o_cnt = c.take<double>((size_t)nstarts * g);
    const size_t o_mean = c.take<double>((size_t)nstarts * g * p);
    const size_t o_S = c.take<double>((size_t)nstarts * g * p * p);
    const size_t o_m3 = c.take<double>((size_t)nstarts * g * p);
    const size_t o_pi = c.take<double>((size_t)C * g);
    const size_t o_mu = c.take<double>((size_t)C * g * p);
    const size_t o_Sg = c.take<double>((size_t)C * g * p * p);
    const size_t o_Dl = c.take<double>((size_t)C * g * p * q);
    const size_t o_nu = c.take<double>((size_t)C * g);
    const size_t o_vch = c.take<int32_t>((size_t)C * g);
    const size_t o_ll = c.take<double>((size_t)C);
    const size_t o_al = c.take<double>((size_t)nalpha);
    void *ws = nullptr;
    if (hipMalloc(&ws, c.off) != hipSuccess) return fail(h, CFUST_ENOMEM, "initialiser scratch of %zu bytes", c.off);
    auto P = [&](size_t off) { return (double *)((char *)ws + off); };
    InitArgs A;
    A.y = y; A.n = d.n; A.p = p; A.q = q; A.g = g;
    A.nstarts = nstarts; A.nalpha = nalpha; A.labels = labels; A.alpha = P(o_al); A.nu0 = nu0; A.nblk = nblk;
    A.part0 = P(o_p0); A.part1 = P(o_p1); A.cnt = P(o_cnt); A.mean = P(o_mean); A.S = P(o_S); A.m3 = P(o_m3);
    A.pi = P(o_pi); A.mu = P(o_mu); A.Sigma = P(o_Sg); A.Delta = P(o_Dl); A.nu = P(o_nu);
    A.valid_ch = (int32_t *)((char *)ws + o_vch);
    double *llc = P(o_ll);
    // one density-only fit per candidate, on the shared data
    std::vector<cfust_fit> fits(C);
    for (int k = 0; k < C; ++k) {
        cfust_fit &F = fits[k];
        memset(&F, 0, sizeof F);
        F.dims = d;
        F.y = y;
        F.params.pi = A.pi + (size_t)k * g;
        F.params.mu = A.mu + (size_t)k * g * p;
        F.params.Sigma = A.Sigma + (size_t)k * g * p * p;
        F.params.Delta = A.Delta + (size_t)k * g * p * q;
        F.params.nu = A.nu + (size_t)k * g;
        F.out.loglik = llc + k;
    }
    cfust_batch b = nullptr;
    hipError_t e = hipMemcpy((void *)A.alpha, alpha, sizeof(double) * nalpha, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        st = cfust_batch_create(h, C, fits.data(), qmc, &b);
        if (st != CFUST_OK) { (void)hipFree(ws); return st; }
    }
    // statistics, candidates, and their validity as the batch's active mask
    if (e == hipSuccess) e = launch_init_stats(A, s);
    if (e == hipSuccess) e = launch_init_candidates(A, b->active, s);
    if (e == hipSuccess) e = enqueue_estep(b, s);
    if (e == hipSuccess) e = launch_init_select(A, b->active, llc, loglik, best_index, *best, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (b) cfust_batch_destroy(b);
    (void)hipFree(ws);
    return hip_check(h, e, "cfust_init");
}

}  // extern "C"
