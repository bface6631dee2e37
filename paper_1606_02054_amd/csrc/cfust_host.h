// cfust_host.h -- host-side state of a handle and the argument checks shared
// by the entry points (private).
#pragma once
#include <stdarg.h>
#include <stdio.h>

#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "cfust_kernels.h"

struct ProfRec {
    int m;
    hipEvent_t e0, e1;
};

struct cfust_ctx {
    int device = 0;
    int ncu = 0;                     // compute units of the device
    std::string err;
    void *ws = nullptr;
    size_t ws_size = 0;
    bool prof = false;
    std::vector<ProfRec> rec;        // recorded (pending) event pairs
    std::vector<hipEvent_t> pool;    // free events
    std::string arch;                // gcnArchName of the device
    // autotuner cache: (m, N, S, precision) -> lattice points per lane
    std::map<std::tuple<int, int, int, int>, int> tuned;
    // device address of this device's fixed workspace array (allocation-free
    // E-step), or null when its lookup failed (scratch_err holds the HIP error)
    void *scratch = nullptr;
    int scratch_err = 0;
};

namespace cfust_host {

using namespace cfust;

inline cfust_status fail(cfust_handle h, cfust_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (h) h->err = buf;
    return st;
}

inline cfust_status hip_check(cfust_handle h, hipError_t e, const char *what) {
    if (e == hipSuccess) return CFUST_OK;
    return fail(h, CFUST_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Bump allocator over a workspace.
struct Carve {
    size_t off = 0;
    template <class T> size_t take(size_t count) {
        const size_t o = off;
        off = align256(off + count * sizeof(T));
        return o;
    }
};

inline cfust_status ensure_ws(cfust_handle h, size_t bytes) {
    if (bytes <= h->ws_size) return CFUST_OK;
    if (h->ws) {
        hipError_t e = hipFree(h->ws);   // synchronises the device
        h->ws = nullptr;
        h->ws_size = 0;
        if (e != hipSuccess) return hip_check(h, e, "hipFree(workspace)");
    }
    const size_t sz = align256(bytes + bytes / 4);
    if (hipMalloc(&h->ws, sz) != hipSuccess) {
        h->ws = nullptr;
        return fail(h, CFUST_ENOMEM, "workspace allocation of %zu bytes failed", sz);
    }
    h->ws_size = sz;
    return CFUST_OK;
}

template <class T> T *at(cfust_handle h, size_t off) { return (T *)((char *)h->ws + off); }

inline cfust_status check_dims(cfust_handle h, const cfust_dims &d) {
    if (d.n < 0) return fail(h, CFUST_EINVAL, "n = %d < 0", d.n);
    if (d.p < 1 || d.p > MAXP) return fail(h, CFUST_EINVAL, "p = %d outside [1, %d]", d.p, MAXP);
    if (d.q < 1 || d.q > MAXQ) return fail(h, CFUST_EINVAL, "q = %d outside [1, %d]", d.q, MAXQ);
    if (d.g < 1 || d.g > MAXG) return fail(h, CFUST_EINVAL, "g = %d outside [1, %d]", d.g, MAXG);
    return CFUST_OK;
}

inline int ilog2_exact(int N) {
    if (N <= 0 || (N & (N - 1))) return -1;
    int k = 0;
    while ((1 << k) < N) ++k;
    return k;
}

// Lattice coordinates the FP32 integrand reads from a table, for integrals of
// dimension up to q: coordinates 0 .. q-2 (the largest integral has q - 1
// lattice coordinates), when the lattice allows it (mixed precision, N a
// power of two >= 64) and the table stays within COORDS_MAX_BYTES; else 0
// (the integrand forms the coordinates itself).
constexpr size_t COORDS_MAX_BYTES = (size_t)16 << 20;
inline int lattice_coord_count(int q, const cfust_qmc *Q) {
    if (!Q || Q->precision != CFUST_MIXED || q < 2) return 0;
    if (ilog2_exact(Q->N) < 6) return 0;
    const int C = q - 1;
    if (lattice_coords_floats(Q->N, Q->S, C) * sizeof(float) > COORDS_MAX_BYTES) return 0;
    return C;
}

inline cfust_status check_qmc(cfust_handle h, const cfust_qmc *Q, bool lattice_needed) {
    if (!Q) return fail(h, CFUST_EINVAL, "qmc is NULL");
    if (Q->precision != CFUST_FP64 && Q->precision != CFUST_MIXED)
        return fail(h, CFUST_EINVAL, "precision %d is neither CFUST_FP64 nor CFUST_MIXED", Q->precision);
    if (!lattice_needed) return CFUST_OK;
    if (Q->N < 2 || Q->N > 65536) return fail(h, CFUST_EINVAL, "lattice size N = %d outside [2, 65536]", Q->N);
    if (Q->S < 1 || Q->S > MAXS) return fail(h, CFUST_EINVAL, "shift count S = %d outside [1, %d]", Q->S, MAXS);
    if (!Q->z || !Q->shifts) return fail(h, CFUST_EINVAL, "lattice vector or shifts are NULL");
    if (Q->precision == CFUST_MIXED && ilog2_exact(Q->N) < 0)
        return fail(h, CFUST_EINVAL, "mixed precision needs N a power of two (N = %d)", Q->N);
    return CFUST_OK;
}

inline LatticeArgs lattice_of(const cfust_qmc *Q) {
    LatticeArgs L;
    L.N = Q->N;
    L.S = Q->S;
    L.log2N = ilog2_exact(Q->N);
    L.z = Q->z;
    L.shifts = Q->shifts;
    return L;
}

inline cfust_status check_params(cfust_handle h, const cfust_params *P) {
    if (!P || !P->pi || !P->mu || !P->Sigma || !P->Delta || !P->nu)
        return fail(h, CFUST_EINVAL, "a parameter array is NULL");
    return CFUST_OK;
}

// Blocks per component of the M-step reduction: about three resident blocks
// per compute unit over the g components (a grid-stride loop over the tiles
// balances them), never more than one per tile.  Few blocks keep the block
// partials, which the solve sums per statistic, short.
inline int mstep_nblk(const cfust_dims &d, int ncu) {
    const int ntiles = (d.n + 63) / 64;
    const int want = (3 * (ncu > 0 ? ncu : 256) + d.g - 1) / (d.g > 0 ? d.g : 1);
    int nb = ntiles < want ? ntiles : want;
    if (nb < 1) nb = 1;
    if (nb > 1024) nb = 1024;
    // a multiple of 8: blocks go to the 8 XCDs in turn, so the g blocks that
    // walk the same tiles of y (same x, one per component) share an XCD and
    // its L2, which then serves y to all but the first of them
    if (nb >= 8) nb -= nb % 8;
    return nb;
}

inline size_t mstep_bytes(const cfust_dims &d, int ncu) {
    return align256((size_t)d.g * mstep_nblk(d, ncu) * nstat(d.p, d.q) * sizeof(double) + (size_t)d.g * sizeof(int32_t));
}

// Lattice points per lane chosen by the autotuner for (m, N, S, precision).
inline int tuned_ppl(cfust_handle h, int m, const LatticeArgs &L, bool mixed) {
    auto it = h->tuned.find(std::make_tuple(m, L.N, L.S, mixed ? 1 : 0));
    if (it != h->tuned.end()) return it->second;
    return 1;
}

// An event from the handle's pool (created when the pool is empty).
inline hipEvent_t pool_event(cfust_handle h) {
    if (!h->pool.empty()) {
        hipEvent_t e = h->pool.back();
        h->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

}  // namespace cfust_host
