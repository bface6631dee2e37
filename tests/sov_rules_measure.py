"""Measurement of two alternatives to the library's lattice estimates (test
infrastructure: it calls only the oracle and the seeded input generators).

1. Chi-radial SOV rule (oracle/chiradial.py) against the library's t-SOV rule
   (the oracle's or_mvt): for m = 2..8, NPROB seeded problems T_m(b; 0, R, nu)
   per m (limits U[-1.5, 2.5], correlations of Wishart unit-diagonal matrices,
   dof U[5, 25] -- the dofs nu + p of the E-step integrals), each rule at
   lattice sizes N = 1024, 4096, 16384 with 8 shifts; error = |estimate -
   reference| / reference with the reference the t rule at N = 65536 x 8.
2. Direct SOV moment estimator (oracle.mvt_moments: lattice means of f, f z,
   f z z^T) against the gradient-identity route (oracle.tmoments: the
   T_{m-1}, T_{m-2} integrals) for the truncated t moments of dimension 8:
   NPROB problems, error of the second-moment matrix (max entry, relative to
   its largest entry) against the identity route at 16384 x 8.

Prints one JSON document (medians per m and N, fitted slopes of log error
against log N).  Usage: python tests/sov_rules_measure.py [--procs P] [--nprob K]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

NS = (1024, 4096, 16384)
S = 8
REF_N = 65536


def problem(m: int, k: int):
    from cfust_inputs import random_spd
    rng = np.random.default_rng(9000 + 100 * m + k)
    R = random_spd(rng, m, df=max(6, m + 2))
    b = rng.uniform(-1.5, 2.5, m)
    nu = rng.uniform(5.0, 25.0)
    return b, np.linalg.cholesky(R), nu


def chiradial_case(args):
    m, k = args
    import oracle
    from oracle.chiradial import mvt_chiradial
    from cfust_inputs import make_design
    oracle.set_threads(1)
    b, L, nu = problem(m, k)
    ref, ref_se = oracle.mvt(b, L, nu, make_design(REF_N, S, seed=77))
    out = {"m": m, "k": k, "ref": ref, "ref_se": ref_se, "t": {}, "chi": {}}
    for N in NS:
        d = make_design(N, S, seed=1606)
        et, st = oracle.mvt(b, L, nu, d)
        ec, sc = mvt_chiradial(b, L, nu, d)
        out["t"][N] = (abs(et - ref) / ref, st / ref)
        out["chi"][N] = (abs(ec - ref) / ref, sc / ref)
    return out


def moments_case(k):
    import oracle
    from cfust_inputs import make_design
    oracle.set_threads(1)
    m = 8
    b, L, nu = problem(m, 50 + k)
    R = L @ L.T
    _, _, ref, _ = oracle.tmoments(b, R, nu, make_design(16384, S, seed=78))
    scale = np.abs(ref).max()
    out = {"k": k, "identity": {}, "direct": {}}
    for N in (1024, 4096):
        _, _, m2, _ = oracle.tmoments(b, R, nu, make_design(N, S, seed=1606))
        out["identity"][N] = float(np.abs(m2 - ref).max() / scale)
    for N in (1024, 4096, 16384):
        _, _, M2 = oracle.mvt_moments(b, L, nu, make_design(N, S, seed=1606))
        out["direct"][N] = float(np.abs(M2 - ref).max() / scale)
    return out


def slope(ns, errs):
    x, y = np.log(np.asarray(ns, float)), np.log(np.maximum(np.asarray(errs, float), 1e-300))
    return float(np.polyfit(x, y, 1)[0])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=7)
    ap.add_argument("--nprob", type=int, default=20)
    ap.add_argument("--skip-moments", action="store_true")
    a = ap.parse_args()
    cases = [(m, k) for m in range(2, 9) for k in range(a.nprob)]
    with Pool(a.procs) as pool:
        res = pool.map(chiradial_case, cases, chunksize=1)
        mom = [] if a.skip_moments else pool.map(moments_case, range(a.nprob), chunksize=1)
    summary = {"lattice_sizes": NS, "shifts": S, "reference_N": REF_N, "problems_per_m": a.nprob, "chiradial": {}}
    for m in range(2, 9):
        rs = [r for r in res if r["m"] == m]
        row = {}
        for rule in ("t", "chi"):
            med_err = [float(np.median([r[rule][N][0] for r in rs])) for N in NS]
            med_se = [float(np.median([r[rule][N][1] for r in rs])) for N in NS]
            row[rule] = {"median_rel_err": med_err, "median_rel_stderr": med_se,
                         "slope_err": slope(NS, med_err), "slope_stderr": slope(NS, med_se)}
        row["median_err_ratio_chi_over_t"] = [
            float(np.median([r["chi"][N][0] / max(r["t"][N][0], 1e-300) for r in rs])) for N in NS]
        row["median_stderr_ratio_chi_over_t"] = [
            float(np.median([r["chi"][N][1] / max(r["t"][N][1], 1e-300) for r in rs])) for N in NS]
        row["median_ref_rel_stderr"] = float(np.median([r["ref_se"] / r["ref"] for r in rs]))
        summary["chiradial"][m] = row
    if mom:
        summary["direct_moments_m8"] = {
            "identity_median_rel_err": {N: float(np.median([r["identity"][N] for r in mom])) for N in (1024, 4096)},
            "direct_median_rel_err": {N: float(np.median([r["direct"][N] for r in mom])) for N in (1024, 4096, 16384)},
            "problems": len(mom)}
    print(json.dumps(summary, indent=1))


if __name__ == "__main__":
    main()
