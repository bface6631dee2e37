"""Write the stored oracle E-step outputs that the full-size parity tests read.

Test infrastructure: this script calls only the FP64 oracle (``oracle/``) and
the seeded input generators (``cfust_inputs/``).  It runs on the CPU, once,
and its outputs are committed next to it:

  estep_cfust_n20000_p4_q4_g3_N4096_S8.npz
      the n = 20000, p = q = 4, g = 3 workload at its own lattice
      (4096 points x 8 shifts, the configuration the bench times);
  estep_cfust_n1e6_p8_q8_g5_box1024_N8192_S8.npz
      the cytometry-shaped n = 10^6, p = q = 8, g = 5 workload (values mapped
      to [0, 1024]) at its own lattice (8192 x 8).

What is stored is the E-step of Sec. 3.1 for the sampled observations: the
posterior memberships tau (eq. 12), log f(y_j) (eq. 4 with eq. 12's mixture),
each component's log density, and the conditional expectations w (eq. 13),
e1 (eq. 15), e2 (eq. 16), e3 (eq. 17, packed upper triangle), plus the two
lattice CDF values A and B of eqs. (4) and (13).

Sampled observations: evenly spaced rows, and for every component h the
member of h (by the generating label) furthest from mu_h in the metric of
Omega_h = Sigma_h + Delta_h Delta_h^T -- the far tail of each component, where
the lattice probabilities are smallest.  For the large workload the evenly
spaced rows lie in the first 32768 observations, so a GPU test can run the
E-step on that block plus the tail rows.

Usage: python tests/golden/make_golden.py [small|large|all] [--threads T]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from cfust_inputs import make_design, workload  # noqa: E402

SPECS = {
    "small": dict(workload="cfust_n20000_p4_q4_g3", N=4096, S=8, design_seed=1606, n_even=32, block=20000),
    "large": dict(workload="cfust_n1e6_p8_q8_g5_box1024", N=8192, S=8, design_seed=1606, n_even=6, block=32768),
}


def golden_path(key: str) -> str:
    s = SPECS[key]
    return os.path.join(HERE, f"estep_{s['workload']}_N{s['N']}_S{s['S']}.npz")


def tail_rows(ds) -> list[int]:
    """Per component, the generating member furthest from mu_h in the Omega_h metric."""
    P = ds.params
    out = []
    for h in range(P.g):
        members = np.flatnonzero(ds.labels == h)
        Om = P.Sigma[h] + P.Delta[h] @ P.Delta[h].T
        Lc = np.linalg.cholesky(Om)
        r = np.linalg.solve(Lc, (ds.y[members] - P.mu[h]).T)
        out.append(int(members[np.argmax((r * r).sum(0))]))
    return out


def sample_rows(key: str, ds) -> np.ndarray:
    s = SPECS[key]
    even = np.linspace(0, s["block"] - 1, s["n_even"]).astype(np.int64)
    rows = list(even) + [r for r in tail_rows(ds) if r not in set(even)]
    return np.array(rows, dtype=np.int64)


def make(key: str) -> str:
    s = SPECS[key]
    ds = workload(s["workload"])
    des = make_design(s["N"], s["S"], seed=s["design_seed"])
    rows = sample_rows(key, ds)
    t0 = time.time()
    o = oracle.estep(ds.y, ds.params, des, rows=rows.astype(np.int32))
    dt = time.time() - t0
    meta = dict(workload=s["workload"], workload_seed=1606, N=s["N"], S=s["S"], design_seed=s["design_seed"],
                block=s["block"], n_even=s["n_even"], oracle_threads=oracle.get_threads(), oracle_seconds=dt,
                note="FP64 oracle E-step (Sec. 3.1, eqs. 4, 12-17) on the sampled rows; same lattice and shifts "
                     "as the GPU path")
    path = golden_path(key)
    np.savez_compressed(path, rows=rows, y=ds.y[rows], tau=o.tau, logf_obs=o.logf_obs, logf_comp=o.logf_comp,
                        w=o.w, e1=o.e1, e2=o.e2, e3=o.e3, A=o.A, B=o.B, meta=json.dumps(meta))
    print(f"{path}: {len(rows)} rows, oracle {dt:.1f} s", flush=True)
    return path


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", nargs="?", default="all", choices=["small", "large", "all"])
    ap.add_argument("--threads", type=int, default=0)
    a = ap.parse_args()
    if a.threads > 0:
        oracle.set_threads(a.threads)
    for key in (["small", "large"] if a.which == "all" else [a.which]):
        make(key)


if __name__ == "__main__":
    main()
