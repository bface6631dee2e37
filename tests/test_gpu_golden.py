"""GPU parity at the workloads' own sizes and lattices, against stored FP64
oracle E-steps (tests/golden/, written by make_golden.py from the oracle only):

  * n = 20000, p = q = 4, g = 3 at 4096 x 8 in mixed precision -- the launch
    configuration the bench times (the whole data set in one call), checked on
    32 evenly spaced observations and each component's furthest member;
  * the cytometry-shaped n = 10^6, p = q = 8, g = 5 workload (values mapped to
    [0, 1024]) at 8192 x 8: 38 lattice integrals of dimensions 6, 7, 8 per
    pair, the E-step run on the first 32768 observations plus each
    component's furthest member, checked on the stored rows.

Element-wise bars (mixed precision): |d log f(y_j)| <= 1e-4, |d tau| <= 1e-5,
e-terms within 1e-3 of their natural scale (Sec. 3.1, eqs. 4, 12-17)."""
import json
import os

import numpy as np
import pytest
import torch

from cfust_inputs import make_design, workload
from gpu_common import TOL, compare_estep

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def lib():
    import paper_1606_02054_amd as cf
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    cf.default_handle()
    return cf


class _Gold:
    def __init__(self, path):
        z = np.load(path, allow_pickle=False)
        self.meta = json.loads(str(z["meta"]))
        for k in ("rows", "y", "tau", "logf_obs", "logf_comp", "w", "e1", "e2", "e3", "A", "B"):
            setattr(self, k, z[k])


def _load(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.fail(f"missing golden file {path}: run tests/golden/make_golden.py")
    return _Gold(path)


def _run(cf, y_rows_major, P, des, prec):
    yd = torch.as_tensor(np.ascontiguousarray(y_rows_major.T)).cuda()
    out = cf.cfust_estep(yd, cf.device_params(P), cf.device_qmc(des, prec))
    torch.cuda.synchronize()
    return out


def test_golden_bench_workload_full_n(lib):
    cf = lib
    gd = _load("estep_cfust_n20000_p4_q4_g3_N4096_S8.npz")
    print(f"golden n=20000 p=q=4 g=3 N=4096 S=8, {len(gd.rows)} rows", flush=True)
    ds = workload(gd.meta["workload"])
    assert np.array_equal(ds.y[gd.rows], gd.y), "workload recipe changed since the golden was written"
    des = make_design(gd.meta["N"], gd.meta["S"], seed=gd.meta["design_seed"])
    gpu = _run(cf, ds.y, ds.params, des, cf.CFUST_MIXED)
    dmax = compare_estep(gpu, gd, "mixed", rows=gd.rows, label="n20000 golden")
    np.testing.assert_allclose(gpu.logf_comp.cpu().numpy()[:, gd.rows], gd.logf_comp, rtol=0,
                               atol=TOL["mixed"]["logf"])
    assert int(gpu.status.cpu()[0]) == 0
    np.testing.assert_allclose(gpu.tau.cpu().numpy().sum(0), 1.0, atol=1e-12)
    print(f"  max |dlogf| = {dmax:.2e}", flush=True)


def test_golden_cytometry_workload(lib):
    cf = lib
    gd = _load("estep_cfust_n1e6_p8_q8_g5_box1024_N8192_S8.npz")
    print(f"golden cytometry p=q=8 g=5 N=8192 S=8, {len(gd.rows)} rows", flush=True)
    ds = workload(gd.meta["workload"])
    assert np.array_equal(ds.y[gd.rows], gd.y), "workload recipe changed since the golden was written"
    block = int(gd.meta["block"])
    extra = [int(r) for r in gd.rows if r >= block]
    sel = np.concatenate([np.arange(block), np.array(extra, dtype=np.int64)])
    pos = {int(r): i for i, r in enumerate(sel)}
    cols = np.array([pos[int(r)] for r in gd.rows])
    des = make_design(gd.meta["N"], gd.meta["S"], seed=gd.meta["design_seed"])
    gpu = _run(cf, ds.y[sel], ds.params, des, cf.CFUST_MIXED)
    dmax = compare_estep(gpu, gd, "mixed", rows=cols, label="cytometry golden")
    np.testing.assert_allclose(gpu.logf_comp.cpu().numpy()[:, cols], gd.logf_comp, rtol=0,
                               atol=TOL["mixed"]["logf"])
    assert int(gpu.status.cpu()[0]) == 0
    print(f"  max |dlogf| = {dmax:.2e}", flush=True)
