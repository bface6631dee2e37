"""End to end on the small configuration (n = 1000, p = q = 2, g = 2, lattice
1024 x 4, FP64): starting values by Algorithm 1 from k-means partitions,
then 20 EM iterations on the GPU, checked along the way against the oracle:

  * every iteration, the oracle's M-step (eqs. 18-22) applied to the GPU's
    E-step output and parameters equals the GPU's M-step;
  * at iterations 1, 10 and 20, the oracle's E-step at the GPU's parameters
    equals the GPU's E-step on a sample of rows (the full oracle E-step of
    this workload takes tens of seconds per iteration);
  * the log-likelihood does not decrease (fixed lattice, FP64);
  * the batched, graph-captured fit reproduces the same trace bit for bit.
"""
import numpy as np
import pytest
import torch

from cfust_inputs import Params, kmeans_partitions, make_design, workload
from gpu_common import compare_estep

pytestmark = pytest.mark.gpu
ITERS = 20


@pytest.fixture(scope="module")
def cf():
    import paper_1606_02054_amd as cf
    assert torch.cuda.is_available()
    cf.default_handle()
    return cf


def _host_params(dp):
    pi, mu, Sg, Dl, nu = dp.to_host()
    return Params(pi, mu, Sg, Dl, nu)


def _host_estep(es):
    from types import SimpleNamespace
    c = lambda t: t.cpu().numpy().astype(np.float64)
    return SimpleNamespace(tau=c(es.tau), logf_obs=c(es.logf_obs), w=c(es.w), e1=c(es.e1), e2=c(es.e2),
                           e3=c(es.e3))


def test_small_config_init_and_em(cf, orc):
    ds = workload("cfust_n1000_p2_q2_g2")
    n, p = ds.y.shape
    g, q = ds.params.g, ds.params.q
    des = make_design(ds.meta["N"], ds.meta["S"], seed=1606)
    qmc = cf.device_qmc(des, cf.CFUST_FP64)
    y = torch.as_tensor(ds.y_soa).cuda()
    labels = torch.as_tensor(kmeans_partitions(ds.y, g, 4, seed=7)).cuda()
    start, ll0, k = cf.initialise(y, g, q, labels, qmc)
    torch.cuda.synchronize()
    assert k >= 0 and np.isfinite(ll0.cpu().numpy().ravel()[k])
    print(f"start: candidate {k}, loglik {ll0.cpu().numpy().ravel()[k]:.4f}", flush=True)

    dp = start.clone()
    sample = np.arange(0, n, 25)
    trace = []
    for it in range(ITERS):
        es = cf.cfust_estep(y, dp, qmc)
        torch.cuda.synchronize()
        trace.append(float(es.loglik.cpu()[0]))
        cur = _host_params(dp)
        if it in (0, 9, ITERS - 1):
            ora = orc.estep(ds.y, cur, des, rows=sample)
            compare_estep(es, ora, "fp64", rows=sample, label=f"iteration {it + 1}")
        nxt = cf.cfust_mstep(y, es, dp)
        torch.cuda.synchronize()
        ref, _ = orc.mstep(ds.y, _host_estep(es), cur)
        got = nxt.to_host()
        for a, b, name in zip(got, (ref.pi, ref.mu, ref.Sigma, ref.Delta, ref.nu), ("pi", "mu", "Sigma", "Delta", "nu")):
            assert np.abs(a - b).max() <= 1e-9 * max(1.0, np.abs(b).max()), (it, name, np.abs(a - b).max())
        dp = nxt
    trace = np.array(trace)
    print("trace", np.round(trace, 4), flush=True)
    assert np.all(np.diff(trace) >= -1e-6 * n), np.diff(trace).min()
    assert trace[-1] > trace[0]

    # the batched, graph-captured fit from the same start reproduces the trace
    es_b = cf.alloc_estep(n, p, q, g, cf.CFUST_FP64, stderr=False)
    B = cf.Batch([(y, start.clone(), es_b)], qmc)
    tb, done = B.fit(ITERS, tol=0.0, use_graph=True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(tb.cpu().numpy()[:, 0], trace)
    assert int(done.cpu()[0]) == ITERS
    B.close()
