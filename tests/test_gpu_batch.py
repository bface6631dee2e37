"""GPU tests of batched fits (include/cfust.h, "Batches of independent fits").

Every fit of a batch must get, bit for bit, what cfust_estep / cfust_mstep
give on that fit alone (the batch runs the same per-item arithmetic; only the
scheduling differs).  The graph-captured EM iteration must equal the eager
launches and the plain sequential loop over several replays, and the fits the
device retires must be those that the oracle's Aitken rule (Sec. 3.4) retires
on the recorded log-likelihoods.  The shapes mix q = 1..8 (closed forms and
every lattice dimension), ragged n (partial tiles), an empty fit and a
component far from its data (FP32 underflow, FP64 redo list)."""
import numpy as np
import pytest
import torch

import oracle
from cfust_inputs import make_design, workload
from cfust_inputs.synth import Params, draw_params, sample_hierarchy

pytestmark = pytest.mark.gpu

FIELDS = ("tau", "logf_obs", "loglik", "w", "e1", "e2", "e3", "logf_comp", "cdf_stderr", "status")


@pytest.fixture(scope="module")
def cf():
    import paper_1606_02054_amd as cf
    assert torch.cuda.is_available()
    cf.default_handle()
    return cf


def _far_params(rng, p, q, g):
    """Component 1 sits 300 units from the data with a strong skew away from
    it: with q = 8 the SOV factors after the first multiply to about e^-110,
    below what FP32 holds, so its lattice items go to the FP64 redo list."""
    P = draw_params(rng, p, q, g, sigma="aat", nu_range=(4.0, 8.0))
    P.mu[1] = P.mu[0] + 300.0
    P.Delta[1] = np.abs(P.Delta[1]) + 100.0
    return P


def small_specs(seed=11):
    rng = np.random.default_rng(seed)
    shapes = [(0, 2, 2, 2), (1, 3, 1, 1), (37, 2, 2, 2), (130, 3, 3, 3), (257, 4, 4, 2),
              (300, 5, 5, 3), (64, 6, 2, 4), (515, 3, 3, 2), (45, 8, 8, 2)]
    out = []
    for (n, p, q, g) in shapes:
        P = draw_params(rng, p, q, g, sigma="aat", nu_range=(4.0, 8.0))
        y = sample_hierarchy(rng, P, n)[0] if n > 0 else np.zeros((0, p))
        out.append((y, P))
    P = _far_params(rng, 8, 8, 2)
    y = sample_hierarchy(rng, Params(np.array([1.0, 0.0]), P.mu, P.Sigma, P.Delta, P.nu), 30)[0]
    out.append((y, P))
    return out


def _to_dev(cf, specs, precision):
    fits = []
    for (y, P) in specs:
        yt = torch.tensor(np.ascontiguousarray(y.T), dtype=torch.float64).cuda()
        dp = cf.device_params(P)
        es = cf.alloc_estep(y.shape[0], P.mu.shape[1], P.Delta.shape[2], P.pi.shape[0], precision)
        fits.append((yt, dp, es))
    return fits


def _assert_same_estep(a, b, where):
    for f in FIELDS:
        ta, tb = getattr(a, f), getattr(b, f)
        assert torch.equal(ta, tb), (where, f)


def _assert_same_params(a, b, where):
    for f in ("pi", "mu", "Sigma", "Delta", "nu"):
        assert torch.equal(getattr(a, f), getattr(b, f)), (where, f)


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_estep_mstep_equal_single(cf, precision):
    print(f"batch vs single, precision {precision}", flush=True)
    specs = small_specs()
    qmc = cf.device_qmc(make_design(256, 4, seed=5), precision)
    fb = _to_dev(cf, specs, precision)
    fs = _to_dev(cf, specs, precision)
    B = cf.Batch(fb, qmc)
    B.estep()
    for k, (y, P, es) in enumerate(fs):
        cf.cfust_estep(y, P, qmc, out=es)
    torch.cuda.synchronize()
    for k in range(len(specs)):
        _assert_same_estep(fb[k][2], fs[k][2], k)
    B.mstep()
    for k, (y, P, es) in enumerate(fs):
        cf.cfust_mstep(y, es, P, out=P, status=es.status)
    torch.cuda.synchronize()
    for k in range(len(specs)):
        _assert_same_params(fb[k][1], fs[k][1], k)
        assert torch.equal(fb[k][2].status, fs[k][2].status), k
    B.close()


def test_batch_far_component_matches_oracle(cf):
    """Mixed precision on the fit with a far component: the FP64 redo of the
    underflowed FP32 items must land (compare with the oracle)."""
    print("batch far component vs oracle", flush=True)
    specs = small_specs()
    y, P = specs[-1]
    des = make_design(256, 4, seed=5)
    qmc = cf.device_qmc(des, cf.CFUST_MIXED)
    fb = _to_dev(cf, [(y, P)], cf.CFUST_MIXED)
    B = cf.Batch(fb, qmc)
    B.estep()
    torch.cuda.synchronize()
    rows = np.array([0, 10, 20, 29])
    ora = oracle.estep(y, P, des, rows=rows)
    got = fb[0][2].logf_comp.cpu().numpy()[:, rows]
    assert np.all(np.isfinite(got))
    assert np.all(got[1] < -100.0)          # the far component is far
    np.testing.assert_allclose(got, ora.logf_comp, rtol=1e-4, atol=1e-4)
    B.close()


def _reset(fits, specs, cf):
    for (yt, dp, es), (y, P) in zip(fits, specs):
        src = cf.device_params(P)
        for f in ("pi", "mu", "Sigma", "Delta", "nu"):
            getattr(dp, f).copy_(getattr(src, f))
        es.status.zero_()


def test_fit_batch_graph_equals_eager_and_sequential(cf):
    print("fit_batch graph / eager / sequential", flush=True)
    # fits whose log-likelihood keeps changing (an all-frozen fit would stop
    # on an unchanged value even at tol = 0)
    specs = small_specs()[2:-1]
    prec = cf.CFUST_MIXED
    qmc = cf.device_qmc(make_design(256, 4, seed=5), prec)
    iters = 3
    # sequential reference
    fs = _to_dev(cf, specs, prec)
    seq_trace = np.zeros((iters, len(specs)))
    for k, (y, P, es) in enumerate(fs):
        for it in range(iters):
            cf.cfust_estep(y, P, qmc, out=es)
            seq_trace[it, k] = float(es.loglik.cpu()[0])
            cf.cfust_mstep(y, es, P, out=P, status=es.status)
    torch.cuda.synchronize()
    fb = _to_dev(cf, specs, prec)
    B = cf.Batch(fb, qmc)
    for mode in ("graph", "graph again", "eager"):
        _reset(fb, specs, cf)
        torch.cuda.synchronize()
        trace, done = B.fit(iters, tol=0.0, use_graph=mode != "eager")
        torch.cuda.synchronize()
        assert np.array_equal(trace.cpu().numpy(), seq_trace), mode
        assert np.all(done.cpu().numpy() == iters), mode
        for k in range(len(specs)):
            _assert_same_params(fb[k][1], fs[k][1], (mode, k))
            _assert_same_estep(fb[k][2], fs[k][2], (mode, k))
    B.close()


def test_fit_batch_aitken_retirement(cf):
    print("fit_batch Aitken retirement", flush=True)
    specs = small_specs()[1:-1]
    prec = cf.CFUST_FP64
    qmc = cf.device_qmc(make_design(128, 4, seed=7), prec)
    iters, tol = 10, 0.5
    fb = _to_dev(cf, specs, prec)
    B = cf.Batch(fb, qmc)
    trace, done = B.fit(iters, tol=tol, use_graph=True)
    torch.cuda.synchronize()
    tr, dn = trace.cpu().numpy(), done.cpu().numpy()
    assert dn.min() < iters, "no fit retired: the test would not exercise retirement"
    fs = _to_dev(cf, specs, prec)
    for k, (y, P, es) in enumerate(fs):
        expect = oracle.aitken_iterations(tr[:, k], tol)
        assert dn[k] == expect, (k, dn[k], expect, tr[:, k])
        assert np.all(np.isnan(tr[dn[k]:, k]))
        # the same fit run alone: dn[k] E-steps, each followed by an M-step
        # unless the rule stops the fit right there
        hist = []
        for it in range(dn[k]):
            cf.cfust_estep(y, P, qmc, out=es)
            hist.append(float(es.loglik.cpu()[0]))
            stops_here = oracle.aitken_iterations(hist + [float("nan")], tol) == len(hist)
            if not stops_here:
                cf.cfust_mstep(y, es, P, out=P, status=es.status)
        assert np.array_equal(np.array(hist), tr[:dn[k], k]), k
        torch.cuda.synchronize()
        _assert_same_params(fb[k][1], P, k)
    B.close()


def test_batch_tune_keeps_results(cf):
    print("batch tune", flush=True)
    specs = small_specs()
    prec = cf.CFUST_MIXED
    qmc = cf.device_qmc(make_design(1024, 4, seed=5), prec)
    fb = _to_dev(cf, specs, prec)
    fs = _to_dev(cf, specs, prec)
    B = cf.Batch(fb, qmc)
    chosen = B.tune()
    print("tuned", chosen, flush=True)
    assert set(chosen) == {2, 3, 4, 5, 6, 7, 8}
    for m, (rows, mult, ppl) in chosen.items():
        assert rows in (4, 8, 16) and mult in (0, 1, 2) and ppl in (1, 2)
        assert mult > 0 or rows == 4
    B.estep()
    for (y, P, es) in fs:
        cf.cfust_estep(y, P, qmc, out=es)
    torch.cuda.synchronize()
    for k in range(len(specs)):
        _assert_same_estep(fb[k][2], fs[k][2], k)
    B.close()


def test_batched_workload_scaled(cf, orc):
    """The 64-fit restart workload (p = q in 3..8, g in 2..6) at reduced n:
    every fit equals its single-fit E-step; sampled rows of the q = 8 fits
    match the oracle."""
    print("batched workload, 64 fits, n in [300, 3000]", flush=True)
    sets = workload("batched_fit", nfits=64, n_lo=300, n_hi=3000)
    des = make_design(1024, 4, seed=1606)
    prec = cf.CFUST_MIXED
    qmc = cf.device_qmc(des, prec)
    specs = [(ds.y, ds.params) for ds in sets]
    fb = _to_dev(cf, specs, prec)
    fs = _to_dev(cf, specs, prec)
    B = cf.Batch(fb, qmc)
    B.estep()
    for (y, P, es) in fs:
        cf.cfust_estep(y, P, qmc, out=es)
    torch.cuda.synchronize()
    for k in range(len(specs)):
        _assert_same_estep(fb[k][2], fs[k][2], k)
    q8 = [k for k, (y, P) in enumerate(specs) if P.Delta.shape[2] == 8][:2]
    assert q8
    for k in q8:
        y, P = specs[k]
        rows = np.array([0, y.shape[0] // 2, y.shape[0] - 1])
        ora = orc.estep(y, P, des, rows=rows)
        es = fb[k][2]
        got_lf = es.logf_comp.cpu().numpy()[:, rows]
        np.testing.assert_allclose(got_lf, ora.logf_comp, rtol=1e-4, atol=1e-4)
        np.testing.assert_allclose(es.tau.cpu().numpy()[:, rows], ora.tau, atol=1e-5)
    B.close()
