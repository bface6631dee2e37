"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on
the same seeded inputs and the same lattice (Secs. 2-3 of the paper; eq. 4,
eqs. 12-17, 18-22, 27)."""
import numpy as np
import pytest
import torch

from cfust_inputs import draw_mvt_problems, draw_params, make_design, sample_hierarchy, workload
from gpu_common import TOL, compare_estep, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import paper_1606_02054_amd as cf
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    cf.default_handle()
    return cf


def _mode(cf, mode):
    return cf.CFUST_MIXED if mode == "mixed" else cf.CFUST_FP64


def _gpu_estep(cf, y, P, design, mode):
    yd = torch.as_tensor(np.ascontiguousarray(y.T)).cuda()
    out = cf.cfust_estep(yd, cf.device_params(P), cf.device_qmc(design, _mode(cf, mode)))
    torch.cuda.synchronize()
    return out


# ---------------------------------------------------------------- mvt batch --

@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 8])
@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_mvt_batch_vs_oracle(lib, orc, m, mode):
    cf = lib
    print(f"mvt m={m} mode={mode}", flush=True)
    rng = np.random.default_rng(500 + m)
    batch = 37                                    # ragged: not a multiple of 4 waves
    b, L, idx, nu = draw_mvt_problems(rng, m, batch, nmat=3, lim=(-2.5, 2.5), dof=(2.0, 30.0))
    des = make_design(256, 4, seed=77)
    p, logp, se = cf.mvt_cdf_batch(torch.as_tensor(b).cuda(), torch.as_tensor(L).cuda(),
                                   torch.as_tensor(idx).cuda(), torch.as_tensor(nu).cuda(),
                                   cf.device_qmc(des, _mode(cf, mode)))
    p, logp = p.cpu().numpy(), logp.cpu().numpy()
    ref = np.array([orc.mvt(b[i], L[idx[i]], nu[i], des)[0] for i in range(batch)])
    tol = 1e-10 if mode == "fp64" else 5e-5
    assert np.all(rel_err(p, ref, 1e-300) <= tol), rel_err(p, ref, 1e-300).max()
    assert np.all(np.abs(logp - np.log(ref)) <= tol * 2)


def test_mvt_batch_far_tail_uses_log(lib, orc):
    cf = lib
    des = make_design(256, 4, seed=78)
    m = 3
    L = np.linalg.cholesky(0.5 * np.eye(m) + 0.5)[None]
    b = np.array([[-40.0, -1.0, 0.5], [-9.0, -9.0, -9.0]])
    nu = np.array([3.0, 6.0])
    idx = np.zeros(2, dtype=np.int32)
    for mode in ("fp64", "mixed"):
        p, logp, se = cf.mvt_cdf_batch(torch.as_tensor(b).cuda(), torch.as_tensor(L).cuda(),
                                       torch.as_tensor(idx).cuda(), torch.as_tensor(nu).cuda(),
                                       cf.device_qmc(des, _mode(cf, mode)))
        ref = np.array([orc.mvt(b[i], L[0], nu[i], des)[0] for i in range(2)])
        np.testing.assert_allclose(logp.cpu().numpy(), np.log(ref), rtol=0, atol=1e-9 if mode == "fp64" else 1e-4)


# ------------------------------------------------------------------- E-step --

CASES = [  # (p, q, g, n, seed)
    (2, 2, 2, 203, 1),
    (3, 2, 2, 65, 2),
    (2, 1, 3, 50, 3),
    (3, 3, 2, 41, 4),
    (4, 4, 3, 23, 5),
    (5, 5, 2, 9, 6),
]


@pytest.mark.parametrize("p,q,g,n,seed", CASES)
@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_estep_vs_oracle(lib, orc, p, q, g, n, seed, mode):
    cf = lib
    print(f"estep p={p} q={q} g={g} n={n} mode={mode}", flush=True)
    rng = np.random.default_rng(seed)
    P = draw_params(rng, p, q, g, sigma="wishart" if p > 2 else "aat")
    y, _ = sample_hierarchy(rng, P, n)
    des = make_design(256, 4, seed=90 + seed)
    ora = orc.estep(y, P, des)
    gpu = _gpu_estep(cf, y, P, des, mode)
    compare_estep(gpu, ora, mode, label=f"p{p}q{q}g{g}")
    ll = float(gpu.loglik.cpu()[0])
    assert abs(ll - ora.loglik) <= TOL[mode]["logf"] * n
    np.testing.assert_allclose(gpu.logf_comp.cpu().numpy(), ora.logf_comp, atol=TOL[mode]["logf"])
    assert int(gpu.status.cpu()[0]) == 0


@pytest.mark.parametrize("p,q", [(2, 2), (4, 4)])
def test_fp64_tables_track_exact_transforms(lib, orc, p, q):
    """FP64 mode draws its univariate t probabilities and quantiles from FP64
    Chebyshev tables of each dof; the oracle uses the continued fraction and
    a root search.  On the same lattice the two agree far inside the FP64
    tolerance: dofs from 1.05 to 150 (integral dofs up to 150 + p + q + 1),
    and observations far in the tails (log-densities of several hundred)."""
    cf = lib
    print(f"fp64 tables vs exact transforms p={p} q={q}", flush=True)
    rng = np.random.default_rng(4200 + p)
    P = draw_params(rng, p, q, 2, sigma="wishart" if p > 2 else "aat")
    P.nu[:] = [1.05, 150.0]
    y, _ = sample_hierarchy(rng, P, 30)
    y[-1] = P.mu[0] + 40.0
    y[-2] = P.mu[1] - 25.0
    des = make_design(256, 4, seed=4300 + p)
    ora = orc.estep(y, P, des)
    gpu = _gpu_estep(cf, y, P, des, "fp64")
    lf = gpu.logf_comp.cpu().numpy()
    assert lf.min() < -100.0
    np.testing.assert_allclose(lf, ora.logf_comp, rtol=0, atol=1e-10)
    compare_estep(gpu, ora, "fp64", label=f"tables p{p}", tol=dict(logf=1e-10, tau=1e-12, eterm=1e-10))


def test_fp64_dof_past_tables_uses_exact_transforms(lib, orc):
    """A component with dof 3000: its integrals use dofs past the range the
    FP64 tables serve, so they are flagged and evaluated with the exact
    transforms (single fit: the flagged pass; batch: the redo list).  Both
    match the oracle far inside the FP64 tolerance (e-terms to 1e-9: at dof
    3000 the exact transforms of the two implementations differ by ~3e-10
    in the second moments, which are differences of nearly equal terms),
    and the batch gives the single fit's bits."""
    cf = lib
    print("fp64, dof past the tables", flush=True)
    rng = np.random.default_rng(4400)
    P = draw_params(rng, 3, 3, 2, sigma="wishart")
    P.nu[:] = [6.0, 3000.0]
    y, _ = sample_hierarchy(rng, P, 25)
    des = make_design(256, 4, seed=4401)
    ora = orc.estep(y, P, des)
    gpu = _gpu_estep(cf, y, P, des, "fp64")
    np.testing.assert_allclose(gpu.logf_comp.cpu().numpy(), ora.logf_comp, rtol=0, atol=1e-10)
    compare_estep(gpu, ora, "fp64", label="dof 3000", tol=dict(logf=1e-10, tau=1e-12, eterm=1e-9))
    yd = torch.as_tensor(np.ascontiguousarray(y.T)).cuda()
    es = cf.alloc_estep(y.shape[0], 3, 3, 2, cf.CFUST_FP64)
    B = cf.Batch([(yd, cf.device_params(P), es)], cf.device_qmc(des, cf.CFUST_FP64))
    B.estep()
    torch.cuda.synchronize()
    for name in ("tau", "logf_obs", "loglik", "w", "e1", "e2", "e3", "logf_comp"):
        assert torch.equal(getattr(es, name), getattr(gpu, name)), name
    B.close()


@pytest.mark.parametrize("p,q,g,n,seed,N,S", [(16, 8, 2, 6, 61, 128, 2), (2, 2, 64, 24, 62, 256, 4)])
def test_estep_max_sizes(lib, orc, p, q, g, n, seed, N, S):
    """The largest p and q the C ABI takes (16 and 8: 38 lattice integrals
    per pair, of every dimension 2..8) and the most components (64), in both
    modes, against the oracle on the same lattice."""
    cf = lib
    print(f"estep max sizes p={p} q={q} g={g} n={n}", flush=True)
    rng = np.random.default_rng(seed)
    P = draw_params(rng, p, q, g, sigma="wishart")
    y, _ = sample_hierarchy(rng, P, n)
    des = make_design(N, S, seed=seed)
    ora = orc.estep(y, P, des)
    for mode in ("fp64", "mixed"):
        gpu = _gpu_estep(cf, y, P, des, mode)
        compare_estep(gpu, ora, mode, label=f"p{p}q{q}g{g} {mode}")
        np.testing.assert_allclose(gpu.logf_comp.cpu().numpy(), ora.logf_comp, rtol=0, atol=TOL[mode]["logf"])
        assert abs(float(gpu.loglik.cpu()[0]) - ora.loglik) <= TOL[mode]["logf"] * n


def test_estep_small_workload_full(lib, orc):
    """The n=1000, p=q=2, g=2 workload in FP64 at its lattice (N=1024 x 4), every observation."""
    cf = lib
    ds = workload("cfust_n1000_p2_q2_g2")
    des = make_design(1024, 4, seed=1606)
    P = ds.params.copy()
    P.mu = P.mu + 0.3
    ora = orc.estep(ds.y, P, des)
    gpu = _gpu_estep(cf, ds.y, P, des, "fp64")
    compare_estep(gpu, ora, "fp64", label="n1000")


def test_estep_determinism(lib):
    cf = lib
    rng = np.random.default_rng(21)
    P = draw_params(rng, 4, 4, 3, sigma="wishart")
    y, _ = sample_hierarchy(rng, P, 77)
    des = make_design(512, 4, seed=5)
    a = _gpu_estep(cf, y, P, des, "mixed")
    b = _gpu_estep(cf, y, P, des, "mixed")
    for name in ("tau", "w", "e1", "e2", "e3", "logf_obs", "loglik"):
        assert torch.equal(getattr(a, name), getattr(b, name)), name


def test_estep_edge_cases(lib, orc):
    cf = lib
    rng = np.random.default_rng(31)
    P = draw_params(rng, 3, 3, 2, sigma="aat")
    des = make_design(256, 4, seed=6)
    # n = 0: valid, loglik = 0
    y0 = torch.zeros((3, 0), dtype=torch.float64, device="cuda")
    out = cf.cfust_estep(y0, cf.device_params(P), cf.device_qmc(des, cf.CFUST_MIXED))
    torch.cuda.synchronize()
    assert float(out.loglik.cpu()[0]) == 0.0
    # g = 1 gives tau = 1
    P1 = draw_params(rng, 3, 3, 1, pi=[1.0], sigma="aat")
    y, _ = sample_hierarchy(rng, P1, 11)
    g1 = _gpu_estep(cf, y, P1, des, "fp64")
    assert np.all(g1.tau.cpu().numpy() == 1.0)
    # an observation far from one component: that component's tau underflows to 0
    y, _ = sample_hierarchy(rng, P, 6)
    y[0] = P.mu[0] + 1e4
    ora = orc.estep(y, P, des)
    gpu = _gpu_estep(cf, y, P, des, "fp64")
    compare_estep(gpu, ora, "fp64", label="far")
    # bad dims are rejected on the host
    with pytest.raises(RuntimeError, match="EINVAL"):
        Pbad = draw_params(rng, 3, 9, 1, pi=[1.0])
        cf.cfust_estep(torch.zeros((3, 4), dtype=torch.float64, device="cuda"), cf.device_params(Pbad),
                       cf.device_qmc(des, cf.CFUST_FP64))


def test_estep_bench_workload_sampled(lib, orc):
    """The n=20000, p=q=4, g=3 workload in the launch configuration the bench
    times (mixed, N=4096 x 8): sampled observations against the oracle."""
    cf = lib
    ds = workload("cfust_n20000_p4_q4_g3")
    des = make_design(4096, 8, seed=1606)
    gpu = _gpu_estep(cf, ds.y, ds.params, des, "mixed")
    rows = np.array([0, 7777, 19999])
    ora = orc.estep(ds.y, ds.params, des, rows=rows)
    compare_estep(gpu, ora, "mixed", rows=rows, label="bench-sampled")
    # tau sums to one everywhere
    np.testing.assert_allclose(gpu.tau.cpu().numpy().sum(0), 1.0, atol=1e-12)


def test_estep_cytometry_shape_sampled(lib, orc):
    """The cytometry-shaped recipe (p = q = 8, g = 5: integrals of dimension
    6, 7 and 8) at n = 2048 in mixed precision, lattice 1024 x 4: sampled
    observations against the oracle (the full-size lattice is left to the
    bench: the FP64 oracle needs minutes per observation there)."""
    cf = lib
    print("estep cytometry shape, sampled", flush=True)
    ds = workload("cfust_n1e6_p8_q8_g5_box1024", n=2048)
    des = make_design(1024, 4, seed=1606)
    gpu = _gpu_estep(cf, ds.y, ds.params, des, "mixed")
    rows = np.array([5, 1500])
    ora = orc.estep(ds.y, ds.params, des, rows=rows)
    compare_estep(gpu, ora, "mixed", rows=rows, label="cytometry-sampled")
    np.testing.assert_allclose(gpu.logf_comp.cpu().numpy()[:, rows], ora.logf_comp, atol=1e-4)
    assert int(gpu.status.cpu()[0]) == 0


def test_loglik_matches_estep_and_oracle(lib, orc):
    cf = lib
    rng = np.random.default_rng(41)
    P = draw_params(rng, 3, 3, 3, sigma="wishart")
    y, _ = sample_hierarchy(rng, P, 57)
    des = make_design(256, 4, seed=7)
    yd = torch.as_tensor(np.ascontiguousarray(y.T)).cuda()
    for mode in ("fp64", "mixed"):
        lo = torch.zeros(y.shape[0], dtype=torch.float64, device="cuda")
        ll, _ = cf.cfust_loglik(yd, cf.device_params(P), cf.device_qmc(des, _mode(cf, mode)), logf_obs=lo)
        es = _gpu_estep(cf, y, P, des, mode)
        assert torch.equal(lo, es.logf_obs)
        ora = orc.estep(y, P, des)
        assert np.abs(lo.cpu().numpy() - ora.logf_obs).max() <= TOL[mode]["logf"]


# ------------------------------------------------------------------- M-step --

def _point_mass_estep(rng, P, n):
    """E-step outputs of posteriors that are point masses at drawn latent values
    (a valid input to eqs. 18-22, and far cheaper than the oracle E-step at
    q = 8): tau from a Dirichlet, w ~ Gamma(nu/2, rate nu/2), u >= 0
    half-normal; w, e1 = log w, e2 = w u, e3 = w u u^T (upper triangle, row by
    row)."""
    from types import SimpleNamespace
    g, q = P.g, P.q
    tau = rng.dirichlet(np.ones(g), size=n).T.copy()
    w = np.stack([rng.gamma(P.nu[h] / 2.0, 2.0 / P.nu[h], size=n) for h in range(g)])
    u = np.abs(rng.standard_normal((g, q, n)))
    iu = [(i, k) for i in range(q) for k in range(i, q)]
    e3 = np.stack([np.stack([w[h] * u[h, i] * u[h, k] for (i, k) in iu]) for h in range(g)])
    return SimpleNamespace(tau=tau, w=w, e1=np.log(w), e2=w[:, None, :] * u, e3=e3, logf_obs=np.zeros(n))


@pytest.mark.parametrize("p,q,g,n,seed", [(2, 2, 2, 300, 11), (4, 4, 3, 200, 12), (5, 3, 2, 130, 13),
                                          (8, 8, 2, 3000, 14), (12, 5, 2, 700, 15), (16, 8, 2, 300, 16)])
@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_mstep_vs_oracle(lib, orc, p, q, g, n, seed, mode):
    """Same E-step outputs into both M-steps (in mixed mode the e-terms are the
    FP32 roundings the GPU path stores).  The shapes cover both sizes of the
    reduction (p <= 8, p <= 16), the largest p and q, and many tiles per block
    with a ragged last tile."""
    cf = lib
    print(f"mstep vs oracle p={p} q={q} g={g} n={n} {mode}", flush=True)
    rng = np.random.default_rng(seed)
    P = draw_params(rng, p, q, g, sigma="aat")
    y, _ = sample_hierarchy(rng, P, n)
    if p <= 5:
        es = orc.estep(y, P, make_design(256, 4, seed=seed))
    else:
        es = _point_mass_estep(rng, P, n)
    if mode == "mixed":
        for name in ("w", "e1", "e2", "e3"):
            setattr(es, name, getattr(es, name).astype(np.float32).astype(np.float64))
    ref, frozen = orc.mstep(y, es, P)
    et = torch.float32 if mode == "mixed" else torch.float64
    to = lambda a, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(a), dtype=dt).cuda()
    ges = cf.EStepResult(to(es.tau), to(es.logf_obs), to(np.zeros(1)), to(es.w, et), to(es.e1, et),
                         to(es.e2, et), to(es.e3, et), precision=_mode(cf, mode))
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    out = cf.cfust_mstep(to(y.T), ges, cf.device_params(P), status=st)
    torch.cuda.synchronize()
    got = out.to_host()
    for a, b, name in zip(got, (ref.pi, ref.mu, ref.Sigma, ref.Delta, ref.nu), ("pi", "mu", "Sigma", "Delta", "nu")):
        assert np.abs(a - b).max() <= 1e-9 * max(1.0, np.abs(b).max()), (name, np.abs(a - b).max())
    assert int(st.cpu()[0]) & ~64 == 0


def test_em_iterations_gpu_vs_oracle(lib, orc):
    """Three FP64 EM iterations on the GPU track the oracle's iterates."""
    cf = lib
    ds = workload("cfust_n1000_p2_q2_g2", n=400)
    des = make_design(256, 4, seed=3)
    P = ds.params.copy()
    P.mu += 0.4
    P.nu = np.array([10.0, 10.0])
    dp = cf.device_params(P)
    qm = cf.device_qmc(des, cf.CFUST_FP64)
    yd = torch.as_tensor(ds.y_soa).cuda()
    cur = P
    for it in range(3):
        es = orc.estep(ds.y, cur, des)
        cur, _ = orc.mstep(ds.y, es, cur)
        ges = cf.cfust_estep(yd, dp, qm)
        dp = cf.cfust_mstep(yd, ges, dp)
        torch.cuda.synchronize()
        assert abs(float(ges.loglik.cpu()[0]) - es.loglik) <= 1e-6 * ds.y.shape[0]
    got = dp.to_host()
    for a, b in zip(got, (cur.pi, cur.mu, cur.Sigma, cur.Delta, cur.nu)):
        assert np.abs(a - b).max() <= 1e-6 * max(1.0, np.abs(b).max())
