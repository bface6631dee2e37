"""GPU test of the allocation-free E-step (cfust_estep_noalloc): through the C
ABI it gives cfust_estep's outputs bit for bit, on two calls in a row (the
second with a smaller input, so the fixed workspace still holds the first
call's larger contents), in both precisions; a call whose workspace exceeds
the fixed array is refused on the host before any launch."""
import numpy as np
import pytest
import torch

from cfust_inputs import draw_params, make_design, sample_hierarchy

pytestmark = pytest.mark.gpu

FIELDS = ("tau", "logf_obs", "loglik", "w", "e1", "e2", "e3", "logf_comp", "cdf_stderr", "status")


@pytest.fixture(scope="module")
def lib():
    import paper_1606_02054_amd as cf
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    cf.default_handle()
    return cf


def _case(seed, p, q, g, n, N, S):
    rng = np.random.default_rng(seed)
    P = draw_params(rng, p, q, g, sigma="wishart" if p > 2 else "aat")
    y, _ = sample_hierarchy(rng, P, n)
    return y, P, make_design(N, S, seed=seed)


@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_noalloc_matches_estep_on_two_calls(lib, mode):
    cf = lib
    prec = cf.CFUST_FP64 if mode == "fp64" else cf.CFUST_MIXED
    cases = [(8101, 4, 4, 3, 1537, 512, 4),     # first call: the larger workspace
             (8102, 3, 3, 2, 203, 256, 4)]      # second call: smaller n, p, q, g and lattice
    for seed, p, q, g, n, N, S in cases:
        print(f"noalloc {mode} p={p} q={q} g={g} n={n} N={N} S={S}", flush=True)
        y, P, des = _case(seed, p, q, g, n, N, S)
        yd = torch.as_tensor(np.ascontiguousarray(y.T)).cuda()
        dp = cf.device_params(P)
        qm = cf.device_qmc(des, prec)
        ref = cf.cfust_estep(yd, dp, qm)
        out = cf.alloc_estep(n, p, q, g, prec)
        for t in (out.tau, out.logf_obs, out.w, out.e1, out.e2, out.e3, out.logf_comp, out.cdf_stderr):
            t.fill_(float("nan"))                 # every output must be written by the call
        got = cf.cfust_estep_noalloc(yd, dp, qm, out)
        torch.cuda.synchronize()
        for name in FIELDS:
            a, b = getattr(got, name), getattr(ref, name)
            assert torch.equal(a, b), f"{mode} n={n}: {name} differs"
        assert np.isfinite(got.logf_obs.cpu().numpy()).all()


def test_noalloc_rejects_oversized_workspace(lib):
    cf = lib
    p = q = 8
    g = 5
    # about g n (12 J + 16) bytes with J = 38 lattice integrals per pair: n = 40000 needs ~94 MB
    n = 40000
    y, P, des = _case(8103, p, q, g, 8, 256, 2)
    yd = torch.zeros((p, n), dtype=torch.float64, device="cuda")
    out = cf.alloc_estep(n, p, q, g, cf.CFUST_MIXED)
    with pytest.raises(RuntimeError, match="EINVAL.*exceeds the fixed"):
        cf.cfust_estep_noalloc(yd, cf.device_params(P), cf.device_qmc(des, cf.CFUST_MIXED), out)
    # the handle stays usable
    y, P, des = _case(8104, 2, 2, 2, 50, 256, 2)
    yd = torch.as_tensor(np.ascontiguousarray(y.T)).cuda()
    out = cf.alloc_estep(50, 2, 2, 2, cf.CFUST_MIXED)
    cf.cfust_estep_noalloc(yd, cf.device_params(P), cf.device_qmc(des, cf.CFUST_MIXED), out)
    torch.cuda.synchronize()
    assert np.isfinite(out.logf_obs.cpu().numpy()).all()
