"""Argument errors of the C ABI (include/cfust.h): each is found on the host
and returned as CFUST_EINVAL before any kernel is launched, and the handle
stays usable afterwards."""
import numpy as np
import pytest
import torch

from cfust_inputs import draw_params, make_design, sample_hierarchy

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cf():
    import paper_1606_02054_amd as cf
    assert torch.cuda.is_available()
    cf.default_handle()
    return cf


def _qmc(cf, N, S, precision):
    z = torch.ones(cf.LATTICE_DIM, dtype=torch.int32, device="cuda")
    shifts = torch.zeros((S, cf.LATTICE_DIM), dtype=torch.float64, device="cuda")
    return cf.DeviceQmc(N, S, z, shifts, precision)


@pytest.mark.parametrize("N,S,precision,why", [
    (100, 2, 1, "power of two"),          # mixed precision needs N = 2^k
    (1, 2, 0, "outside"),                 # N < 2
    (70000, 2, 0, "outside"),             # N > 65536
    (256, 0, 0, "outside"),               # no shift
    (256, 65, 0, "outside"),              # more shifts than CFUST_MAX_SHIFTS
    (256, 2, 7, "neither"),               # unknown precision
])
def test_bad_lattice_is_rejected(cf, N, S, precision, why):
    print(f"bad lattice N={N} S={S} precision={precision}", flush=True)
    rng = np.random.default_rng(3)
    P = draw_params(rng, 3, 3, 2, sigma="aat")
    y = torch.as_tensor(np.ascontiguousarray(sample_hierarchy(rng, P, 10)[0].T)).cuda()
    with pytest.raises(RuntimeError, match=f"EINVAL.*{why}"):
        cf.cfust_estep(y, cf.device_params(P), _qmc(cf, N, S, precision))
    with pytest.raises(RuntimeError, match="EINVAL"):
        cf.cfust_loglik(y, cf.device_params(P), _qmc(cf, N, S, precision))
    # the handle still works
    ok = cf.cfust_estep(y, cf.device_params(P), cf.device_qmc(make_design(256, 2, seed=1), cf.CFUST_FP64))
    torch.cuda.synchronize()
    assert np.isfinite(float(ok.loglik.cpu()[0]))


def test_bad_mvt_dimension_is_rejected(cf):
    print("mvt m = 9", flush=True)
    m = 9
    b = torch.zeros((3, m), dtype=torch.float64, device="cuda")
    L = torch.eye(m, dtype=torch.float64, device="cuda")[None].contiguous()
    idx = torch.zeros(3, dtype=torch.int32, device="cuda")
    nu = torch.full((3,), 5.0, dtype=torch.float64, device="cuda")
    with pytest.raises(RuntimeError, match="EINVAL"):
        cf.mvt_cdf_batch(b, L, idx, nu, cf.device_qmc(make_design(256, 2, seed=1), cf.CFUST_FP64))
