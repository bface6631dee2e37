"""GPU tests of the surrogate network (forward/backward/loss/Adam kernels
against the FP64 reference in oracle/mlp.py), of its training, and of the
E-step that uses it with the lattice as fallback."""
import os
import time

import numpy as np
import pytest
import torch

from cfust_inputs import make_design, workload
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sur():
    import paper_1606_02054_amd as cf
    from paper_1606_02054_amd import surrogate as S
    assert torch.cuda.is_available()
    cf.default_handle()
    return cf, S


def _host_net(net):
    Ws = [omlp.bf16_round(w.cpu().numpy().astype(np.float64)) for w in net.W32]
    bs = [b.cpu().numpy().astype(np.float64) for b in net.b32]
    return Ws, bs


def _bf16_input(rng, rows):
    X = rng.uniform(-1, 1, (rows, 16))
    Xb = omlp.bf16_round(X)
    t = torch.tensor(Xb, dtype=torch.float32).to(torch.bfloat16).view(torch.int16).cuda()
    return Xb, t


def test_forward_backward_vs_reference(sur):
    cf, S = sur
    print("mlp forward/backward", flush=True)
    rng = np.random.default_rng(3)
    net = S.SurrogateNet(2, seed=5)
    rows = 192                      # three 64-row tiles
    Xb, X0 = _bf16_input(rng, rows)
    acts = S.Activations(rows, "cuda")
    out = torch.zeros((rows, 16), dtype=torch.float32, device="cuda")
    S.mlp_forward(net, X0, out, acts)
    label = rng.uniform(-1.5, 0.0, rows)
    dout = torch.zeros_like(out)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    S.mlp_loss(out, torch.tensor(label, dtype=torch.float32).cuda(), rows, 0.2, dout, loss)
    S.mlp_backward(net, acts, dout)
    torch.cuda.synchronize()
    Ws, bs = _host_net(net)
    ref_out, cache = omlp.forward(Ws, bs, Xb, bf16=True)
    got = out.cpu().numpy().astype(np.float64)
    scale = np.abs(ref_out).max()
    assert np.abs(got - ref_out).max() <= 2e-2 * scale
    rl, rdout = omlp.loss_and_grad(got, label.astype(np.float32).astype(np.float64), 0.2)
    assert abs(float(loss.cpu()[0]) / rows - rl) <= 1e-4 * max(1.0, rl)
    np.testing.assert_allclose(dout.cpu().numpy(), rdout, rtol=1e-4, atol=1e-7)
    # Gradients entry by entry.  The reference back-propagates from the
    # activations the kernels saved (BF16 layer inputs X_l, FP32
    # pre-activations Z_l) and the kernels' dL/dout, so the two differ only by
    # the FP32 accumulation order and by the BF16 rounding of dZ, where an FP32
    # and an FP64 product on either side of a rounding boundary round one BF16
    # step (2^-8 relative) apart.  Bound per entry: 2 x 2^-8 sum_b |dZ_bi||X_bj|
    # (two such steps) plus 1e-5 of the layer's largest gradient.
    xs = [torch.as_tensor(acts.X[l]).view(torch.bfloat16).float().cpu().numpy().astype(np.float64)
          for l in range(5)]
    zs = [acts.Z[l].cpu().numpy().astype(np.float64) for l in range(4)]
    gdout = dout.cpu().numpy().astype(np.float64)
    dWs, dbs, _ = omlp.backward(Ws, bs, (xs, zs), gdout, bf16=True)
    dzs = omlp.backward_dz(Ws, (xs, zs), gdout, bf16=True)
    for l in range(5):
        gW = net.dW[l].cpu().numpy().astype(np.float64)
        bound = 2.0 * 2.0 ** -8 * (np.abs(dzs[l]).T @ np.abs(xs[l])) + 1e-5 * np.abs(dWs[l]).max()
        bad = np.abs(gW - dWs[l]) > bound
        assert not bad.any(), (l, int(bad.sum()), float(np.abs(gW - dWs[l]).max()))
        gb = net.db[l].cpu().numpy().astype(np.float64)
        bound_b = 2.0 * 2.0 ** -8 * np.abs(dzs[l]).sum(0) + 1e-5 * np.abs(dbs[l]).max()
        badb = np.abs(gb - dbs[l]) > bound_b
        assert not badb.any(), (l, int(badb.sum()), float(np.abs(gb - dbs[l]).max()))
        # and the bound is tight enough to see one wrong term: an average
        # row's contribution to an entry is above half of it (entries with a
        # gradient; outputs 2..15 carry no loss)
        contrib = np.abs(dzs[l]).T @ np.abs(xs[l]) / dzs[l].shape[0]
        live = contrib > 0
        assert np.median(contrib[live] / bound[live]) > 0.5


@pytest.mark.parametrize("rows", [64, 192, 8192])
def test_fused_inference_equals_layered_forward(sur, rows):
    """The inference pass (no activations kept: one fused kernel, the tile's
    activations in LDS) against the per-layer pass the training uses: the
    same MFMA operands, K order and roundings, so the outputs are equal bit
    for bit; and against the FP64 reference with BF16 rounding."""
    cf, S = sur
    print(f"fused inference rows={rows}", flush=True)
    rng = np.random.default_rng(17)
    net = S.SurrogateNet(3, seed=9)
    Xb, X0 = _bf16_input(rng, rows)
    out_f = torch.zeros((rows, 16), dtype=torch.float32, device="cuda")
    out_l = torch.zeros_like(out_f)
    S.mlp_forward(net, X0, out_f)
    S.mlp_forward(net, X0, out_l, S.Activations(rows, "cuda"))
    torch.cuda.synchronize()
    assert torch.equal(out_f, out_l)
    Ws, bs = _host_net(net)
    ref_out, _ = omlp.forward(Ws, bs, Xb, bf16=True)
    assert np.abs(out_f.cpu().numpy() - ref_out).max() <= 2e-2 * np.abs(ref_out).max()


def test_adam_step_vs_reference(sur):
    cf, S = sur
    net = S.SurrogateNet(3, seed=9)
    rng = np.random.default_rng(4)
    for l in range(5):
        net.dW[l].copy_(torch.tensor(rng.standard_normal(net.dW[l].shape), dtype=torch.float32))
        net.db[l].copy_(torch.tensor(rng.standard_normal(net.db[l].shape), dtype=torch.float32))
    W0 = [w.cpu().numpy().astype(np.float64) for w in net.W32]
    g = [d.cpu().numpy().astype(np.float64) for d in net.dW]
    S.mlp_adam(net, 1e-3)
    torch.cuda.synchronize()
    for l in range(5):
        m = 0.1 * g[l]; v = 0.001 * g[l] ** 2
        ref = W0[l] - 1e-3 * (m / 0.1) / (np.sqrt(v / 0.001) + 1e-8)
        np.testing.assert_allclose(net.W32[l].cpu().numpy(), ref, rtol=1e-5, atol=1e-7)
        bf = torch.tensor(net.W32[l].cpu().numpy()).to(torch.bfloat16).view(torch.int16)
        assert torch.equal(net.Wb[l].cpu(), bf)
        assert torch.equal(net.WbT[l].cpu(), bf.t().contiguous())


def test_training_reduces_error(sur):
    cf, S = sur
    print("surrogate short training", flush=True)
    des = make_design(1024, 4, seed=31)
    net, rep = S.train(2, 262144, des, epochs=6, batch=4096, lr=2e-3, seed=7, n_val=8192, log=print)
    print(rep, flush=True)
    # the typical problem is learned to a few hundredths in ln T and the tail
    # to a few tenths (the short run: 2.6e5 problems, 6 epochs), and the error
    # head ranks its own errors (it decides which answers are used)
    assert rep.val_p50_abs_lnT < 0.05
    assert rep.val_p99_abs_lnT < 0.5
    assert rep.err_head_corr > 0.3
    # after calibration, the answers accepted at each tolerance meet it at the
    # 99th percentile on held-out problems the calibration did not see (a
    # 20% margin for the sampling of a 99th percentile)
    for tol, share, p99 in rep.calibration:
        assert p99 <= 1.2 * tol, (tol, share, p99)


def _c1(cf):
    ds = workload("cfust_n1000_p2_q2_g2")
    y = torch.as_tensor(ds.y_soa).cuda()
    return ds, y, cf.device_params(ds.params)


def test_surrogate_tol_zero_is_plain_lattice(sur):
    cf, S = sur
    ds, y, dp = _c1(cf)
    qmc = cf.device_qmc(make_design(1024, 4, seed=1606), cf.CFUST_MIXED)
    net = S.SurrogateNet(2, seed=1)
    nf = torch.zeros(1, dtype=torch.int32, device="cuda")
    a = S.cfust_estep_surrogate(y, dp, qmc, {2: net}, tol=0.0, n_fallback=nf)
    b = cf.cfust_estep(y, dp, qmc)
    torch.cuda.synchronize()
    for name in ("tau", "w", "e1", "e2", "e3", "logf_obs", "loglik"):
        assert torch.equal(getattr(a, name), getattr(b, name)), name
    assert int(nf.cpu()[0]) == 2 * 2 * 1000


def _trained(S, m, des):
    path = os.path.join(os.path.dirname(S.__file__), "weights", f"surrogate_m{m}.npz")
    if os.path.exists(path):
        return S.SurrogateNet.load(path)
    net, _ = S.train(m, 262144, des, epochs=4, seed=11, log=print)
    return net


def test_surrogate_estep_accuracy_and_gain(sur, orc):
    """E-step of the n=1000, p=q=2, g=2 data with the trained network for
    T_2 against the lattice (reference: 65536 x 16 points).

    Asserted: the fallback rule works -- at the tightest tolerance some
    integrals go to the lattice, and at every tolerance the observations'
    log-densities stay within it of the oracle's at the 99th percentile (the answers accepted are
    those whose calibrated predicted error in ln T is below it); and the
    measured outcome: at equal log-likelihood accuracy the network gives no
    speed-up over the lattice (a lattice of a few hundred points is already
    more accurate than the BF16 network and cheaper than its evaluation)."""
    cf, S = sur
    print("surrogate E-step gain", flush=True)
    ds, y, dp = _c1(cf)
    net = _trained(S, 2, make_design(8192, 8, seed=2024))
    ref_qmc = cf.device_qmc(make_design(65536, 16, seed=99), cf.CFUST_MIXED)
    ref = cf.cfust_estep(y, dp, ref_qmc)
    torch.cuda.synchronize()
    l_ref = float(ref.loglik.cpu()[0])

    def timed(fn, reps=5):
        fn(); torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            out = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps, out

    rows = []
    for N, Sh in [(64, 2), (128, 2), (256, 2), (256, 4), (512, 4), (1024, 4), (2048, 8), (4096, 8)]:
        q = cf.device_qmc(make_design(N, Sh, seed=1606), cf.CFUST_MIXED)
        t, o = timed(lambda: cf.cfust_estep(y, dp, q))
        rows.append((N, Sh, t, abs(float(o.loglik.cpu()[0]) - l_ref)))
        print(f"lattice {N}x{Sh}: {t * 1e3:.3f} ms, |dl| = {rows[-1][3]:.3e}", flush=True)
    qmc_s = cf.device_qmc(make_design(1024, 4, seed=1606), cf.CFUST_MIXED)
    des_s = make_design(1024, 4, seed=1606)
    ora = orc.estep(ds.y, ds.params, des_s)
    speedups = []
    for tol in (0.02, 0.05, 0.1):
        nf = torch.zeros(1, dtype=torch.int32, device="cuda")
        t_sur, o_sur = timed(lambda: S.cfust_estep_surrogate(y, dp, qmc_s, {2: net}, tol=tol, n_fallback=nf))
        err_sur = abs(float(o_sur.loglik.cpu()[0]) - l_ref)
        nfb = int(nf.cpu()[0])
        match = [r for r in rows if r[3] <= err_sur]
        t_eq = min(r[2] for r in match) if match else rows[-1][2]
        speedups.append(t_eq / t_sur)
        d = np.abs(o_sur.logf_obs.cpu().numpy() - ora.logf_obs)
        print(f"surrogate tol={tol}: {t_sur * 1e3:.3f} ms, |dl| = {err_sur:.3e}, lattice fallback {nfb}/4000, "
              f"|dlogf| p99 {np.quantile(d, 0.99):.3e} max {d.max():.3e}, "
              f"speed-up at equal log-likelihood accuracy {t_eq / t_sur:.2f}x", flush=True)
        if tol == 0.02:
            assert nfb > 0          # the network is not trusted everywhere at the tightest tolerance
        assert np.quantile(d, 0.99) <= tol + 1e-3, (tol, np.quantile(d, 0.99))
    assert max(speedups) < 1.0, speedups
