"""Learned surrogate for the lattice estimate of T_m(b; 0, R, nu), m = 2..4.

The E-step needs, per (observation, component), the multivariate t
probabilities T_q, T_{q-1}, T_{q-2} of the density (Sec. 2 eq. 4), of the
weights (Sec. 3.1 eq. 13) and of the truncated-t moments (eqs. 16-17).  A
small perceptron (16 -> 4 x 256 GELU -> 16; BF16 weights, FP32 accumulate on
the matrix cores) predicts ln T_m from standardised limits, correlations and
the dof, plus a second head that predicts the log10 of its own absolute error.
The E-step uses the prediction where the predicted error is below a
tolerance and the inputs lie in the training domain, and the lattice
estimate otherwise (the lattice also produces the training labels and judges
the network's error).

Training runs on the GPU through the library's own kernels (forward,
backward, loss, Adam); PyTorch only allocates buffers and shuffles indices.
"""
from __future__ import annotations

import ctypes as C
import math
import time
from dataclasses import dataclass
from typing import Dict, Optional

import numpy as np
import torch

from . import _binding as B
from . import (DeviceQmc, EStepResult, Handle, _check_y, _ptr, _stream, alloc_estep, default_handle,
               mvt_cdf_batch)

RESID_SCALE = 5.0          # network output 0 = (ln T - sum of marginal ln T_nu) / RESID_SCALE


def _arr(ptrs):
    a = (C.c_void_p * len(ptrs))()
    for i, t in enumerate(ptrs):
        a[i] = None if t is None else t.data_ptr()
    return a


class SurrogateNet:
    """Weights, master copy, Adam state and gradients of one network, on the device."""

    def __init__(self, m: int, seed: int = 0, device="cuda"):
        self.m = int(m)
        self.device = torch.device(device)
        g = torch.Generator(device="cpu").manual_seed(seed)
        self.W32, self.b32 = [], []
        for K, N in zip(B.MLP_K, B.MLP_N):
            std = math.sqrt(2.0 / K)
            self.W32.append((torch.randn(N, K, generator=g, dtype=torch.float32) * std).to(self.device))
            self.b32.append(torch.zeros(N, dtype=torch.float32, device=self.device))
        self._alloc()
        self.refresh_bf16()
        self.step = 0

    def _alloc(self):
        d = self.device
        self.mW = [torch.zeros_like(w) for w in self.W32]
        self.vW = [torch.zeros_like(w) for w in self.W32]
        self.mb = [torch.zeros_like(b) for b in self.b32]
        self.vb = [torch.zeros_like(b) for b in self.b32]
        self.dW = [torch.zeros_like(w) for w in self.W32]
        self.db = [torch.zeros_like(b) for b in self.b32]
        self.Wb = [torch.zeros(w.shape, dtype=torch.int16, device=d) for w in self.W32]
        self.WbT = [torch.zeros((w.shape[1], w.shape[0]), dtype=torch.int16, device=d) for w in self.W32]

    def refresh_bf16(self):
        """BF16 copies (both layouts) of the FP32 master weights (setup only;
        during training the Adam kernel refreshes them)."""
        for l, w in enumerate(self.W32):
            self.Wb[l].copy_(w.to(torch.bfloat16).view(torch.int16))
            self.WbT[l].copy_(w.t().contiguous().to(torch.bfloat16).view(torch.int16))

    # ---- C structs ---------------------------------------------------------
    def weights_c(self) -> B.MlpWeightsC:
        return B.MlpWeightsC(_arr(self.Wb), _arr(self.WbT), _arr(self.b32))

    def grads_c(self) -> B.MlpGradsC:
        return B.MlpGradsC(_arr(self.dW), _arr(self.db))

    def master_c(self) -> B.MlpMasterC:
        return B.MlpMasterC(_arr(self.W32), _arr(self.mW), _arr(self.vW), _arr(self.b32), _arr(self.mb),
                            _arr(self.vb))

    # ---- persistence ---------------------------------------------------------
    def state(self) -> Dict[str, np.ndarray]:
        out = {"m": np.array(self.m)}
        for l in range(B.MLP_LAYERS):
            out[f"W{l}"] = self.W32[l].cpu().numpy()
            out[f"b{l}"] = self.b32[l].cpu().numpy()
        return out

    def save(self, path: str):
        np.savez(path, **self.state())

    @classmethod
    def load(cls, path: str, device="cuda") -> "SurrogateNet":
        z = np.load(path, allow_pickle=False)
        net = cls(int(z["m"]), device=device)
        for l in range(B.MLP_LAYERS):
            net.W32[l].copy_(torch.as_tensor(z[f"W{l}"]))
            net.b32[l].copy_(torch.as_tensor(z[f"b{l}"]))
        net.refresh_bf16()
        return net


class Activations:
    def __init__(self, rows: int, device):
        self.X = [torch.zeros((rows, K), dtype=torch.int16, device=device) for K in B.MLP_K]
        self.XT = [torch.zeros((K, rows), dtype=torch.int16, device=device) for K in B.MLP_K]
        self.Z = [torch.zeros((rows, N), dtype=torch.float32, device=device) for N in B.MLP_N[:-1]]

    def c(self) -> B.MlpActsC:
        return B.MlpActsC(_arr(self.X), _arr(self.XT), _arr(self.Z))


def mlp_forward(net: SurrogateNet, X0: torch.Tensor, out: torch.Tensor, acts: Optional[Activations] = None,
                handle: Optional[Handle] = None, stream=None):
    h = handle or default_handle()
    rows = int(X0.shape[0])
    w = net.weights_c()
    ac = acts.c() if acts is not None else None
    st = h.lib.cfust_mlp_forward(h.h, C.byref(w), C.c_void_p(X0.data_ptr()), rows, C.c_void_p(out.data_ptr()),
                                 C.byref(ac) if ac is not None else None, _stream(stream))
    B.check(st, h.h, "cfust_mlp_forward")
    return out


def mlp_backward(net: SurrogateNet, acts: Activations, dout: torch.Tensor, handle: Optional[Handle] = None,
                 stream=None):
    h = handle or default_handle()
    w, ac, gc = net.weights_c(), acts.c(), net.grads_c()
    st = h.lib.cfust_mlp_backward(h.h, C.byref(w), C.byref(ac), C.c_void_p(dout.data_ptr()), int(dout.shape[0]),
                                  C.byref(gc), _stream(stream))
    B.check(st, h.h, "cfust_mlp_backward")


def mlp_adam(net: SurrogateNet, lr: float, b1=0.9, b2=0.999, eps=1e-8, handle: Optional[Handle] = None,
             stream=None):
    h = handle or default_handle()
    net.step += 1
    mc, gc, w = net.master_c(), net.grads_c(), net.weights_c()
    st = h.lib.cfust_mlp_adam(h.h, C.byref(mc), C.byref(gc), C.byref(w), float(lr), float(b1), float(b2),
                              float(eps), int(net.step), _stream(stream))
    B.check(st, h.h, "cfust_mlp_adam")


def mlp_loss(out, label, nvalid, lam, dout, loss_sum, handle: Optional[Handle] = None, stream=None):
    h = handle or default_handle()
    st = h.lib.cfust_mlp_loss(h.h, _ptr(out), _ptr(label), int(out.shape[0]), int(nvalid), float(lam),
                              _ptr(dout), _ptr(loss_sum), _stream(stream))
    B.check(st, h.h, "cfust_mlp_loss")


def mvt_features(m, b, L, mat_idx, nu, rows_pad, handle: Optional[Handle] = None, stream=None):
    """Network inputs (BF16 as int16 [rows_pad][16]), training-domain flags and
    the independence log-probability sum_i ln T_nu(z_i) of T_m problems."""
    h = handle or default_handle()
    batch = int(b.shape[0])
    X0 = torch.zeros((rows_pad, B.MLP_IN), dtype=torch.int16, device=b.device)
    inr = torch.zeros(max(batch, 1), dtype=torch.int32, device=b.device)
    base = torch.zeros(max(batch, 1), dtype=torch.float64, device=b.device)
    st = h.lib.cfust_mlp_features(h.h, int(m), batch, int(rows_pad), _ptr(b), _ptr(L), _ptr(mat_idx),
                                  int(L.shape[0]), _ptr(nu), _ptr(X0), _ptr(inr), _ptr(base), _stream(stream))
    B.check(st, h.h, "cfust_mlp_features")
    return X0, inr[:batch], base[:batch]


# ------------------------------------------------------------------ training --

@dataclass
class TrainReport:
    m: int
    n_train: int
    epochs: int
    seconds_label: float
    seconds_train: float
    train_loss: float
    val_rmse_lnT: float          # RMSE of ln T on held-out problems
    val_max_abs_lnT: float
    err_head_corr: float         # correlation of predicted vs actual log10 |error|
    val_p50_abs_lnT: float = float("nan")
    val_p90_abs_lnT: float = float("nan")
    val_p99_abs_lnT: float = float("nan")
    accepted_frac_at_0p05: float = float("nan")    # share whose predicted error is <= 0.05
    accepted_p99_abs_lnT: float = float("nan")     # actual error of those, 99th percentile
    err_head_log10_scale: float = 0.0              # calibration added to output 1 (log10 of the error)
    calibration: tuple = ()                        # (tol, accepted share, p99 actual error) on the report half


def draw_training_problems(m: int, n: int, seed: int, nmat: int = 16384):
    """Limits U[-6,6], correlations of random SPD matrices (Wishart, unit
    diagonal), dof U[2,30]: the training distribution of the network."""
    from cfust_inputs import draw_mvt_problems
    rng = np.random.default_rng(seed)
    return draw_mvt_problems(rng, m, n, nmat=min(nmat, max(n, 1)), lim=(-6.0, 6.0), dof=(2.0, 30.0))


def label_problems(m, b, L, idx, nu, design, handle=None, chunk=1 << 18):
    """ln T_m of every problem by the lattice (mixed precision), on the device."""
    from . import device_qmc, CFUST_MIXED
    h = handle or default_handle()
    qmc = device_qmc(design, CFUST_MIXED)
    dev = "cuda"
    Ld = torch.as_tensor(L, device=dev)
    out = torch.empty(b.shape[0], dtype=torch.float64, device=dev)
    for s in range(0, b.shape[0], chunk):
        e = min(b.shape[0], s + chunk)
        _, logp, _ = mvt_cdf_batch(torch.as_tensor(b[s:e], device=dev), Ld, torch.as_tensor(idx[s:e], device=dev),
                                   torch.as_tensor(nu[s:e], device=dev), qmc, handle=h)
        out[s:e] = logp
    return out


def train(m: int, n_train: int, design, epochs: int = 4, batch: int = 4096, lr: float = 2e-3, lam: float = 0.05,
          seed: int = 0, n_val: int = 16384, handle=None, log=print) -> (SurrogateNet, TrainReport):
    h = handle or default_handle()
    dev = "cuda"
    t0 = time.perf_counter()
    b, L, idx, nu = draw_training_problems(m, n_train + n_val, seed)
    lnT = label_problems(m, b, L, idx, nu, design, handle=h)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rows = n_train + n_val
    rows_pad = (rows + 63) // 64 * 64
    X0, inr, base = mvt_features(m, torch.as_tensor(b, device=dev), torch.as_tensor(L, device=dev),
                                 torch.as_tensor(idx, device=dev), torch.as_tensor(nu, device=dev), rows_pad,
                                 handle=h)
    label = ((lnT - base) / RESID_SCALE).to(torch.float32)
    net = SurrogateNet(m, seed=seed + 1, device=dev)
    acts = Activations(batch, dev)
    out = torch.zeros((batch, B.MLP_OUT), dtype=torch.float32, device=dev)
    dout = torch.zeros_like(out)
    loss_sum = torch.zeros(1, dtype=torch.float32, device=dev)
    xb = torch.zeros((batch, B.MLP_IN), dtype=torch.int16, device=dev)
    lb = torch.zeros(batch, dtype=torch.float32, device=dev)
    steps_per_epoch = n_train // batch
    total = max(1, steps_per_epoch * epochs)
    gen = torch.Generator(device=dev).manual_seed(seed + 2)
    last = float("nan")
    k = 0
    for ep in range(epochs):
        perm = torch.randperm(n_train, generator=gen, device=dev)
        acc = torch.zeros(1, dtype=torch.float64, device=dev)
        for s in range(steps_per_epoch):
            sel = perm[s * batch:(s + 1) * batch]
            xb.copy_(X0[sel])
            lb.copy_(label[sel])
            mlp_forward(net, xb, out, acts, handle=h)
            mlp_loss(out, lb, batch, lam, dout, loss_sum, handle=h)
            mlp_backward(net, acts, dout, handle=h)
            rate = lr * 0.5 * (1.0 + math.cos(math.pi * k / total))     # cosine schedule
            mlp_adam(net, rate, handle=h)
            acc += loss_sum
            k += 1
        last = float(acc.item()) / max(1, steps_per_epoch * batch)
        if log:
            log(f"surrogate m={m} epoch {ep + 1}/{epochs} loss {last:.3e}")
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    # held-out evaluation
    vpad = (n_val + 63) // 64 * 64
    xv = torch.zeros((vpad, B.MLP_IN), dtype=torch.int16, device=dev)
    xv[:n_val] = X0[n_train:n_train + n_val]
    ov = torch.zeros((vpad, B.MLP_OUT), dtype=torch.float32, device=dev)
    mlp_forward(net, xv, ov, None, handle=h)
    pred = torch.clamp(base[n_train:n_train + n_val] + ov[:n_val, 0].double() * RESID_SCALE, max=0.0)
    truth = lnT[n_train:n_train + n_val]
    err = (pred - truth).abs().cpu().numpy()
    pe = ov[:n_val, 1].double().cpu().numpy()
    inside = (inr[n_train:n_train + n_val] > 0).cpu().numpy()
    ae = np.log10(err / RESID_SCALE + 1e-6)
    corr = float(np.corrcoef(pe, ae)[0, 1])
    qs = np.quantile(err, [0.5, 0.9, 0.99]).tolist()
    # Calibration of the error head: the E-step accepts an answer when its
    # predicted error RESID_SCALE 10^(o1) is at most tol.  On the first half of
    # the held-out set, the smallest shift of o1 (log10 scale, grid of 0.05)
    # for which the accepted answers' actual error is at most tol at the 99th
    # percentile, for every tol of CALIB_TOLS; it is added to the bias of
    # output 1, and the second half reports the result.
    half = n_val // 2
    shift = calibrate_error_head(pe[:half], err[:half], inside[:half])
    net.b32[B.MLP_LAYERS - 1][1] += float(shift)
    pe = pe + shift
    rows_rep = []
    for tol in CALIB_TOLS:
        acc = (RESID_SCALE * 10.0 ** pe[half:] <= tol) & inside[half:]
        rows_rep.append((tol, float(acc.mean()), float(np.quantile(err[half:][acc], 0.99)) if acc.any() else 0.0))
    acc5 = (RESID_SCALE * 10.0 ** pe[half:] <= 0.05) & inside[half:]
    acc_frac = float(acc5.mean())
    acc_p99 = float(np.quantile(err[half:][acc5], 0.99)) if acc5.any() else float("nan")
    rep = TrainReport(m, n_train, epochs, t1 - t0, t2 - t1, last, float(np.sqrt((err ** 2).mean())),
                      float(err.max()), corr, qs[0], qs[1], qs[2], acc_frac, acc_p99, float(shift), tuple(rows_rep))
    return net, rep


CALIB_TOLS = (0.01, 0.02, 0.05, 0.1)


def calibrate_error_head(pe: np.ndarray, err: np.ndarray, inside: np.ndarray, tols=CALIB_TOLS) -> float:
    """Smallest shift d (a multiple of 0.05, >= 0) of the predicted log10
    error pe such that, for each tol, the answers accepted at tol
    (RESID_SCALE 10^(pe + d) <= tol, inside the training domain) have actual
    error err at most tol at the 99th percentile."""
    for k in range(0, 161):
        d = 0.05 * k
        ok = True
        for tol in tols:
            acc = (RESID_SCALE * 10.0 ** (pe + d) <= tol) & inside
            if acc.sum() >= 1 and np.quantile(err[acc], 0.99) > tol:
                ok = False
                break
        if ok:
            return d
    return 8.0


# ------------------------------------------------------------------- E-step --

def cfust_estep_surrogate(y: torch.Tensor, params, qmc: DeviceQmc, models: Dict[int, SurrogateNet], tol: float,
                          out: Optional[EStepResult] = None, n_fallback: Optional[torch.Tensor] = None,
                          stream=None, handle: Optional[Handle] = None) -> EStepResult:
    """E-step with the surrogate answering T_m (m = 2..4) where its predicted
    error is below ``tol`` (in ln T) and the lattice elsewhere."""
    h = handle or default_handle()
    n = _check_y(y, params.p)
    if out is None:
        out = alloc_estep(n, params.p, params.q, params.g, qmc.precision, y.device)
    keep = {m: net.weights_c() for m, net in models.items()}
    mp = (C.c_void_p * (B.MAX_Q + 1))()
    for m, w in keep.items():
        mp[m] = C.cast(C.pointer(w), C.c_void_p)
    sur = B.SurrogateC(mp, float(tol), None if n_fallback is None else n_fallback.data_ptr())
    pc, oc = params.c(), out.c()
    st = h.lib.cfust_estep_surrogate(h.h, _ptr(y), B.Dims(n, params.p, params.q, params.g), C.byref(pc),
                                     C.byref(qmc.c), C.byref(sur), C.byref(oc), _stream(stream))
    B.check(st, h.h, "cfust_estep_surrogate")
    return out
