"""MI355X (gfx950) CFUST mixture E-step / M-step.

Thin PyTorch-facing wrappers with the names of the C ABI (include/cfust.h):
``cfust_estep``, ``cfust_mstep``, ``cfust_loglik``, ``mvt_cdf_batch``.
Tensors live on the GPU; the wrappers only marshal pointers, sizes and the
current HIP stream.  See Lee, Leemaqz & McLachlan, "A simple multithreaded
implementation of the EM algorithm for mixture models", Secs. 2-3, for the
quantities computed.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Optional

import torch

from . import _binding as B
from ._binding import CFUST_FP64, CFUST_MIXED, LATTICE_DIM

__all__ = ["Handle", "DeviceParams", "DeviceQmc", "EStepResult", "cfust_estep", "cfust_estep_noalloc", "cfust_mstep",
           "cfust_loglik", "mvt_cdf_batch", "CFUST_FP64", "CFUST_MIXED", "default_handle",
           "device_params", "device_qmc", "decode_status"]


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _need(t: torch.Tensor, dtype, name: str, shape=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


class Handle:
    """Owns a cfust_handle (workspace) bound to one device."""

    def __init__(self, device: int = 0):
        self.lib = B.load()
        self.device = device
        h = C.c_void_p()
        st = self.lib.cfust_create(C.byref(h), int(device))
        B.check(st, None, "cfust_create")
        self.h = h

    def reserve(self, n, p, q, g, qmc: "DeviceQmc" = None):
        st = self.lib.cfust_reserve(self.h, B.Dims(n, p, q, g), C.byref(qmc.c) if qmc else None)
        B.check(st, self.h, "cfust_reserve")

    def autotune(self, y: torch.Tensor, params: "DeviceParams", qmc: "DeviceQmc", stream=None):
        """Time the lattice-kernel variants for these shapes and cache the fastest.
        Returns {m: points_per_lane}."""
        n = _check_y(y, params.p)
        ch = (C.c_int32 * (B.MAX_Q + 1))()
        pc = params.c()
        st = self.lib.cfust_autotune(self.h, _ptr(y), B.Dims(n, params.p, params.q, params.g), C.byref(pc),
                                     C.byref(qmc.c), ch, _stream(stream))
        B.check(st, self.h, "cfust_autotune")
        return {m: ch[m] for m in range(B.MAX_Q + 1) if ch[m]}

    def profile(self, enable: bool = True):
        """Bracket the lattice kernels with HIP events (see cfust_profile_enable)."""
        B.check(self.lib.cfust_profile_enable(self.h, int(bool(enable))), self.h, "cfust_profile_enable")

    def profile_read(self):
        """{m: (total_ms, launches)} for the lattice kernels recorded since the last read."""
        ms = (C.c_double * (B.MAX_Q + 1))()
        cnt = (C.c_int32 * (B.MAX_Q + 1))()
        B.check(self.lib.cfust_profile_read(self.h, ms, cnt), self.h, "cfust_profile_read")
        return {m: (ms[m], cnt[m]) for m in range(B.MAX_Q + 1) if cnt[m] > 0}

    def close(self):
        if getattr(self, "h", None):
            self.lib.cfust_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default = {}


def default_handle(device: Optional[int] = None) -> Handle:
    dev = torch.cuda.current_device() if device is None else device
    if dev not in _default:
        _default[dev] = Handle(dev)
    return _default[dev]


@dataclass
class DeviceParams:
    """Psi on the device: pi[g], mu[g][p], Sigma[g][p][p], Delta[g][p][q], nu[g] (float64)."""
    pi: torch.Tensor
    mu: torch.Tensor
    Sigma: torch.Tensor
    Delta: torch.Tensor
    nu: torch.Tensor

    @property
    def g(self): return int(self.pi.shape[0])

    @property
    def p(self): return int(self.mu.shape[1])

    @property
    def q(self): return int(self.Delta.shape[2])

    def c(self) -> B.ParamsC:
        for name in ("pi", "mu", "Sigma", "Delta", "nu"):
            _need(getattr(self, name), torch.float64, name)
        return B.ParamsC(self.pi.data_ptr(), self.mu.data_ptr(), self.Sigma.data_ptr(),
                         self.Delta.data_ptr(), self.nu.data_ptr())

    def clone(self) -> "DeviceParams":
        return DeviceParams(*(t.clone() for t in (self.pi, self.mu, self.Sigma, self.Delta, self.nu)))

    def to_host(self):
        return tuple(t.cpu().numpy() for t in (self.pi, self.mu, self.Sigma, self.Delta, self.nu))


def device_params(P, device="cuda") -> DeviceParams:
    """Copy a host parameter set (attributes pi, mu, Sigma, Delta, nu) to the device."""
    f = lambda a: torch.as_tensor(a, dtype=torch.float64).contiguous().to(device)
    return DeviceParams(f(P.pi), f(P.mu), f(P.Sigma), f(P.Delta), f(P.nu))


class DeviceQmc:
    """Lattice rule on the device: N points, S shifts, generating vector z[8], shifts[S][8]."""

    def __init__(self, N: int, S: int, z: torch.Tensor, shifts: torch.Tensor, precision: int):
        self.N, self.S, self.precision = int(N), int(S), int(precision)
        self.z = _need(z, torch.int32, "z", (LATTICE_DIM,))
        self.shifts = _need(shifts, torch.float64, "shifts", (S, LATTICE_DIM))
        self.c = B.QmcC(self.N, self.S, self.z.data_ptr(), self.shifts.data_ptr(), self.precision)

    @property
    def mixed(self) -> bool:
        return self.precision == CFUST_MIXED


def device_qmc(design, precision: int = CFUST_MIXED, device="cuda") -> DeviceQmc:
    """Upload a lattice design (attributes N, S, z, shifts)."""
    z = torch.as_tensor(design.z, dtype=torch.int32).contiguous().to(device)
    sh = torch.as_tensor(design.shifts, dtype=torch.float64).contiguous().to(device)
    return DeviceQmc(design.N, design.S, z, sh, precision)


@dataclass
class EStepResult:
    tau: torch.Tensor        # [g][n] float64
    logf_obs: torch.Tensor   # [n] float64
    loglik: torch.Tensor     # [1] float64
    w: torch.Tensor          # [g][n]        float64 (FP64) / float32 (mixed)
    e1: torch.Tensor         # [g][n]
    e2: torch.Tensor         # [g][q][n]
    e3: torch.Tensor         # [g][q(q+1)/2][n]
    logf_comp: Optional[torch.Tensor] = None
    cdf_stderr: Optional[torch.Tensor] = None
    status: Optional[torch.Tensor] = None
    precision: int = CFUST_FP64

    def c(self) -> B.EstepOutC:
        return B.EstepOutC(*(None if t is None else t.data_ptr() for t in
                             (self.tau, self.logf_obs, self.loglik, self.w, self.e1, self.e2, self.e3,
                              self.logf_comp, self.cdf_stderr, self.status)))


def alloc_estep(n, p, q, g, precision, device="cuda", logf_comp=True, stderr=True) -> EStepResult:
    et = torch.float32 if precision == CFUST_MIXED else torch.float64
    z = lambda *s, dt=torch.float64: torch.zeros(s, dtype=dt, device=device)
    return EStepResult(z(g, n), z(n), z(1), z(g, n, dt=et), z(g, n, dt=et), z(g, q, n, dt=et),
                       z(g, q * (q + 1) // 2, n, dt=et), z(g, n) if logf_comp else None,
                       z(g, n) if stderr else None, torch.zeros(1, dtype=torch.int32, device=device),
                       precision)


def _check_y(y: torch.Tensor, p: int):
    _need(y, torch.float64, "y")
    if y.dim() != 2 or y.shape[0] != p:
        raise ValueError(f"y must be [p][n] with p = {p}, got {tuple(y.shape)}")
    return int(y.shape[1])


def cfust_estep(y: torch.Tensor, params: DeviceParams, qmc: DeviceQmc, out: Optional[EStepResult] = None,
                stream=None, handle: Optional[Handle] = None) -> EStepResult:
    """E-step (Sec. 3.1): tau, w, e1, e2, e3, log f and the log-likelihood.  y: [p][n] float64."""
    h = handle or default_handle()
    n = _check_y(y, params.p)
    if out is None:
        out = alloc_estep(n, params.p, params.q, params.g, qmc.precision, y.device)
    pc, oc = params.c(), out.c()
    st = h.lib.cfust_estep(h.h, _ptr(y), B.Dims(n, params.p, params.q, params.g), C.byref(pc),
                           C.byref(qmc.c), C.byref(oc), _stream(stream))
    B.check(st, h.h, "cfust_estep")
    return out


def cfust_estep_noalloc(y: torch.Tensor, params: DeviceParams, qmc: DeviceQmc, out: EStepResult,
                        stream=None, handle: Optional[Handle] = None) -> EStepResult:
    """cfust_estep with the library's fixed per-device workspace (no device
    allocation inside the call).  ``out`` must be preallocated by the caller."""
    h = handle or default_handle()
    n = _check_y(y, params.p)
    pc, oc = params.c(), out.c()
    st = h.lib.cfust_estep_noalloc(h.h, _ptr(y), B.Dims(n, params.p, params.q, params.g), C.byref(pc),
                                   C.byref(qmc.c), C.byref(oc), _stream(stream))
    B.check(st, h.h, "cfust_estep_noalloc")
    return out


def cfust_mstep(y: torch.Tensor, es: EStepResult, params: DeviceParams, out: Optional[DeviceParams] = None,
                status: Optional[torch.Tensor] = None, stream=None, handle: Optional[Handle] = None) -> DeviceParams:
    """M-step (Sec. 3.2, eqs. 18-22).  Returns Psi^(k+1) (``out`` may be ``params``)."""
    h = handle or default_handle()
    n = _check_y(y, params.p)
    if out is None:
        out = DeviceParams(*(torch.empty_like(t) for t in (params.pi, params.mu, params.Sigma,
                                                             params.Delta, params.nu)))
    pin, pout, ec = params.c(), out.c(), es.c()
    st = h.lib.cfust_mstep(h.h, _ptr(y), B.Dims(n, params.p, params.q, params.g), C.byref(ec),
                           int(es.precision), C.byref(pin), C.byref(pout), _ptr(status), _stream(stream))
    B.check(st, h.h, "cfust_mstep")
    return out


def cfust_loglik(y: torch.Tensor, params: DeviceParams, qmc: DeviceQmc, logf_obs: Optional[torch.Tensor] = None,
                 status: Optional[torch.Tensor] = None, stream=None, handle: Optional[Handle] = None):
    """Log-likelihood (eq. 27).  Returns (loglik [1], logf_obs [n] or None)."""
    h = handle or default_handle()
    n = _check_y(y, params.p)
    ll = torch.zeros(1, dtype=torch.float64, device=y.device)
    pc = params.c()
    st = h.lib.cfust_loglik(h.h, _ptr(y), B.Dims(n, params.p, params.q, params.g), C.byref(pc),
                            C.byref(qmc.c), _ptr(ll), _ptr(logf_obs), _ptr(status), _stream(stream))
    B.check(st, h.h, "cfust_loglik")
    return ll, logf_obs


def mvt_cdf_batch(b: torch.Tensor, L: torch.Tensor, mat_idx: torch.Tensor, nu: torch.Tensor, qmc: DeviceQmc,
                  stream=None, handle: Optional[Handle] = None):
    """T_m(b; 0, L L^T, nu) per item.  b [batch][m], L [nmat][m][m], mat_idx [batch] int32,
    nu [batch].  Returns (p, logp, stderr), each [batch] float64."""
    h = handle or default_handle()
    _need(b, torch.float64, "b"); _need(L, torch.float64, "L")
    _need(mat_idx, torch.int32, "mat_idx"); _need(nu, torch.float64, "nu")
    batch, m = int(b.shape[0]), int(b.shape[1])
    if L.dim() != 3 or L.shape[1] != m or L.shape[2] != m:
        raise ValueError("L must be [nmat][m][m]")
    p = torch.empty(batch, dtype=torch.float64, device=b.device)
    logp = torch.empty_like(p)
    se = torch.empty_like(p)
    st = h.lib.mvt_cdf_batch(h.h, m, batch, _ptr(b), _ptr(L), _ptr(mat_idx), int(L.shape[0]), _ptr(nu),
                             C.byref(qmc.c), _ptr(p), _ptr(logp), _ptr(se), _stream(stream))
    B.check(st, h.h, "mvt_cdf_batch")
    return p, logp, se


class Batch:
    """Many independent fits run together (include/cfust.h, "Batches of
    independent fits").  ``fits`` is a list of (y [p][n] float64, DeviceParams,
    EStepResult) on one device; the parameters are updated in place by the
    M-step.  All fits share one lattice rule and precision."""

    def __init__(self, fits, qmc: DeviceQmc, handle: Optional[Handle] = None):
        self.handle = handle or default_handle()
        self.qmc = qmc
        self.fits = list(fits)
        if not 1 <= len(self.fits) <= B.MAX_FITS:
            raise ValueError(f"1 <= number of fits <= {B.MAX_FITS}")
        arr = (B.FitC * len(self.fits))()
        for k, (y, P, es) in enumerate(self.fits):
            n = _check_y(y, P.p)
            if es.precision != qmc.precision:
                raise ValueError(f"fit {k}: E-step outputs of another precision")
            arr[k] = B.FitC(B.Dims(n, P.p, P.q, P.g), _ptr(y), P.c(), es.c(), _ptr(es.status))
        self._arr = arr
        b = C.c_void_p()
        B.check(self.handle.lib.cfust_batch_create(self.handle.h, len(self.fits), arr, C.byref(qmc.c), C.byref(b)),
                self.handle.h, "cfust_batch_create")
        self.b = b

    @property
    def nfits(self) -> int:
        return len(self.fits)

    def estep(self, stream=None):
        B.check(self.handle.lib.cfust_batch_estep(self.b, _stream(stream)), self.handle.h, "cfust_batch_estep")

    def mstep(self, stream=None):
        B.check(self.handle.lib.cfust_batch_mstep(self.b, _stream(stream)), self.handle.h, "cfust_batch_mstep")

    def fit(self, iters: int, tol: float = 0.0, use_graph: bool = True, trace: Optional[torch.Tensor] = None,
            iters_done: Optional[torch.Tensor] = None, stream=None):
        """``iters`` EM iterations with Aitken's stopping rule (Sec. 3.4) at
        tolerance ``tol`` (<= 0: all iterations).  Returns (trace [iters][nfits]
        float64, NaN where a fit had stopped; iters_done [nfits] int32)."""
        dev = self.fits[0][0].device
        if trace is None:
            trace = torch.full((max(iters, 1), self.nfits), float("nan"), dtype=torch.float64, device=dev)
        if iters_done is None:
            iters_done = torch.zeros(self.nfits, dtype=torch.int32, device=dev)
        _need(trace, torch.float64, "trace", (max(iters, 1), self.nfits))
        _need(iters_done, torch.int32, "iters_done", (self.nfits,))
        st = self.handle.lib.cfust_fit_batch(self.b, int(iters), float(tol), 1 if use_graph else 0,
                                             _ptr(trace), _ptr(iters_done), _stream(stream))
        B.check(st, self.handle.h, "cfust_fit_batch")
        return trace, iters_done

    def tune(self, stream=None):
        """Autotune the lattice queues; returns {m: (rows per tile, persistent blocks per
        resident slot (0: one block per tile), points per lane)}."""
        arr = (C.c_int32 * ((B.MAX_Q + 1) * 3))()
        B.check(self.handle.lib.cfust_batch_tune(self.b, arr, _stream(stream)), self.handle.h, "cfust_batch_tune")
        return {m: tuple(arr[3 * m:3 * m + 3]) for m in range(B.MAX_Q + 1) if arr[3 * m] > 0}

    def close(self):
        if getattr(self, "b", None):
            self.handle.lib.cfust_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def initialise(y: torch.Tensor, g: int, q: int, labels: torch.Tensor, qmc: DeviceQmc,
               alphas=(0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9), nu0: float = 10.0, stream=None,
               handle: Optional[Handle] = None):
    """Starting values of Sec. 3.3 (eq. 23, Algorithm 1) over the partitions
    labels [nstarts][n] (int32, device) and the alpha grid.  Returns
    (DeviceParams of the best candidate, loglik [nstarts][nalpha] with -inf
    for invalid candidates, best flat index or -1)."""
    h = handle or default_handle()
    p = int(y.shape[0])
    n = _check_y(y, p)
    _need(labels, torch.int32, "labels")
    nstarts = int(labels.shape[0])
    if labels.dim() != 2 or labels.shape[1] != n:
        raise ValueError("labels must be [nstarts][n]")
    dev = y.device
    best = DeviceParams(torch.zeros(g, dtype=torch.float64, device=dev),
                        torch.zeros((g, p), dtype=torch.float64, device=dev),
                        torch.zeros((g, p, p), dtype=torch.float64, device=dev),
                        torch.zeros((g, p, q), dtype=torch.float64, device=dev),
                        torch.zeros(g, dtype=torch.float64, device=dev))
    al = (C.c_double * len(alphas))(*[float(a) for a in alphas])
    ll = torch.zeros((nstarts, len(alphas)), dtype=torch.float64, device=dev)
    bi = torch.zeros(1, dtype=torch.int32, device=dev)
    bc = best.c()
    st = h.lib.cfust_init(h.h, _ptr(y), B.Dims(n, p, q, g), nstarts, _ptr(labels), len(alphas), al, float(nu0),
                          C.byref(qmc.c), C.byref(bc), _ptr(ll), _ptr(bi), _stream(stream))
    B.check(st, h.h, "cfust_init")
    return best, ll, int(bi.cpu()[0])


def decode_status(word: int):
    return [name for bit, name in B.DEV_BITS.items() if word & bit]
