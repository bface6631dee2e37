"""FP64 CPU oracle for the CFUST E-step / M-step -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the bench's CPU-baseline leg may import
this package.  The product library never calls it.  The arithmetic lives in
``cfust_oracle.c`` (plain C, FP64, OpenMP over observations); this module
compiles it with gcc and wraps it with ctypes + numpy.

Array layouts follow the library boundary: outputs are [g][.][rows]
structure-of-arrays; e3 holds the packed upper triangle of each q x q matrix.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cfust_oracle.c")
_LIB = os.path.join(_HERE, "libcfust_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-fno-fast-math", "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = C.CDLL(_LIB)
        d, i, pd, pi = C.c_double, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int32)
        lib.or_digamma.restype = d; lib.or_digamma.argtypes = [d]
        lib.or_betai.restype = d; lib.or_betai.argtypes = [d, d, d]
        lib.or_tcdf.restype = d; lib.or_tcdf.argtypes = [d, d]
        lib.or_tinv.restype = d; lib.or_tinv.argtypes = [d, d]
        lib.or_t1pdf.restype = d; lib.or_t1pdf.argtypes = [d, d, d]
        lib.or_mvt_c.restype = d
        lib.or_mvt_c.argtypes = [i, pd, pd, d, i, i, pi, pd, pd]
        lib.or_tmoments_c.restype = None
        lib.or_tmoments_c.argtypes = [i, pd, pd, d, i, i, pi, pd, pd, pd, pd, pd]
        lib.or_estep.restype = i
        lib.or_estep.argtypes = [i, i, i, i, pd, pd, pd, pd, pd, pd, i, i, pi, pd, pi, i, i,
                                 pd, pd, pd, pd, pd, pd, pd, pd, pd]
        lib.or_mvt_mom_c.restype = None
        lib.or_mvt_mom_c.argtypes = [i, pd, pd, d, i, i, pi, pd, pd, pd, pd]
        lib.or_mstep.restype = i
        lib.or_mstep.argtypes = [i, i, i, i, pd, pd, pd, pd, pd, pd, pd, pd, pd, pd, pd,
                                 pd, pd, pd, pd, pd, pi]
        lib.or_set_threads.restype = None; lib.or_set_threads.argtypes = [i]
        lib.or_get_threads.restype = i; lib.or_get_threads.argtypes = []
        _lib = lib
    return _lib


def _pd(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _pi(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32)) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def set_threads(n: int) -> None:
    _load().or_set_threads(int(n))


def get_threads() -> int:
    return int(_load().or_get_threads())


# -- special functions --------------------------------------------------------
def digamma(x):
    f = _load().or_digamma
    return np.vectorize(lambda v: f(float(v)))(x)


def betai(a, b, x):
    f = _load().or_betai
    return np.vectorize(lambda aa, bb, xx: f(float(aa), float(bb), float(xx)))(a, b, x)


def tcdf(t, nu):
    f = _load().or_tcdf
    return np.vectorize(lambda tt, nn: f(float(tt), float(nn)))(t, nu)


def tinv(p, nu):
    f = _load().or_tinv
    return np.vectorize(lambda pp, nn: f(float(pp), float(nn)))(p, nu)


def t1pdf(x, s, nu):
    f = _load().or_t1pdf
    return np.vectorize(lambda xx, ss, nn: f(float(xx), float(ss), float(nn)))(x, s, nu)


# -- multivariate t CDF and truncated moments ----------------------------------
def _design(design):
    z = np.ascontiguousarray(design.z, dtype=np.int32)
    sh = _f64(design.shifts)
    return int(design.N), int(design.S), z, sh


def mvt(b, L, nu, design):
    """T_m(b; 0, L L^T, nu) by the SOV lattice rule.  Returns (estimate, stderr)."""
    b = _f64(b); L = _f64(L)
    m = b.shape[0]
    N, S, z, sh = _design(design)
    se = np.zeros(1)
    v = _load().or_mvt_c(m, _pd(b), _pd(L), float(nu), N, S, _pi(z), _pd(sh), _pd(se))
    return v, float(se[0])


def tmoments(a, R, nu, design):
    """(M0, M1, M2, T2) of Z ~ t_m(0,R,nu) on {Z <= a}; see cfust_oracle.c."""
    a = _f64(a); R = _f64(R)
    m = a.shape[0]
    N, S, z, sh = _design(design)
    M0 = np.zeros(1); M1 = np.zeros(m); M2 = np.zeros((m, m)); T2 = np.zeros(1)
    _load().or_tmoments_c(m, _pd(a), _pd(R), float(nu), N, S, _pi(z), _pd(sh),
                          _pd(M0), _pd(M1), _pd(M2), _pd(T2))
    return float(M0[0]), M1, M2, float(T2[0])


def mvt_moments(b, L, nu, design):
    """Direct SOV moments of Z ~ t_m(0, L L^T, nu) on {Z <= b}: (P, M1 [m],
    M2 [m][m]) = lattice means of f, f z, f z z^T with every coordinate drawn."""
    b = _f64(b); L = _f64(L)
    m = b.shape[0]
    N, S, z, sh = _design(design)
    P = np.zeros(1); M1 = np.zeros(m); M2 = np.zeros((m, m))
    _load().or_mvt_mom_c(m, _pd(b), _pd(L), float(nu), N, S, _pi(z), _pd(sh), _pd(P), _pd(M1), _pd(M2))
    return float(P[0]), M1, M2


# -- E-step / M-step ------------------------------------------------------------
@dataclass
class EStepOut:
    tau: np.ndarray        # [g][r]
    logf_obs: np.ndarray   # [r]
    logf_comp: np.ndarray  # [g][r]
    w: np.ndarray          # [g][r]
    e1: np.ndarray         # [g][r]
    e2: np.ndarray         # [g][q][r]
    e3: np.ndarray         # [g][q(q+1)/2][r]
    A: np.ndarray          # [g][r] density CDF
    B: np.ndarray          # [g][r] w-numerator CDF

    @property
    def loglik(self) -> float:
        return float(self.logf_obs.sum())


def estep(y, params, design, rows=None, moments: str = "identity") -> EStepOut:
    """Oracle E-step.  y: [n][p] float64.  rows: optional subset of observations.
    moments: "identity" (truncated-t moments from the gradient identity, with
    the lower-dimensional T_{q-1}, T_{q-2}) or "direct" (lattice means of f z,
    f z z^T inside the B integral; q >= 2, q = 1 keeps the closed forms)."""
    if moments not in ("identity", "direct"):
        raise ValueError(f"moments = {moments!r}")
    y = _f64(y)
    n, p = y.shape
    g, q = params.g, params.q
    N, S, z, sh = _design(design)
    if rows is not None:
        rows = np.ascontiguousarray(rows, dtype=np.int32)
        r = rows.shape[0]
    else:
        r = n
    nq2 = q * (q + 1) // 2
    out = EStepOut(*(np.zeros(s) for s in [(g, r), (r,), (g, r), (g, r), (g, r), (g, q, r),
                                           (g, nq2, r), (g, r), (g, r)]))
    st = _load().or_estep(n, p, q, g, _pd(y), _pd(_f64(params.pi)), _pd(_f64(params.mu)),
                          _pd(_f64(params.Sigma)), _pd(_f64(params.Delta)), _pd(_f64(params.nu)),
                          N, S, _pi(z), _pd(sh), _pi(rows), r, 1 if moments == "direct" else 0,
                          _pd(out.tau), _pd(out.logf_obs), _pd(out.logf_comp), _pd(out.w),
                          _pd(out.e1), _pd(out.e2), _pd(out.e3), _pd(out.A), _pd(out.B))
    if st != 0:
        raise ValueError(f"oracle E-step: component {-st - 1} has a non-SPD Omega or Lambda")
    return out


def mstep(y, es: EStepOut, params):
    """Oracle M-step (eqs. 18-22).  Returns (Params, frozen_mask)."""
    from cfust_inputs import Params
    y = _f64(y)
    n, p = y.shape
    g, q = params.g, params.q
    out = Params(np.zeros(g), np.zeros((g, p)), np.zeros((g, p, p)), np.zeros((g, p, q)), np.zeros(g))
    frozen = np.zeros(1, dtype=np.int32)
    st = _load().or_mstep(n, p, q, g, _pd(y), _pd(_f64(es.tau)), _pd(_f64(es.w)), _pd(_f64(es.e1)),
                          _pd(_f64(es.e2)), _pd(_f64(es.e3)), _pd(_f64(params.pi)), _pd(_f64(params.mu)),
                          _pd(_f64(params.Sigma)), _pd(_f64(params.Delta)), _pd(_f64(params.nu)),
                          _pd(out.pi), _pd(out.mu), _pd(out.Sigma), _pd(out.Delta), _pd(out.nu),
                          _pi(frozen))
    if st != 0:
        raise ValueError(f"oracle M-step: component {-st - 1} produced a non-SPD matrix")
    return out, int(frozen[0])


def loglik(y, params, design) -> float:
    return estep(y, params, design).loglik


def aitken_iterations(trace, tol: float) -> int:
    """Number of EM iterations (E-steps) after which Aitken's criterion of
    Sec. 3.4 stops a fit whose log-likelihoods are trace[0], trace[1], ...

    With l^(k+1) the newest value: a^(k) = (l^(k+1) - l^(k)) / (l^(k) -
    l^(k-1)) (eq. 26), l_inf^(k+1) = l^(k) + (l^(k+1) - l^(k)) / (1 - a^(k))
    (eq. 25), stop when |l_inf^(k+1) - l^(k+1)| < tol (eq. 24), which needs
    three values.  Readings where the formulas are undefined: an unchanged
    log-likelihood stops (a is 0/0; the iteration has reached a fixed point);
    l^(k) = l^(k-1) with a change after it gives a = +-inf and l_inf = l^(k);
    a = 1 gives an infinite l_inf (no stop); a non-finite value stops.
    tol <= 0 never stops on the criterion."""
    t = np.asarray(trace, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        for k in range(len(t)):
            l1 = t[k]
            if not np.isfinite(l1):
                return k + 1
            if k >= 1 and l1 == t[k - 1]:
                return k + 1
            if k >= 2 and tol > 0:
                l0, lm = t[k - 1], t[k - 2]
                d1, d0 = l1 - l0, l0 - lm
                if d0 == 0.0:
                    gap = abs(d1)
                else:
                    a = np.float64(d1) / np.float64(d0)
                    linf = l0 + np.float64(d1) / (np.float64(1.0) - a)
                    gap = abs(linf - l1)
                if gap < tol:
                    return k + 1
    return len(t)
