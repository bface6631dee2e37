"""Helpers shared by the GPU parity tests (not collected by pytest)."""
import numpy as np

# Tolerances: log-density per observation (absolute), tau (absolute), e-terms
# relative to each entry's natural scale (see compare_estep), on pairs with
# tau > 1e-8.
TOL = {
    "fp64": dict(logf=1e-6, tau=1e-9, eterm=1e-8),
    "mixed": dict(logf=1e-4, tau=1e-5, eterm=1e-3),
}


def rel_err(a, b, floor=1.0):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.abs(a - b) / np.maximum(np.abs(b), floor)


def compare_estep(gpu, ora, mode, rows=None, label="", tol=None):
    """Element-wise comparison of a GPU E-step (torch tensors) with the oracle
    (tolerances TOL[mode], or the dict ``tol``)."""
    t = tol or TOL[mode]
    sel = (lambda x: x[..., rows]) if rows is not None else (lambda x: x)
    lf_g = sel(gpu.logf_obs.cpu().numpy())
    d_lf = np.abs(lf_g - ora.logf_obs)
    assert np.all(np.isfinite(lf_g)), label
    assert d_lf.max() <= t["logf"], f"{label} max |dlogf| = {d_lf.max():.3e}"
    tau_g = sel(gpu.tau.cpu().numpy())
    assert np.abs(tau_g - ora.tau).max() <= t["tau"], f"{label} tau err {np.abs(tau_g - ora.tau).max():.3e}"
    mask = ora.tau > 1e-8
    q = ora.e2.shape[1]
    iu = np.triu_indices(q)
    diag = np.array([k for k, (i, j) in enumerate(zip(*iu)) if i == j])
    e3d = np.abs(ora.e3[:, diag, :])                    # [g][q][n] = w E[U_i^2]
    # natural scale of each entry: |e1| floored at 1, w; for e2_i the RMS
    # sqrt(w e3_ii); for e3_ik (Cauchy-Schwarz) sqrt(e3_ii e3_kk)
    scales = {
        "w": np.abs(ora.w),
        "e1": np.maximum(np.abs(ora.e1), 1.0),
        "e2": np.maximum(np.abs(ora.e2), np.sqrt(np.abs(ora.w)[:, None, :] * e3d)),
        "e3": np.sqrt(e3d[:, iu[0], :] * e3d[:, iu[1], :]),
    }
    for name in ("w", "e1", "e2", "e3"):
        g = sel(getattr(gpu, name).cpu().numpy().astype(np.float64))
        o = getattr(ora, name)
        m = mask if g.ndim == 2 else mask[:, None, :]
        m = np.broadcast_to(m, o.shape)
        err = (np.abs(g - o) / np.maximum(scales[name], 1e-300))[m]
        if err.size:
            assert err.max() <= t["eterm"], f"{label} {name} max scaled err {err.max():.3e}"
    return d_lf.max()
