"""Helpers shared by the GPU parity tests (not collected by pytest)."""
import numpy as np

# Tolerances (the reading of the design notes): log-density per observation,
# tau (absolute), e-terms (relative, on pairs with tau > 1e-8).
TOL = {
    "fp64": dict(logf=1e-6, tau=1e-9, eterm=1e-8),
    "mixed": dict(logf=1e-4, tau=1e-5, eterm=1e-3),
}


def rel_err(a, b, floor=1.0):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.abs(a - b) / np.maximum(np.abs(b), floor)


def compare_estep(gpu, ora, mode, rows=None, label=""):
    """Element-wise comparison of a GPU E-step (torch tensors) with the oracle."""
    t = TOL[mode]
    sel = (lambda x: x[..., rows]) if rows is not None else (lambda x: x)
    lf_g = sel(gpu.logf_obs.cpu().numpy())
    d_lf = np.abs(lf_g - ora.logf_obs)
    assert np.all(np.isfinite(lf_g)), label
    assert d_lf.max() <= t["logf"], f"{label} max |dlogf| = {d_lf.max():.3e}"
    tau_g = sel(gpu.tau.cpu().numpy())
    assert np.abs(tau_g - ora.tau).max() <= t["tau"], f"{label} tau err {np.abs(tau_g - ora.tau).max():.3e}"
    mask = ora.tau > 1e-8
    for name in ("w", "e1", "e2", "e3"):
        g = sel(getattr(gpu, name).cpu().numpy().astype(np.float64))
        o = getattr(ora, name)
        m = mask if g.ndim == 2 else mask[:, None, :]
        m = np.broadcast_to(m, o.shape)
        floor = 1.0 if name == "e1" else 1e-6
        err = rel_err(g, o, floor)[m]
        if err.size:
            assert err.max() <= t["eterm"], f"{label} {name} max rel err {err.max():.3e}"
    return d_lf.max()
