"""Shared helpers of the GPU tests (comparison metrics, device transfer)."""
import numpy as np


def normrel(a, b, mask=None):
    """Per-field norm-relative difference max|a-b| / max|b| over the compared
    points (pointwise relative error is meaningless where a field crosses 0).
    A field whose reference is identically 0 reports max|a-b| instead."""
    a = np.asarray(a)
    b = np.asarray(b)
    if mask is not None:
        a = a[:, mask]
        b = b[:, mask]
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    d = np.abs(a - b).max(axis=1)
    s = np.abs(b).max(axis=1)
    return np.where(s > 0, d / np.where(s > 0, s, 1.0), d)


def to_dev(u):
    import torch
    return torch.as_tensor(np.ascontiguousarray(u), dtype=torch.float64, device="cuda")


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def pi_mirror_equal(u, parity):
    return np.array_equal(u, u[:, :, ::-1, ::-1] * parity[:, None, None, None])


def ulp_sensitivity(oz, u0, g, dt, nsteps, shell=None, seed=0):
    """Per-field norm-relative change of the ORACLE's own result after
    nsteps when its input is perturbed by one ulp at every point.  Two
    correct float64 implementations that round differently disagree by about
    this much: the stencils amplify ulp-level differences of O(1) fields by
    ~1/h^2, which dominates fields whose own values are tiny (noise-level
    off-diagonal components, a 1e-6 wave)."""
    a = u0.copy()
    oz.rk4(a, g.as_dict(), dt, nsteps, shell=shell)
    b = u0.copy()
    rng = np.random.default_rng(seed)
    b = b + np.spacing(b) * rng.choice([-1.0, 1.0], size=b.shape)
    oz.rk4(b, g.as_dict(), dt, nsteps, shell=shell)
    return a, normrel(b, a)


def assert_state_parity(got, ref, sens, tol=1e-12, factor=20.0):
    """State comparison after time steps: every field within max(tol,
    factor x the oracle's own ulp sensitivity) norm-relative, and within tol
    of the largest state magnitude in absolute terms."""
    e = normrel(got, ref)
    bound = np.maximum(tol, factor * sens)
    scale = np.abs(ref).max()
    absd = np.abs(np.asarray(got) - np.asarray(ref)).reshape(ref.shape[0], -1).max(axis=1)
    print("per-field normrel:", " ".join(f"{x:.1e}" for x in e))
    print("oracle ulp sensitivity:", " ".join(f"{x:.1e}" for x in sens))
    assert np.all(e <= bound), (e, bound)
    assert np.all(absd <= tol * scale), absd
