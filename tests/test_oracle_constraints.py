"""Pins of the oracle's constraint monitor (paper Sec. 2.3: Hamiltonian and
momentum constraints, volume-normalised L2 norms), against the ADM
constraints of the same analytic data differentiated exactly by autodiff:
H = R + K^2 - K_ij K^ij and M^i = gamma^ij (D_k K^k_j - d_j K)."""
import numpy as np
import pytest

import analytic as A
from paper_2607_08743_amd import inputs as I


def _errs(oz, prim, centre, sizes=(8, 16), extent=1.0):
    errs, scales = [], []
    for n in sizes:
        g = I.centered_grid(n, extent / n, center=centre, bc=I.BC_COPY)
        u = A.evaluate(A.conformal_state_fn(prim), g)
        ex = A.evaluate(A.adm_constraints_fn(prim), g, only_active=True)[:4]
        c, norms = oz.constraints(u, g.as_dict())
        m = g.active_mask()
        errs.append(np.abs(c - ex)[:, m].max(axis=1))
        scales.append(np.abs(ex)[:, m].max(axis=1))
        # the norm is the volume-normalised L2 norm over the active cells
        np.testing.assert_allclose(norms, np.sqrt((c[:, m] ** 2).mean(axis=1)), rtol=1e-13)
    return np.array(errs), np.array(scales)


def test_generic_data_constraints_converge(oz):
    errs, scales = _errs(oz, A.generic_prim(), (0.3, -0.2, 0.1))
    assert scales[-1].min() > 1e-3  # the data violate both constraints
    assert np.all(errs[0] / errs[1] > 11), errs


@pytest.mark.parametrize("name", ["kerr_schild", "brill_lindquist"])
def test_vacuum_solutions_satisfy_constraints(oz, name):
    if name == "kerr_schild":
        prim, centre = A.kerr_schild_prim(), (3.0, 2.5, 2.0)
    else:
        prim, centre = A.brill_lindquist_prim(), (2.0, 1.0, 0.5)
    errs, scales = _errs(oz, prim, centre)
    assert scales.max() < 1e-12  # the analytic constraints vanish
    H, M = errs[:, 0], errs[:, 1:]
    assert H[0] / H[1] > 11
    if name == "brill_lindquist":
        assert M.max() < 1e-14  # K = 0 and At = 0: M vanishes identically
    else:
        assert np.all(M[0] / M[1] > 11)
