"""The convergence-factor harness on the CPU, with oracle-built hierarchies.

These tests check the harness itself (it is what the GPU check relies on):
the Arnoldi spectral-radius estimate against a dense eigensolver, the
Galerkin coarse operators, and that the two-level and multilevel V(1,1)
iterations built from the oracle converge on the 32x32 problem.  The absolute
convergence factors are not the paper's (its are for DG matrices) and are not
pinned.
"""
import numpy as np
import scipy.sparse as sp

from paper_2307_00229_amd import problems as P

from . import _vcycle as V


def test_arnoldi_rho_matches_dense_eigenvalues():
    p = P.cfg1()
    A = p.scipy()
    M = sp.diags(1.0 / A.diagonal()) @ A
    ref = np.max(np.abs(np.linalg.eigvals(M.toarray())))
    est = V.arnoldi_rho(M, steps=15)
    # 15 Arnoldi steps: Ritz values approach the extreme eigenvalue from inside
    assert 0.9 * ref <= est <= ref * (1 + 1e-12), (est, ref)


def test_cf_grid_matches_generator_rule():
    assert np.array_equal(V.cf_grid((32, 32), 2), P.cfg1().cf)
    assert np.array_equal(V.cf_grid((7, 5, 3), 2), P.cf_every_k((7, 5, 3), 2))


def test_galerkin_coarse_operator_shape_and_injection():
    p = P.cfg1()
    lev = V.build_hierarchy(p.scipy(), (32, 32), 2, p.ell, V.oracle_builder(), max_levels=2)
    A1 = lev[1].A
    assert A1.shape == (256, 256)
    # R and P inject the C-points: (R A P)_cc couples to the fine C-block
    R, Pm = lev[0].R, lev[0].P
    C = np.nonzero(p.cf)[0]
    assert np.allclose(R[:, C].toarray(), np.eye(256))
    assert np.allclose(Pm[C, :].toarray(), np.eye(256))


def test_two_level_and_vcycle_converge_on_32x32():
    p = P.cfg1()
    two = V.build_hierarchy(p.scipy(), (32, 32), 2, p.ell, V.oracle_builder(), max_levels=2)
    g2 = V.convergence_factor(two)
    multi = V.build_hierarchy(p.scipy(), (32, 32), 2, p.ell, V.oracle_builder(), min_coarse=16)
    gm = V.convergence_factor(multi)
    assert len(multi) >= 3
    assert 0.0 < g2 < 1.0 and 0.0 < gm < 1.0, (g2, gm)
    # deterministic: the same hierarchy gives the same factor
    assert V.convergence_factor(two) == g2
