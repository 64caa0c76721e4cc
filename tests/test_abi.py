"""The C-ABI library loads on any host and exports every entry point declared in include/pd.h
(no compute calls: those need a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "pd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pd_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ["pd_setup", "pd_apply", "pd_cg_solve", "pd_project_velocity", "pd_step"]:
        assert name in syms


def test_library_exports_every_declared_symbol(pd):
    lib = ctypes.CDLL(pd.LIB_PATH)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    assert sorted(pd.EXPORTED) == declared_symbols()


def test_binding_constants_match_header(pd):
    """Every enumerator of include/pd.h (PD_... = value) has the same value in the binding."""
    src = open(os.path.join(ROOT, "include", "pd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    consts = dict((k, int(v)) for k, v in re.findall(r"\b(PD_[A-Z0-9_]+)\s*=\s*(-?\d+)", src))
    assert "PD_CFG_DEFER_X" in consts and "PD_BCFG_CHUNK" in consts
    wrong = {k: (v, getattr(pd, k, None)) for k, v in consts.items() if getattr(pd, k, None) != v}
    assert not wrong, wrong


def test_setup_rejects_bad_arguments_without_touching_the_device(pd):
    import pytest
    for args in [(4, (4, 4), (1.0, 1.0), 2, 1e-3, 0.6, 0.0),      # dim
                 (2, (0, 4), (1.0, 1.0), 2, 1e-3, 0.6, 0.0),      # cells
                 (2, (4, 4), (1.0, 1.0), 9, 1e-3, 0.6, 0.0),      # N
                 (2, (4, 4), (1.0, 1.0), 2, -1.0, 0.6, 0.0),      # dt
                 (2, (4, 4), (1.0, 1.0), 2, 1e-3, 0.3, 0.0)]:     # theta
        with pytest.raises(pd.PdError) as e:
            pd.pd_setup(*args, stream=0)
        assert e.value.code == pd.PD_EINVAL
    # periodic_mask bits at or above dim (clear bits below dim are Dirichlet walls)
    with pytest.raises(pd.PdError) as e:
        pd.pd_setup(2, (4, 4), (1.0, 1.0), 2, 1e-3, 0.6, 0.0, periodic_mask=0b111, stream=0)
    assert e.value.code == pd.PD_EINVAL


def test_host_tables_match_oracle(pd):
    """The library's host-built FP64 tables (nodes, weights, pressure blocks and the null-space
    projector the solves use) equal the oracle's for every degree. Odd degrees have a
    two-dimensional cell-periodic kernel; for N = 1, R~ - L~ vanishes identically, so the
    projector is the identity."""
    import numpy as np
    from oracle.basis import tables
    from oracle.operators import null_basis_dirichlet, null_basis_tiled
    for N in range(9):
        t = tables(N)
        n = N + 1
        got = {w: np.array(pd.pd_table_1d(N, w)) for w in range(7)}
        assert np.abs(got[pd.PD_TAB_NODES] - t.xi).max() <= 1e-15
        assert np.abs(got[pd.PD_TAB_WEIGHTS] - t.w).max() <= 1e-15
        for which, blk in ((pd.PD_TAB_L, t.Lblk), (pd.PD_TAB_C, t.Cblk), (pd.PD_TAB_R, t.Rblk)):
            assert np.abs(got[which].reshape(n, n) - blk).max() <= 1e-11 * np.abs(blk).max()
        Z = null_basis_tiled(1, N)
        assert np.abs(got[pd.PD_TAB_PNULL].reshape(n, n) - Z @ Z.T).max() <= 1e-12
        assert round(float(np.trace(got[pd.PD_TAB_PNULL].reshape(n, n)))) == (1 if N % 2 == 0 else 2)
        # the 1D null space along a Dirichlet direction: the odd part of that kernel
        Zo = null_basis_dirichlet(1, N)
        podd = np.array(pd.pd_table_1d(N, pd.PD_TAB_PNULL_ODD)).reshape(n, n)
        assert np.abs(podd - Zo @ Zo.T).max() <= 1e-12
        assert round(float(np.trace(podd))) == (0 if N % 2 == 0 else 1)
    import pytest
    with pytest.raises(pd.PdError):
        pd.pd_table_1d(9, 0)


def test_host_time_tables_match_oracle(pd):
    """The library's host-built time tables of the space-time step (nodes, weights, psi(0),
    psi(1), MV of eq. tmatrix3 and the inverse of At = M1 - MV) equal the oracle's for M = 0..4."""
    import numpy as np
    from oracle.spacetime import TimeTables
    for M in range(5):
        t = TimeTables(M)
        m = M + 1
        got = {w: np.array(pd.pd_time_table(M, w)) for w in range(6)}
        assert np.abs(got[pd.PD_TTAB_NODES] - t.tau).max() <= 1e-15
        assert np.abs(got[pd.PD_TTAB_WEIGHTS] - t.omega).max() <= 1e-15
        assert np.abs(got[pd.PD_TTAB_PSI0] - t.psi0).max() <= 1e-13
        assert np.abs(got[pd.PD_TTAB_PSI1] - t.psi1).max() <= 1e-13
        assert np.abs(got[pd.PD_TTAB_MV].reshape(m, m) - t.MV).max() <= 1e-12
        assert np.abs(got[pd.PD_TTAB_AINV].reshape(m, m) - np.linalg.inv(t.At)).max() <= 1e-12
    import pytest
    with pytest.raises(pd.PdError):
        pd.pd_time_table(5, 0)
