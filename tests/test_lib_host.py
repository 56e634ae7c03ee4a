"""Host-side tests of the library (no GPU): the C ABI loads and exports every declared symbol, and
the library's own setup (Kronecker assembly, ILUT, transfers, exact p = 1 solve, schedules)
agrees with the independently written oracle."""
import ctypes as C

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import paper_2107_05337_amd as pm


def host_solver(p, n, domain=0, Nt=16, kappa=1.0, T=0.1, m=4, trsv_block=-1, **kw):
    prob = pm.problem(p, n, Nt, kappa=kappa, T=T, domain=domain)
    so = pm.default_solver_opts(trsv_block=trsv_block, **kw)
    mo = pm.default_mgrit_opts(cfactor=m, coarsest_max=2)
    return pm.Solver([prob], mo, so, device=-1)


def test_exports_every_declared_symbol():
    names = pm.header_functions()
    assert "pmgrit_create" in names and "pmgrit_solve_mgrit" in names and len(names) >= 20
    L = C.CDLL(pm.LIB_PATH)
    for nm in names:
        assert hasattr(L, nm), nm


@pytest.mark.parametrize("p,n,domain", [(2, 5, 0), (3, 6, 0), (5, 4, 0), (2, 6, 1), (4, 5, 1)])
def test_assembly_matches_oracle(p, n, domain):
    S = host_solver(p, n, domain)
    P = O.Problem(p, n, domain)
    for name in ("M", "K", "P", "M1", "K1"):
        A = S.host_matrix(name).toarray()
        B = P.dense(name)
        assert A.shape == B.shape, name
        # same sparsity pattern (tensor-product support overlap)
        assert np.array_equal(S.host_matrix(name).nnz, P.scipy(name).nnz), name
        assert np.abs(A - B).max() <= 1e-13 * np.abs(B).max(), name
    v = S.host_vectors()
    mlp, ml1 = P.lumped()
    assert np.allclose(v["mlp"], mlp, rtol=1e-13)
    assert np.allclose(v["ml1"], ml1, rtol=1e-13)


def test_level_operator_and_ilut_match_oracle():
    p, n, Nt, T, kappa = 3, 8, 64, 0.1, 1.0
    S = host_solver(p, n, 0, Nt=Nt, kappa=kappa, T=T, m=4)
    P = O.Problem(p, n, 0)
    for level in (0, 1):
        dt = T / Nt * 4 ** level
        A = S.host_matrix("A", level=level)
        Ao = P.scipy("M") + kappa * dt * P.scipy("K")
        assert abs(A - Ao).max() <= 1e-13 * abs(Ao).max()
        L, U = S.host_matrix("L", level=level), S.host_matrix("U", level=level)
        rc, Lo, Uo = P.ilut(kappa * dt, tau=1e-12)
        assert rc == 0
        # identical definition (same caps, drop rule and tie order): same pattern, values to rounding
        assert L.nnz == Lo.nnz and U.nnz == Uo.nnz
        assert (abs(L - Lo) > 1e-10 * abs(Lo).max()).nnz == 0
        assert (abs(U - Uo) > 1e-10 * abs(Uo).max()).nnz == 0


@pytest.mark.parametrize("domain", [0, 1])
def test_sources_and_projection_match_oracle(domain):
    p, n = 3, 7
    S = host_solver(p, n, domain)
    P = O.Problem(p, n, domain)
    modes = [(1, 1, 2.0), (2, 3, -0.5), (0, 2, 0.25)]
    S.set_source(0, modes, 0)
    S.set_initial_modes(0, [(1, 2, 1.5)])
    v = S.host_vectors()
    Fo = P.load_vector(modes)
    assert np.abs(v["load"] - Fo).max() <= 1e-13 * np.abs(Fo).max()
    uo = P.project([(1, 2, 1.5)])
    assert np.abs(v["u0"] - uo).max() <= 1e-11 * np.abs(uo).max()


@pytest.mark.parametrize("domain,level", [(0, 0), (0, 2), (1, 0), (1, 1)])
def test_exact_p1_solve(domain, level):
    p, n, Nt, T, kappa = 2, 9, 64, 0.1, 0.7
    S = host_solver(p, n, domain, Nt=Nt, kappa=kappa, T=T, m=4)
    P = O.Problem(p, n, domain)
    dt = T / Nt * 4 ** level
    A1 = P.dense("M1") + kappa * dt * P.dense("K1")
    b = np.random.default_rng(2).standard_normal(A1.shape[0])
    x = S.host_coarse_solve(b, level=level)
    assert np.allclose(x, np.linalg.solve(A1, b), rtol=1e-11, atol=1e-13)


def _row_levels(T, lower):
    n = T.shape[0]
    lev = np.zeros(n, dtype=int)
    rng = range(n) if lower else range(n - 1, -1, -1)
    for i in rng:
        cols = T.indices[T.indptr[i]:T.indptr[i + 1]]
        cols = cols[cols < i] if lower else cols[cols > i]
        lev[i] = lev[cols].max() + 1 if len(cols) else 0
    return lev.max() + 1


def test_schedules():
    p, n = 3, 12
    S1 = host_solver(p, n, 0, trsv_block=1)
    L, U = S1.host_matrix("L"), S1.host_matrix("U")
    s = S1.host_schedule(factor=0)
    assert s["block_size"] == 1 and s["levels"] == _row_levels(L, True)
    s = S1.host_schedule(factor=1)
    assert s["levels"] == _row_levels(U, False)
    Sl = host_solver(p, n, 0, trsv_block=-1)
    nin = n + p - 2
    for f in (0, 1):
        s = Sl.host_schedule(factor=f)
        assert s["block_size"] == nin and s["blocks"] == nin
        # one grid line per block: lines depend on the previous line only
        assert s["levels"] == nin and s["max_rows"] == nin


@pytest.mark.parametrize("p,n", [(3, 12), (2, 70), (5, 9)])
def test_default_schedule_blocks_of_64_rows(p, n):
    """The default blocking takes 64 consecutive rows per block whatever the grid lines (the whole
    system when it is smaller), placed in dependency order: the level counts match an independent
    greedy placement of the same blocks, and no level holds more than 128 rows."""
    S = host_solver(p, n, 0, trsv_block=0, Nt=8)
    L, U = S.host_matrix("L"), S.host_matrix("U")
    ndof = (n + p - 2) ** 2
    bs = min(64, ndof)
    for f, T, lower in ((0, L, True), (1, U, False)):
        s = S.host_schedule(factor=f)
        assert s["block_size"] == bs and s["blocks"] == (ndof + bs - 1) // bs
        levels, rows = _block_levels(T, lower, bs, 128)
        assert s["levels"] == levels and s["max_rows"] == rows <= 128


def test_invalid_arguments_rejected():
    with pytest.raises(pm.PmgritError) as e:
        host_solver(1, 8)
    assert e.value.code == -1
    with pytest.raises(pm.PmgritError) as e:
        host_solver(2, 8, m=1)
    assert e.value.code == -1
    S = host_solver(2, 6)
    with pytest.raises(pm.PmgritError) as e:
        S.solve_mgrit(outs=[])
    with pytest.raises(pm.PmgritError) as e:
        S.set_source(0, [(-1, 1, 1.0)])
    assert e.value.code == -1


@pytest.mark.parametrize("kw", [dict(lds_mask=-1), dict(lds_mask=32), dict(lds_mask=3, autotune=1),
                                dict(lds_mask=3 | 16, precision=0), dict(lds_mask=7 | 16, precision=1),
                                dict(lds_mask=2 | 16, precision=1), dict(lds_mask=64), dict(lds_mask=2 | 64),
                                dict(lds_mask=1 | 16 | 64, precision=1), dict(lds_mask=1 | 32 | 64),
                                dict(lds_mask=128)])
def test_rejects_invalid_placement(kw):
    """The forced LDS placement is checked at create: in range, not with the autotuner, the
    two-workgroups-per-CU build only in precision 1 with y (and at most d) in LDS, the 8-lane
    builds only with y in LDS and one at a time."""
    with pytest.raises(pm.PmgritError):
        host_solver(3, 6, **kw)


@pytest.mark.parametrize("kw", [dict(lds_mask=3 | 16, precision=1), dict(lds_mask=1 | 16, precision=1),
                                dict(lds_mask=15), dict(lds_mask=1), dict(lds_mask=15 | 64), dict(lds_mask=1 | 64),
                                dict(lds_mask=15 | 32)])
def test_accepts_valid_placement(kw):
    host_solver(3, 6, **kw).close()


def _block_levels(T, lower, bs, cap):
    """Level count of bs-row blocks in dependency order, each at the first level after its
    dependencies with room for its rows (cap rows per level, 0: no cap)."""
    n = T.shape[0]
    nb = (n + bs - 1) // bs
    lev = np.zeros(nb, dtype=int)
    used = []
    for b in (range(nb) if lower else range(nb - 1, -1, -1)):
        r0, r1 = b * bs, min(n, b * bs + bs)
        deps = T.indices[T.indptr[r0]:T.indptr[r1]] // bs
        deps = deps[deps != b]
        lv = lev[deps].max() + 1 if len(deps) else 0
        while cap and lv < len(used) and used[lv] + (r1 - r0) > cap:
            lv += 1
        if lv >= len(used):
            used.extend([0] * (lv + 1 - len(used)))
        used[lv] += r1 - r0
        lev[b] = lv
    return len(used), max(used)


def test_schedule_levels_capped_at_row_slots():
    """Grid lines split into 65-row blocks let the first block of a line run beside the last
    blocks of the previous one: 130 rows, more than the 128 row slots of the prefetched triangular
    solve.  The schedule then moves a block to a later level: at most 128 rows per level, every
    block still after the blocks it depends on (the level count matches an independent greedy
    placement)."""
    p, n, bs = 2, 260, 65
    S = host_solver(p, n, 0, trsv_block=bs, Nt=8)
    L, U = S.host_matrix("L"), S.host_matrix("U")
    for f, T, lower in ((0, L, True), (1, U, False)):
        s = S.host_schedule(factor=f)
        free_levels, free_rows = _block_levels(T, lower, bs, 0)
        assert free_rows > 128  # the uncapped schedule would overflow the row slots
        assert s["max_rows"] <= 128
        assert s["levels"] == _block_levels(T, lower, bs, 128)[0] > free_levels


@pytest.mark.parametrize("kw", [dict(theta=-0.1), dict(theta=1.5), dict(theta=float("nan"))])
def test_rejects_invalid_theta(kw):
    with pytest.raises(pm.PmgritError) as e:
        prob = pm.problem(2, 6, 16, **kw)
        pm.Solver([prob], pm.default_mgrit_opts(), pm.default_solver_opts(), device=-1)
    assert e.value.code == -1


@pytest.mark.parametrize("so,mo", [(dict(solver=2), {}), (dict(coarse=2), {}), (dict(solver=1, precision=1), {}),
                                   (dict(solver=-1), {}), ({}, dict(cycle=3)), ({}, dict(cycle=-1))])
def test_rejects_invalid_solver_variants(so, mo):
    with pytest.raises(pm.PmgritError) as e:
        pm.Solver([pm.problem(2, 6, 16)], pm.default_mgrit_opts(**mo), pm.default_solver_opts(**so), device=-1)
    assert e.value.code == -1


def test_factor_failure_reported():
    """A non-finite operator (kappa dt K overflows) makes the factorisation fail: PMGRIT_E_FACTOR with a
    message, no handle."""
    with pytest.raises(pm.PmgritError) as e:
        host_solver(2, 6, kappa=1e308, T=1.0, Nt=1)
    assert e.value.code == -4
    assert "SPD" in str(e.value) or "pivot" in str(e.value) or "factor" in str(e.value).lower()


@pytest.mark.parametrize("theta", [0.0, 0.5])
def test_theta_level_operator_matches_oracle(theta):
    """A_l = M + theta kappa dt_l K is the operator the library factors (theta-scheme, Sec. 2)"""
    p, n, Nt, T, kappa = 3, 6, 32, 0.1, 0.7
    prob = pm.problem(p, n, Nt, kappa=kappa, T=T, theta=theta)
    S = pm.Solver([prob], pm.default_mgrit_opts(cfactor=4, coarsest_max=2), pm.default_solver_opts(), device=-1)
    P = O.Problem(p, n, 0)
    for level in (0, 1):
        dt = T / Nt * 4 ** level
        A = S.host_matrix("A", level=level)
        Ao = P.scipy("M") + theta * kappa * dt * P.scipy("K")
        assert abs(A - Ao).max() <= 1e-13 * abs(Ao).max()


@pytest.mark.parametrize("precision,bs", [(1, 128), (0, 128)])
def test_window_instances_get_128_row_blocks(precision, bs):
    """An instance whose FP64-sized triangular-solve vector cannot be in LDS (h = 2^-8) is scheduled in
    blocks of 128 rows in either precision (window mode, slab tables), 64 otherwise"""
    S = host_solver(2, 256, Nt=8, trsv_block=0, precision=precision)
    s = S.host_schedule()
    assert s["block_size"] == bs and s["max_rows"] <= 128
    assert host_solver(3, 32, Nt=8, trsv_block=0, precision=precision).host_schedule()["block_size"] == 64
