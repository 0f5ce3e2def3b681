"""GPU parity against the oracle where the earlier tests left holes: the
device's own triplet residuals per triplet, the 64-wide block path the
headline workload runs, exact counts at the headline shape on a
known-spectrum surrogate, mixed precision, and the guards that keep one solve
per context.

Tolerances follow from the arithmetic: residuals are compared per triplet
with a relative slack for summation order only; singular values against exact
or oracle values at 1e-9 (FP64) or 1e-6 (mixed precision, with the residual
target of that mode).
"""
import numpy as np
import pytest

import paper_2109_13655_amd as cs
import synth
from oracle import method, sparse, truth

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-test]", *a, flush=True)


def make_ctx(I):
    return cs.csvd_create(I.m, I.n, I.rowptr, I.colidx, I.vals)


def check_device_residuals(I, sig, U, V, res, normA, rtol=1e-6):
    """The residuals the library reports (k_resid_cols on the device) equal
    the oracle's dense residual definition per triplet (Sec. 4.2,
    max(||A v - s u||, ||A^T u - s v||) / ||A||_2), up to summation order.
    At rounding level the two sums differ by the forward error of a sparse
    product, at most 2 k eps ||A||_F for unit vectors (k the longest row or
    column), which sets the absolute floor."""
    r_host = truth.triplet_residuals(I, sig, U, V, normA=normA)
    assert res.shape == r_host.shape
    k = max(np.diff(I.rowptr).max(), np.bincount(I.colidx, minlength=I.n).max())
    floor = 2.0 * (k + 2) * np.finfo(np.float64).eps * np.linalg.norm(I.vals) / normA
    np.testing.assert_allclose(res, r_host, rtol=rtol, atol=max(floor, 1e-15))
    return r_host


def compare_with_oracle(I, sig, U, V, res, ref, tol_sigma, tol_res, normA):
    """Triplets of the GPU against the oracle's (same count, values, vectors of
    simple values) and the device residuals against the host's."""
    s_o, U_o, V_o = ref
    assert sig.size == s_o.size, (sig, s_o)
    np.testing.assert_allclose(sig, s_o, rtol=tol_sigma, atol=0)
    r_host = check_device_residuals(I, sig, U, V, res, normA)
    assert r_host.max() <= tol_res
    for i in range(sig.size):
        if (i > 0 and sig[i] - sig[i - 1] < 1e-6) or (i + 1 < sig.size and sig[i + 1] - sig[i] < 1e-6):
            continue
        assert abs(abs(V[:, i] @ V_o[:, i]) - 1.0) < 1e-6
        assert abs(abs(U[:, i] @ U_o[:, i]) - 1.0) < 1e-6


def _mid_problem():
    sig = np.linspace(0.02, 1.0, 1100)
    return synth.givens_known(1300, 1100, sigma=sig, nrot=3000, config=85, a=0.40, b=0.41)


@pytest.mark.parametrize("solver", [cs.CSVD_SOLVER_SINGLE, cs.CSVD_SOLVER_BLOCK])
def test_device_residuals_per_triplet_loose_solves(solver):
    """Loose shifted solves (solve_rtol 1e-6) leave triplet residuals far
    above rounding, so a residual kernel that returned zeros, dropped the
    sigma term or took the wrong column would differ from the host's values
    here; the values must agree per triplet."""
    I = _mid_problem()
    V = synth.v_in(I.n, 8, 21)
    ctx = make_ctx(I)
    try:
        p = cs.csvd_params_default(L=8, M=4, N=16, solve_rtol=1e-6, norm_a=1.0, solver=solver)
        st = cs.csvd_solve_interval(ctx, I.a, I.b, p, V)
        assert st == cs.CSVD_OK
        sig, U, Vv, res = cs.csvd_get_triplets(ctx, I.m, I.n)
        info = cs.csvd_get_info(ctx)
    finally:
        cs.csvd_destroy(ctx)
    say("loose solves: solver", info.solver, "t_hat", sig.size, "resid range", res.min(), res.max())
    assert sig.size >= 5 and res.min() > 1e-13
    r_host = check_device_residuals(I, sig, U, Vv, res, 1.0)
    assert info.max_triplet_resid == pytest.approx(r_host.max(), rel=1e-6)
    assert info.svd_sweeps_exhausted == 0


def test_givens_ell2_triplets_against_oracle():
    """The 1200 x 1000 Givens workload (exact sigma, [0.40, 0.45], N = 16,
    L = 16, M = 8, ell = 2) against the oracle's triplets: values, vectors and
    the device's residual per triplet on the 50 strict-interior values.  The
    value 0.45000000000000007 sits on the end b up to rounding (an edge
    value): either side may report it, and where reported it must be exact
    and meet the residual target."""
    I = synth.givens_known()
    V = synth.v_in(I.n, 16, 9)
    ctx = make_ctx(I)
    try:
        p = cs.csvd_params_default(L=16, M=8, N=16, ell=2, norm_a=1.0)
        assert cs.csvd_solve_interval(ctx, I.a, I.b, p, V) == cs.CSVD_OK
        sig, U, Vv, res = cs.csvd_get_triplets(ctx, I.m, I.n)
    finally:
        cs.csvd_destroy(ctx)
    o = method.ss_svd(I, I.a, I.b, V, 16, 8, 16, ell=2)
    band = 1e-12
    core = (sig > I.a + band) & (sig < I.b - band)
    core_o = (o["sigma"] > I.a + band) & (o["sigma"] < I.b - band)
    assert core.sum() == core_o.sum() == 50
    compare_with_oracle(I, sig[core], U[:, core], Vv[:, core], res[core],
                        (o["sigma"][core_o], o["U"][:, core_o], o["V"][:, core_o]), 1e-9, 1e-8, 1.0)
    for s_ in np.concatenate([sig[~core], o["sigma"][~core_o]]):
        assert np.min(np.abs(I.sigma - s_)) <= 1e-9 * s_
    assert check_device_residuals(I, sig, U, Vv, res, 1.0).max() <= 1e-8


def test_block_width_64_against_oracle_and_truth():
    """The 64-wide block path of the headline workload (bs_tall_rg<64>,
    bs_small1<64>, b_shift<64>, b_moments<64>): a random sparse 9216 x 4608
    matrix (10 nonzeros per column) with L = 64, so the automatic choice takes
    the block solver at width 64.  Moments against the oracle's direct
    solves, triplets against the oracle and the dense truth (exact count of
    an interval whose ends sit between eigenvalues)."""
    I = synth.random_sparse(9216, 4608, 10, config=96)
    A = I.dense()
    G = A.T @ A
    ev = np.linalg.eigvalsh(G)
    a, b = synth.interval_by_count(ev, ev.size // 2, 24)
    L, M, N = 64, 4, 16
    V = synth.v_in(I.n, L, 22)
    say("block width 64: n", I.n, "interval", a, b)
    ctx = make_ctx(I)
    try:
        p = cs.csvd_params_default(L=L, M=M, N=N, solve_rtol=1e-12)
        st = cs.csvd_solve_interval(ctx, a, b, p, V)
        info = cs.csvd_get_info(ctx)
        say("steps", info.iterations, "Lp", info.L_padded, "t_hat", info.t_hat, "stored", info.basis_stored)
        assert st == cs.CSVD_OK and info.solver == cs.CSVD_SOLVER_BLOCK and info.L_padded == 64
        Sg = [cs.csvd_get_moment(ctx, k, I.n, L) for k in range(M + 1)]
        sig, U, Vv, res = cs.csvd_get_triplets(ctx, I.m, I.n)
    finally:
        cs.csvd_destroy(ctx)
    o = method.ss_svd(I, a, b, V, L, M, N, G=G)
    ymax = max(np.linalg.norm(o["Y"][j]) for j in range(N // 2))
    for k in range(M + 1):
        scale = 2 * np.abs(o["c"][:, k]).sum() * ymax
        assert np.linalg.norm(Sg[k] - o["S"][k]) <= 1e-9 * scale, k
    s_t, U_t, V_t, sall = truth.dense_truth(I, a, b)
    assert s_t.size == 24
    compare_with_oracle(I, sig, U, Vv, res, (o["sigma"], o["U"], o["V"]), 1e-9, 1e-8, sall[0])
    np.testing.assert_allclose(sig, s_t, rtol=1e-9)
    assert truth.subspace_gap(Vv, V_t) <= 1e-7


def test_headline_shape_known_spectrum_count():
    """Count parity at the headline shape: a 2e5 x 1e5 surrogate with exactly
    known singular values (distributed like the random c2 matrix's, from the
    quantile function of a same-distribution sample) wrapped in two levels of
    random Givens rotations on rows and columns (16 nonzeros per column).
    With the bench's parameters (N = 32, L = 64, M = 8) and an interval whose
    ends sit halfway between neighbouring exact values around 64 values at the
    median, the GPU returns exactly those 64 values to 1e-9, each triplet
    certified by the oracle's host sparse residuals <= 1e-8."""
    m, n = 200000, 100000
    sig_all = synth.sample_spectrum(m, n, 10, config=2)
    I = synth.known_spectrum_sparse(m, n, sig_all, levels=2, config=21)
    lam = np.sort(sig_all ** 2)
    a, b = synth.interval_by_count(lam, lam.size // 2, 64)
    exact = np.sort(sig_all[(sig_all >= a) & (sig_all <= b)])
    assert exact.size == 64
    nA = float(sig_all.max())
    say("surrogate", m, "x", n, "nnz", I.nnz, "interval", a, b)
    ctx = make_ctx(I)
    try:
        p = cs.csvd_params_default(L=64, M=8, N=32, norm_a=nA)
        st = cs.csvd_solve_interval(ctx, a, b, p, synth.v_in(n, 64, 2, 1))
        info = cs.csvd_get_info(ctx)
        say("status", st, "steps", info.iterations, "t_hat", info.t_hat, "max resid", info.max_triplet_resid)
        assert st == cs.CSVD_OK and info.solver == cs.CSVD_SOLVER_BLOCK and info.L_padded == 64
        sig, U, V, res = cs.csvd_get_triplets(ctx, m, n)
    finally:
        cs.csvd_destroy(ctx)
    assert sig.size == 64
    np.testing.assert_allclose(sig, exact, rtol=1e-9)
    r_host = truth.sparse_triplet_residuals(I.rowptr, I.colidx, I.vals, m, n, sig, U, V, nA)
    assert r_host.max() <= 1e-8
    np.testing.assert_allclose(res, r_host, rtol=1e-6, atol=1e-15)
    rows = np.random.default_rng(6).choice(m, 64, replace=False)
    AV = sparse.product_rows(I.rowptr, I.colidx, I.vals, V, rows)
    np.testing.assert_allclose(AV, U[rows] * sig[None, :], rtol=0, atol=1e-8 * nA)


@pytest.mark.parametrize("solver", [cs.CSVD_SOLVER_SINGLE, cs.CSVD_SOLVER_BLOCK])
@pytest.mark.parametrize("transform", [cs.CSVD_PLAIN, cs.CSVD_EXP])
def test_mixed_precision_against_oracle(transform, solver):
    """CSVD_MIXED against the FP64 oracle, on both solvers (the block solver
    with its FP32 stored basis): same count as the oracle and the exact
    spectrum, values to 1e-6 and residuals within the 1e-6 target of that
    mode."""
    I = _mid_problem()
    V = synth.v_in(I.n, 8, 23)
    ctx = make_ctx(I)
    try:
        p = cs.csvd_params_default(L=8, M=4, N=16, ell=2, norm_a=1.0, transform=transform,
                                   precision=cs.CSVD_MIXED, solver=solver)
        st = cs.csvd_solve_interval(ctx, I.a, I.b, p, V)
        info = cs.csvd_get_info(ctx)
        sig, U, Vv, res = cs.csvd_get_triplets(ctx, I.m, I.n)
    finally:
        cs.csvd_destroy(ctx)
    say("mixed: solver", info.solver, "status", st, "t_hat", sig.size, "max resid", res.max() if res.size else None)
    assert st == cs.CSVD_OK and info.solver == solver
    if solver == cs.CSVD_SOLVER_BLOCK:
        assert info.basis_stored == 1
    o = method.ss_svd(I, I.a, I.b, V, 8, 4, 16, ell=2, transform=transform)
    exact = np.sort(I.sigma[(I.sigma >= I.a) & (I.sigma <= I.b)])
    assert sig.size == o["sigma"].size == exact.size
    np.testing.assert_allclose(sig, exact, rtol=1e-6)
    r_host = check_device_residuals(I, sig, U, Vv, res, 1.0)
    assert r_host.max() <= 1e-6


def test_one_live_solve_per_context():
    """A context with a queued server request refuses a second request, a
    solo solve and result reads (CSVD_ESTATE); a batch refuses a context
    listed twice (CSVD_EINVAL).  After the request is done the context is
    usable again and its results are the request's."""
    I = _mid_problem()
    p = cs.csvd_params_default(L=8, M=2, N=16, norm_a=1.0)
    V = synth.v_in(I.n, 8, 24)
    ctx = make_ctx(I)
    srv = cs.csvd_server_create(8 << 30, 2)
    try:
        rid = cs.csvd_server_submit(srv, ctx, I.a, I.b, p, V)
        with pytest.raises(cs.CsvdError) as e:
            cs.csvd_server_submit(srv, ctx, I.a, I.b, p, V)
        assert e.value.code == cs.CSVD_ESTATE
        with pytest.raises(cs.CsvdError) as e:
            cs.csvd_solve_interval(ctx, I.a, I.b, p, V)
        assert e.value.code == cs.CSVD_ESTATE
        with pytest.raises(cs.CsvdError) as e:
            cs.csvd_get_triplets(ctx, I.m, I.n)
        assert e.value.code == cs.CSVD_ESTATE
        with pytest.raises(cs.CsvdError) as e:
            cs.csvd_solve_batch([ctx], [I.a], [I.b], [p], [V])
        assert e.value.code == cs.CSVD_ESTATE
        for _ in range(100000):
            if cs.csvd_server_step(srv, 64) == 0:
                break
        done, st = cs.csvd_server_poll(srv, rid)
        assert done and st == cs.CSVD_OK
        served = cs.csvd_get_triplets(ctx, I.m, I.n)
        assert cs.csvd_solve_interval(ctx, I.a, I.b, p, V) == cs.CSVD_OK
        solo = cs.csvd_get_triplets(ctx, I.m, I.n)
        for x, y in zip(served, solo):
            assert np.array_equal(x, y)
        ctx2 = make_ctx(I)
        try:
            with pytest.raises(cs.CsvdError) as e:
                cs.csvd_solve_batch([ctx2, ctx2], [I.a, I.a], [I.b, I.b], [p, p], [V, V])
            assert e.value.code == cs.CSVD_EINVAL
        finally:
            cs.csvd_destroy(ctx2)
    finally:
        cs.csvd_server_destroy(srv)
        cs.csvd_destroy(ctx)


def test_block_mixed_stored_basis_and_its_fallback():
    """The block solver in mixed precision on the 64-wide path (random sparse
    9216 x 4608, L = 64): the dense truth's count and values to 1e-9 and
    residuals below the 1e-6 target of mixed precision.  Here the basis (112
    blocks of 64 for n = 4608) is far from orthogonal, the moments from its
    FP32 copies miss the target (1.8e-6 measured), and the FP64 refinement
    (moments again from the basis regenerated in FP64) makes the result the
    FP64 solver's.  Capping the stored basis (keep_basis = 40) sends the
    solve to the FP64 ring and a second pass after 40 blocks: the FP64
    solver's result without a stored basis, bit for bit."""
    I = synth.random_sparse(9216, 4608, 10, config=96)
    A = I.dense()
    ev = np.linalg.eigvalsh(A.T @ A)
    a, b = synth.interval_by_count(ev, ev.size // 2, 24)
    s_t, U_t, V_t, sall = truth.dense_truth(I, a, b)
    V = synth.v_in(I.n, 64, 25)
    ctx = make_ctx(I)
    try:
        out = {}
        for name, prec, keep in (("mixed", cs.CSVD_MIXED, 1), ("mixed_cap", cs.CSVD_MIXED, 40),
                                 ("fp64_ring", cs.CSVD_FP64, 0)):
            p = cs.csvd_params_default(L=64, M=4, N=16, precision=prec, keep_basis=keep)
            st = cs.csvd_solve_interval(ctx, a, b, p, V)
            info = cs.csvd_get_info(ctx)
            say(name, "status", st, "steps", info.iterations, "stored", info.basis_stored, "t_hat", info.t_hat,
                "max resid", info.max_triplet_resid)
            assert st == cs.CSVD_OK and info.solver == cs.CSVD_SOLVER_BLOCK and info.L_padded == 64
            assert info.basis_stored == (name == "mixed")
            if name == "mixed":
                refined = info.mixed_refined
            out[name] = cs.csvd_get_triplets(ctx, I.m, I.n) + (cs.csvd_get_moment(ctx, 1, I.n, 64),)
    finally:
        cs.csvd_destroy(ctx)
    sig, U, Vv, res, _ = out["mixed"]
    assert sig.size == s_t.size == 24
    np.testing.assert_allclose(sig, s_t, rtol=1e-9)
    r_host = check_device_residuals(I, sig, U, Vv, res, sall[0])
    assert r_host.max() <= 1e-6
    if refined:
        for x, y in zip(out["mixed"], out["fp64_ring"]):
            assert np.array_equal(x, y)
    for x, y in zip(out["mixed_cap"], out["fp64_ring"]):
        assert np.array_equal(x, y)


def test_wide_block_as_column_groups():
    """L = 80 > 64 on the block solver: two independent column groups (64 and
    16 columns) stepped together in one engine.  Each group's moments are
    bit for bit those of a solo solve on its own columns (the moments are
    linear in the right-hand side, column by column), and the triplets match
    the oracle with L = 80 and the dense truth."""
    I = synth.random_sparse(9216, 4608, 10, config=96)
    A = I.dense()
    G = A.T @ A
    ev = np.linalg.eigvalsh(G)
    a, b = synth.interval_by_count(ev, ev.size // 2, 24)
    L, M, N = 80, 4, 16
    V = synth.v_in(I.n, L, 26)
    ctx = make_ctx(I)
    try:
        p = cs.csvd_params_default(L=L, M=M, N=N, solve_rtol=1e-12)
        st = cs.csvd_solve_interval(ctx, a, b, p, V)
        info = cs.csvd_get_info(ctx)
        say("L = 80: groups", info.column_groups, "steps", info.iterations, "t_hat", info.t_hat)
        assert st == cs.CSVD_OK and info.solver == cs.CSVD_SOLVER_BLOCK and info.column_groups == 2
        Sw = [cs.csvd_get_moment(ctx, k, I.n, L) for k in range(M + 1)]
        sig, U, Vv, res = cs.csvd_get_triplets(ctx, I.m, I.n)
        for lo, hi in ((0, 64), (64, 80)):
            ps = cs.csvd_params_default(L=hi - lo, M=M, N=N, solve_rtol=1e-12)
            assert cs.csvd_solve_interval(ctx, a, b, ps, np.asfortranarray(V[:, lo:hi])) == cs.CSVD_OK
            for k in range(M + 1):
                assert np.array_equal(cs.csvd_get_moment(ctx, k, I.n, hi - lo), Sw[k][:, lo:hi]), (lo, k)
    finally:
        cs.csvd_destroy(ctx)
    o = method.ss_svd(I, a, b, V, L, M, N, G=G)
    s_t, U_t, V_t, sall = truth.dense_truth(I, a, b)
    compare_with_oracle(I, sig, U, Vv, res, (o["sigma"], o["U"], o["V"]), 1e-9, 1e-8, sall[0])
    np.testing.assert_allclose(sig, s_t, rtol=1e-9)


def _long_row_matrix():
    """Zipf(1.8) row lengths (up to 400 nonzeros per row) plus six dense-ish
    columns (300 nonzeros each): rows of A and of A^T longer than the
    128-nonzero segment length of the block products."""
    import scipy.sparse as sp
    m, n = 8192, 4096
    Z = synth.zipf_rows(m, n, kmax=400, config=97)
    rng = np.random.default_rng(np.random.SeedSequence([2109, 13655, 97, 1]))
    rows = np.concatenate([rng.choice(m, 300, replace=False) for _ in range(6)])
    cols = np.repeat(rng.choice(n, 6, replace=False), 300)
    D = sp.csr_matrix((rng.standard_normal(rows.size), (rows, cols)), shape=(m, n))
    A = (Z.scipy() + D).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return synth.Instance(m, n, A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.astype(np.float64),
                          name="zipf_long_rows")


def test_block_long_rows_against_oracle():
    """Rows with more than 128 nonzeros in A (Zipf lengths up to 2000) and in
    A^T (dense-ish columns) are summed from 128-nonzero segments in a fixed
    order: the block solver's moments match the oracle's direct solves and
    its triplets the dense truth (exact count of an interval whose ends sit
    between eigenvalues).  The interval sits at the 85% point of the
    spectrum: the long rows stretch the spectrum to about 4e2 and the block
    solves around its median need more steps than the solver's cap at this
    small n."""
    I = _long_row_matrix()
    rl, cl = np.diff(I.rowptr), np.bincount(I.colidx, minlength=I.n)
    assert rl.max() > 300 and (rl > 128).sum() > 20 and (cl > 128).sum() >= 6
    A = I.dense()
    G = A.T @ A
    ev = np.linalg.eigvalsh(G)
    a, b = synth.interval_by_count(ev, int(0.85 * ev.size), 12)
    L, M, N = 32, 4, 16
    V = synth.v_in(I.n, L, 27)
    say("long rows: max row", rl.max(), "long rows", (rl > 128).sum(), "long cols", (cl > 128).sum())
    ctx = make_ctx(I)
    try:
        p = cs.csvd_params_default(L=L, M=M, N=N, solve_rtol=1e-12)
        st = cs.csvd_solve_interval(ctx, a, b, p, V)
        info = cs.csvd_get_info(ctx)
        say("steps", info.iterations, "t_hat", info.t_hat)
        assert st == cs.CSVD_OK and info.solver == cs.CSVD_SOLVER_BLOCK and info.L_padded == 32
        Sg = [cs.csvd_get_moment(ctx, k, I.n, L) for k in range(M + 1)]
        sig, U, Vv, res = cs.csvd_get_triplets(ctx, I.m, I.n)
    finally:
        cs.csvd_destroy(ctx)
    o = method.ss_svd(I, a, b, V, L, M, N, G=G)
    ymax = max(np.linalg.norm(o["Y"][j]) for j in range(N // 2))
    for k in range(M + 1):
        scale = 2 * np.abs(o["c"][:, k]).sum() * ymax
        assert np.linalg.norm(Sg[k] - o["S"][k]) <= 1e-9 * scale, k
    s_t, U_t, V_t, sall = truth.dense_truth(I, a, b)
    assert s_t.size == 12
    compare_with_oracle(I, sig, U, Vv, res, (o["sigma"], o["U"], o["V"]), 1e-9, 1e-8, sall[0])
    np.testing.assert_allclose(sig, s_t, rtol=1e-9)


@pytest.mark.parametrize("kind,transform,L,solver", [(1, cs.CSVD_PLAIN, 14, cs.CSVD_SOLVER_SINGLE),
                                                     (2, cs.CSVD_EXP, 10, cs.CSVD_SOLVER_SINGLE),
                                                     (0, cs.CSVD_PLAIN, 8, cs.CSVD_SOLVER_BLOCK)])
def test_residual_estimates_against_oracle(kind, transform, L, solver):
    """Sec. 3.4.1 on the device: the residual estimates from the moments
    (eq. residual; eq. res_nonlinear with mu from the largest computed
    residual) against the oracle's, on deliberately small subspaces whose
    residuals sit far above the solve accuracy (model problems 1 and 2 of
    Sec. 4.2 with N = 16; the 1300 x 1100 Givens matrix with M = 2 on the
    block solver)."""
    from oracle import quadrature as Q
    if kind:
        I = synth.model_problem(kind)
        nA, M, N = float(I.sigma[0]), 4, 16
    else:
        I = _mid_problem()
        nA, M, N = 1.0, 2, 16
    V = synth.v_in(I.n, L, 9)
    ctx = make_ctx(I)
    try:
        p = cs.csvd_params_default(L=L, M=M, N=N, transform=transform, norm_a=nA, solve_rtol=1e-13, solver=solver)
        st = cs.csvd_solve_interval(ctx, I.a, I.b, p, V)
        assert st == cs.CSVD_OK
        sig, U, Vv, res = cs.csvd_get_triplets(ctx, I.m, I.n)
        est = cs.csvd_get_residual_estimates(ctx, sig.size)
    finally:
        cs.csvd_destroy(ctx)
    o = method.ss_svd(I, I.a, I.b, V, L, M, N, transform=Q.EXP if transform == cs.CSVD_EXP else Q.PLAIN)
    assert sig.size == o["sigma"].size and sig.size >= 5
    np.testing.assert_allclose(sig, o["sigma"], rtol=1e-6)
    A = I.dense()
    exact_o = np.linalg.norm(A.T @ o["U"] - o["V"] * o["sigma"], axis=0)
    ref = o["resid_est"] if transform == cs.CSVD_PLAIN else method.nt_mu(o["resid_est"], exact_o) * o["resid_est"]
    say("residual estimates: kind", kind, "gpu", est.min(), est.max(), "oracle", (ref / nA).min(), (ref / nA).max())
    assert (ref / nA).min() > 1e-9  # far above the solve accuracy
    np.testing.assert_allclose(est, ref / nA, rtol=1e-4)
    if transform == cs.CSVD_PLAIN:  # eq. residual is exact for Alg. 1 (Prop. 1)
        exact = np.linalg.norm(A.T @ U - Vv * sig, axis=0) / nA
        np.testing.assert_allclose(est, exact, rtol=1e-4)


def test_resid_target_drops_and_reports():
    """resid_target: triplets whose residual exceeds it are not returned, the
    rest are exactly those of the solve without a target (same values, same
    vectors, same order), csvd_info.dropped counts the others and the status
    is CSVD_ENOTCONV.  Loose shifted solves spread the residuals so that a
    target between them splits the set."""
    I = _mid_problem()
    V = synth.v_in(I.n, 8, 21)
    ctx = make_ctx(I)
    try:
        p = cs.csvd_params_default(L=8, M=4, N=16, solve_rtol=1e-6, norm_a=1.0)
        assert cs.csvd_solve_interval(ctx, I.a, I.b, p, V) == cs.CSVD_OK
        full = cs.csvd_get_triplets(ctx, I.m, I.n)
        target = float(np.median(full[3]))
        p.resid_target = target
        st = cs.csvd_solve_interval(ctx, I.a, I.b, p, V)
        info = cs.csvd_get_info(ctx)
        kept = cs.csvd_get_triplets(ctx, I.m, I.n)
    finally:
        cs.csvd_destroy(ctx)
    keep = full[3] <= target
    say("resid_target", target, "kept", keep.sum(), "of", keep.size, "dropped", info.dropped)
    assert 0 < keep.sum() < keep.size
    assert st == cs.CSVD_ENOTCONV and info.dropped == keep.size - keep.sum() and info.t_hat == keep.sum()
    assert np.array_equal(kept[0], full[0][keep]) and np.array_equal(kept[3], full[3][keep])
    assert np.array_equal(kept[1], full[1][:, keep]) and np.array_equal(kept[2], full[2][:, keep])
    assert info.max_triplet_resid <= target


def test_step_graph_replays_equal_eager_steps():
    """The block steps replayed from the captured step graph
    (CSVD_STEP_GRAPH=1: the kernels read the step clock from device memory)
    give the same bits as eager launches: moments and triplets, alone and
    batched."""
    import os
    I = _mid_problem()
    V = synth.v_in(I.n, 8, 12)
    probs = [(synth.random_sparse(m, m // 2, 8, config=98, instance=i), i) for i, m in enumerate((3000, 4400))]
    out = {}
    for mode in ("graph", "eager"):
        if mode == "graph":
            os.environ["CSVD_STEP_GRAPH"] = "1"
        try:
            ctx = make_ctx(I)
            try:
                p = cs.csvd_params_default(L=8, M=4, N=16, norm_a=1.0, solver=cs.CSVD_SOLVER_BLOCK)
                assert cs.csvd_solve_interval(ctx, I.a, I.b, p, V) == cs.CSVD_OK
                res = list(cs.csvd_get_triplets(ctx, I.m, I.n)) + [cs.csvd_get_moment(ctx, k, I.n, 8) for k in range(5)]
            finally:
                cs.csvd_destroy(ctx)
            ctxs = [make_ctx(J) for J, _ in probs]
            try:
                ev = [np.linalg.eigvalsh(J.dense().T @ J.dense()) for J, _ in probs]
                ab = [synth.interval_by_count(e, e.size // 2, 6) for e in ev]
                pb = [cs.csvd_params_default(L=16, M=4, N=16, solver=cs.CSVD_SOLVER_BLOCK) for _ in probs]
                st = cs.csvd_solve_batch(ctxs, [x[0] for x in ab], [x[1] for x in ab], pb,
                                         [synth.v_in(J.n, 16, 13, i) for J, i in probs])
                assert all(x == cs.CSVD_OK for x in st)
                for c, (J, _) in zip(ctxs, probs):
                    res += list(cs.csvd_get_triplets(c, J.m, J.n))
            finally:
                for c in ctxs:
                    cs.csvd_destroy(c)
        finally:
            os.environ.pop("CSVD_STEP_GRAPH", None)
        out[mode] = res
    for x, y in zip(out["graph"], out["eager"]):
        assert np.array_equal(x, y)


def test_served_results_against_oracle():
    """Requests of different sizes served together (continuous batching,
    budgeted admission, stored bases where the budget allows) against the
    oracle's direct solves: same count, values to 1e-9, vectors and the
    device residuals per triplet."""
    specs = [(2400, 1200, 8, 5, 0), (3400, 1700, 16, 8, 1), (1800, 900, 8, 4, 2)]
    probs = []
    for m, n, L, cnt, i in specs:
        I = synth.random_sparse(m, n, 12, config=99, instance=i)
        A = I.dense()
        G = A.T @ A
        ev = np.linalg.eigvalsh(G)
        a, b = synth.interval_by_count(ev, ev.size // 2, cnt)
        probs.append((I, G, a, b, L, synth.v_in(n, L, 28, i)))
    ctxs = [make_ctx(P[0]) for P in probs]
    srv = cs.csvd_server_create(8 << 30, 3)
    try:
        reqs = [cs.csvd_server_submit(srv, c, a, b, cs.csvd_params_default(L=L, M=4, N=16, solve_rtol=1e-12), V)
                for c, (I, G, a, b, L, V) in zip(ctxs, probs)]
        for _ in range(100000):
            if cs.csvd_server_step(srv, 64) == 0:
                break
        for r in reqs:
            done, st = cs.csvd_server_poll(srv, r)
            assert done and st == cs.CSVD_OK
        for c, (I, G, a, b, L, V) in zip(ctxs, probs):
            sig, U, Vv, res = cs.csvd_get_triplets(c, I.m, I.n)
            o = method.ss_svd(I, a, b, V, L, 4, 16, G=G)
            s_t, _, _, sall = truth.dense_truth(I, a, b)
            say("served n", I.n, "t_hat", sig.size, "oracle", o["sigma"].size, "truth", s_t.size)
            compare_with_oracle(I, sig, U, Vv, res, (o["sigma"], o["U"], o["V"]), 1e-9, 1e-8, sall[0])
    finally:
        cs.csvd_server_destroy(srv)
        for c in ctxs:
            cs.csvd_destroy(c)


def test_block_nearly_invariant_start():
    """A second round starts from the filtered block of the first, which is
    nearly invariant: its new Krylov blocks are about 1e-8 of the products
    they come from, so the second projection must act on the explicitly
    projected block (with the two projections combined the moments carried
    errors near 1e-8 and the triplets 6e-8 on this problem), and a warm
    start (ell = 1 from the oracle's exact filtered block, as many values in
    the interval as columns) needs Householder QR for its first steps (with
    Cholesky QR: 7.5e-8).  Both against the exact values and the FP64
    residual target."""
    I, t = synth.batch_pool(count=8)[7]
    A = I.dense()
    G = A.T @ A
    # the interval of the batched workload: about t values near the median,
    # read off a same-distribution sample (here 32 values for t = 31)
    k = max(1, int(round(I.nnz / I.n)))
    a, b, _, _ = synth.interval_from_sample(I.m, I.n, k, t, scale=max(1, I.n // 1000), config=3)
    s_t, _, _, sall = truth.dense_truth(I, a, b)
    V = synth.v_in(I.n, 32, 3, 7)
    sh, c = method.Q.moment_coeffs(a, b, 16, 4, 0.1, method.Q.PLAIN)
    R = method.moment_sums(method.shifted_solves(G, sh, V), c[:, :1])[0]
    ctx = make_ctx(I)
    try:
        for name, ell, Vin in (("ell 2", 2, V), ("warm start", 1, np.ascontiguousarray(R))):
            p = cs.csvd_params_default(L=32, M=4, N=16, ell=ell, solver=cs.CSVD_SOLVER_BLOCK)
            st = cs.csvd_solve_interval(ctx, a, b, p, Vin)
            sig, U, Vv, res = cs.csvd_get_triplets(ctx, I.m, I.n)
            info = cs.csvd_get_info(ctx)
            say(name, "status", st, "steps", info.iterations_total, "t_hat", sig.size, "max resid", res.max())
            assert st == cs.CSVD_OK
            assert sig.size == s_t.size
            np.testing.assert_allclose(sig, s_t, rtol=1e-9, atol=0)
            r_host = check_device_residuals(I, sig, U, Vv, res, sall[0])
            assert r_host.max() <= 1e-8
    finally:
        cs.csvd_destroy(ctx)


def test_block_rank_deficient_starting_block():
    """A starting block with a repeated and a zero column is numerically rank
    deficient: the first steps take Householder QR (the rank test on B_0),
    the repeated column's moments equal its twin's and the zero column's are
    zero, and moments and triplets match the oracle's direct solves from the
    same block and the exact spectrum."""
    I = synth.random_sparse(4000, 2000, 10, config=97)
    A = I.dense()
    G = A.T @ A
    ev = np.linalg.eigvalsh(G)
    a, b = synth.interval_by_count(ev, ev.size // 2, 12)
    L, M, N = 16, 4, 16
    V = synth.v_in(I.n, L, 23)
    V[:, 5] = V[:, 3]
    V[:, 9] = 0.0
    ctx = make_ctx(I)
    try:
        p = cs.csvd_params_default(L=L, M=M, N=N, solve_rtol=1e-12, solver=cs.CSVD_SOLVER_BLOCK)
        st = cs.csvd_solve_interval(ctx, a, b, p, V)
        info = cs.csvd_get_info(ctx)
        say("rank-deficient start: status", st, cs.csvd_last_error(ctx), "steps", info.iterations, "deflated",
            info.deflated, "t_hat", info.t_hat, "converged", info.converged, "sweeps", info.svd_sweeps_exhausted)
        assert st == cs.CSVD_OK and info.solver == cs.CSVD_SOLVER_BLOCK
        Sg = [cs.csvd_get_moment(ctx, k, I.n, L) for k in range(M + 1)]
        sig, U, Vv, res = cs.csvd_get_triplets(ctx, I.m, I.n)
    finally:
        cs.csvd_destroy(ctx)
    o = method.ss_svd(I, a, b, V, L, M, N, G=G)
    ymax = max(np.linalg.norm(o["Y"][j]) for j in range(N // 2))
    for k in range(M + 1):
        scale = 2 * np.abs(o["c"][:, k]).sum() * ymax
        assert np.linalg.norm(Sg[k] - o["S"][k]) <= 1e-9 * scale, k
        assert np.linalg.norm(Sg[k][:, 5] - Sg[k][:, 3]) <= 1e-9 * scale, k
        assert np.linalg.norm(Sg[k][:, 9]) <= 1e-12 * scale, k
    s_t, U_t, V_t, sall = truth.dense_truth(I, a, b)
    assert s_t.size == 12
    compare_with_oracle(I, sig, U, Vv, res, (o["sigma"], o["U"], o["V"]), 1e-9, 1e-8, sall[0])
    np.testing.assert_allclose(sig, s_t, rtol=1e-9)
