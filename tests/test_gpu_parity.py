"""GPU parity tests: the HIP path (through the C ABI) against the CPU oracle.

Tolerances follow from the arithmetic: a shifted solve stopped at relative
residual rtol has forward error at most ||(zI - A^T A)^{-1}|| * rtol * ||V||
<= rtol ||V|| / Im z; the final triplets are held to the residual targets
(<= 1e-8 relative in FP64) and to the oracle's singular values.
"""
import sys

import numpy as np
import pytest

import paper_2109_13655_amd as cs
import synth
from oracle import method, quadrature as Q, sparse, truth

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-test]", *a, flush=True)


def make_ctx(I):
    return cs.csvd_create(I.m, I.n, I.rowptr, I.colidx, I.vals)


# ------------------------------------------------------------ sparse kernels

@pytest.mark.parametrize("k,dense_rows", [(1, False), (7, False), (64, False), (16, True)])
def test_spmm_matches_definition(k, dense_rows):
    I = synth.random_sparse(3001, 1703, 7, config=80) if not dense_rows else \
        synth.givens_known(400, 300, nrot=900, config=85)
    say("spmm", I.m, I.n, k)
    ctx = make_ctx(I)
    try:
        X = np.asfortranarray(np.random.default_rng(1).standard_normal((I.n, k)))
        Y = cs.csvd_spmm(ctx, 0, X, I.m)
        ref = sparse.product_rows(I.rowptr, I.colidx, I.vals, X, range(I.m))
        np.testing.assert_allclose(Y, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
        Xt = np.asfortranarray(np.random.default_rng(2).standard_normal((I.m, k)))
        Yt = cs.csvd_spmm(ctx, 1, Xt, I.n)
        rpT, ciT, vaT = sparse.transpose(I.m, I.n, I.rowptr, I.colidx, I.vals)
        reft = sparse.product_rows(rpT, ciT, vaT, Xt, range(I.n))
        np.testing.assert_allclose(Yt, reft, rtol=1e-13, atol=1e-13 * np.abs(reft).max())
        # deterministic: a second call is bitwise identical
        assert np.array_equal(Y, cs.csvd_spmm(ctx, 0, X, I.m))
    finally:
        cs.csvd_destroy(ctx)


def test_transpose_bit_exact():
    I = synth.random_sparse(2000, 1500, 9, config=81)
    say("transpose", I.m, I.n)
    ctx = make_ctx(I)
    try:
        rp, ci, va = cs.csvd_get_transpose(ctx, I.n, I.nnz)
        rpo, cio, vao = sparse.transpose(I.m, I.n, I.rowptr, I.colidx, I.vals)
        assert np.array_equal(rp, rpo) and np.array_equal(ci, cio) and np.array_equal(va, vao)
    finally:
        cs.csvd_destroy(ctx)


# ------------------------------------------------------- solves and moments

def _small_problem():
    sig = np.linspace(0.02, 1.0, 250)
    I = synth.givens_known(300, 250, sigma=sig, nrot=700, config=82, a=0.40, b=0.46)
    return I


@pytest.mark.parametrize("transform", [cs.CSVD_PLAIN, cs.CSVD_EXP])
def test_solutions_and_moments_match_oracle(transform):
    I = _small_problem()
    L, M, N = 8, 4, 16
    V = synth.v_in(I.n, L, 3)
    say("solve small", I.m, I.n, "transform", transform)
    ctx = make_ctx(I)
    try:
        p = cs.csvd_params_default(L=L, M=M, N=N, transform=transform, solve_rtol=1e-12, check_solves=1,
                                   solver=cs.CSVD_SOLVER_SINGLE)
        st = cs.csvd_solve_interval(ctx, I.a, I.b, p, V)
        assert st == cs.CSVD_OK
        info = cs.csvd_get_info(ctx)
        assert info.converged == 1 and info.max_solve_resid_true < 1e-10
        S_o, Y_o, shifts, c = method.filtered_moments(I, I.a, I.b, V, M, N, transform=transform)
        vn = np.linalg.norm(V)
        for j in range(N // 2):
            Y = cs.csvd_get_solution(ctx, j, I.n, L)
            bound = 1e-10 * vn / abs(shifts[j].imag)
            assert np.linalg.norm(Y - Y_o[j]) <= bound, (j, np.linalg.norm(Y - Y_o[j]), bound)
        ymax = max(np.linalg.norm(Y_o[j]) for j in range(N // 2))
        for k in range(M + 1):
            Sk = cs.csvd_get_moment(ctx, k, I.n, L)
            scale = 2 * np.abs(c[:, k]).sum() * ymax
            assert np.linalg.norm(Sk - S_o[k]) <= 1e-9 * scale, (k, np.linalg.norm(Sk - S_o[k]), scale)
    finally:
        cs.csvd_destroy(ctx)


def _mid_problem():
    sig = np.linspace(0.02, 1.0, 1100)
    return synth.givens_known(1300, 1100, sigma=sig, nrot=3000, config=85, a=0.40, b=0.41)


@pytest.mark.parametrize("transform", [cs.CSVD_PLAIN, cs.CSVD_EXP])
@pytest.mark.parametrize("L,small", [(8, False), (5, False), (8, True)])
def test_block_moments_match_oracle(transform, L, small):
    """Block solver (one block Lanczos basis for all shifts, two passes):
    moments S_0..S_M against the oracle's direct solves.  L = 5 exercises the
    seeded padding columns (the block is 16 wide).  small = True forces the
    block basis on n = 250, where 16 columns exhaust the space in about 16
    steps and deflation takes over: a looser bound (the automatic choice
    uses the per-column solver there)."""
    I = _small_problem() if small else _mid_problem()
    M, N = 4, 16
    V = synth.v_in(I.n, L, 3)
    say("block moments", transform, L, "n", I.n)
    ctx = make_ctx(I)
    try:
        p = cs.csvd_params_default(L=L, M=M, N=N, transform=transform, solve_rtol=1e-12,
                                   solver=cs.CSVD_SOLVER_BLOCK)
        st = cs.csvd_solve_interval(ctx, I.a, I.b, p, V)
        info = cs.csvd_get_info(ctx)
        say("block steps", info.iterations, "Lp", info.L_padded, "deflated", info.deflated)
        assert st == cs.CSVD_OK and info.solver == cs.CSVD_SOLVER_BLOCK
        S_o, Y_o, shifts, c = method.filtered_moments(I, I.a, I.b, V, M, N, transform=transform)
        ymax = max(np.linalg.norm(Y_o[j]) for j in range(N // 2))
        for k in range(M + 1):
            Sk = cs.csvd_get_moment(ctx, k, I.n, L)
            scale = 2 * np.abs(c[:, k]).sum() * ymax
            bound = (1e-6 if small else 1e-9) * scale
            assert np.linalg.norm(Sk - S_o[k]) <= bound, (k, np.linalg.norm(Sk - S_o[k]), scale)
    finally:
        cs.csvd_destroy(ctx)


@pytest.mark.parametrize("solver", [cs.CSVD_SOLVER_SINGLE, cs.CSVD_SOLVER_BLOCK])
def test_interval_from_zero(solver):
    """a = 0 (allowed for the plain form): the 34 smallest singular values of
    a Givens-wrapped diagonal (exact values known), against the exact values
    and the oracle's dense residuals.  The shifts then lie within 2.5e-3 of
    the origin with imaginary parts near 1.3e-4."""
    sig = np.linspace(0.02, 1.0, 1100)
    I = synth.givens_known(1300, 1100, sigma=sig, nrot=3000, config=93, a=0.0, b=0.05)
    exact = np.sort(I.sigma[(I.sigma >= 0.0) & (I.sigma <= 0.05)])
    ctx = make_ctx(I)
    try:
        p = cs.csvd_params_default(L=16, M=8, N=32, solve_rtol=1e-12, solver=solver)
        st = cs.csvd_solve_interval(ctx, 0.0, 0.05, p, synth.v_in(I.n, 16, 93))
        info = cs.csvd_get_info(ctx)
        s, U, V, r = cs.csvd_get_triplets(ctx, I.m, I.n)
    finally:
        cs.csvd_destroy(ctx)
    say("interval [0, 0.05]: solver", info.solver, "steps", info.iterations, "t_hat", s.size, "exact", exact.size)
    assert st == cs.CSVD_OK and s.size == exact.size == 34
    np.testing.assert_allclose(s, exact, rtol=1e-9)
    res = truth.triplet_residuals(I, s, U, V, normA=1.0)
    assert res.max() <= 1e-8


@pytest.mark.parametrize("solver", [cs.CSVD_SOLVER_SINGLE, cs.CSVD_SOLVER_BLOCK])
def test_top_of_spectrum_and_multiple_value(solver):
    """Two degenerate intervals on a Givens-wrapped diagonal with exact
    values, ends at midpoints between neighbouring values: one ends half a
    spacing past sigma_max = 1 (the 10 largest values), the other holds 0.5 with
    multiplicity 4 and one neighbour on each side.  A multiple value has no
    unique vectors, so its four triplets are compared by the principal angles
    between the computed and the exact subspaces."""
    sig = np.linspace(0.02, 1.0, 1100)
    sig[540:544] = 0.5  # multiplicity 4
    sig = np.sort(sig)[::-1]
    I = synth.givens_known(1300, 1100, sigma=sig, nrot=3000, config=94, a=0.98, b=1.5)
    so = np.sort(I.sigma)
    i5 = int(np.searchsorted(so, 0.5))  # first copy of 0.5
    top = (0.5 * (so[-11] + so[-10]), so[-1] + 0.5 * (so[-1] - so[-2]))
    mult = (0.5 * (so[i5 - 2] + so[i5 - 1]), 0.5 * (so[i5 + 4] + so[i5 + 5]))
    for (a, b), want in ((top, 10), (mult, 6)):
        exact = np.sort(I.sigma[(I.sigma >= a) & (I.sigma <= b)])
        ctx = make_ctx(I)
        try:
            p = cs.csvd_params_default(L=16, M=8, N=32, solve_rtol=1e-12, solver=solver)
            st = cs.csvd_solve_interval(ctx, a, b, p, synth.v_in(I.n, 16, 94))
            s, U, V, r = cs.csvd_get_triplets(ctx, I.m, I.n)
        finally:
            cs.csvd_destroy(ctx)
        say("interval", a, b, "solver", solver, "t_hat", s.size, "exact", exact.size)
        assert st == cs.CSVD_OK and s.size == exact.size == want
        np.testing.assert_allclose(s, exact, rtol=1e-9)
        assert truth.triplet_residuals(I, s, U, V, normA=1.0).max() <= 1e-8
        if want == 6:
            sel = np.nonzero(np.abs(I.sigma - 0.5) < 1e-12)[0]
            mine = np.nonzero(np.abs(s - 0.5) < 1e-9)[0]
            assert sel.size == mine.size == 4
            assert truth.subspace_gap(V[:, mine], I.V[:, sel]) <= 1e-7
            assert truth.subspace_gap(U[:, mine], I.U[:, sel]) <= 1e-7


@pytest.mark.parametrize("solver", [cs.CSVD_SOLVER_BLOCK, cs.CSVD_SOLVER_SINGLE])
def test_wide_interval_end_with_adaptive_rounds(solver):
    """An interval reaching far past sigma_max (b = 1.5 over a spectrum ending
    at 1) sizes the ellipse by [a^2, b^2], so the filter's transition at a is
    wide and one round leaves the value nearest a at 1.0e-8 (block) or 3.4e-8
    (per column).  With ell_adaptive and target 1e-8 a second round runs
    where it is missed, and all ten values end within the target."""
    sig = np.linspace(0.02, 1.0, 1100)
    sig[540:544] = 0.5
    sig = np.sort(sig)[::-1]
    I = synth.givens_known(1300, 1100, sigma=sig, nrot=3000, config=94, a=0.98, b=1.5)
    so = np.sort(I.sigma)
    a, b = 0.5 * (so[-11] + so[-10]), 1.5
    exact = np.sort(I.sigma[(I.sigma >= a) & (I.sigma <= b)])
    ctx = make_ctx(I)
    try:
        p = cs.csvd_params_default(L=16, M=8, N=32, solve_rtol=1e-12, solver=solver, ell=2, ell_adaptive=1,
                                   resid_target=1e-8)
        st = cs.csvd_solve_interval(ctx, a, b, p, synth.v_in(I.n, 16, 94))
        s, U, V, r = cs.csvd_get_triplets(ctx, I.m, I.n)
        info = cs.csvd_get_info(ctx)
    finally:
        cs.csvd_destroy(ctx)
    say("wide interval, solver", solver, "status", st, "rounds", info.rounds, "t_hat", s.size, "resid", r.max())
    assert st == cs.CSVD_OK and info.dropped == 0 and s.size == exact.size == 10
    assert info.rounds == 2 or (solver == cs.CSVD_SOLVER_BLOCK and info.rounds == 1)
    np.testing.assert_allclose(s, exact, rtol=1e-12)
    assert truth.triplet_residuals(I, s, U, V, normA=1.0).max() <= 1e-8


def test_block_and_single_solvers_agree():
    """Both solvers give the same triplets on the same problem."""
    I = _mid_problem()
    V = synth.v_in(I.n, 8, 12)
    ctx = make_ctx(I)
    try:
        out = []
        for solver in (cs.CSVD_SOLVER_BLOCK, cs.CSVD_SOLVER_SINGLE):
            p = cs.csvd_params_default(L=8, M=4, N=16, ell=2, norm_a=1.0, solver=solver)
            st = cs.csvd_solve_interval(ctx, I.a, I.b, p, V)
            info = cs.csvd_get_info(ctx)
            out.append(cs.csvd_get_triplets(ctx, I.m, I.n))
            say("solver", solver, "status", st, "steps", info.iterations, "total", info.iterations_total,
                "converged", info.converged, "deflated", info.deflated, "est", info.max_solve_resid_est,
                "resid", out[-1][3].max() if out[-1][3].size else None)
        (s1, U1, V1, r1), (s2, U2, V2, r2) = out
        assert s1.size == s2.size > 0
        np.testing.assert_allclose(s1, s2, rtol=1e-10)
        assert r1.max() <= 1e-8 and r2.max() <= 1e-8
        for i in range(s1.size):
            assert abs(abs(V1[:, i] @ V2[:, i]) - 1.0) < 1e-8
    finally:
        cs.csvd_destroy(ctx)


def test_block_stored_basis_equals_regenerated():
    """Keeping the block basis in device memory and regenerating it in a
    second pass accumulate the same moments from the same blocks: the bits
    agree.  The basis spans several storage chunks of 64 blocks here.  A cap
    of 40 stored blocks makes the solve start in store mode and move to the
    ring in the middle of pass 1 (Q_{k-1} and Q_k copied over), then
    regenerate the basis: the same bits again."""
    I = _mid_problem()
    V = synth.v_in(I.n, 8, 12)
    ctx = make_ctx(I)
    try:
        out = []
        for keep in (1, 0, 40):
            p = cs.csvd_params_default(L=8, M=4, N=16, ell=2, norm_a=1.0, solver=cs.CSVD_SOLVER_BLOCK,
                                       keep_basis=keep)
            st = cs.csvd_solve_interval(ctx, I.a, I.b, p, V)
            info = cs.csvd_get_info(ctx)
            say("keep_basis", keep, "status", st, "steps", info.iterations, "stored", info.basis_stored)
            assert st == cs.CSVD_OK and info.basis_stored == (keep == 1)
            assert info.iterations > 64  # the last round's basis spans two storage chunks
            out.append(cs.csvd_get_triplets(ctx, I.m, I.n) + (cs.csvd_get_moment(ctx, 0, I.n, 8),))
        # the kept chunks are reused by the next solve, and freed on request
        st = cs.csvd_solve_interval(ctx, I.a, I.b, cs.csvd_params_default(
            L=8, M=4, N=16, ell=2, norm_a=1.0, solver=cs.CSVD_SOLVER_BLOCK), V)
        assert st == cs.CSVD_OK and cs.csvd_get_info(ctx).basis_stored == 1
        out.append(cs.csvd_get_triplets(ctx, I.m, I.n) + (cs.csvd_get_moment(ctx, 0, I.n, 8),))
        cs.csvd_trim(ctx)
        for other in out[1:]:
            for x, y in zip(out[0], other):
                assert np.array_equal(x, y)
    finally:
        cs.csvd_destroy(ctx)


def test_prop1_on_gpu_moments():
    """Proposition 1 on the GPU output: S_k = (A^T A)^k S_0 (plain rule)."""
    I = _small_problem()
    L, M, N = 6, 3, 16
    V = synth.v_in(I.n, L, 4)
    ctx = make_ctx(I)
    try:
        p = cs.csvd_params_default(L=L, M=M, N=N, solve_rtol=1e-13)
        cs.csvd_solve_interval(ctx, I.a, I.b, p, V)
        S0 = cs.csvd_get_moment(ctx, 0, I.n, L)
        X = S0
        for k in range(1, M + 1):
            X = cs.csvd_spmm(ctx, 1, cs.csvd_spmm(ctx, 0, X, I.m), I.n)
            Sk = cs.csvd_get_moment(ctx, k, I.n, L)
            assert np.linalg.norm(Sk - X) <= 1e-8 * np.linalg.norm(X)
    finally:
        cs.csvd_destroy(ctx)


# --------------------------------------------------------- end-to-end triplets

def _compare_triplets(I, sig, U, V, res, ref, tol_sigma, tol_res, normA):
    s_o, U_o, V_o = ref
    assert sig.size == s_o.size, (sig, s_o)
    np.testing.assert_allclose(sig, s_o, rtol=tol_sigma, atol=0)
    assert res.max() <= tol_res
    # independent residual check on the host (FP64, dense)
    r_host = truth.triplet_residuals(I, sig, U, V, normA=normA)
    assert r_host.max() <= tol_res
    for i in range(sig.size):
        if i > 0 and sig[i] - sig[i - 1] < 1e-6:
            continue
        if i + 1 < sig.size and sig[i + 1] - sig[i] < 1e-6:
            continue
        assert abs(abs(V[:, i] @ V_o[:, i]) - 1.0) < 1e-6


def test_givens_1200x1000_ell2():
    """A = G1 D G2 (1200 x 1000, exact sigma), [0.40, 0.45], N=16, L=16, M=8,
    ell=2: the 50 strict-interior triplets (plus the edge value 0.45) at
    residual <= 1e-8, matching the oracle and the exact spectrum."""
    I = synth.givens_known()
    V = synth.v_in(I.n, 16, 9)
    say("givens 1200x1000 ell=2")
    ctx = make_ctx(I)
    try:
        p = cs.csvd_params_default(L=16, M=8, N=16, ell=2, norm_a=1.0)
        st = cs.csvd_solve_interval(ctx, I.a, I.b, p, V)
        assert st == cs.CSVD_OK
        sig, U, Vv, res = cs.csvd_get_triplets(ctx, I.m, I.n)
        info = cs.csvd_get_info(ctx)
        say("iters", info.iterations_total, "rank", info.rank, "t", info.t_hat, "res", info.max_triplet_resid,
            "ms", info.t_total_ms)
        o = method.ss_svd(I, I.a, I.b, V, 16, 8, 16, ell=2)
        core = (sig > I.a + 1e-12) & (sig < I.b - 1e-12)
        core_o = (o["sigma"] > I.a + 1e-12) & (o["sigma"] < I.b - 1e-12)
        assert core.sum() == 50 and core_o.sum() == 50
        exact = np.sort(I.sigma[(I.sigma > I.a + 1e-12) & (I.sigma < I.b - 1e-12)])
        np.testing.assert_allclose(sig[core], exact, rtol=1e-9)
        np.testing.assert_allclose(sig[core], o["sigma"][core_o], rtol=1e-9)
        assert res.max() <= 1e-8
        r_host = truth.triplet_residuals(I, sig, U, Vv, normA=1.0)
        assert r_host.max() <= 1e-8
        for i in np.nonzero(core)[0]:
            j = np.argmin(np.abs(o["sigma"] - sig[i]))
            assert abs(abs(Vv[:, i] @ o["V"][:, j]) - 1.0) < 1e-7
    finally:
        cs.csvd_destroy(ctx)


def _adaptive_params(solver, **kw):
    # N = 8 makes the filter weak, so every round of eq. iter1 gains orders of
    # magnitude on the mid problem (largest residual after one, two and three
    # rounds: the oracle's direct solves 4.0e-5, 3.0e-9, 1.8e-11; the block
    # solver 4.0e-5, 5.9e-9, 1.1e-10)
    return cs.csvd_params_default(L=8, M=4, N=8, norm_a=1.0, solve_rtol=1e-12, solver=solver, **kw)


@pytest.mark.parametrize("solver", [cs.CSVD_SOLVER_BLOCK, cs.CSVD_SOLVER_SINGLE])
def test_adaptive_rounds(solver):
    """ell_adaptive stops after the first round whose triplets all meet
    resid_target: a target met after one round gives the bits of ell = 1;
    1e-7 takes two rounds and 1e-9 three, each matching the oracle's and the
    device's fixed-ell results; with ell = 2 the rounds stop at the cap and
    the triplets above 1e-9 are dropped."""
    I = _mid_problem()
    V = synth.v_in(I.n, 8, 12)
    ctx = make_ctx(I)

    def run(**kw):
        st = cs.csvd_solve_interval(ctx, I.a, I.b, _adaptive_params(solver, **kw), V)
        info = cs.csvd_get_info(ctx)
        trip = cs.csvd_get_triplets(ctx, I.m, I.n)
        say("adaptive", solver, kw, "status", st, "rounds", info.rounds, "t_hat", info.t_hat, "dropped",
            info.dropped, "resid", info.max_triplet_resid)
        return st, info, trip

    try:
        fixed = {}
        for ell in (1, 2, 3):
            st, info, trip = run(ell=ell)
            assert st == cs.CSVD_OK and info.rounds == ell
            fixed[ell] = trip
        st, info, trip = run(ell=3, ell_adaptive=1, resid_target=1e-3)
        assert st == cs.CSVD_OK and info.rounds == 1 and info.dropped == 0
        for x, y in zip(trip, fixed[1]):
            assert np.array_equal(x, y)
        for target, rounds in ((1e-7, 2), (1e-9, 3)):
            st, info, (sig, U, Vv, res) = run(ell=3, ell_adaptive=1, resid_target=target)
            assert st == cs.CSVD_OK and info.rounds == rounds and info.dropped == 0
            assert 0 < res.max() <= target
            o = method.ss_svd(I, I.a, I.b, V, 8, 4, 8, ell=rounds)
            assert sig.size == o["sigma"].size == fixed[rounds][0].size
            np.testing.assert_allclose(sig, o["sigma"], rtol=1e-9)
            np.testing.assert_allclose(sig, fixed[rounds][0], rtol=1e-10)
            assert truth.triplet_residuals(I, sig, U, Vv, normA=1.0).max() <= target
        st, info, (sig, _, _, res) = run(ell=2, ell_adaptive=1, resid_target=1e-9)
        assert info.rounds == 2 and info.dropped >= 1 and st == cs.CSVD_ENOTCONV
        assert sig.size + info.dropped == fixed[2][0].size
        assert res.size == 0 or res.max() <= 1e-9
        with pytest.raises(cs.CsvdError) as e:  # the stop needs a target
            cs.csvd_solve_interval(ctx, I.a, I.b, _adaptive_params(solver, ell=2, ell_adaptive=1), V)
        assert e.value.code == cs.CSVD_EINVAL
    finally:
        cs.csvd_destroy(ctx)


def test_adaptive_rounds_batched_and_served_equal_solo():
    """Problems that stop after one, two and three rounds in one batch, and
    served together, give the bits of their solo solves (a batch runs steps
    3-5 on worker threads and hands a problem that needs another round back
    to the engine)."""
    I = _mid_problem()
    V = synth.v_in(I.n, 8, 12)
    ps = [_adaptive_params(cs.CSVD_SOLVER_BLOCK, ell=3, ell_adaptive=1, resid_target=t) for t in (1e-3, 1e-7, 1e-9)]
    ctxs = [make_ctx(I) for _ in ps]
    srv = None
    try:
        solo = []
        for p in ps:
            assert cs.csvd_solve_interval(ctxs[0], I.a, I.b, p, V) == cs.CSVD_OK
            solo.append((cs.csvd_get_info(ctxs[0]).rounds, cs.csvd_get_triplets(ctxs[0], I.m, I.n)))
        assert [r for r, _ in solo] == [1, 2, 3]

        def check(how):
            for c, (rounds, ref) in zip(ctxs, solo):
                assert cs.csvd_get_info(c).rounds == rounds, how
                for x, y in zip(cs.csvd_get_triplets(c, I.m, I.n), ref):
                    assert np.array_equal(x, y), how

        say("adaptive batch of", len(ps))
        st = cs.csvd_solve_batch(ctxs, [I.a] * 3, [I.b] * 3, ps, [V] * 3)
        assert st == [cs.CSVD_OK] * 3
        check("batched")
        say("adaptive served")
        srv = cs.csvd_server_create(8 << 30, 3)
        reqs = [cs.csvd_server_submit(srv, c, I.a, I.b, p, V) for c, p in zip(ctxs, ps)]
        for _ in range(10000):
            if cs.csvd_server_step(srv, 64) == 0:
                break
        for r in reqs:
            done, s = cs.csvd_server_poll(srv, r)
            assert done and s == cs.CSVD_OK
        check("served")
    finally:
        if srv is not None:
            cs.csvd_server_destroy(srv)
        for c in ctxs:
            cs.csvd_destroy(c)


def test_model1_plain_and_model2_exp():
    """Experiment II model problems with (L,M,N,ell,delta) = (20,4,32,1,1e-20)."""
    for kind, tr in ((1, cs.CSVD_PLAIN), (2, cs.CSVD_EXP)):
        I = synth.model_problem(kind)
        V = synth.v_in(I.n, 20, 9)
        say("model", kind, "transform", tr)
        ctx = make_ctx(I)
        try:
            p = cs.csvd_params_default(L=20, M=4, N=32, transform=tr, norm_a=float(I.sigma[0]), solve_rtol=1e-12)
            cs.csvd_solve_interval(ctx, I.a, I.b, p, V)
            sig, U, Vv, res = cs.csvd_get_triplets(ctx, I.m, I.n)
            o = method.ss_svd(I, I.a, I.b, V, 20, 4, 32, transform=tr)
            ref = truth.dense_truth(I, I.a, I.b)
            # count parity on the strict interior; sigma equal to a or b (model
            # problem 2 has both 1e-3 and 1e-1 in its spectrum) may fall on
            # either side after rounding, so an edge value is only checked
            # against the truth when it is reported
            band = 1e-12
            inner = lambda s_: s_[(s_ > I.a + band * I.b) & (s_ < I.b - band * I.b)]
            assert inner(sig).size == inner(ref[0]).size == inner(o["sigma"]).size
            np.testing.assert_allclose(inner(sig), inner(ref[0]), rtol=1e-9)
            np.testing.assert_allclose(inner(sig), inner(o["sigma"]), rtol=1e-9)
            for s_ in sig:
                assert np.min(np.abs(ref[3] - s_)) <= 1e-9 * s_
            r_host = truth.triplet_residuals(I, sig, U, Vv, normA=I.sigma[0])
            assert r_host.max() <= 1e-8
        finally:
            cs.csvd_destroy(ctx)


@pytest.mark.parametrize("L,M", [(1, 4), (5, 3), (12, 2)])
def test_random_sparse_vs_dense_truth(L, M):
    """Random sparse matrix, ragged L (padding to the next power of two)."""
    I = synth.random_sparse(900, 500, 7, config=83)
    A = I.dense()
    ev = np.linalg.eigvalsh(A.T @ A)
    a, b = synth.interval_by_count(ev, 250, 6)
    s_o, U_o, V_o, sall = truth.dense_truth(I, a, b)
    V = synth.v_in(I.n, L, 5)
    say("random sparse L", L, "M", M)
    ctx = make_ctx(I)
    try:
        p = cs.csvd_params_default(L=L, M=M, N=32, solve_rtol=1e-12)
        cs.csvd_solve_interval(ctx, a, b, p, V)
        sig, U, Vv, res = cs.csvd_get_triplets(ctx, I.m, I.n)
        o = method.ss_svd(I, a, b, V, L, M, 32)
        # the oracle with the same subspace size is the parity target
        assert sig.size == o["sigma"].size
        np.testing.assert_allclose(sig, o["sigma"], rtol=1e-8)
        if o["sigma"].size == s_o.size and np.allclose(o["sigma"], s_o, rtol=1e-10):
            r_host = truth.triplet_residuals(I, sig, U, Vv, normA=sall[0])
            assert r_host.max() <= 1e-8
    finally:
        cs.csvd_destroy(ctx)


@pytest.mark.parametrize("L", [12, 16])
def test_block_random_sparse_vs_dense_truth(L):
    """The automatic choice takes the block basis once n >= 64 x padded L:
    random sparse 4000 x 2048, interval of about 10 values mid-spectrum."""
    I = synth.random_sparse(4000, 2048, 7, config=84)
    A = I.dense()
    ev = np.linalg.eigvalsh(A.T @ A)
    a, b = synth.interval_by_count(ev, 1024, 10)
    s_o, U_o, V_o, sall = truth.dense_truth(I, a, b)
    V = synth.v_in(I.n, L, 6)
    say("block random sparse L", L)
    ctx = make_ctx(I)
    try:
        p = cs.csvd_params_default(L=L, M=4, N=32, solve_rtol=1e-12)
        st = cs.csvd_solve_interval(ctx, a, b, p, V)
        info = cs.csvd_get_info(ctx)
        say("block steps", info.iterations, "deflated", info.deflated)
        assert st == cs.CSVD_OK and info.solver == cs.CSVD_SOLVER_BLOCK
        sig, U, Vv, res = cs.csvd_get_triplets(ctx, I.m, I.n)
        o = method.ss_svd(I, a, b, V, L, 4, 32)
        assert sig.size == o["sigma"].size
        np.testing.assert_allclose(sig, o["sigma"], rtol=1e-9)
        assert o["sigma"].size == s_o.size
        np.testing.assert_allclose(sig, s_o, rtol=1e-9)
        r_host = truth.triplet_residuals(I, sig, U, Vv, normA=sall[0])
        assert r_host.max() <= 1e-8
        assert truth.subspace_gap(Vv, V_o) <= 1e-6
    finally:
        cs.csvd_destroy(ctx)


def test_block_one_and_two_cholqr_passes_agree():
    """A well-conditioned new block takes one Cholesky QR pass (random sparse
    matrices give cond(B_k) close to 1); forcing two passes everywhere gives
    the same triplets to the residual accuracy, and both match dense truth."""
    I = synth.random_sparse(4000, 2048, 7, config=84)
    A = I.dense()
    ev = np.linalg.eigvalsh(A.T @ A)
    a, b = synth.interval_by_count(ev, 1024, 10)
    s_o, U_o, V_o, sall = truth.dense_truth(I, a, b)
    V = synth.v_in(I.n, 16, 6)
    ctx = make_ctx(I)
    try:
        out = []
        for passes in (0, 2):
            p = cs.csvd_params_default(L=16, M=4, N=32, solve_rtol=1e-12, cholqr_passes=passes)
            st = cs.csvd_solve_interval(ctx, a, b, p, V)
            info = cs.csvd_get_info(ctx)
            say("cholqr_passes", passes, "steps", info.iterations, "one-pass steps", info.one_pass_steps)
            assert st == cs.CSVD_OK and info.solver == cs.CSVD_SOLVER_BLOCK
            if passes == 0:
                assert info.one_pass_steps > info.iterations // 2
            else:
                assert info.one_pass_steps == 0
            sig, U, Vv, res = cs.csvd_get_triplets(ctx, I.m, I.n)
            np.testing.assert_allclose(sig, s_o, rtol=1e-9)
            r_host = truth.triplet_residuals(I, sig, U, Vv, normA=sall[0])
            assert r_host.max() <= 1e-8
            assert truth.subspace_gap(Vv, V_o) <= 1e-6
            out.append(sig)
        np.testing.assert_allclose(out[0], out[1], rtol=1e-10)
        with pytest.raises(cs.CsvdError) as e:
            cs.csvd_solve_interval(ctx, a, b, cs.csvd_params_default(L=16, cholqr_passes=1), V)
        assert e.value.code == cs.CSVD_EINVAL
    finally:
        cs.csvd_destroy(ctx)


def test_block_ell2_with_more_columns_than_values():
    """Two rounds with L = 32 columns and 16 values in the interval: the
    second round starts from a filtered block that is numerically rank
    deficient, whose first Krylov blocks are orthonormalised by Householder
    QR.  Matches dense truth and the per-column solver."""
    I = synth.random_sparse(5200, 2600, 9, config=86)
    A = I.dense()
    ev = np.linalg.eigvalsh(A.T @ A)
    a, b = synth.interval_by_count(ev, 1300, 16)
    s_o, U_o, V_o, sall = truth.dense_truth(I, a, b)
    V = synth.v_in(I.n, 32, 9)
    ctx = make_ctx(I)
    try:
        out = []
        for solver in (cs.CSVD_SOLVER_BLOCK, cs.CSVD_SOLVER_SINGLE):
            p = cs.csvd_params_default(L=32, M=4, N=16, ell=2, solver=solver)
            st = cs.csvd_solve_interval(ctx, a, b, p, V)
            info = cs.csvd_get_info(ctx)
            say("ell2 solver", solver, "status", st, "steps", info.iterations, "total", info.iterations_total)
            assert st == cs.CSVD_OK
            sig, U, Vv, res = cs.csvd_get_triplets(ctx, I.m, I.n)
            np.testing.assert_allclose(sig, s_o, rtol=1e-10)
            r_host = truth.triplet_residuals(I, sig, U, Vv, normA=sall[0])
            assert r_host.max() <= 1e-10
            assert truth.subspace_gap(Vv, V_o) <= 1e-7
            out.append(sig)
        np.testing.assert_allclose(out[0], out[1], rtol=1e-11)
    finally:
        cs.csvd_destroy(ctx)


def test_empty_interval_and_determinism():
    I = _small_problem()
    V = synth.v_in(I.n, 4, 6)
    ctx = make_ctx(I)
    try:
        p = cs.csvd_params_default(L=4, M=2, N=16)
        # an interval that holds no singular value (spacing is ~0.004)
        s = np.sort(I.sigma)
        a = s[100] + 1e-4
        b = s[100] + 2e-4
        cs.csvd_solve_interval(ctx, a, b, p, V)
        sig, U, Vv, res = cs.csvd_get_triplets(ctx, I.m, I.n)
        assert sig.size == 0
        # determinism: two solves are bitwise identical
        cs.csvd_solve_interval(ctx, I.a, I.b, p, V)
        r1 = cs.csvd_get_triplets(ctx, I.m, I.n)
        S1 = cs.csvd_get_moment(ctx, 1, I.n, 4)
        cs.csvd_solve_interval(ctx, I.a, I.b, p, V)
        r2 = cs.csvd_get_triplets(ctx, I.m, I.n)
        S2 = cs.csvd_get_moment(ctx, 1, I.n, 4)
        assert np.array_equal(S1, S2)
        for x, y in zip(r1, r2):
            assert np.array_equal(x, y)
    finally:
        cs.csvd_destroy(ctx)


def test_not_converged_status_and_errors():
    I = _small_problem()
    ctx = make_ctx(I)
    try:
        p = cs.csvd_params_default(L=4, M=2, N=16, max_iters=8)
        st = cs.csvd_solve_interval(ctx, I.a, I.b, p, synth.v_in(I.n, 4, 7))
        assert st == cs.CSVD_ENOTCONV
        cs.csvd_get_triplets(ctx, I.m, I.n)      # still readable
        bad = cs.csvd_params_default(L=4, M=2, N=15)
        with pytest.raises(cs.CsvdError) as e:
            cs.csvd_solve_interval(ctx, I.a, I.b, bad)
        assert e.value.code == cs.CSVD_EINVAL
        bad = cs.csvd_params_default(L=4, M=2, N=16, transform=cs.CSVD_EXP)
        with pytest.raises(cs.CsvdError):
            cs.csvd_solve_interval(ctx, 0.0, 0.5, bad)
        with pytest.raises(cs.CsvdError):
            cs.csvd_solve_interval(ctx, 0.5, 0.4, cs.csvd_params_default(L=4, M=2))
        big = cs.csvd_params_default(L=200, M=2)
        with pytest.raises(cs.CsvdError):
            cs.csvd_solve_interval(ctx, I.a, I.b, big)
        with pytest.raises(cs.CsvdError) as e:
            cs.csvd_solve_interval(ctx, I.a, I.b, cs.csvd_params_default(L=4, M=2, N=16, keep_basis=-1))
        assert e.value.code == cs.CSVD_EINVAL
        # the context stays usable after the rejected calls
        assert cs.csvd_solve_interval(ctx, I.a, I.b, cs.csvd_params_default(L=4, M=2, N=16, keep_basis=3)) in (
            cs.CSVD_OK, cs.CSVD_ENOTCONV)
    finally:
        cs.csvd_destroy(ctx)


def test_seeded_vin_uses_counter_generator():
    """V_in = NULL draws from the counter-based SplitMix64/Box-Muller stream;
    the same stream built independently on the host gives identical results."""
    I = _small_problem()
    ctx = make_ctx(I)
    try:
        # the two starting blocks may differ in the last bit, so the moments
        # agree to about the solve tolerance: fix it well below the bound
        p = cs.csvd_params_default(L=4, M=2, N=16, seed=12345, solve_rtol=1e-13)
        cs.csvd_solve_interval(ctx, I.a, I.b, p, None)
        S_a = cs.csvd_get_moment(ctx, 0, I.n, 4)
        V = synth.splitmix_normal(12345, I.n, 4)
        cs.csvd_solve_interval(ctx, I.a, I.b, p, V)
        S_b = cs.csvd_get_moment(ctx, 0, I.n, 4)
        # the two sides share the integer stream exactly; log/cos may differ
        # in the last bit between the host libm and NumPy
        np.testing.assert_allclose(S_a, S_b, rtol=0, atol=1e-12 * np.abs(S_b).max())
        cs.csvd_solve_interval(ctx, I.a, I.b, cs.csvd_params_default(L=4, M=2, N=16, seed=777), None)
        S_c = cs.csvd_get_moment(ctx, 0, I.n, 4)
        assert np.abs(S_c - S_b).max() > 1e-3 * np.abs(S_b).max()
    finally:
        cs.csvd_destroy(ctx)


# ------------------------------------------------------------ batch / serve

def _three_problems():
    out = []
    for i, (m, n) in enumerate([(700, 400), (1100, 600), (500, 300)]):
        I = synth.random_sparse(m, n, 8, config=84, instance=i)
        ev = np.linalg.eigvalsh(I.dense().T @ I.dense())
        a, b = synth.interval_by_count(ev, n // 2, 5)
        out.append((I, a, b))
    return out


@pytest.mark.parametrize("solver", [cs.CSVD_SOLVER_SINGLE, cs.CSVD_SOLVER_BLOCK])
def test_batch_equals_solo_bitwise(solver):
    probs = _three_problems()
    p = cs.csvd_params_default(L=8, M=2, N=16, solver=solver)
    say("batch solver", solver)
    solo = []
    ctxs = [make_ctx(I) for I, _, _ in probs]
    try:
        for (I, a, b), c in zip(probs, ctxs):
            cs.csvd_solve_interval(c, a, b, p, synth.v_in(I.n, 8, 11))
            solo.append(cs.csvd_get_triplets(c, I.m, I.n))
        say("batch of", len(probs))
        st = cs.csvd_solve_batch(ctxs, [a for _, a, _ in probs], [b for _, _, b in probs], [p] * 3,
                                 [synth.v_in(I.n, 8, 11) for I, _, _ in probs])
        assert all(s == cs.CSVD_OK for s in st)
        for (I, _, _), c, ref in zip(probs, ctxs, solo):
            got = cs.csvd_get_triplets(c, I.m, I.n)
            for x, y in zip(got, ref):
                assert np.array_equal(x, y)
    finally:
        for c in ctxs:
            cs.csvd_destroy(c)


def test_batch_mixed_block_widths_bitwise():
    """A block batch of widths 16, 32 and 64 (L = 8, 24, 40): every step runs
    each width's kernels on its jobs, and the epilogues of finished jobs run
    on worker threads; each result equals the job's solo solve bit for bit."""
    specs = [(2200, 1100, 8), (4200, 2100, 24), (8400, 4200, 40)]
    probs = []
    for i, (m, n, L) in enumerate(specs):
        I = synth.random_sparse(m, n, 8, config=95, instance=i)
        a, b, _, _ = synth.interval_from_sample(m, n, 8, 6, scale=max(1, n // 1000), config=95)
        probs.append((I, a, b, L))
    params = [cs.csvd_params_default(L=L, M=4, N=16, solver=cs.CSVD_SOLVER_BLOCK) for _, _, _, L in probs]
    vins = [synth.v_in(I.n, L, 12, i) for i, (I, _, _, L) in enumerate(probs)]
    ctxs = [make_ctx(I) for I, _, _, _ in probs]
    try:
        solo = []
        for (I, a, b, L), c, p, V in zip(probs, ctxs, params, vins):
            st = cs.csvd_solve_interval(c, a, b, p, V)
            info = cs.csvd_get_info(c)
            say("solo n", I.n, "L", L, "Lp", info.L_padded, "steps", info.iterations, "t_hat", info.t_hat)
            assert st == cs.CSVD_OK and info.solver == cs.CSVD_SOLVER_BLOCK
            solo.append(cs.csvd_get_triplets(c, I.m, I.n))
        st = cs.csvd_solve_batch(ctxs, [a for _, a, _, _ in probs], [b for _, _, b, _ in probs], params, vins)
        assert all(s == cs.CSVD_OK for s in st)
        for (I, _, _, _), c, ref in zip(probs, ctxs, solo):
            got = cs.csvd_get_triplets(c, I.m, I.n)
            assert got[0].size >= 1
            for x, y in zip(got, ref):
                assert np.array_equal(x, y)
    finally:
        for c in ctxs:
            cs.csvd_destroy(c)


@pytest.mark.parametrize("solver", [cs.CSVD_SOLVER_SINGLE, cs.CSVD_SOLVER_BLOCK])
def test_server_results_match_solo_and_cancel(solver):
    probs = _three_problems()
    p = cs.csvd_params_default(L=8, M=2, N=16, solver=solver)
    say("server solver", solver)
    ctxs = [make_ctx(I) for I, _, _ in probs]
    solo_ctx = [make_ctx(I) for I, _, _ in probs]
    extra_ctx = make_ctx(probs[0][0])  # one live request per context
    srv = cs.csvd_server_create(8 << 30, 2)
    try:
        solo = []
        for (I, a, b), c in zip(probs, solo_ctx):
            cs.csvd_solve_interval(c, a, b, p, synth.v_in(I.n, 8, 11))
            solo.append(cs.csvd_get_triplets(c, I.m, I.n))
        reqs = [cs.csvd_server_submit(srv, c, a, b, p, synth.v_in(I.n, 8, 11))
                for (I, a, b), c in zip(probs, ctxs)]
        extra = cs.csvd_server_submit(srv, extra_ctx, probs[0][1], probs[0][2], p,
                                      synth.v_in(probs[0][0].n, 8, 11))
        cs.csvd_server_cancel(srv, extra)
        for _ in range(10000):
            if cs.csvd_server_step(srv, 64) == 0:
                break
        for r in reqs:
            done, st = cs.csvd_server_poll(srv, r)
            assert done and st == cs.CSVD_OK
        done, st = cs.csvd_server_poll(srv, extra)
        assert done and st == cs.CSVD_ESTATE
        for (I, _, _), c, ref in zip(probs, ctxs, solo):
            got = cs.csvd_get_triplets(c, I.m, I.n)
            for x, y in zip(got, ref):
                assert np.array_equal(x, y)
        # a request larger than the whole budget is rejected up front
        tiny = cs.csvd_server_create(1 << 20, 2)
        with pytest.raises(cs.CsvdError) as e:
            cs.csvd_server_submit(tiny, ctxs[1], probs[1][1], probs[1][2], p)
        assert e.value.code == cs.CSVD_ENOMEM
        cs.csvd_server_destroy(tiny)
    finally:
        cs.csvd_server_destroy(srv)
        for c in ctxs + solo_ctx + [extra_ctx]:
            cs.csvd_destroy(c)


def test_served_mixed_block_keeps_fp64_basis():
    """A served block request in mixed precision keeps an FP64 basis (the
    FP64 refinement of an FP32 basis runs only in csvd_solve_interval): its
    triplets are those of the FP64 solve, bit for bit."""
    I = _mid_problem()
    V = synth.v_in(I.n, 8, 12)
    ctxs = [make_ctx(I), make_ctx(I)]
    srv = None
    try:
        base = dict(L=8, M=4, N=16, norm_a=1.0, solver=cs.CSVD_SOLVER_BLOCK)
        assert cs.csvd_solve_interval(ctxs[0], I.a, I.b, cs.csvd_params_default(**base), V) == cs.CSVD_OK
        ref = cs.csvd_get_triplets(ctxs[0], I.m, I.n)
        srv = cs.csvd_server_create(8 << 30, 2)
        req = cs.csvd_server_submit(srv, ctxs[1], I.a, I.b, cs.csvd_params_default(precision=cs.CSVD_MIXED, **base), V)
        for _ in range(10000):
            if cs.csvd_server_step(srv, 64) == 0:
                break
        done, st = cs.csvd_server_poll(srv, req)
        assert done and st == cs.CSVD_OK
        info = cs.csvd_get_info(ctxs[1])
        say("served mixed block: solver", info.solver, "mixed_resid_fp32", info.mixed_resid_fp32)
        assert info.solver == cs.CSVD_SOLVER_BLOCK and info.mixed_resid_fp32 == 0.0 and info.mixed_refined == 0
        for x, y in zip(cs.csvd_get_triplets(ctxs[1], I.m, I.n), ref):
            assert np.array_equal(x, y)
    finally:
        if srv is not None:
            cs.csvd_server_destroy(srv)
        for c in ctxs:
            cs.csvd_destroy(c)


@pytest.mark.parametrize("R,N,K", [(16, 16, 4), (70, 33, 21), (1024, 50, 110), (3, 200, 1)])
def test_dense_gemm_mfma(R, N, K):
    """FP64 MFMA GEMM against the textbook product (edges and ragged tiles)."""
    rng = np.random.default_rng(R + N + K)
    A = rng.standard_normal((R, K))
    B = rng.standard_normal((K, N))
    Cm = cs.csvd_dense_gemm(A, B)
    ref = np.einsum("ik,kj->ij", A, B)
    np.testing.assert_allclose(Cm, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
    # single nonzeros land where the definition puts them
    for (i, k, j) in [(min(3, R - 1), 0, min(5, N - 1)), (R - 1, K - 1, N - 1), (0, K // 2, N // 3)]:
        A = np.zeros((R, K)); A[i, k] = 2.0
        B = np.zeros((K, N)); B[k, j] = 3.0
        Cm = cs.csvd_dense_gemm(A, B)
        assert Cm[i, j] == 6.0 and np.count_nonzero(Cm) == 1


# ------------------------------------------------------------ full size

def test_c2_full_size_certificate():
    """The headline workload at full size (2e5 x 1e5, 10^6 nonzeros, L = 64,
    M = 8, N = 32, the bench's parameters and starting block).  No oracle
    solve fits here, so the oracle certifies the GPU's triplets: residuals
    from host sparse products (checked on sampled rows against the row-by-row
    definition) over a lower bound of ||A||_2, orthonormal U and V, every
    value in [a, b]."""
    import bench
    W = bench.workload("c2")
    I = W["I"]
    say("c2 full size: m", I.m, "n", I.n, "nnz", I.nnz, "interval", W["a"], W["b"])
    ctx = make_ctx(I)
    try:
        p = cs.csvd_params_default(L=W["L"], M=W["M"], N=W["N"], ell=W["ell"], norm_a=W["norm_a"])
        st = cs.csvd_solve_interval(ctx, W["a"], W["b"], p, synth.v_in(I.n, W["L"], 2, 0))
        info = cs.csvd_get_info(ctx)
        say("status", st, "block steps", info.iterations, "t_hat", info.t_hat, "one-pass steps",
            info.one_pass_steps, "basis stored", info.basis_stored)
        assert st == cs.CSVD_OK and info.converged
        # counters of the steps the solution uses (the convergence poll lags
        # by one interval; the steps run meanwhile are not counted)
        assert 0 <= info.one_pass_steps <= info.iterations and info.deflated == 0
        sig, U, V, r = cs.csvd_get_triplets(ctx, I.m, I.n)
    finally:
        cs.csvd_destroy(ctx)
    t = sig.size
    assert t >= 32
    assert np.all(np.diff(sig) >= 0) and sig[0] >= W["a"] and sig[-1] <= W["b"]
    nA = truth.sparse_norm2_lower(I.rowptr, I.colidx, I.vals, I.m, I.n, iters=60)
    res = truth.sparse_triplet_residuals(I.rowptr, I.colidx, I.vals, I.m, I.n, sig, U, V, nA)
    say("oracle certificate: max residual", res.max(), "reported", r.max())
    assert res.max() <= 1e-8
    rows = np.random.default_rng(5).choice(I.m, 64, replace=False)
    AV = sparse.product_rows(I.rowptr, I.colidx, I.vals, V, rows)
    np.testing.assert_allclose(AV, U[rows] * sig[None, :], rtol=0, atol=1e-8 * nA)
    assert np.abs(U.T @ U - np.eye(t)).max() <= 1e-10
    assert np.abs(V.T @ V - np.eye(t)).max() <= 1e-10
