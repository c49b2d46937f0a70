"""Pins of the least-squares fit oracle against things the problem and linear algebra fix."""
import numpy as np
import pytest

from oracle import fit as of
from paper_1911_02373_amd import synth


def test_pivoted_qr_matches_svd_lstsq_full_rank():
    """The paper's own solver is an SVD (LAPACK); numpy's lstsq (gelsd) is that SVD."""
    rng = np.random.default_rng(1)
    for trial in range(20):
        m, n = rng.integers(20, 200), rng.integers(2, 20)
        A = rng.normal(size=(m, n)) * (10.0 ** rng.uniform(-4, 4, n))[None, :]
        b = rng.normal(size=m)
        y, r, _ = of.pivoted_qr_lstsq(A, b)
        # SVD on the column-equilibrated matrix (powers of two, exact), mapped back
        _, ex = np.frexp(np.linalg.norm(A, axis=0))
        Dg = np.ldexp(1.0, -ex)
        zs, *_ = np.linalg.lstsq(A * Dg, b, rcond=None)
        ys = zs * Dg
        kappa = np.linalg.cond(A * Dg)
        assert r == n
        assert np.linalg.norm(y / Dg - zs) <= 1e-14 * kappa * np.linalg.norm(zs)


def test_min_norm_matches_pseudoinverse_rank_deficient():
    rng = np.random.default_rng(2)
    for trial in range(10):
        m, n, r = 50, 12, 7
        A = rng.normal(size=(m, r)) @ rng.normal(size=(r, n))
        A = A / np.linalg.norm(A, axis=0) * 0.75          # column norms in [0.5, 1): D = I
        b = rng.normal(size=m)
        y, rank, _ = of.pivoted_qr_lstsq(A, b)
        assert rank == r
        assert np.allclose(y, np.linalg.pinv(A) @ b, rtol=0, atol=1e-10)


def test_underdetermined_min_norm_interpolates():
    rng = np.random.default_rng(3)
    A = rng.normal(size=(6, 10)) * 0.2
    A = A / np.linalg.norm(A, axis=0) * 0.75
    b = rng.normal(size=6)
    y, rank, _ = of.pivoted_qr_lstsq(A, b)
    assert rank == 6
    assert np.allclose(A @ y, b, atol=1e-12)
    assert np.allclose(y, np.linalg.pinv(A) @ b, atol=1e-11)


def test_polynomial_special_case_matches_polyfit():
    """n_den = 1: ordinary univariate polynomial least squares."""
    rng = np.random.default_rng(4)
    x = rng.integers(1, 1 << 16, 300).astype(np.int32)
    f = 3.0 + 2.0 * (x / 65536.0) - 0.5 * (x / 65536.0) ** 3 + 0.01 * rng.normal(size=300)
    E = synth.monomials(1, 3)[:, :1]
    y, info = of.fit_one(x[:, None], f, E, E[:1], np.array([16]))
    ref = np.polynomial.polynomial.polyfit(x / 65536.0, f, 3)
    assert info["rank"] == 4
    assert np.allclose(y, ref, rtol=1e-10, atol=1e-10)


def test_interpolation_special_case_zero_residual():
    """m = n distinct unisolvent points: the linear system is square and solved exactly."""
    rng = np.random.default_rng(5)
    E = synth.monomials(2, 2)[:, :2]
    n = E.shape[0] * 2 - 1
    X = np.stack([rng.integers(1, 1 << 10, n), rng.integers(1, 1 << 10, n)], 1).astype(np.int32)
    f = rng.uniform(1.0, 2.0, n)
    y, info = of.fit_one(X, f, E, E, np.array([10, 10]))
    assert info["rank"] == n
    assert info["resid_norm"] <= 1e-10 * np.linalg.norm(f)


def _rel_err(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
def test_exact_recovery_config1(seed):
    """Noise-free samples of a rational function are interpolated exactly (step 2 of the
    paper's algorithm: exact values determine g_i by rational interpolation)."""
    b = synth.config1_fit(seed, noise=0.0)
    coef, infos = of.fit_batch(b)
    assert infos[0]["rank"] == 11 and infos[0]["status"] == 0
    assert _rel_err(coef, b.truth_coef) < 1e-9
    Xi, fi, En, Ed, s = b.fit_arrays(0)
    grid = b.meta["grid"]
    got = of.rational_value(grid, En, Ed, s, coef)
    want = of.rational_value(grid, En, Ed, s, b.truth_coef)
    assert np.max(np.abs(got - want) / np.abs(want)) < 1e-12


def test_exact_recovery_config2b_full_rank():
    b = synth.config2_fits(7, n_fits=12, domain="2b", noise=0.0)
    coef, infos = of.fit_batch(b)
    for i, info in enumerate(infos):
        c0 = b.coef0[i]
        assert info["rank"] == 39
        assert _rel_err(coef[c0:c0 + 39], b.truth_coef[c0:c0 + 39]) < 1e-6


def test_config2a_rank_deficient_values_unique():
    """The literal domain has 8 (bx, by) pairs: the system is structurally rank deficient, the
    coefficients are not unique, but the values on the sample domain are."""
    b = synth.config2_fits(8, n_fits=6, domain="2a", noise=0.0)
    coef, infos = of.fit_batch(b)
    for i, info in enumerate(infos):
        assert info["rank"] < 39 and (info["status"] & of.RANK_DEFICIENT)
        Xi, fi, En, Ed, s = b.fit_arrays(i)
        got = of.rational_value(Xi, En, Ed, s, coef[b.coef0[i]:b.coef0[i] + 39])
        assert np.max(np.abs(got - fi) / np.abs(fi)) < 1e-9


def test_denominator_positive_on_samples_noise_free():
    for bb in (synth.config1_fit(9, noise=0.0), synth.config2_fits(9, 8, "2b", noise=0.0)):
        coef, infos = of.fit_batch(bb)
        for i, info in enumerate(infos):
            Xi, fi, En, Ed, s = bb.fit_arrays(i)
            c0 = bb.coef0[i]
            q = of.q_values(Xi, Ed, s, coef[c0 + En.shape[0]: c0 + En.shape[0] + Ed.shape[0] - 1])
            assert np.all(q > 0) and info["q_nonpos"] == 0


def test_noisy_fit_is_least_squares_stationary():
    """At a least-squares minimum the residual is orthogonal to the columns of A."""
    b = synth.config1_fit(11, noise=0.01)
    coef, _ = of.fit_batch(b)
    Xi, fi, En, Ed, s = b.fit_arrays(0)
    A, rhs = of.design_matrix(Xi, fi, En, Ed, s)
    r = A @ coef - rhs
    assert np.max(np.abs(A.T @ r)) / (np.linalg.norm(A) * np.linalg.norm(r)) < 1e-10


def test_bad_input_and_underdetermined_status():
    b = synth.config1_fit(12, noise=0.0)
    Xi, fi, En, Ed, s = b.fit_arrays(0)
    f2 = fi.copy()
    f2[3] = np.nan
    _, info = of.fit_one(Xi, f2, En, Ed, s)
    assert info["status"] & of.BAD_INPUT
    _, info = of.fit_one(Xi[:0], fi[:0], En, Ed, s)
    assert info["status"] & of.BAD_INPUT
    _, info = of.fit_one(Xi[:7], fi[:7], En, Ed, s)
    assert info["status"] & of.UNDERDETERMINED and info["rank"] == 7
