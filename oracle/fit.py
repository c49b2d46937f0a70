"""Oracle: linearised rational least squares, FP64, by column-pivoted Householder QR.

Test infrastructure only (see the package docstring); never imported by the product path.

What it follows.  Section "Building a Driver Program: Rational function estimation": a metric is
modelled as f = p(X)/q(X), p and q polynomials with unknown coefficients alpha (numerator) and
beta (denominator) over given monomial sets; the coefficients are found by linear least squares
on an over-determined system built from monomial evaluations (a Vandermonde-like matrix that the
paper warns is ill-conditioned and may be rank-deficient, so a rank-revealing solver is needed).

Readings taken where the paper is silent:
  * linearisation f*q - p = 0 with q's constant coefficient fixed to 1, i.e. for sample i
        sum_a alpha_a * x_i^a  -  f_i * sum_{b != 0} beta_b * x_i^b  =  f_i ;
  * variables enter scaled by a power of two, x~_k = x_k * 2^-s_k (exact in binary FP);
  * columns are equilibrated by powers of two (exact), then a Householder QR with column
    pivoting (Businger-Golub) reveals the numerical rank r = #{k : |R_kk| > tau |R_11|},
    tau = 10 * max(m, n) * 2^-52;
  * full rank: back substitution; rank deficient (or m < n): the minimum-norm solution of the
    equilibrated problem via a complete orthogonal decomposition of [R11 R12].
The coefficients are returned in the scaled-variable basis (the basis the fit is solved in).
"""
from __future__ import annotations

import numpy as np

# status bits of a fit (same meaning as the library's; values are the documented interface)
RANK_DEFICIENT = 1
UNDERDETERMINED = 2
NOT_CONVERGED = 4
FELL_BACK_FP64 = 8
BAD_INPUT = 16
Q_NONPOS = 32


def scaled_variables(Xi: np.ndarray, s: np.ndarray) -> np.ndarray:
    """x~ = x * 2^-s, exact in FP64 for |x| < 2^53."""
    return np.ldexp(Xi.astype(np.float64), -np.asarray(s, np.int64)[None, :])


def monomial_columns(xt: np.ndarray, E: np.ndarray) -> np.ndarray:
    """Column j = prod_k xt[:, k]^E[j, k], by repeated multiplication in variable order."""
    m, v = xt.shape
    cols = np.ones((m, E.shape[0]))
    for j in range(E.shape[0]):
        for k in range(v):
            for _ in range(int(E[j, k])):
                cols[:, j] = cols[:, j] * xt[:, k]
    return cols


def design_matrix(Xi, fi, E_num, E_den, s):
    """A = [ x~^a (a in E_num) | -f * x~^b (b in E_den without its constant row) ], b = f."""
    xt = scaled_variables(Xi, s)
    P = monomial_columns(xt, E_num)
    Q = monomial_columns(xt, E_den[1:])
    A = np.hstack([P, -fi[:, None] * Q])
    return A, fi.astype(np.float64).copy()


def _back_substitute(U: np.ndarray, c: np.ndarray) -> np.ndarray:
    n = U.shape[0]
    y = np.zeros(n)
    for i in range(n - 1, -1, -1):
        y[i] = (c[i] - U[i, i + 1:] @ y[i + 1:]) / U[i, i]
    return y


def _forward_substitute(L: np.ndarray, c: np.ndarray) -> np.ndarray:
    n = L.shape[0]
    y = np.zeros(n)
    for i in range(n):
        y[i] = (c[i] - L[i, :i] @ y[:i]) / L[i, i]
    return y


def pivoted_qr_lstsq(A: np.ndarray, b: np.ndarray, tau_factor: float = 10.0):
    """min ||A y - b||_2 by column-equilibrated, column-pivoted Householder QR.

    Returns (y, rank, R_diag).  Rank deficient: minimum-norm solution in the equilibrated
    variable z = D^-1 y."""
    m, n = A.shape
    norms = np.linalg.norm(A, axis=0)
    _, ex = np.frexp(np.where(norms > 0, norms, 1.0))
    D = np.ldexp(1.0, -ex)                     # ||A_j|| * D_j in [0.5, 1)
    R = A * D[None, :]
    c = b.astype(np.float64).copy()
    perm = np.arange(n)
    kmax = min(m, n)
    for k in range(kmax):
        cn = np.linalg.norm(R[k:, k:], axis=0)
        j = k + int(np.argmax(cn))
        if j != k:
            R[:, [k, j]] = R[:, [j, k]]
            perm[[k, j]] = perm[[j, k]]
        x = R[k:, k].copy()
        nx = np.linalg.norm(x)
        if nx == 0.0:
            break
        alpha = -np.copysign(nx, x[0])
        v = x
        v[0] -= alpha
        beta = 2.0 / (v @ v)
        R[k:, k:] -= np.outer(v, beta * (v @ R[k:, k:]))
        c[k:] -= v * (beta * (v @ c[k:]))
        R[k + 1:, k] = 0.0
    diag = np.abs(np.diag(R[:kmax, :kmax])) if kmax else np.zeros(0)
    tau = tau_factor * max(m, n) * 2.0 ** -52
    r = 0
    if kmax and diag[0] > 0:
        while r < kmax and diag[r] > tau * diag[0]:
            r += 1
    if r == n:
        zp = _back_substitute(R[:n, :n], c[:n])
    elif r == 0:
        zp = np.zeros(n)
    else:
        # complete orthogonal decomposition: [R11 R12]^T = Zq Lq  =>  [R11 R12] = Lq^T Zq^T
        M = R[:r, :]
        Zq, Lq = np.linalg.qr(M.T)             # n x r, r x r upper
        u = _forward_substitute(Lq.T, c[:r])
        zp = Zq @ u
    z = np.zeros(n)
    z[perm] = zp
    return D * z, r, diag


def q_values(Xi, E_den, s, beta):
    xt = scaled_variables(Xi, s)
    return 1.0 + monomial_columns(xt, E_den[1:]) @ beta


def rational_value(Xi, E_num, E_den, s, coef):
    """p(x~)/q(x~) at integer points; NaN where q <= 0 or the value is not finite (invalid)."""
    n_num = E_num.shape[0]
    xt = scaled_variables(np.atleast_2d(Xi), s)
    p = monomial_columns(xt, E_num) @ coef[:n_num]
    q = 1.0 + monomial_columns(xt, E_den[1:]) @ coef[n_num:]
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        v = p / q
    return np.where((q > 0) & np.isfinite(v), v, np.nan)


def fit_one(Xi, fi, E_num, E_den, s):
    """One fit.  Returns (coef, info dict)."""
    m = Xi.shape[0]
    n = E_num.shape[0] + E_den.shape[0] - 1
    info = {"status": 0, "rank": 0, "resid_norm": np.nan, "q_nonpos": 0}
    if m == 0 or not np.all(np.isfinite(fi)) or np.any(E_den[0] != 0):
        info["status"] = BAD_INPUT
        return np.zeros(n), info
    A, b = design_matrix(Xi, fi, E_num, E_den, s)
    y, r, _ = pivoted_qr_lstsq(A, b)
    st = 0
    if r < n:
        st |= RANK_DEFICIENT
    if m < n:
        st |= UNDERDETERMINED
    qv = q_values(Xi, E_den, s, y[E_num.shape[0]:])
    qn = int(np.count_nonzero(qv <= 0))
    if qn:
        st |= Q_NONPOS
    info.update(status=st, rank=r, resid_norm=float(np.linalg.norm(A @ y - b)), q_nonpos=qn)
    return y, info


def fit_batch(batch, indices=None):
    """Fit every (or the listed) fit of a synth.FitBatch.  Returns (coef, infos)."""
    coef = np.zeros(batch.n_coef)
    infos = []
    idx = range(batch.n_fits) if indices is None else indices
    for i in idx:
        Xi, fi, En, Ed, s = batch.fit_arrays(i)
        y, info = fit_one(Xi, fi, En, Ed, s)
        c0 = int(batch.coef0[i])
        coef[c0: c0 + y.shape[0]] = y
        infos.append(info)
    return coef, infos


def condition_number(Xi, fi, E_num, E_den, s):
    """2-norm condition number of the column-equilibrated design matrix (for tolerances)."""
    A, _ = design_matrix(Xi, fi, E_num, E_den, s)
    norms = np.linalg.norm(A, axis=0)
    _, ex = np.frexp(np.where(norms > 0, norms, 1.0))
    sv = np.linalg.svd(A * np.ldexp(1.0, -ex)[None, :], compute_uv=False)
    return float(sv[0] / sv[-1]) if sv[-1] > 0 else np.inf
