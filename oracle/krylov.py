"""Oracle implementations of the simultaneous Krylov methods (FP64, numpy/scipy).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Notation follows the paper: A is n x n, blocks are n x s, <X, Y> = tr(Y^H X) is
the inner product of the tensorised system (I (x) A) x = b (Section 2), hatted
quantities are "shadow" blocks living in Krylov spaces of A^H.

Common conventions (Section 5, first paragraph):
  * X0 = 0 by default; with preprocessing the block of initial residuals is
    replaced by Q from its thin QR factorisation R0 = Q R_R, the solver works on
    A D = Q, and X = X0 + D R_R is returned.
  * The shadow is R^_0 = R_0; the economic variants use the arithmetic mean of
    the initial residuals.
  * Stop at the first iterate k with ||R_k||_F <= tol ||R_0||_F, using the
    recursively updated residual (||C_k||_F for the rQ variants, which equals
    ||R_k||_F, Section 4 remarks after Algorithm 5).  The true relative residual
    ||B - A X||_F / ||B||_F is recomputed at exit; larger than 1 is reported as
    divergence (Section 5.2, discussion of Table 2).

Breakdown rule (Section 2 states that a method breaks down when a quotient's
denominator vanishes or an s x s matrix is singular): a scalar denominator
that is exactly zero or not finite, or an LU pivot with
|u_kk| <= s * 2^-52 * max |u_ij|, stops the iteration with status BREAKDOWN and
returns the last complete iterate.

Each method function has the signature
    method(A, AH, R0, tol, maxit, shadow=None, hook=None) -> (D, info)
where ``A`` / ``AH`` are scipy sparse matrices for A and A^H, ``R0`` is the
block of initial residuals (the system solved is A D = R0 from D0 = 0) and
``hook(k, D_k, extras)`` is called after every completed iteration (``extras``
holds the step length omega for the BiCGStab variants).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

STATUS_OK = 0
STATUS_NOT_CONVERGED = 1
STATUS_BREAKDOWN = 2
STATUS_DIVERGED = 3

EPS = 2.0 ** -52


class _Breakdown(Exception):
    pass


def tr(Y: np.ndarray, X: np.ndarray) -> complex:
    """<X, Y> = tr(Y^H X) (Section 2, identities for mat_{n x s})."""
    return np.vdot(Y, X)


def _fro(X: np.ndarray) -> float:
    return float(np.linalg.norm(X))


def _denominator(d) -> None:
    if d == 0 or not np.isfinite(d):
        raise _Breakdown()


def _lu(G: np.ndarray):
    """LU with partial pivoting of an s x s matrix, with the pivot breakdown test."""
    if not np.all(np.isfinite(G)):
        raise _Breakdown()
    lu, piv = sla.lu_factor(G, check_finite=False)
    u = np.abs(np.diag(lu))
    umax = np.abs(np.triu(lu)).max()
    if umax == 0 or np.any(u <= G.shape[0] * EPS * umax):
        raise _Breakdown()
    return lu, piv


def _solve(G: np.ndarray, M: np.ndarray) -> np.ndarray:
    """G^{-1} M."""
    return sla.lu_solve(_lu(G), M, check_finite=False)


def qr_pos(Z: np.ndarray):
    """Thin QR, Z = Q C, with diag(C) real and >= 0 (Householder, numpy)."""
    Q, C = np.linalg.qr(Z, mode="reduced")
    d = np.diag(C)
    a = np.abs(d)
    ph = np.where(a > 0, d / np.where(a > 0, a, 1), 1)
    Q = Q * ph[None, :]
    C = np.conj(ph)[:, None] * C
    return Q, C


@dataclass
class _Info:
    status: int = STATUS_NOT_CONVERGED
    iterations: int = 0
    matvecs: int = 0
    history: list = field(default_factory=list)
    breakdown_iter: int = -1


def _finish(info: _Info, res: float, nr0: float, tol: float, k: int) -> bool:
    info.history.append(res / nr0)
    info.iterations = k
    if res <= tol * nr0:
        info.status = STATUS_OK
        return True
    return False


# ----------------------------------------------------------------------------
# Global BiCG, Algorithm 2
# ----------------------------------------------------------------------------
def gl_bicg(A, AH, R0, tol, maxit, shadow=None, hook=None):
    """Global BiCG (Algorithm 2): BiCG on (I (x) A) x = b, matricised."""
    s = R0.shape[1]
    info = _Info()
    X = np.zeros_like(R0)
    R = R0.copy()
    Rh = R0.copy() if shadow is None else np.array(shadow, dtype=R0.dtype)
    P = R.copy()
    Ph = Rh.copy()
    nr0 = _fro(R0)
    info.history.append(1.0)
    if nr0 == 0:
        info.status = STATUS_OK
        return X, info
    rho = tr(Rh, R)
    try:
        for k in range(maxit):
            Q = A @ P
            Zh = AH @ Ph
            info.matvecs += 2 * s
            sigma = tr(Ph, Q)
            _denominator(sigma)
            alpha = rho / sigma
            X = X + alpha * P
            R = R - alpha * Q
            Rh = Rh - np.conj(alpha) * Zh
            if hook:
                hook(k + 1, X, {})
            if _finish(info, _fro(R), nr0, tol, k + 1):
                return X, info
            rho_new = tr(Rh, R)
            _denominator(rho)
            beta = rho_new / rho
            rho = rho_new
            P = R + beta * P
            Ph = Rh + np.conj(beta) * Ph
    except _Breakdown:
        info.status = STATUS_BREAKDOWN
        info.breakdown_iter = info.iterations
    return X, info


# ----------------------------------------------------------------------------
# Economic global BiCG, Algorithm 4
# ----------------------------------------------------------------------------
def egl_bicg(A, AH, R0, tol, maxit, shadow=None, hook=None):
    """Economic global BiCG (Algorithm 4): the shadow block keeps the form
    r^ 1^T, so A^H is applied to one vector per iteration and
    tr(1 r^H R) = sum(r^H R) (Section 4).  Default r^_0 = mean of R0's columns."""
    s = R0.shape[1]
    info = _Info()
    X = np.zeros_like(R0)
    R = R0.copy()
    rh = R0.mean(axis=1) if shadow is None else np.array(shadow, dtype=R0.dtype)
    P = R.copy()
    ph = rh.copy()
    nr0 = _fro(R0)
    info.history.append(1.0)
    if nr0 == 0:
        info.status = STATUS_OK
        return X, info
    rho = np.sum(np.conj(rh) @ R)
    try:
        for k in range(maxit):
            Q = A @ P
            zh = AH @ ph
            info.matvecs += s + 1
            sigma = np.sum(np.conj(ph) @ Q)
            _denominator(sigma)
            alpha = rho / sigma
            X = X + alpha * P
            R = R - alpha * Q
            rh = rh - np.conj(alpha) * zh
            if hook:
                hook(k + 1, X, {})
            if _finish(info, _fro(R), nr0, tol, k + 1):
                return X, info
            rho_new = np.sum(np.conj(rh) @ R)
            _denominator(rho)
            beta = rho_new / rho
            rho = rho_new
            P = R + beta * P
            ph = rh + np.conj(beta) * ph
    except _Breakdown:
        info.status = STATUS_BREAKDOWN
        info.breakdown_iter = info.iterations
    return X, info


# ----------------------------------------------------------------------------
# Global QMR and economic global QMR (Sections 2 and 4; written out here)
# ----------------------------------------------------------------------------
def _qmr(A, AH, R0, tol, maxit, economic, shadow=None, hook=None):
    """QMR without look-ahead in its coupled two-term form (Freund & Nachtigal),
    applied to (I (x) A) x = b and matricised as in Section 2: vector inner
    products become tr(Y^H X), norms become Frobenius norms.  Lanczos blocks are
    scaled to unit Frobenius norm.  The residual is updated explicitly
    (R <- R - A D) so the stopping rule is the same as for the other variants.

    Economic variant (Section 4, "in a similar way"): the left Lanczos block is
    w 1^T and is stored as the vector w; then ||w 1^T||_F = sqrt(s) ||w||,
    tr((w 1^T)^H V) = sum(w^H V), and A^H is applied to one vector.
    """
    s = R0.shape[1]
    info = _Info()
    X = np.zeros_like(R0)
    R = R0.copy()
    nr0 = _fro(R0)
    info.history.append(1.0)
    if nr0 == 0:
        info.status = STATUS_OK
        return X, info
    Vt = R0.copy()
    rho = _fro(Vt)
    if economic:
        wt = R0.mean(axis=1) if shadow is None else np.array(shadow, dtype=R0.dtype)
        xi = np.sqrt(s) * np.linalg.norm(wt)
    else:
        Wt = R0.copy() if shadow is None else np.array(shadow, dtype=R0.dtype)
        xi = _fro(Wt)
    gamma_p, eta_p, theta_p, eps_p = 1.0, -1.0, 0.0, None
    P = Qd = D = S = None
    try:
        for i in range(maxit):
            _denominator(rho)
            _denominator(xi)
            V = Vt / rho
            if economic:
                w = wt / xi
                delta = np.sum(np.conj(w) @ V)
            else:
                W = Wt / xi
                delta = tr(W, V)
            _denominator(delta)
            if i == 0:
                P = V.copy()
                Qd = (w if economic else W).copy()
            else:
                _denominator(eps_p)
                P = V - (xi * delta / eps_p) * P
                Qd = (w if economic else W) - np.conj(rho * delta / eps_p) * Qd
            Pt = A @ P
            if economic:
                eps = np.sum(np.conj(Qd) @ Pt)
            else:
                eps = tr(Qd, Pt)
            _denominator(eps)
            beta = eps / delta
            Vt = Pt - beta * V
            rho_n = _fro(Vt)
            if economic:
                wt = AH @ Qd - np.conj(beta) * w
                xi_n = np.sqrt(s) * np.linalg.norm(wt)
                info.matvecs += s + 1
            else:
                Wt = AH @ Qd - np.conj(beta) * W
                xi_n = _fro(Wt)
                info.matvecs += 2 * s
            _denominator(beta)
            _denominator(gamma_p)
            theta = rho_n / (gamma_p * abs(beta))
            gamma = 1.0 / np.sqrt(1.0 + theta * theta)
            _denominator(gamma)
            eta = -eta_p * rho * gamma * gamma / (beta * gamma_p * gamma_p)
            if i == 0:
                D = eta * P
                S = eta * Pt
            else:
                f = (theta_p * gamma) ** 2
                D = eta * P + f * D
                S = eta * Pt + f * S
            X = X + D
            R = R - S
            if hook:
                hook(i + 1, X, {})
            if _finish(info, _fro(R), nr0, tol, i + 1):
                return X, info
            rho, xi, gamma_p, eta_p, theta_p, eps_p = rho_n, xi_n, gamma, eta, theta, eps
    except _Breakdown:
        info.status = STATUS_BREAKDOWN
        info.breakdown_iter = info.iterations
    return X, info


def gl_qmr(A, AH, R0, tol, maxit, shadow=None, hook=None):
    """Global QMR (Section 2, not written out in the paper)."""
    return _qmr(A, AH, R0, tol, maxit, False, shadow, hook)


def egl_qmr(A, AH, R0, tol, maxit, shadow=None, hook=None):
    """Economic global QMR (Section 4)."""
    return _qmr(A, AH, R0, tol, maxit, True, shadow, hook)


# ----------------------------------------------------------------------------
# Global BiCGStab (Sections 2-3; van der Vorst's BiCGStab on (I (x) A) x = b)
# ----------------------------------------------------------------------------
def gl_bicgstab(A, AH, R0, tol, maxit, shadow=None, hook=None):
    """Global BiCGStab: BiCGStab (van der Vorst 1992) on the tensorised system,
    matricised; fixed shadow R~ = R0.  Convergence is tested after full steps only."""
    s = R0.shape[1]
    info = _Info()
    X = np.zeros_like(R0)
    R = R0.copy()
    Rt = R0.copy() if shadow is None else np.array(shadow, dtype=R0.dtype)
    P = R.copy()
    nr0 = _fro(R0)
    info.history.append(1.0)
    if nr0 == 0:
        info.status = STATUS_OK
        return X, info
    rho = tr(Rt, R)
    try:
        for k in range(maxit):
            V = A @ P
            info.matvecs += s
            sigma = tr(Rt, V)
            _denominator(sigma)
            alpha = rho / sigma
            S = R - alpha * V
            T = A @ S
            info.matvecs += s
            tt = tr(T, T)
            _denominator(tt)
            omega = tr(T, S) / tt
            X = X + alpha * P + omega * S
            R = S - omega * T
            if hook:
                hook(k + 1, X, {"omega": omega})
            if _finish(info, _fro(R), nr0, tol, k + 1):
                return X, info
            rho_new = tr(Rt, R)
            _denominator(rho)
            _denominator(omega)
            beta = (rho_new / rho) * (alpha / omega)
            rho = rho_new
            P = R + beta * (P - omega * V)
    except _Breakdown:
        info.status = STATUS_BREAKDOWN
        info.breakdown_iter = info.iterations
    return X, info


# ----------------------------------------------------------------------------
# Block BiCG, Algorithm 3 (pin for Algorithm 5)
# ----------------------------------------------------------------------------
def bl_bicg(A, AH, R0, tol, maxit, shadow=None, hook=None):
    """Block BiCG (Algorithm 3), literally: all four s x s coefficient matrices
    from their own Gram matrices."""
    s = R0.shape[1]
    info = _Info()
    X = np.zeros_like(R0)
    R = R0.copy()
    Rh = R0.copy() if shadow is None else np.array(shadow, dtype=R0.dtype)
    P = R.copy()
    Ph = Rh.copy()
    nr0 = _fro(R0)
    info.history.append(1.0)
    if nr0 == 0:
        info.status = STATUS_OK
        return X, info
    try:
        for k in range(maxit):
            Q = A @ P
            Qh = AH @ Ph
            info.matvecs += 2 * s
            RhR = Rh.conj().T @ R
            RRh = R.conj().T @ Rh
            alpha = _solve(Ph.conj().T @ Q, RhR)
            alphah = _solve(P.conj().T @ Qh, RRh)
            X = X + P @ alpha
            R_n = R - Q @ alpha
            Rh_n = Rh - Qh @ alphah
            if hook:
                hook(k + 1, X, {})
            if _finish(info, _fro(R_n), nr0, tol, k + 1):
                return X, info
            beta = _solve(RhR, Rh_n.conj().T @ R_n)
            betah = _solve(RRh, R_n.conj().T @ Rh_n)
            P = R_n + P @ beta
            Ph = Rh_n + Ph @ betah
            R, Rh = R_n, Rh_n
    except _Breakdown:
        info.status = STATUS_BREAKDOWN
        info.breakdown_iter = info.iterations
    return X, info


# ----------------------------------------------------------------------------
# Block BiCG with QR of the block residuals, Algorithm 5
# ----------------------------------------------------------------------------
def bl_bicg_rq(A, AH, R0, tol, maxit, shadow=None, hook=None):
    """Bl-BiCG-rQ (Algorithm 5 with eqs. (newalpha)-(newbetahat)).  R_k = Q_k C_k
    and P_k = V_k C_k; no C^{-1} is formed.  The loop index starts at 0 (the
    initialisation defines the k = 0 quantities).  ||R_k||_F = ||C_k||_F drives
    the stopping test.  alpha^ and beta^ use their own Gram matrices as printed."""
    s = R0.shape[1]
    info = _Info()
    X = np.zeros_like(R0)
    Rh0 = R0 if shadow is None else np.array(shadow, dtype=R0.dtype)
    Q, C = qr_pos(R0)
    Qh, Ch = qr_pos(Rh0)
    V = Q.copy()
    Vh = Qh.copy()
    nr0 = _fro(C)
    info.history.append(1.0)
    if nr0 == 0:
        info.status = STATUS_OK
        return X, info
    try:
        for k in range(maxit):
            W = A @ V
            Wh = AH @ Vh
            info.matvecs += 2 * s
            alpha = _solve(Vh.conj().T @ W, Qh.conj().T @ Q)
            alphah = _solve(V.conj().T @ Wh, Q.conj().T @ Qh)
            X = X + V @ alpha @ C
            Qn, S = qr_pos(Q - W @ alpha)
            C = S @ C
            Qhn, Sh = qr_pos(Qh - Wh @ alphah)
            Ch = Sh @ Ch
            if hook:
                hook(k + 1, X, {})
            if _finish(info, _fro(C), nr0, tol, k + 1):
                return X, info
            beta = _solve(Qh.conj().T @ Q, Sh.conj().T @ (Qhn.conj().T @ Qn))
            betah = _solve(Q.conj().T @ Qh, S.conj().T @ (Qn.conj().T @ Qhn))
            V = Qn + V @ beta
            Vh = Qhn + Vh @ betah
            Q, Qh = Qn, Qhn
    except _Breakdown:
        info.status = STATUS_BREAKDOWN
        info.breakdown_iter = info.iterations
    return X, info


# ----------------------------------------------------------------------------
# Block BiCGStab (El Guennouni, Jbilou, Sadok 2003) -- pin for the rQ variant
# ----------------------------------------------------------------------------
def bl_bicgstab(A, AH, R0, tol, maxit, shadow=None, hook=None):
    """Block BiCGStab: s x s alpha and beta, scalar omega from the Frobenius
    (global) steepest-descent step (Section 2, last paragraph)."""
    s = R0.shape[1]
    info = _Info()
    X = np.zeros_like(R0)
    R = R0.copy()
    Rt = R0.copy() if shadow is None else np.array(shadow, dtype=R0.dtype)
    P = R.copy()
    nr0 = _fro(R0)
    info.history.append(1.0)
    if nr0 == 0:
        info.status = STATUS_OK
        return X, info
    try:
        for k in range(maxit):
            V = A @ P
            info.matvecs += s
            G = Rt.conj().T @ V
            alpha = _solve(G, Rt.conj().T @ R)
            S = R - V @ alpha
            T = A @ S
            info.matvecs += s
            tt = tr(T, T)
            _denominator(tt)
            omega = tr(T, S) / tt
            X = X + P @ alpha + omega * S
            R = S - omega * T
            if hook:
                hook(k + 1, X, {"omega": omega})
            if _finish(info, _fro(R), nr0, tol, k + 1):
                return X, info
            beta = -_solve(G, Rt.conj().T @ T)
            P = R + (P - omega * V) @ beta
    except _Breakdown:
        info.status = STATUS_BREAKDOWN
        info.breakdown_iter = info.iterations
    return X, info


# ----------------------------------------------------------------------------
# Block BiCGStab with QR of the block residuals (Section 4, last paragraph)
# ----------------------------------------------------------------------------
def bl_bicgstab_rq(A, AH, R0, tol, maxit, shadow=None, hook=None):
    """Bl-BiCGStab-rQ.  The paper names this variant but does not write it out;
    this is block BiCGStab with R = Q C and P = U C substituted, following the
    derivation of Algorithm 5 from Algorithm 3:

        W = A U,  G = R~^H W,  a = G^{-1} N            (alpha = C^{-1} a C)
        S~ = Q - W a,  T~ = A S~                        (S = S~ C, T = T~ C)
        omega = tr(T~^H S~ C C^H) / tr(T~^H T~ C C^H)   (= tr(T^H S)/tr(T^H T))
        X <- X + (U a + omega S~) C
        S~ - omega T~ = Q' Sigma,  C' = Sigma C          (R' = Q' C')
        N' = R~^H Q',  b = (1/omega) G^{-1} N'
        U' = Q' + (U - omega W) b                      (P' = U' C')

    The last line uses R~^H S~ = 0, which gives R~^H T~ Sigma^{-1} = -(1/omega) N',
    so neither C^{-1} nor Sigma^{-1} appears.  R~ = R0."""
    s = R0.shape[1]
    info = _Info()
    X = np.zeros_like(R0)
    Rt = R0.copy() if shadow is None else np.array(shadow, dtype=R0.dtype)
    Q, C = qr_pos(R0)
    U = Q.copy()
    N = Rt.conj().T @ Q
    nr0 = _fro(C)
    info.history.append(1.0)
    if nr0 == 0:
        info.status = STATUS_OK
        return X, info
    try:
        for k in range(maxit):
            W = A @ U
            info.matvecs += s
            G = Rt.conj().T @ W
            a = _solve(G, N)
            St = Q - W @ a
            Tt = A @ St
            info.matvecs += s
            K = C @ C.conj().T
            den = np.trace((Tt.conj().T @ Tt) @ K)
            _denominator(den)
            omega = np.trace((Tt.conj().T @ St) @ K) / den
            X = X + (U @ a + omega * St) @ C
            Qn, Sig = qr_pos(St - omega * Tt)
            C = Sig @ C
            if hook:
                hook(k + 1, X, {"omega": omega})
            if _finish(info, _fro(C), nr0, tol, k + 1):
                return X, info
            Nn = Rt.conj().T @ Qn
            _denominator(omega)
            b = _solve(G, Nn) / omega
            U = Qn + (U - omega * W) @ b
            Q, N = Qn, Nn
    except _Breakdown:
        info.status = STATUS_BREAKDOWN
        info.breakdown_iter = info.iterations
    return X, info


# ----------------------------------------------------------------------------
# Loop-interchanged BiCG, Algorithm 1
# ----------------------------------------------------------------------------
def li_bicg(A, AH, R0, tol, maxit, shadow=None, hook=None):
    """Loop-interchanged BiCG (Algorithm 1): s independent BiCG recurrences with
    per-column alpha_i, beta_i."""
    s = R0.shape[1]
    info = _Info()
    X = np.zeros_like(R0)
    R = R0.copy()
    Rh = R0.copy() if shadow is None else np.array(shadow, dtype=R0.dtype)
    P = R.copy()
    Ph = Rh.copy()
    nr0 = _fro(R0)
    info.history.append(1.0)
    if nr0 == 0:
        info.status = STATUS_OK
        return X, info
    rho = np.einsum("ij,ij->j", np.conj(Rh), R)
    try:
        for k in range(maxit):
            Q = A @ P
            Zh = AH @ Ph
            info.matvecs += 2 * s
            sigma = np.einsum("ij,ij->j", np.conj(Ph), Q)
            for d in sigma:
                _denominator(d)
            alpha = rho / sigma
            X = X + P * alpha[None, :]
            R = R - Q * alpha[None, :]
            Rh = Rh - Zh * np.conj(alpha)[None, :]
            if hook:
                hook(k + 1, X, {})
            if _finish(info, _fro(R), nr0, tol, k + 1):
                return X, info
            rho_new = np.einsum("ij,ij->j", np.conj(Rh), R)
            for d in rho:
                _denominator(d)
            beta = rho_new / rho
            rho = rho_new
            P = R + P * beta[None, :]
            Ph = Rh + Ph * np.conj(beta)[None, :]
    except _Breakdown:
        info.status = STATUS_BREAKDOWN
        info.breakdown_iter = info.iterations
    return X, info


def _cdot(Y: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Column-wise inner products y_j^H x_j (one per right-hand side)."""
    return np.einsum("ij,ij->j", np.conj(Y), X)


def _denominators(d) -> None:
    for v in np.atleast_1d(d):
        _denominator(v)


# ----------------------------------------------------------------------------
# Loop-interchanged QMR and BiCGStab (Section 2: the s single-RHS recurrences
# run side by side, their products with A gathered into one block product)
# ----------------------------------------------------------------------------
def li_qmr(A, AH, R0, tol, maxit, shadow=None, hook=None):
    """Loop-interchanged QMR: column j runs the QMR of ``_qmr`` (Freund &
    Nachtigal, no look-ahead, coupled two-term form) on A x_j = r0_j with its own
    scalars rho_j, xi_j, delta_j, eps_j, beta_j, theta_j, gamma_j, eta_j.  The
    block residual R <- R - S is carried for the common stopping rule."""
    s = R0.shape[1]
    info = _Info()
    X = np.zeros_like(R0)
    R = R0.copy()
    nr0 = _fro(R0)
    info.history.append(1.0)
    if nr0 == 0:
        info.status = STATUS_OK
        return X, info
    Vt = R0.copy()
    Wt = R0.copy() if shadow is None else np.array(shadow, dtype=R0.dtype)
    rho = np.linalg.norm(Vt, axis=0)
    xi = np.linalg.norm(Wt, axis=0)
    gamma_p, eta_p, theta_p, eps_p = np.ones(s), -np.ones(s, dtype=R0.dtype), np.zeros(s), None
    P = Qd = D = S = None
    try:
        for i in range(maxit):
            _denominators(rho)
            _denominators(xi)
            V = Vt / rho[None, :]
            W = Wt / xi[None, :]
            delta = _cdot(W, V)
            _denominators(delta)
            if i == 0:
                P, Qd = V.copy(), W.copy()
            else:
                _denominators(eps_p)
                P = V - P * (xi * delta / eps_p)[None, :]
                Qd = W - Qd * np.conj(rho * delta / eps_p)[None, :]
            Pt = A @ P
            eps = _cdot(Qd, Pt)
            _denominators(eps)
            beta = eps / delta
            Vt = Pt - V * beta[None, :]
            Wt = AH @ Qd - W * np.conj(beta)[None, :]
            info.matvecs += 2 * s
            rho_n = np.linalg.norm(Vt, axis=0)
            xi_n = np.linalg.norm(Wt, axis=0)
            _denominators(beta)
            _denominators(gamma_p)
            theta = rho_n / (gamma_p * np.abs(beta))
            gamma = 1.0 / np.sqrt(1.0 + theta * theta)
            _denominators(gamma)
            eta = -eta_p * rho * gamma * gamma / (beta * gamma_p * gamma_p)
            if i == 0:
                D = P * eta[None, :]
                S = Pt * eta[None, :]
            else:
                f = (theta_p * gamma) ** 2
                D = P * eta[None, :] + D * f[None, :]
                S = Pt * eta[None, :] + S * f[None, :]
            X = X + D
            R = R - S
            if hook:
                hook(i + 1, X, {})
            if _finish(info, _fro(R), nr0, tol, i + 1):
                return X, info
            rho, xi, gamma_p, eta_p, theta_p, eps_p = rho_n, xi_n, gamma, eta, theta, eps
    except _Breakdown:
        info.status = STATUS_BREAKDOWN
        info.breakdown_iter = info.iterations
    return X, info


def li_bicgstab(A, AH, R0, tol, maxit, shadow=None, hook=None):
    """Loop-interchanged BiCGStab: column j runs van der Vorst's BiCGStab on
    A x_j = r0_j (shadow r~_j = r0_j) with its own alpha_j, omega_j, beta_j;
    the two products per step are block products.  Convergence is tested on
    the block residual after full steps only."""
    s = R0.shape[1]
    info = _Info()
    X = np.zeros_like(R0)
    R = R0.copy()
    Rt = R0.copy() if shadow is None else np.array(shadow, dtype=R0.dtype)
    P = R.copy()
    nr0 = _fro(R0)
    info.history.append(1.0)
    if nr0 == 0:
        info.status = STATUS_OK
        return X, info
    rho = _cdot(Rt, R)
    try:
        for k in range(maxit):
            V = A @ P
            info.matvecs += s
            sigma = _cdot(Rt, V)
            _denominators(sigma)
            alpha = rho / sigma
            S = R - V * alpha[None, :]
            T = A @ S
            info.matvecs += s
            tt = _cdot(T, T)
            _denominators(tt)
            omega = _cdot(T, S) / tt
            X = X + P * alpha[None, :] + S * omega[None, :]
            R = S - T * omega[None, :]
            if hook:
                hook(k + 1, X, {"omega": omega})
            if _finish(info, _fro(R), nr0, tol, k + 1):
                return X, info
            rho_new = _cdot(Rt, R)
            _denominators(rho)
            _denominators(omega)
            beta = (rho_new / rho) * (alpha / omega)
            rho = rho_new
            P = R + (P - V * omega[None, :]) * beta[None, :]
    except _Breakdown:
        info.status = STATUS_BREAKDOWN
        info.breakdown_iter = info.iterations
    return X, info


METHODS = {
    "gl_bicg": gl_bicg,
    "egl_bicg": egl_bicg,
    "gl_qmr": gl_qmr,
    "egl_qmr": egl_qmr,
    "gl_bicgstab": gl_bicgstab,
    "bl_bicg_rq": bl_bicg_rq,
    "bl_bicgstab_rq": bl_bicgstab_rq,
}
PIN_METHODS = {
    "bl_bicg": bl_bicg,
    "bl_bicgstab": bl_bicgstab,
    "li_bicg": li_bicg,
    "li_qmr": li_qmr,
    "li_bicgstab": li_bicgstab,
}


@dataclass
class Result:
    X: np.ndarray
    status: int
    iterations: int
    matvecs: int
    history: np.ndarray
    rel_res_true: float
    rel_res_recursive: float
    breakdown_iter: int
    method: str


def _as_scipy(A):
    if hasattr(A, "to_scipy"):
        return A.to_scipy().tocsr()
    return sp.csr_array(A)


def solve(A, B, method: str, tol: float = 1e-8, maxit: int = 10000, preprocess: bool = True,
          X0=None, shadow=None, hook=None, precond: str | None = None) -> Result:
    """Solve A X = B with one of the simultaneous methods.

    ``A``: scipy sparse matrix or ``inputs.CSR``; ``B``: n x s.  With
    ``preprocess`` the block of initial residuals R0 = B - A X0 is replaced by
    Q from R0 = Q R_R (Section 5), the method solves A D = Q and
    X = X0 + D R_R is returned.  ``precond='ilu0'``: right no-fill ILU
    preconditioning (``oracle.ilu``): the method runs on A M^-1 and
    X = X0 + M^-1 D R_R."""
    A = _as_scipy(A)
    AH = A.conj().T.tocsr()
    Aplain = A
    M = None
    if precond == "ilu0":
        from .ilu import PrecOp, RightILU
        M = RightILU(A)
        A, AH = PrecOp(Aplain, AH, M, False), PrecOp(Aplain, AH, M, True)
    elif precond is not None:
        raise ValueError(precond)
    fn = METHODS.get(method) or PIN_METHODS[method]
    B = np.asarray(B)
    dtype = np.result_type(Aplain.dtype, B.dtype, np.float64)
    B = B.astype(dtype)
    if X0 is None:
        X0 = np.zeros_like(B)
        R0 = B.copy()
    else:
        X0 = np.asarray(X0, dtype=dtype)
        R0 = B - Aplain @ X0
    if preprocess:
        Qr, Rr = qr_pos(R0)
        D, info = fn(A, AH, Qr, tol, maxit, shadow, hook)
        if M is not None:
            D = M.minv(D)
        X = X0 + D @ Rr
    else:
        D, info = fn(A, AH, R0, tol, maxit, shadow, hook)
        if M is not None:
            D = M.minv(D)
        X = X0 + D
    nb = _fro(B)
    rel_true = _fro(B - Aplain @ X) / nb if nb > 0 else 0.0
    status = info.status
    if status != STATUS_BREAKDOWN and rel_true > 1.0:
        status = STATUS_DIVERGED
    hist = np.asarray(info.history, dtype=np.float64)
    return Result(X, status, info.iterations, info.matvecs, hist, rel_true, float(hist[-1]),
                  info.breakdown_iter, method)
