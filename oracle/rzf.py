"""Plain complex128 reference of the RZF precoder computed by Jacobi-preconditioned CG.

TEST INFRASTRUCTURE ONLY (see the package docstring): used by tests/, the smoke
check and the CPU baseline of the benchmark, never by the product path.

Notation follows the paper, with the renames needed to avoid its symbol clashes:

  H      M x K channel, column k is user k's vector h_k            (Sec. II, eq. 1)
  xi     regularisation factor                                     (eq. 7; xi = 1/SNR)
  A      regularised Gram H^H H + xi I (the paper's P_i)           (eq. 7)
  B      right-hand sides, K x n (the paper's s_i; I_K = inverse)  (eqs. 15-16)
  X      solution of A X = B (the paper's w_i)                     (eqs. 15-16)
  W      power-normalised precoder beta_pow * H X (the paper's G_i) (eq. 7, eq. 15)
  P_tx   total transmit power (the paper's P in beta's definition) (Sec. II, after eq. 7)

Status codes mirror the C ABI: OK = 0, NOT_CONVERGED = 1, BREAKDOWN = -5.
"""

from __future__ import annotations

import numpy as np

OK = 0
NOT_CONVERGED = 1
BREAKDOWN = -5


def _c128(a):
    return np.asarray(a, dtype=np.complex128)


# ---------------------------------------------------------------------------
# O1: regularised Gram matrix  (eq. 7: P_i = H_i^H H_i + xi I)
# ---------------------------------------------------------------------------
def gram(H, xi):
    """A = H^H H + xi I_K (eq. 7), with an exactly Hermitian result.

    Entry (i, j) is sum_m conj(H[m, i]) H[m, j] + xi [i == j]. The upper
    triangle (j >= i) is formed row by row, the lower triangle is its conjugate
    mirror, and the diagonal -- a sum of squared moduli -- is stored as an
    exactly real number.
    """
    H = _c128(H)
    M, K = H.shape
    A = np.zeros((K, K), dtype=np.complex128)
    for i in range(K):
        row = H[:, i].conj() @ H[:, i:]          # entries (i, i..K-1)
        A[i, i:] = row
        A[i:, i] = row.conj()                     # Hermitian mirror
        A[i, i] = float(np.sum(H[:, i].real ** 2 + H[:, i].imag ** 2)) + float(xi)
    return A


# ---------------------------------------------------------------------------
# O2: direct inverse, the "traditional RZF" route (Appendix A)
# ---------------------------------------------------------------------------
def cholesky_lower(A):
    """Cholesky factor L with A = L L^H (Appendix A, step (a): P = M M^H).

    Column-by-column textbook recurrence; raises ValueError on a non-positive
    pivot (A not Hermitian positive definite).
    """
    A = _c128(A)
    K = A.shape[0]
    L = np.zeros((K, K), dtype=np.complex128)
    for j in range(K):
        pivot = A[j, j].real - float(np.sum(np.abs(L[j, :j]) ** 2))
        if not (pivot > 0.0) or not np.isfinite(pivot):
            raise ValueError(f"Cholesky pivot {pivot!r} <= 0 at column {j}: matrix not HPD")
        L[j, j] = np.sqrt(pivot)
        for i in range(j + 1, K):
            L[i, j] = (A[i, j] - np.sum(L[i, :j] * L[j, :j].conj())) / L[j, j]
    return L


def lower_inverse(L):
    """L^{-1} of a lower-triangular L by forward substitution (Appendix A, step (b)).

    Solves L Y = I one column of the identity at a time.
    """
    L = _c128(L)
    K = L.shape[0]
    Y = np.zeros((K, K), dtype=np.complex128)
    for c in range(K):
        for i in range(c, K):
            rhs = (1.0 if i == c else 0.0) - np.sum(L[i, c:i] * Y[c:i, c])
            Y[i, c] = rhs / L[i, i]
    return Y


def chol_inverse(A):
    """A^{-1} = L^{-H} L^{-1} (Appendix A, steps (a)-(c))."""
    Linv = lower_inverse(cholesky_lower(A))
    return Linv.conj().T @ Linv


def gauss_jordan_inverse(A):
    """A^{-1} by Gauss-Jordan elimination with partial pivoting.

    The paper names Gauss-Jordan as the practical O(K^3) inverse (Sec. I,
    footnote 1). Used as an independent second route on small K.
    """
    A = _c128(A)
    K = A.shape[0]
    aug = np.concatenate([A.copy(), np.eye(K, dtype=np.complex128)], axis=1)
    for c in range(K):
        p = c + int(np.argmax(np.abs(aug[c:, c])))
        if aug[p, c] == 0:
            raise ValueError("singular matrix")
        if p != c:
            aug[[c, p]] = aug[[p, c]]
        aug[c] = aug[c] / aug[c, c]
        for r in range(K):
            if r != c and aug[r, c] != 0:
                aug[r] = aug[r] - aug[r, c] * aug[c]
    return aug[:, K:]


# ---------------------------------------------------------------------------
# O3: Jacobi-preconditioned conjugate gradient (Algorithm 1, eq. 21)
# ---------------------------------------------------------------------------
def jacpcg(A, B=None, tol=0.0, max_iter=16, precond="jacobi"):
    """Solve A X = B column by column with Jacobi-preconditioned CG.

    Reading of the paper (Sec. III-B Steps 1-4, eq. 21 and Algorithm 1):
      * preconditioner C = D = diag(A) (eq. 21); ``precond="none"`` gives plain
        CG (C = I), the method the paper compares against;
      * initial guess w^0 = 0, so the first residual is s itself and the first
        preconditioned residual is C^{-1} s (Algorithm 1's initialisation);
      * step length alpha = (residual^H C^{-1} residual) / (m^H A m) and the
        direction update m <- C^{-1} r' + beta m with
        beta = (r'^H C^{-1} r') / (r^H C^{-1} r), i.e. the standard PCG form
        whose step length Step 3 states; Algorithm 1's listing instead takes
        Euclidean products on C^{-1} A, which agrees only when diag(A) is
        constant (see ``cg_on_jacobi_scaled_operator``);
      * the two inner products are real for Hermitian positive definite A
        (eq. 18); their real parts are used;
      * stop rule (Step 2, applied per column, relative to ||b_j||): stop as soon
        as ||r_j|| <= tol * ||b_j|| after an update. tol = 0 runs exactly
        ``max_iter`` iterations unless the residual becomes exactly zero;
      * one iteration is one product A m (Algorithm 1's counter t);
      * a step with m^H A m < 0 or not finite is a breakdown: the column stops
        with its last x and status BREAKDOWN. m^H A m = 0 means m = 0 for HPD A
        (eq. 18), i.e. the residual vanished: the column stops as converged.

    Returns a dict with X (K x n), iters (n,), relres (n,) from the recurrence
    residual, true_relres (n,) = ||b - A x|| / ||b||, status (n,) per column,
    and instance_status (worst column: BREAKDOWN < NOT_CONVERGED < OK).
    """
    A = _c128(A)
    K = A.shape[0]
    Bm = np.eye(K, dtype=np.complex128) if B is None else _c128(B)
    if Bm.ndim == 1:
        Bm = Bm[:, None]
    n = Bm.shape[1]
    if precond == "jacobi":
        d = A.diagonal().real.copy()
    elif precond == "none":
        d = np.ones(K)
    else:
        raise ValueError(precond)

    X = np.zeros((K, n), dtype=np.complex128)
    iters = np.zeros(n, dtype=np.int64)
    relres = np.zeros(n)
    status = np.full(n, OK, dtype=np.int64)
    for j in range(n):
        b = Bm[:, j]
        bnorm = np.linalg.norm(b)
        x = np.zeros(K, dtype=np.complex128)
        if bnorm == 0.0:
            X[:, j] = x
            continue
        r = b.copy()
        z = r / d
        p = z.copy()
        rho = float(np.vdot(r, z).real)
        converged = False
        for t in range(1, max_iter + 1):
            q = A @ p
            gamma = float(np.vdot(p, q).real)
            if not np.isfinite(gamma) or gamma < 0.0:
                status[j] = BREAKDOWN
                break
            if gamma == 0.0:
                # For HPD A, p^H A p = 0 only for p = 0 (eq. 18), i.e. the
                # residual has vanished: the column has converged.
                converged = True
                break
            alpha = rho / gamma
            x = x + alpha * p
            r = r - alpha * q
            iters[j] = t
            if np.linalg.norm(r) <= tol * bnorm:
                converged = True
                break
            z = r / d
            rho_next = float(np.vdot(r, z).real)
            if rho_next == 0.0:
                # r^H D^{-1} r = 0 with D > 0 only for r = 0: converged.
                converged = True
                break
            p = z + (rho_next / rho) * p
            rho = rho_next
        X[:, j] = x
        relres[j] = np.linalg.norm(r) / bnorm
        if status[j] == OK and tol > 0.0 and not converged:
            status[j] = NOT_CONVERGED
    true_relres = np.array([
        np.linalg.norm(Bm[:, j] - A @ X[:, j]) / max(np.linalg.norm(Bm[:, j]), 1e-300) if np.linalg.norm(Bm[:, j]) > 0 else 0.0
        for j in range(n)
    ])
    if np.any(status == BREAKDOWN):
        inst = BREAKDOWN
    elif np.any(status == NOT_CONVERGED):
        inst = NOT_CONVERGED
    else:
        inst = OK
    return dict(X=X, iters=iters, relres=relres, true_relres=true_relres,
                status=status, instance_status=inst)


def _euclidean_cg(apply_op, rhs, T):
    """T steps of textbook conjugate gradient with Euclidean inner products on
    the linear operator ``apply_op`` from x = 0 (Hestenes-Stiefel form). For a
    Hermitian positive definite operator this is the Krylov-optimal method; the
    recurrences are evaluated as written even when the operator is not
    Hermitian."""
    x = np.zeros_like(rhs)
    res = rhs.copy()
    d = res.copy()
    for _ in range(T):
        Ad = apply_op(d)
        step = np.vdot(res, res) / np.vdot(d, Ad)
        x = x + step * d
        res_new = res - step * Ad
        d = res_new + (np.vdot(res_new, res_new) / np.vdot(res, res)) * d
        res = res_new
    return x


def cg_on_jacobi_scaled_operator(A, s, T):
    """The iteration Algorithm 1 prints: it is Euclidean CG (``_euclidean_cg``)
    applied to the operator C^{-1} A with right-hand side C^{-1} s, C =
    diag(A). C^{-1} A is not Hermitian unless diag(A) is constant, so this is
    not the preconditioned CG of Step 3 (the reading ``jacpcg`` takes). Kept
    only to document that choice: the two agree when diag(A) is constant and
    drift apart otherwise. Never a parity target of the GPU path.
    """
    A = _c128(A)
    s = _c128(s).reshape(-1)
    cinv = 1.0 / A.diagonal().real
    return _euclidean_cg(lambda v: cinv * (A @ v), cinv * s, T)


# ---------------------------------------------------------------------------
# O4: power-normalised precoder (eq. 7 and the definition of beta after it)
# ---------------------------------------------------------------------------
def precoder(H, X, P_tx=1.0):
    """W = beta_pow H X with beta_pow = sqrt(P_tx / tr(F^H F)), F = H X.

    The paper defines F = H P^{-1} and beta = sqrt(P / tr(F^H F)); with X an
    approximation of A^{-1} B, F is the computed H X and tr(F^H F) = ||F||_F^2.
    Returns (W, beta_pow).
    """
    F = _c128(H) @ _c128(X)
    fro2 = float(np.sum(F.real ** 2 + F.imag ** 2))
    beta = float(np.sqrt(P_tx / fro2))
    return beta * F, beta


def rzf(H, xi, B=None, tol=0.0, max_iter=16, P_tx=1.0, precond="jacobi"):
    """Whole path: A = gram(H, xi); X = jacpcg(A, B); W = precoder(H, X)."""
    A = gram(H, xi)
    res = jacpcg(A, B, tol=tol, max_iter=max_iter, precond=precond)
    W, beta = precoder(H, res["X"], P_tx)
    res.update(A=A, W=W, beta_pow=beta)
    return res


def direct_rzf(H, xi, B=None, P_tx=1.0):
    """The exact RZF precoder through the Cholesky inverse (Appendix A route).

    X* = A^{-1} B is the target of the FP64-refined GPU result and the
    "error vs FP64" reference for every result. Returns (X*, W*, beta*).
    """
    A = gram(H, xi)
    K = A.shape[0]
    Bm = np.eye(K, dtype=np.complex128) if B is None else _c128(B)
    Xs = chol_inverse(A) @ Bm
    W, beta = precoder(H, Xs, P_tx)
    return Xs, W, beta


# ---------------------------------------------------------------------------
# O6: subarray-block RZF (Sec. II: eqs. 2, 6 and 7)
# ---------------------------------------------------------------------------
def block_slices(M1, Mc, M2, K1, K2):
    """Row and column ranges of the three blocks of eq. 2 / eq. 6.

    Antennas: subarray 1 = rows [0, M1), the common subarray c = rows
    [M1, M1 + Mc), subarray 2 = rows [M1 + Mc, M1 + Mc + M2). Users: group 1 =
    columns [0, K1), group 2 = columns [K1, K1 + K2). Returns a dict
    block -> (row slice, column slice) for blocks "1", "c", "2".
    """
    r1, rc, r2 = slice(0, M1), slice(M1, M1 + Mc), slice(M1 + Mc, M1 + Mc + M2)
    return {"1": (r1, slice(0, K1)), "c": (rc, slice(0, K1 + K2)), "2": (r2, slice(K1, K1 + K2))}


def block_rzf(H, xi, M1, Mc, M2, K1, K2, tol=0.0, max_iter=16, P_tx=1.0, precond="jacobi", direct=False):
    """Subarray-block RZF precoder G of eq. 6 for a channel H of the form of eq. 2.

    Each block i in {1, c, 2} is its own RZF problem (eq. 7):
    G_i = beta_i H_i P_i^{-1}, P_i = H_i^H H_i + xi I, with its own power factor
    beta_i = sqrt(P_tx / tr(F_i^H F_i)). G_1 and G_2 fill the (subarray 1,
    group 1) and (subarray 2, group 2) blocks, G_c = [G_c1, G_c2] the common
    subarray's rows; the (subarray 1, group 2) and (subarray 2, group 1)
    blocks are zero. P_i^{-1} comes from Jacobi-PCG (O3) at (tol, max_iter),
    or from the Cholesky inverse when ``direct``. Returns (G, {block: beta_i}).
    """
    H = _c128(H)
    G = np.zeros_like(H)
    betas = {}
    for name, (rows, cols) in block_slices(M1, Mc, M2, K1, K2).items():
        Hi = H[rows, cols]
        if Hi.size == 0:
            betas[name] = 0.0
            continue
        if direct:
            _, Gi, beta = direct_rzf(Hi, xi, P_tx=P_tx)
        else:
            r = rzf(Hi, xi, tol=tol, max_iter=max_iter, P_tx=P_tx, precond=precond)
            Gi, beta = r["W"], r["beta_pow"]
        G[rows, cols] = Gi
        betas[name] = beta
    return G, betas


# ---------------------------------------------------------------------------
# Application-level evaluation (eqs. 9-10)
# ---------------------------------------------------------------------------
def sinr(H, W, sigma2):
    """Per-user SINR of precoder W on channel H (eq. 9 in its generic form).

    User k receives h_k^H g_k s_k plus the leakage of every other user's
    precoding vector plus noise of power sigma2; with block-structured H and G
    (eqs. 2 and 6) the same expression reproduces the intra-group,
    inter-subarray terms of eq. 9.
    """
    G = _c128(H).conj().T @ _c128(W)              # G[k, j] = h_k^H g_j
    P = G.real ** 2 + G.imag ** 2
    sig = np.diagonal(P).copy()
    interf = P.sum(axis=1) - sig
    return sig / (interf + float(sigma2))


def sum_rate(H, W, sigma2):
    """Sum of log2(1 + SINR_k) over users for one channel realisation (eq. 10)."""
    return float(np.sum(np.log2(1.0 + sinr(H, W, sigma2))))
