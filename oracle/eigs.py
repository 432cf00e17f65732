"""Oracle: eigenpairs of the Dey--Mittra cavity problem (TEST INFRASTRUCTURE ONLY).

Result definition.  The wanted eigenpairs are the smallest lambda > 0 of the
symmetric pencil K b = lambda A b with K = C L C^T (eq. discWaveBDM
multiplied by A), restricted to the active faces.  Grad-div augmentation,
A-scaling, the shift and the projection (eqs. discLaplBDM, discLaplDM,
proj, fullMat) leave these pairs unchanged; they only change the cost.  So:

* ``dense_eigs``   writes the definition out: scipy.linalg.eigh(K, A) and
                   drop the gradient null space (lambda below 1e-8 lambda_max).
* ``lanczos_eigs`` is the plain iterative route of Sec. 4.1 / eq. fullMat:
                   block Lanczos with full re-orthogonalisation in the
                   A-inner product (eq. bInner) on T = P_DM M^-1 A, inner
                   solves by preconditioned CG at an SPD shift, projection
                   P_DM = I - D^T (D A D^T)^+ D A by CG, and Rayleigh--Ritz on
                   (K, A) in the Krylov basis.
* ``eig_residual`` is rho = ||K b - lambda A b||_{A^-1} / (lambda ||b||_A),
                   the residual of the symmetric form A^-1/2 K A^-1/2 (the
                   scaled operator of eq. transformation).

Pinned in tests against the closed-form PEC-box spectrum, dense eigh on
small grids, and the analytic TM/TE sphere modes (second-order
convergence, Sec. 6.2).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sl
import scipy.sparse.csgraph as csg


def dense_eigs(op, k=None):
    """Smallest nonzero eigenpairs of (K, A) by dense eigh (tiny grids)."""
    K = op.K_a.toarray()
    w, V = sl.eigh(K, np.diag(op.a_a))
    keep = w > 1e-8 * w.max()
    w, V = w[keep], V[:, keep]
    if k is not None:
        w, V = w[:k], V[:, :k]
    return w, V


def eig_residual(op, lam, b):
    r = op.K_a @ b - lam * op.a_a * b
    num = math.sqrt(float(np.sum(r * r / op.a_a)))
    den = lam * math.sqrt(float(np.sum(op.a_a * b * b)))
    return num / den


def div_residual(op, b):
    """||V^-1/2 D A b|| / ||b||_A : the divergence left in b (Sec. 5.1)."""
    g = op.D_a @ (op.a_a * b)
    return math.sqrt(float(np.sum(g * g / op.v_a))) / math.sqrt(float(np.sum(op.a_a * b * b)))


def pcg(apply, rhs, tol, maxiter, precond=None, deflate=None):
    """Plain preconditioned conjugate gradients for an SPD operator.

    ``deflate`` (optional) is a projector onto the complement of a known
    null space, applied to the right-hand side and to every preconditioned
    residual (consistent singular systems).
    """
    if deflate is not None:
        rhs = deflate(rhs)
    x = np.zeros_like(rhs)
    r = rhs.copy()
    bnorm = np.linalg.norm(rhs)
    if bnorm == 0.0:
        return x, 0
    z = precond(r) if precond else r.copy()
    if deflate is not None:
        z = deflate(z)
    p = z.copy()
    rz = float(r @ z)
    for it in range(1, maxiter + 1):
        q = apply(p)
        alpha = rz / float(p @ q)
        x += alpha * p
        r -= alpha * q
        if np.linalg.norm(r) <= tol * bnorm:
            return x, it
        z = precond(r) if precond else r.copy()
        if deflate is not None:
            z = deflate(z)
        rz_new = float(r @ z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    raise RuntimeError(f"pcg: no convergence in {maxiter} iterations")


class Projector:
    """P_DM b = b - D^T S^+ D A b with S = D A D^T (eq. proj).

    S is singular on every connected group of active cells that no
    boundary pins (its constants); the right-hand side D A b sums to zero
    over such a group, so the mean-free solution is taken.
    """

    def __init__(self, op, tol=1e-13, maxiter=20000):
        self.op = op
        self.tol = tol
        self.maxiter = maxiter
        S = op.S_a
        ncomp, labels = csg.connected_components(S, directed=False)
        self.floating = []
        for c in range(ncomp):
            ind = np.flatnonzero(labels == c)
            one = np.zeros(S.shape[0])
            one[ind] = 1.0
            if np.linalg.norm(S @ one) <= 1e-12 * max(1.0, abs(S.diagonal()).max()) * math.sqrt(ind.size):
                self.floating.append(ind)
        d = S.diagonal()
        self.dinv = np.where(d > 0.0, 1.0 / np.where(d > 0.0, d, 1.0), 0.0)

    def _deflate(self, x):
        x = x.copy()
        for ind in self.floating:
            x[ind] -= x[ind].mean()
        return x

    def __call__(self, b):
        op = self.op
        rhs = op.D_a @ (op.a_a * b)
        psi, _ = pcg(lambda p: op.S_a @ p, rhs, self.tol, self.maxiter,
                     precond=lambda r: self.dinv * r, deflate=self._deflate)
        return b - op.D_a.T @ psi


def _a_orthonormalize(W, a, basis=None):
    """CGS2 against ``basis`` then Cholesky-QR (twice) in the A-inner product."""
    if basis is not None and basis.shape[1]:
        for _ in range(2):
            W = W - basis @ (basis.T @ (a[:, None] * W))
    for _ in range(2):
        G = W.T @ (a[:, None] * W)
        Rf = np.linalg.cholesky(0.5 * (G + G.T)).T
        W = sl.solve_triangular(Rf, W.T, trans="T").T
    return W


def augmented_eigs(op, k, sigma_o=0.0, block=4, tol=1e-10, max_blocks=60, seed=1301,
                   cg_tol=1e-12, precond=None, maxiter=100000, div_tol=1e-6, log=None):
    """k smallest electromagnetic eigenpairs via the augmented pencil.

    Sec. 5.1 (after eq. discLaplBDM): every eigenpair of (K, A) with
    lambda > 0 is an eigenpair of the grad-div augmented pencil (K + G, A),
    whose remaining eigenpairs are the gradient modes (D A b != 0).  So:
    block Lanczos with full re-orthogonalisation on M^-1 A (M = K + G -
    sigma_o A SPD, no projection), Rayleigh--Ritz on (K + G, A), and keep the
    Ritz pairs whose divergence ||V^-1/2 D A b|| / ||b||_A is below div_tol.
    Used where the projection's CG would be too slow (large grids); pinned
    against ``lanczos_eigs`` and dense eigh on small grids.
    """
    M = op.M_a if op.sigma == sigma_o else op.with_shift(sigma_o).M_a
    KG = (op.K_a + op.G_a).tocsr()
    a = op.a_a
    n = a.size
    if precond is None:
        dinv = 1.0 / M.diagonal()
        precond = lambda r: dinv * r  # noqa: E731
    rng = np.random.default_rng(seed)
    V = _a_orthonormalize(rng.standard_normal((n, block)), a)
    KV = KG @ V
    n_solves = cg_its = 0
    lam = B = res = None
    for it in range(max_blocks):
        last = V[:, -block:]
        W = np.empty_like(last)
        for c in range(block):
            W[:, c], its = pcg(lambda p: M @ p, a * last[:, c], cg_tol, maxiter, precond=precond)
            n_solves += 1
            cg_its += its
        W = _a_orthonormalize(W, a, V)
        V = np.hstack([V, W])
        KV = np.hstack([KV, KG @ W])
        H = V.T @ KV
        theta, Y = np.linalg.eigh(0.5 * (H + H.T))
        em = []
        for c in np.argsort(theta):
            b = V @ Y[:, c]
            if div_residual(op, b) < div_tol:
                em.append((theta[c], b))
            if len(em) == k:
                break
        if len(em) < k:
            continue
        lam = np.array([e[0] for e in em])
        B = np.column_stack([e[1] for e in em])
        res = np.array([eig_residual(op, lam[c], B[:, c]) for c in range(k)])
        if log:
            log(f"augmented block {it}: dim {V.shape[1]} max res {res.max():.3e}")
        if res.max() <= tol:
            break
    return lam, B, dict(n_solves=n_solves, cg_iters=cg_its, dim=V.shape[1], residuals=res)


def lanczos_eigs(op, k, sigma_o=0.0, block=4, tol=1e-10, max_blocks=60, seed=1301,
                 cg_tol=1e-13, proj_tol=1e-13, precond=None, maxiter=100000, log=None,
                 project=True):
    """k smallest nonzero eigenpairs of (K, A) by shift-and-invert block Lanczos.

    ``sigma_o`` must keep M = K + G - sigma_o A positive definite (below both
    the lowest electromagnetic eigenvalue and the lowest nonzero eigenvalue
    of (S, V)); sigma_o = 0 is always safe because K + G has a trivial null
    space (Sec. 4.3, text after eq. hodge).  ``precond`` is an optional SPD
    preconditioner for M (default Jacobi).  With ``project=False`` the
    projection P_DM is skipped: the Krylov basis then also holds gradient
    modes b = D^T psi, which Rayleigh--Ritz on (K, A) maps to lambda = 0 and
    discards (eq. hodge: K D^T = 0), so the returned pairs are the same.

    Returns (lam, B, info) with B A-orthonormal columns.
    """
    M = op.M_a if op.sigma == sigma_o else op.with_shift(sigma_o).M_a
    a = op.a_a
    n = a.size
    if precond is None:
        dinv = 1.0 / M.diagonal()
        precond = lambda r: dinv * r  # noqa: E731
    proj = Projector(op, tol=proj_tol) if project else (lambda b: b)
    rng = np.random.default_rng(seed)
    V0 = rng.standard_normal((n, block))
    V0 = np.column_stack([proj(V0[:, c]) for c in range(block)])
    V = _a_orthonormalize(V0, a)
    KV = op.K_a @ V
    n_solves = 0
    cg_its = 0
    lam = B = res = None
    for it in range(max_blocks):
        last = V[:, -block:]
        W = np.empty_like(last)
        for c in range(block):
            y, its = pcg(lambda p: M @ p, a * last[:, c], cg_tol, maxiter, precond=precond)
            W[:, c] = proj(y)
            n_solves += 1
            cg_its += its
        W = _a_orthonormalize(W, a, V)
        V = np.hstack([V, W])
        KV = np.hstack([KV, op.K_a @ W])
        H = V.T @ KV
        theta, Y = np.linalg.eigh(0.5 * (H + H.T))
        pos = np.flatnonzero(theta > 1e-8 * abs(theta).max())
        if pos.size < k:
            continue
        sel = pos[:k]
        lam = theta[sel]
        B = V @ Y[:, sel]
        res = np.array([eig_residual(op, lam[c], B[:, c]) for c in range(k)])
        if log:
            log(f"lanczos block {it}: dim {V.shape[1]} max res {res.max():.3e}")
        if res.max() <= tol:
            break
    info = dict(n_solves=n_solves, cg_iters=cg_its, dim=V.shape[1], residuals=res)
    return lam, B, info
