"""The exterior Neumann problem through the integral equation of Sec. 1 (eq. ext-neumann-ie).

With the solution written as a single layer potential u = S mu outside the curves, the Neumann
condition n . grad u -> g from outside becomes the second-kind equation

    -mu/2 + S' mu = g   on the curves,

S' mu the normal derivative of S mu at the curve (the principal value: the average of the two
one-sided limits, which is what the library's GQ_SP evaluation returns at on-surface targets).
Once mu is known, u = S mu anywhere outside.

The equation is solved for many right-hand sides at once by GMRES (no restart): every right-hand
side keeps its own Krylov space and Hessenberg matrix, and each iteration applies the operator to
all of them with one batched GQ_SP evaluation of the library. The orthogonalisation and the small
least-squares updates are vector operations on the device arrays the evaluation reads and writes.
"""
from __future__ import annotations

import torch

from ._lib import GQ_SP


def neumann_operator(fmm):
    """mu (n_rhs, n_src) device tensor -> -mu/2 + S' mu, by the library (targets = the nodes,
    target normals set with ``fmm.set_target_normals``)."""
    def apply(mu):
        return -0.5 * mu + fmm.eval(GQ_SP, mu).reshape(mu.shape)
    return apply


def gmres(apply, b, tol: float = 1e-10, maxiter: int = 100):
    """Solve apply(x) = b for every row of b (n_rhs, n) at once.

    Returns (x, iterations, relative residuals): x like b; for each right-hand side the number of
    iterations after which its residual estimate |g_{j+1}| / |b| first fell to tol (maxiter if
    never) and the final estimate. Modified Gram-Schmidt, Givens rotations; a right-hand side
    that has converged keeps iterating with the others (its residual only shrinks further).
    """
    if b.dim() == 1:
        b = b[None, :]
    k, n = b.shape
    dt, dev = b.dtype, b.device
    beta = torch.linalg.vector_norm(b, dim=1)
    safe = torch.where(beta > 0, beta, torch.ones_like(beta))
    V = torch.zeros((maxiter + 1, k, n), dtype=dt, device=dev)
    V[0] = b / safe[:, None]
    H = torch.zeros((k, maxiter + 1, maxiter), dtype=dt, device=dev)
    cs = torch.zeros((k, maxiter), dtype=dt, device=dev)
    sn = torch.zeros((k, maxiter), dtype=dt, device=dev)
    g = torch.zeros((k, maxiter + 1), dtype=dt, device=dev)
    g[:, 0] = beta
    its = torch.full((k,), maxiter, dtype=torch.int64, device=dev)
    m = 0
    for j in range(maxiter):
        w = apply(V[j])
        for i in range(j + 1):
            h = (w * V[i]).sum(dim=1)
            H[:, i, j] = h
            w = w - h[:, None] * V[i]
        hn = torch.linalg.vector_norm(w, dim=1)
        H[:, j + 1, j] = hn
        V[j + 1] = w / torch.where(hn > 0, hn, torch.ones_like(hn))[:, None]
        for i in range(j):
            a, c = H[:, i, j].clone(), H[:, i + 1, j].clone()
            H[:, i, j] = cs[:, i] * a + sn[:, i] * c
            H[:, i + 1, j] = -sn[:, i] * a + cs[:, i] * c
        d = torch.hypot(H[:, j, j], H[:, j + 1, j])
        d = torch.where(d > 0, d, torch.ones_like(d))
        cs[:, j] = H[:, j, j] / d
        sn[:, j] = H[:, j + 1, j] / d
        H[:, j, j] = d
        H[:, j + 1, j] = 0.0
        g[:, j + 1] = -sn[:, j] * g[:, j]
        g[:, j] = cs[:, j] * g[:, j]
        m = j + 1
        res = g[:, j + 1].abs() / safe
        newly = (res <= tol) & (its == maxiter)
        its = torch.where(newly, torch.full_like(its, m), its)
        if bool((its < maxiter).all()) or bool((res <= tol).all()):
            break
    # back substitution in the m x m triangular systems, then x = sum_i y_i v_i
    R = H[:, :m, :m]
    y = torch.linalg.solve_triangular(R, g[:, :m, None], upper=True)[..., 0]
    x = torch.einsum("ki,ikn->kn", y, V[:m])
    res = g[:, m].abs() / safe
    return x, its.cpu().numpy(), res.cpu().numpy()
