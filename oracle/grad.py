"""Gradients of a solved SDP through the ADMM fixed point (TEST INFRASTRUCTURE).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may use
this module.

With z = u - v~ the iteration of eqs. (Step1)-(Step3) is
    z+ = T(z) = z + R (2 Pi(z) - z) - Pi(z),   R = (I + Q)^{-1},
since u = Pi_K(z) and v~ = Pi_K(z) - z (Moreau).  A fixed point satisfies
v~* = Q u* (eq. HomogeneousEmbedding).  For data theta = (c, b) entering Q,
differentiating z* = T(z*, theta) gives
    (I - T') dz = dR (2 Pi - z) = -R dQ u*,   T' = I + R (2 DPi - I) - DPi,
and for a loss L(u*) with g = DPi dL/du:
    (I - T')^T mu = g,   nu = R^T mu = (I - Q)^{-1} mu,   dL = -nu^T dQ u*.
Q holds c in its (x, tau) block, -c^T in (tau, x), -b in (y, tau) and b^T in
(tau, y), so
    dL/dc = -(tau nu_x - nu_tau x),   dL/db = tau nu_y - nu_tau y.
The fixed point is a ray (T is positively homogeneous), so I - T' is singular
along z*; a degree-0 homogeneous loss (X = x / tau) keeps the adjoint system
consistent and any solution gives the same gradient.

The loss here is L = <W, X*> = w^T x / tau with w = svec(W) over E'.
DPi on a PSD block at Y = V diag(lam) V^T maps dY to V (B o (V^T dY V)) V^T
with B_ij = 1 (both lam > 0), 0 (both <= 0), (lam_i^+ - lam_j^+)/(lam_i - lam_j)
otherwise (Daleckii-Krein).
"""
from __future__ import annotations

import numpy as np

from . import hsde, literal


def dproj_block(Y, dY):
    """Derivative of the PSD projection at Y applied to dY (symmetric matrices)."""
    lam, V = np.linalg.eigh(Y)
    pos = lam > 0
    lp = np.maximum(lam, 0.0)
    K = len(lam)
    B = np.zeros((K, K))
    for i in range(K):
        for j in range(K):
            if pos[i] and pos[j]:
                B[i, j] = 1.0
            elif pos[i] != pos[j]:
                B[i, j] = (lp[i] - lp[j]) / (lam[i] - lam[j])
    return V @ (B * (V.T @ dY @ V)) @ V.T


def dproj_packed(zs, d, prob):
    """DPi_S at the slot vector zs applied to d (both packed svec clique blocks)."""
    out = np.empty_like(d)
    sizes = hsde.clique_sizes(prob)
    for k, K in enumerate(sizes):
        sl = slice(prob.slot_off[k], prob.slot_off[k + 1])
        Y = hsde.smat_blocks(zs[sl], int(K))
        dY = hsde.smat_blocks(d[sl], int(K))
        out[sl] = hsde.svec_blocks(dproj_block(Y, dY), int(K))
    return out


def flat(parts):
    return np.concatenate([np.atleast_1d(np.asarray(p, dtype=np.float64)) for p in parts])


def offsets(prob):
    return np.cumsum([0, prob.nE, prob.ns, prob.m, prob.ns, 1])


def dproj_full(z, prob):
    """DPi_K at z as a dense matrix (free, PSD blocks, free, free, R_+)."""
    off = offsets(prob)
    N = off[-1]
    D = np.zeros((N, N))
    D[off[0]:off[1], off[0]:off[1]] = np.eye(prob.nE)
    D[off[2]:off[3], off[2]:off[3]] = np.eye(prob.m)
    D[off[3]:off[4], off[3]:off[4]] = np.eye(prob.ns)
    D[off[4], off[4]] = 1.0 if z[off[4]] > 0 else 0.0
    zs = z[off[1]:off[2]]
    for j in range(prob.ns):
        e = np.zeros(prob.ns)
        e[j] = 1.0
        D[off[1]:off[2], off[1] + j] = dproj_packed(zs, e, prob)
    return D


def loss_and_du(prob, u, w):
    """L = w^T x / tau and dL/du for u = (x, s, y, v, tau)."""
    x, tau = u[0], u[4]
    L = float(w @ x) / tau
    g = [w / tau, np.zeros(prob.ns), np.zeros(prob.m), np.zeros(prob.ns), -float(w @ x) / tau ** 2]
    return L, flat(g)


def adjoint_gradient_dense(res, w):
    """dL/dc and dL/db at a solved instance (dense linear algebra; small problems)."""
    prob = res.prob
    u = flat(res.u)
    vt = flat(res.vt)
    z = u - vt
    IQ, off = literal.dense_affine_matrix_svec(prob)
    N = off[-1]
    R = np.linalg.inv(IQ)
    DP = dproj_full(z, prob)
    Tp = np.eye(N) + R @ (2 * DP - np.eye(N)) - DP
    _, gu = loss_and_du(prob, res.u, w)
    g = DP @ gu
    Aadj = (np.eye(N) - Tp).T
    try:
        mu = np.linalg.lstsq(Aadj, g, rcond=None)[0]
    except np.linalg.LinAlgError:
        # the divide-and-conquer SVD of gelsd does not converge on some of
        # these matrices: the same minimum-norm least-squares solution from
        # the QR-iteration SVD (gelss)
        import scipy.linalg as sla
        mu = sla.lstsq(Aadj, g, lapack_driver="gelss")[0]
    nu = R.T @ mu
    tau = u[off[4]]
    x = u[off[0]:off[1]]
    y = u[off[2]:off[3]]
    nux = nu[off[0]:off[1]]
    nuy = nu[off[2]:off[3]]
    nut = nu[off[4]]
    return -(tau * nux - nut * x), tau * nuy - nut * y


def adjoint_step(prob, cache_T, z, mu, g):
    """One step of the adjoint fixed-point iteration mu <- T'^T mu + g,
    T'^T mu = mu - q + DPi(2q - mu) with q = (I - Q)^{-1} mu."""
    q = cache_T.solve_transpose(mu)
    return mu - q + dproj_apply(prob, z, 2 * q - mu) + g


def dproj_apply(prob, z, d):
    off = offsets(prob)
    out = d.copy()
    out[off[1]:off[2]] = dproj_packed(z[off[1]:off[2]], d[off[1]:off[2]], prob)
    out[off[4]] = d[off[4]] if z[off[4]] > 0 else 0.0
    return out


class TransposeSolver:
    """(I - Q)^{-1} = ((I + Q)^{-1})^T by a dense LU (small problems)."""

    def __init__(self, prob):
        IQ, off = literal.dense_affine_matrix_svec(prob)
        import scipy.linalg as sla
        self.lu = sla.lu_factor(IQ.T)
        self._sla = sla

    def solve_transpose(self, mu):
        return self._sla.lu_solve(self.lu, mu)


def objective_weight_loss(inst, w, eps_tol=1e-10, max_iter=200000):
    """L(C, b) = <W, X*> on a tightly solved instance (for finite differences)."""
    res = hsde.solve(inst, eps_tol=eps_tol, max_iter=max_iter)
    if res.status != hsde.SOLVED:
        raise RuntimeError(f"not solved: {hsde.STATUS_NAMES[res.status]}")
    return float(w @ res.u[0]) / res.u[4], res
