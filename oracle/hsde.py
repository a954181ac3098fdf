"""Plain FP64 CPU oracle of the HSDE-ADMM for chordally decomposed SDPs.

TEST INFRASTRUCTURE.  Only tests/, __graft_entry__.smoke() and bench.py's
cpu_baseline leg may import or run anything in this package.  It shares no
code with the GPU library (different language, different algebra route) and
is written from Zheng, Fantuzzi, Papachristodoulou, Goulart & Wynn, "Fast
ADMM for homogeneous self-dual embedding of sparse SDPs":

  * vectorised decomposed pair            Section 3.1, eqs. (PrimalVectorForm),
                                          (DualVectorForm); H_k = E_k (x) E_k
  * homogeneous self-dual embedding Q     Section 3.2, eq. (HomogeneousEmbedding)
  * ADMM steps 1-3                        Section 4.1, eqs. (Step1)-(Step3)
    + optional over-relaxation            the relaxed steps of O'Donoghue et al.
                                          2016, whose algorithm Section 4.1 applies
  * step 1 by block elimination           Section 4.2, eqs. (LinearSystem),
    + Sherman-Morrison                    (MatrixInverse), (FirstBlockElimination),
                                          (MatrixInverseResult)
  * inner system                          Section 4.3, eqs. (SecondBlockElimination)
                                          - (FactorizationMatrix), inverted with
                                          the matrix inversion lemma (Woodbury)

Coordinates.  The paper stacks full columns (vec, n^2 entries).  Here every
symmetric matrix is stored as svec over the lower-triangular entries of the
chordal pattern E' = U_k C_k x C_k (off-diagonals scaled by sqrt 2): an
isometry on symmetric matrices, under which H_k stays a 0/1 entry selector
and inner products and norms are unchanged.  `oracle.literal` runs the
paper's n^2 form on tiny problems to pin this reading.

Readings of the paper where it is silent or inconsistent:
  R1  svec over E' instead of vec over n^2 (above).
  R2  The inner system is eliminated onto the first block,
      (I + Ahat^T Ahat) u1 = w1 - Ahat^T w2, which is the matrix eq.
      (ThirdBlkElm) actually prints and leads to the factorised matrix
      I + D/2 + A^T A of eq. (FactorizationMatrix).
  R3  u0 = v0 = (0, 0, 0, 0, 1).
  R4  Residuals (O'Donoghue et al. 2016 normalisation, KKT rows of
      eqs. (PrimalFeasible)-(ZeroGap)):
        eps_p = ||(A x - tau b, H x - s)|| / (tau (1 + ||b||))
        eps_d = ||(A^T y + H^T v - tau c, v - z)|| / (tau (1 + ||c||))
        eps_g = |c^T x - b^T y| / (tau + |c^T x| + |b^T y|)
  R5  Infeasibility: primal if b^T y > 0 and
      ||(A^T y + H^T v, v - z)|| <= eps_tol b^T y; dual if c^T x < 0 and
      ||(A x, H x - s)|| <= eps_tol (-c^T x).  Checked every iteration in the
      order solved (tau > 0), primal infeasible, dual infeasible.
  R6  eps_tol = 1e-4, at most 2000 iterations (Section 5).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

SQRT2 = math.sqrt(2.0)

RUNNING, SOLVED, PRIMAL_INFEASIBLE, DUAL_INFEASIBLE, MAX_ITER = 0, 1, 2, 3, 4
STATUS_NAMES = {0: "running", 1: "solved", 2: "primal_infeasible",
                3: "dual_infeasible", 4: "max_iter"}


# ----------------------------------------------------------------------------
# conversion (Section 3.1)
# ----------------------------------------------------------------------------

@dataclass
class Problem:
    n: int
    m: int
    cliques: list
    erow: np.ndarray        # E' lower entries, sorted by (col, row)
    ecol: np.ndarray
    c: np.ndarray           # svec(C)
    A: sp.csr_matrix        # m x nE, rows svec(A_i)
    b: np.ndarray
    H: sp.csr_matrix        # ns x nE 0/1 selector
    slot_off: np.ndarray    # p+1 offsets of the clique blocks in s, z, v
    D: np.ndarray           # diag(H^T H)

    @property
    def nE(self):
        return len(self.erow)

    @property
    def ns(self):
        return int(self.slot_off[-1])


def _entry_index(n, erow, ecol):
    keys = erow.astype(np.int64) * n + ecol
    order = np.argsort(keys)
    return keys[order], order


def _lookup(n, keys_sorted, order, r, c):
    r = np.asarray(r, dtype=np.int64)
    c = np.asarray(c, dtype=np.int64)
    hi = np.maximum(r, c)
    lo = np.minimum(r, c)
    k = hi * n + lo
    pos = np.searchsorted(keys_sorted, k)
    if len(k) and (np.any(pos >= len(keys_sorted)) or np.any(keys_sorted[np.minimum(pos, len(keys_sorted) - 1)] != k)):
        raise ValueError("data entry outside the chordal pattern E'")
    return order[pos]


def clique_slots(K):
    """Local (a, b), a >= b, of a K-clique in the packed column-major order."""
    a, b = [], []
    for j in range(K):
        for i in range(j, K):
            a.append(i)
            b.append(j)
    return np.asarray(a, dtype=np.int64), np.asarray(b, dtype=np.int64)


def build_problem(inst) -> Problem:
    """O1-O4: E', svec data, the selectors H_k (Section 3.1)."""
    n, m = inst.n, inst.m
    cliques = [np.asarray(c, dtype=np.int64) for c in inst.cliques]
    for c in cliques:
        if len(c) == 0 or np.any(np.diff(c) <= 0) or c[0] < 0 or c[-1] >= n:
            raise ValueError("cliques must be non-empty, sorted, in range")
    cover = np.zeros(n, dtype=bool)
    for c in cliques:
        cover[c] = True
    if not cover.all():
        raise ValueError("every vertex needs a clique")
    keys = set()
    for c in cliques:
        a, b = clique_slots(len(c))
        keys.update(zip(c[b].tolist(), c[a].tolist()))   # (col, row), row >= col
    arr = np.array(sorted(keys), dtype=np.int64).reshape(-1, 2)
    ecol, erow = arr[:, 0].copy(), arr[:, 1].copy()
    nE = len(erow)
    ks, order = _entry_index(n, erow, ecol)

    def svec_coo(r, cidx, v):
        idx = _lookup(n, ks, order, r, cidx)
        scale = np.where(np.asarray(r) == np.asarray(cidx), 1.0, SQRT2)
        return idx, scale * np.asarray(v, dtype=np.float64)

    cr, cc, cv = inst.C
    idx, val = svec_coo(cr, cc, cv)
    c = np.zeros(nE)
    np.add.at(c, idx, val)

    con, ar, ac, av = inst.A
    idx, val = svec_coo(ar, ac, av)
    A = sp.csr_matrix((val, (np.asarray(con, dtype=np.int64), idx)), shape=(m, nE))
    A.sum_duplicates()

    rows, cols = [], []
    off = [0]
    for c_ in cliques:
        a, b = clique_slots(len(c_))
        ent = _lookup(n, ks, order, c_[a], c_[b])
        rows.append(np.arange(off[-1], off[-1] + len(a)))
        cols.append(ent)
        off.append(off[-1] + len(a))
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    ns = off[-1]
    H = sp.csr_matrix((np.ones(ns), (rows, cols)), shape=(ns, nE))
    D = np.asarray(H.multiply(H).sum(axis=0)).ravel()
    return Problem(n, m, cliques, erow, ecol, c, A, np.asarray(inst.b, dtype=np.float64),
                   H, np.asarray(off, dtype=np.int64), D)


# ----------------------------------------------------------------------------
# step 1: affine projection (Sections 4.2-4.3)
# ----------------------------------------------------------------------------

class AffineCache:
    """Everything eq. (MatrixInverseResult) lets us cache before iterating:
    the factor of the inner matrix and M^{-1} zeta, 1 + zeta^T M^{-1} zeta."""

    def __init__(self, prob: Problem):
        self.prob = prob
        P = 1.0 + 0.5 * prob.D                      # I + D/2 (diagonal)
        self.Pinv = 1.0 / P
        A = prob.A
        # I + D/2 + A^T A = P + A^T A; matrix inversion lemma: only
        # K = I_m + A P^{-1} A^T (m x m) is factorised.
        K = (sp.identity(prob.m, format="csr") + A @ sp.diags(self.Pinv) @ A.T).toarray()
        self.K = K
        self.Kfac = sla.cho_factor(K, lower=True)
        # zeta = (c_hat; b_hat) = (c, 0, -b, 0)
        zeta = self.split_zeros()
        zeta[0][:] = prob.c
        zeta[2][:] = -prob.b
        self.zeta = zeta
        self.zt = self.inner_solve(zeta)
        self.den = 1.0 + self.dot(zeta, self.zt)

    def split_zeros(self):
        p = self.prob
        return [np.zeros(p.nE), np.zeros(p.ns), np.zeros(p.m), np.zeros(p.ns)]

    @staticmethod
    def dot(a, b):
        return sum(float(x @ y) for x, y in zip(a, b))

    def F_solve(self, r):
        """(I + D/2 + A^T A)^{-1} r by the matrix inversion lemma."""
        A = self.prob.A
        q = self.Pinv * r
        w = sla.cho_solve(self.Kfac, A @ q)
        return q - self.Pinv * (A.T @ w)

    def inner_solve(self, t):
        """M^{-1} t with M = [[I, Ahat^T], [-Ahat, I]], Ahat = [[-A, 0], [-H, I]].

        Eliminate onto the first block (reading R2):
          (I + Ahat^T Ahat) p1 = t1 - Ahat^T t2,
          I + Ahat^T Ahat = [[I + D + A^T A, -H^T], [-H, 2I]],
        then the s-block once more, leaving I + D/2 + A^T A for p_x;
        finally p2 = t2 + Ahat p1.
        """
        A, H = self.prob.A, self.prob.H
        tx, ts, ty, tv = t
        # r = t1 - Ahat^T t2 ;  Ahat^T = [[-A^T, -H^T], [0, I]]
        rx = tx + A.T @ ty + H.T @ tv
        rs = ts - tv
        px = self.F_solve(rx + 0.5 * (H.T @ rs))
        ps = 0.5 * (rs + H @ px)
        # p2 = t2 + Ahat p1 ;  Ahat p1 = (-A px, -H px + ps)
        py = ty - A @ px
        pv = tv - H @ px + ps
        return [px, ps, py, pv]

    def solve(self, omega):
        """Step 1: u_hat = (I+Q)^{-1} omega via eqs. (MatrixInverse),
        (FirstBlockElimination), (MatrixInverseResult)."""
        w12, w3 = omega[:4], omega[4]
        t = [a - w3 * z for a, z in zip(w12, self.zeta)]
        p = self.inner_solve(t)
        # Sherman-Morrison: u12 = p - M^{-1} zeta (zeta^T p) / (1 + zeta^T M^{-1} zeta)
        g = self.dot(self.zeta, p) / self.den
        u12 = [a - g * z for a, z in zip(p, self.zt)]
        c_hat_u1 = float(self.prob.c @ u12[0])
        b_hat_u2 = float(-self.prob.b @ u12[2])
        u3 = w3 + c_hat_u1 + b_hat_u2
        return u12 + [u3]


def apply_Q(prob: Problem, u):
    """Q u for the HSDE matrix of eq. (HomogeneousEmbedding), matrix-free."""
    x, s, y, v, tau = u
    A, H, c, b = prob.A, prob.H, prob.c, prob.b
    h = -(A.T @ y) - (H.T @ v) + c * tau
    z = v.copy()
    r = A @ x - b * tau
    w = H @ x - s
    kap = -float(c @ x) + float(b @ y)
    return [h, z, r, w, kap]


# ----------------------------------------------------------------------------
# step 2: projection onto K (Section 3.2 cone, Section 4.1)
# ----------------------------------------------------------------------------

def smat_blocks(vec, K):
    """Packed svec block(s) -> full symmetric K x K matrices (batched)."""
    a, b = clique_slots(K)
    scale = np.where(a == b, 1.0, 1.0 / SQRT2)
    M = np.zeros(vec.shape[:-1] + (K, K))
    M[..., a, b] = vec * scale
    M[..., b, a] = vec * scale
    return M


def svec_blocks(M, K):
    a, b = clique_slots(K)
    scale = np.where(a == b, 1.0, SQRT2)
    return M[..., a, b] * scale


def proj_psd(M):
    """Euclidean projection onto the PSD cone: V max(Lambda, 0) V^T."""
    lam, V = np.linalg.eigh(M)
    return (V * np.maximum(lam, 0.0)[..., None, :]) @ np.swapaxes(V, -1, -2)


def proj_psd_packed(vec, sizes, offsets):
    """Project every packed clique block (batched by equal size)."""
    out = np.empty_like(vec)
    sizes = np.asarray(sizes)
    for K in np.unique(sizes):
        ks = np.where(sizes == K)[0]
        nk = K * (K + 1) // 2
        idx = offsets[ks][:, None] + np.arange(nk)[None, :]
        blocks = vec[idx]
        out[idx] = svec_blocks(proj_psd(smat_blocks(blocks, int(K))), int(K))
    return out


# ----------------------------------------------------------------------------
# the iteration and the solver
# ----------------------------------------------------------------------------

def initial_point(prob: Problem):
    """Reading R3: u0 = v0 = (0, 0, 0, 0, 1)."""
    z = lambda k: np.zeros(k)
    u = [z(prob.nE), z(prob.ns), z(prob.m), z(prob.ns), 1.0]
    vt = [z(prob.nE), z(prob.ns), z(prob.m), z(prob.ns), 1.0]
    return u, vt


def iterate(prob: Problem, cache: AffineCache, u, vt, sizes, alpha=1.0):
    """One ADMM iteration, eqs. (Step1)-(Step3).

    alpha != 1 is the over-relaxed form of the same algorithm (O'Donoghue et
    al. 2016, the method Section 4.1 applies): steps 2 and 3 take
    alpha u_hat + (1 - alpha) u in place of u_hat.  alpha = 1 is the paper's
    iteration exactly."""
    omega = [a + b for a, b in zip(u, vt)]
    uh = cache.solve(omega)                                   # (Step1)
    if alpha != 1.0:
        uh = [alpha * a + (1.0 - alpha) * b for a, b in zip(uh, u)]
    d = [a - b for a, b in zip(uh, vt)]                       # u_hat - v
    un = [d[0].copy(),                                        # free (x)
          proj_psd_packed(d[1], sizes, prob.slot_off[:-1]),    # S = S_1 x ... x S_p
          d[2].copy(),                                        # free (y)
          d[3].copy(),                                        # free (v)
          max(0.0, d[4])]                                     # R_+ (tau)
    vn = [a - b + c for a, b, c in zip(vt, uh, un)]           # (Step3)
    return un, vn


def residuals(prob: Problem, u, vt, nb=None, nc=None):
    """Readings R4/R5 on the current iterate."""
    x, s, y, v, tau = u
    z, kap = vt[1], vt[4]
    A, H, b, c = prob.A, prob.H, prob.b, prob.c
    nb = float(np.linalg.norm(b)) if nb is None else nb
    nc = float(np.linalg.norm(c)) if nc is None else nc
    Ax = A @ x
    Hx_s = H @ x - s
    dual_lin = A.T @ y + H.T @ v
    v_z = v - z
    cx = float(c @ x)
    by = float(b @ y)
    r = dict(cx=cx, by=by, tau=tau, kappa=kap)
    r["pri_sq"] = float((Ax - tau * b) @ (Ax - tau * b) + Hx_s @ Hx_s)
    r["dua_sq"] = float((dual_lin - tau * c) @ (dual_lin - tau * c) + v_z @ v_z)
    r["pinf_sq"] = float(dual_lin @ dual_lin + v_z @ v_z)
    r["dinf_sq"] = float(Ax @ Ax + Hx_s @ Hx_s)
    if tau > 0:
        r["eps_p"] = math.sqrt(r["pri_sq"]) / (tau * (1.0 + nb))
        r["eps_d"] = math.sqrt(r["dua_sq"]) / (tau * (1.0 + nc))
    else:
        r["eps_p"] = r["eps_d"] = math.inf
    r["eps_g"] = abs(cx - by) / (tau + abs(cx) + abs(by)) if (tau + abs(cx) + abs(by)) > 0 else math.inf
    return r


def status_of(r, eps_tol):
    if r["tau"] > 0 and r["eps_p"] <= eps_tol and r["eps_d"] <= eps_tol and r["eps_g"] <= eps_tol:
        return SOLVED
    if r["by"] > 0 and math.sqrt(r["pinf_sq"]) <= eps_tol * r["by"]:
        return PRIMAL_INFEASIBLE
    if r["cx"] < 0 and math.sqrt(r["dinf_sq"]) <= eps_tol * (-r["cx"]):
        return DUAL_INFEASIBLE
    return RUNNING


@dataclass
class Result:
    status: int
    iters: int
    u: list
    vt: list
    res: dict
    history: list
    prob: Problem


def solve(inst_or_prob, eps_tol=1e-4, max_iter=2000, record=0, stop=True, cache=None, state=None,
          alpha=1.0):
    """Run the ADMM until a status other than running (R5) or max_iter
    (alpha: relaxation of steps 2-3, see iterate)."""
    prob = inst_or_prob if isinstance(inst_or_prob, Problem) else build_problem(inst_or_prob)
    cache = cache or AffineCache(prob)
    sizes = np.diff(prob.slot_off)
    sizes = ((np.sqrt(8 * sizes + 1) - 1) / 2).round().astype(np.int64)
    u, vt = state if state is not None else initial_point(prob)
    nb, nc = float(np.linalg.norm(prob.b)), float(np.linalg.norm(prob.c))
    history = []
    st = RUNNING
    r = {}
    k = 0
    for k in range(1, max_iter + 1):
        u, vt = iterate(prob, cache, u, vt, sizes, alpha)
        if k <= record:
            history.append(([a.copy() if isinstance(a, np.ndarray) else a for a in u],
                            [a.copy() if isinstance(a, np.ndarray) else a for a in vt]))
        r = residuals(prob, u, vt, nb, nc)
        st = status_of(r, eps_tol)
        if stop and st != RUNNING:
            break
    if st == RUNNING and k >= max_iter:
        st = MAX_ITER
    return Result(st, k, u, vt, r, history, prob)


def clique_sizes(prob: Problem):
    return np.array([len(c) for c in prob.cliques], dtype=np.int64)


# ----------------------------------------------------------------------------
# recovery (O'Donoghue et al. 2016, as cited in Section 3.2)
# ----------------------------------------------------------------------------

def recover(res: Result):
    """Solved: X on E', y, Z = sum_k E_k^T Z_k E_k with Z_k = smat(z_k)/tau
    (Agler, Theorem 2).  Infeasible: the certificate scaled as R5 states."""
    prob = res.prob
    x, s, y, v, tau = res.u
    z = res.vt[1]
    out = dict(status=res.status)
    if res.status == SOLVED:
        out["x"] = x / tau
        out["y"] = y / tau
        out["Zvec"] = (prob.H.T @ z) / tau     # svec(Z) over E'
        out["obj_p"] = float(prob.c @ x) / tau
        out["obj_d"] = float(prob.b @ y) / tau
    elif res.status == PRIMAL_INFEASIBLE:
        by = float(prob.b @ y)
        out["y_cert"] = y / by
        out["v_cert"] = v / by
    elif res.status == DUAL_INFEASIBLE:
        cx = float(prob.c @ x)
        out["x_cert"] = x / (-cx)
        out["s_cert"] = s / (-cx)
    return out


def svec_to_dense(prob: Problem, xvec):
    """Symmetric n x n matrix with the E' entries of an svec vector (zeros elsewhere)."""
    X = np.zeros((prob.n, prob.n))
    scale = np.where(prob.erow == prob.ecol, 1.0, 1.0 / SQRT2)
    X[prob.erow, prob.ecol] = xvec * scale
    X[prob.ecol, prob.erow] = xvec * scale
    return X


def state_vector(u, vt):
    """Flatten (u, v~) in the fixed order x, s, y, v, tau, h, z, r, w, kappa."""
    parts = []
    for blk in list(u) + list(vt):
        parts.append(np.atleast_1d(np.asarray(blk, dtype=np.float64)))
    return np.concatenate(parts)
