"""Plain FP64 CPU oracle of the primal-only and dual-only ADMM for chordally
decomposed SDPs (TEST INFRASTRUCTURE: only tests/, __graft_entry__.smoke()
and bench.py's cpu_baseline leg may import or run anything in this package).

Section 5 of Zheng, Fantuzzi, Papachristodoulou, Goulart & Wynn, "Fast ADMM
for homogeneous self-dual embedding of sparse SDPs" compares the self-dual
method with the primal and dual methods of the authors' earlier work on
chordal decomposition in operator-splitting methods (its reference
zheng2016fast; the CDCS-primal and CDCS-dual columns of Tables 2-4).  Both
work on the decomposed pair of Section 3.1 in the coordinates of oracle/hsde
(svec over E', packed clique blocks, H the entry selector, D = diag(H^T H)):

  primal (eq. DecomposedPriaml):  min c^T x  s.t.  A x = b,  s = H x,  s in S
  dual   (eq. DecomposedDual):    min -b^T y s.t.  A^T y + H^T v = c,  v = z,  z in S

with S the product of the clique PSD cones, and apply the textbook ADMM
(Boyd et al. 2011, Section 3) with penalty rho to the consensus constraint.

Primal method, multiplier lam of s = H x:
  1. x = argmin_{A x = b} c^T x + rho/2 ||s - H x + lam/rho||^2:
     the KKT system [[rho D, -A^T], [A, 0]] (x, y) = (H^T(rho s + lam) - c, b),
     eliminated onto the m x m matrix A D^-1 A^T:
       (A D^-1 A^T) y = rho b - A D^-1 r,   r = H^T(rho s + lam) - c,
       x = D^-1 (r + A^T y) / rho
  2. s = Pi_S(H x - lam/rho)
  3. lam = lam + rho (s - H x)
Dual method, multiplier lam of v = z:
  1. (y, v) = argmin_{A^T y + H^T v = c} -b^T y + rho/2 ||v - z + lam/rho||^2:
     with x the multiplier of the equality,
       (A D^-1 A^T) y = b / rho - A D^-1 r,   r = H^T(z - lam/rho) - c,
       x = rho D^-1 (A^T y + r),   v = z - lam/rho - H x / rho
  2. z = Pi_S(v + lam/rho)
  3. lam = lam + rho (v - z)
At a fixed point the primal method's lam is the dual slack (lam in S,
<lam, s> = 0, A^T y + H^T lam = c) and the dual method's x is the primal
matrix (A x = b, H x = -lam in S).

Readings (the paper states none of this; each is listed with its reason):
  S1  rho fixed (default 1), no adaptive penalty.
  S2  Start from zero: s = lam = 0 (primal), z = lam = 0 (dual).
  S3  Stopping (Boyd et al. 2011, Section 3.3, relative form): primal method
        eps_p = ||s - H x|| / max(||s||, ||H x||),
        eps_d = rho ||s+ - s|| / ||lam+||;
      dual method
        eps_p = ||v - z+|| / max(||v||, ||z+||),
        eps_d = rho ||z+ - z|| / ||lam+||;
      both <= eps_tol (1e-4, at most 2000 iterations, as in Section 5),
      checked after every iteration; a zero denominator counts as not
      converged.
  S4  Objectives: primal c^T x and b^T y of the step-1 multiplier (primal
      method); b^T y and c^T x of the step-1 multiplier (dual method).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

from . import hsde

PRIMAL, DUAL = "primal", "dual"


class SplitCache:
    """The m x m matrix A D^-1 A^T of both methods' step 1, factorised once."""

    def __init__(self, prob: hsde.Problem, rho: float = 1.0):
        self.prob = prob
        self.rho = float(rho)
        self.Dinv = 1.0 / prob.D
        A = prob.A
        self.K = (A @ (A.multiply(self.Dinv[None, :])).T).toarray()
        self.Kfac = sla.cho_factor(self.K, lower=True)

    def solve_K(self, g):
        return sla.cho_solve(self.Kfac, g)


@dataclass
class SplitState:
    s: np.ndarray          # primal: s (= x_k blocks); dual: z
    lam: np.ndarray
    x: np.ndarray          # from the last step 1
    y: np.ndarray
    v: np.ndarray          # dual method only (v of step 1)


def initial_state(prob: hsde.Problem):
    """Reading S2."""
    return SplitState(np.zeros(prob.ns), np.zeros(prob.ns), np.zeros(prob.nE), np.zeros(prob.m),
                      np.zeros(prob.ns))


def primal_step1(prob, cache, s, lam):
    rho = cache.rho
    r = prob.H.T @ (rho * s + lam) - prob.c
    q = cache.Dinv * r
    y = cache.solve_K(rho * prob.b - prob.A @ q)
    x = cache.Dinv * (r + prob.A.T @ y) / rho
    return x, y


def dual_step1(prob, cache, z, lam):
    rho = cache.rho
    r = prob.H.T @ (z - lam / rho) - prob.c
    q = cache.Dinv * r
    y = cache.solve_K(prob.b / rho - prob.A @ q)
    x = rho * cache.Dinv * (prob.A.T @ y + r)
    v = z - lam / rho - (prob.H @ x) / rho
    return x, y, v


def iterate(prob, cache, st: SplitState, method, sizes):
    """One iteration of the primal or dual method; returns the new state and
    the residual figures of reading S3."""
    rho = cache.rho
    offs = prob.slot_off[:-1]
    if method == PRIMAL:
        x, y = primal_step1(prob, cache, st.s, st.lam)
        hx = prob.H @ x
        s_new = hsde.proj_psd_packed(hx - st.lam / rho, sizes, offs)
        lam = st.lam + rho * (s_new - hx)
        rp = float(np.linalg.norm(s_new - hx))
        pden = max(float(np.linalg.norm(s_new)), float(np.linalg.norm(hx)))
        rd = rho * float(np.linalg.norm(s_new - st.s))
        new = SplitState(s_new, lam, x, y, np.zeros(prob.ns))
    else:
        x, y, v = dual_step1(prob, cache, st.s, st.lam)
        z_new = hsde.proj_psd_packed(v + st.lam / rho, sizes, offs)
        lam = st.lam + rho * (v - z_new)
        rp = float(np.linalg.norm(v - z_new))
        pden = max(float(np.linalg.norm(v)), float(np.linalg.norm(z_new)))
        rd = rho * float(np.linalg.norm(z_new - st.s))
        new = SplitState(z_new, lam, x, y, v)
    dden = float(np.linalg.norm(lam))
    res = {"eps_p": rp / pden if pden > 0 else math.inf,
           "eps_d": rd / dden if dden > 0 else math.inf,
           "cx": float(prob.c @ x), "by": float(prob.b @ y)}
    return new, res


@dataclass
class SplitResult:
    status: int
    iters: int
    state: SplitState
    res: dict
    history: list
    prob: hsde.Problem


def solve(inst_or_prob, method, eps_tol=1e-4, max_iter=2000, rho=1.0, record=0, stop=True):
    prob = inst_or_prob if isinstance(inst_or_prob, hsde.Problem) else hsde.build_problem(inst_or_prob)
    cache = SplitCache(prob, rho)
    sizes = hsde.clique_sizes(prob)
    st = initial_state(prob)
    history = []
    res = {}
    status = hsde.RUNNING
    k = 0
    for k in range(1, max_iter + 1):
        st, res = iterate(prob, cache, st, method, sizes)
        if k <= record:
            history.append(SplitState(st.s.copy(), st.lam.copy(), st.x.copy(), st.y.copy(), st.v.copy()))
        if res["eps_p"] <= eps_tol and res["eps_d"] <= eps_tol:
            status = hsde.SOLVED
            if stop:
                break
    if status == hsde.RUNNING:
        status = hsde.MAX_ITER
    return SplitResult(status, k, st, res, history, prob)


def recover(r: SplitResult, method):
    """X on E' (svec), y, Z = sum_k E_k^T Z_k E_k (svec over E') and the
    objectives (reading S4)."""
    prob, st = r.prob, r.state
    if method == PRIMAL:
        Z = prob.H.T @ st.lam
    else:
        Z = prob.H.T @ st.s
    return {"x": st.x, "y": st.y, "Zvec": Z, "obj_p": float(prob.c @ st.x), "obj_d": float(prob.b @ st.y)}


def state_vector(prob, st: SplitState, method):
    """Flatten the iterate as the solver reports it: primal (x, s, y, lam),
    dual (x, z, y, lam, v)."""
    if method == PRIMAL:
        return np.concatenate([st.x, st.s, st.y, st.lam])
    return np.concatenate([st.x, st.s, st.y, st.lam, st.v])
