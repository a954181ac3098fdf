"""The paper's literal coordinates, for tiny problems only (TEST INFRASTRUCTURE).

Section 3.1 vectorises with vec (column stacking, n^2 entries) and
H_k = E_k (x) E_k; Section 3.2 assembles the HSDE matrix Q of eq.
(HomogeneousEmbedding) over K = R^{n^2} x S x R^m x R^{n_d} x R_+; step 1 of
Section 4.1 is the plain definition u_hat = (I+Q)^{-1}(u + v), solved here by
a dense LU of the assembled I + Q.  Nothing here is shared with the svec
oracle in `oracle.hsde` except the seeded instance it is given; comparing
the two pins reading R1 (svec over E') and the block-elimination route.
"""
from __future__ import annotations

import math

import numpy as np


def selector(clique, n):
    """E_C: (E_C)_{ij} = 1 iff C(i) = j (Section 2.2)."""
    E = np.zeros((len(clique), n))
    E[np.arange(len(clique)), np.asarray(clique)] = 1.0
    return E


def vec(M):
    return M.reshape(-1, order="F")


def unvec(x, k):
    return x.reshape((k, k), order="F")


def dense_sym(n, coo):
    r, c, v = coo
    M = np.zeros((n, n))
    for i, j, val in zip(r, c, v):
        M[i, j] += val
        if i != j:
            M[j, i] += val
    return M


class Literal:
    def __init__(self, inst):
        n, m = inst.n, inst.m
        self.n, self.m = n, m
        self.cliques = [np.asarray(c) for c in inst.cliques]
        self.c = vec(dense_sym(n, inst.C))
        con, r, cc, v = inst.A
        As = []
        for i in range(m):
            sel = np.asarray(con) == i
            As.append(vec(dense_sym(n, (np.asarray(r)[sel], np.asarray(cc)[sel], np.asarray(v)[sel]))))
        self.A = np.array(As).reshape(m, n * n)
        self.b = np.asarray(inst.b, dtype=np.float64)
        Hs = [np.kron(selector(c, n), selector(c, n)) for c in self.cliques]
        self.H = np.vstack(Hs)
        self.sizes = [len(c) for c in self.cliques]
        self.nd = self.H.shape[0]
        N = n * n
        nd = self.nd
        # Q of eq. (HomogeneousEmbedding), blocks ordered (x, s, y, v, tau)
        dims = [N, nd, m, nd, 1]
        off = np.cumsum([0] + dims)
        T = off[-1]
        Q = np.zeros((T, T))

        def blk(i, j, M):
            Q[off[i]:off[i + 1], off[j]:off[j + 1]] = M

        blk(0, 2, -self.A.T)
        blk(0, 3, -self.H.T)
        blk(0, 4, self.c[:, None])
        blk(1, 3, np.eye(nd))
        blk(2, 0, self.A)
        blk(2, 4, -self.b[:, None])
        blk(3, 0, self.H)
        blk(3, 1, -np.eye(nd))
        blk(4, 0, -self.c[None, :])
        blk(4, 2, self.b[None, :])
        self.Q = Q
        self.off = off
        self.IQ = np.eye(T) + Q

    def split(self, w):
        o = self.off
        return [w[o[i]:o[i + 1]] for i in range(5)]

    def project(self, w):
        """Pi_K: free, S (PSD blocks), free, free, R_+."""
        x, s, y, v, t = self.split(w)
        out = []
        pos = 0
        for k in self.sizes:
            Y = unvec(s[pos:pos + k * k], k)
            Y = 0.5 * (Y + Y.T)
            lam, V = np.linalg.eigh(Y)
            out.append(vec((V * np.maximum(lam, 0)) @ V.T))
            pos += k * k
        s2 = np.concatenate(out)
        return np.concatenate([x, s2, y, v, np.maximum(t, 0)])

    def initial(self):
        T = self.off[-1]
        u = np.zeros(T)
        vt = np.zeros(T)
        u[-1] = 1.0
        vt[-1] = 1.0
        return u, vt

    def iterate(self, u, vt):
        uh = np.linalg.solve(self.IQ, u + vt)      # (Step1), plain definition
        un = self.project(uh - vt)                 # (Step2)
        vn = vt - uh + un                          # (Step3)
        return un, vn

    # ------------------------------------------------------------------
    # map to the svec coordinates of oracle.hsde (lower entries of E',
    # clique blocks packed column-major, off-diagonals times sqrt 2)
    # ------------------------------------------------------------------
    def to_svec(self, w, erow, ecol):
        n = self.n
        x, s, y, v, t = self.split(w)
        X = unvec(x, n)
        sc = np.where(erow == ecol, 1.0, math.sqrt(2.0))
        xs = X[erow, ecol] * sc

        def blocks(z):
            out = []
            pos = 0
            for k in self.sizes:
                M = unvec(z[pos:pos + k * k], k)
                for j in range(k):
                    for i in range(j, k):
                        out.append(M[i, j] * (1.0 if i == j else math.sqrt(2.0)))
                pos += k * k
            return np.asarray(out)

        return [xs, blocks(s), y.copy(), blocks(v), float(t[0])]


def dense_affine_matrix_svec(prob):
    """I + Q assembled densely in the svec coordinates of oracle.hsde from
    the block layout of eq. (HomogeneousEmbedding) (for the step-1 pin)."""
    A = prob.A.toarray()
    H = prob.H.toarray()
    nE, ns, m = prob.nE, prob.ns, prob.m
    dims = [nE, ns, m, ns, 1]
    off = np.cumsum([0] + dims)
    T = off[-1]
    Q = np.zeros((T, T))

    def blk(i, j, M):
        Q[off[i]:off[i + 1], off[j]:off[j + 1]] = M

    blk(0, 2, -A.T)
    blk(0, 3, -H.T)
    blk(0, 4, prob.c[:, None])
    blk(1, 3, np.eye(ns))
    blk(2, 0, A)
    blk(2, 4, -prob.b[:, None])
    blk(3, 0, H)
    blk(3, 1, -np.eye(ns))
    blk(4, 0, -prob.c[None, :])
    blk(4, 2, prob.b[None, :])
    return np.eye(T) + Q, off
