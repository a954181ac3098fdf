"""torch.autograd.Function around the solver (argument marshalling only).

A batch of SDPs with fixed structure (constraint matrices A_i and cliques)
and variable data: c = svec(C) over each instance's pattern E' (canonical
entry order, off-diagonals scaled by sqrt 2) and b.  forward() solves every
instance on the GPU and returns X* = x/tau (svec over E', instances
concatenated); backward() calls cdcs_adjoint, which differentiates the
converged fixed point of the ADMM iteration implicitly.  Gradients are with
respect to c and b in those coordinates (for an off-diagonal pair,
dL/dC_ij = sqrt(2) dL/dc_e when C_ij = C_ji is one parameter).
"""
from __future__ import annotations

import warnings

import numpy as np
import torch

from . import cdcs


class SDPLayer:
    def __init__(self, instances, eps_tol=1e-8, max_iter=200000, check_every=50,
                 adjoint_tol=1e-10, adjoint_max_iter=200000):
        self.templates = list(instances)
        self.settings = dict(eps_tol=eps_tol, max_iter=max_iter, check_every=check_every)
        self.adjoint_tol = adjoint_tol
        self.adjoint_max_iter = adjoint_max_iter
        probe = cdcs.Solver(self.templates, **self.settings)
        self.entries = [probe.entries(i) for i in range(len(self.templates))]
        self.nE = [len(r) for r, _ in self.entries]
        self.m = [t.m for t in self.templates]
        probe.close()

    def svec_of(self, inst_index, C):
        """svec over the instance's pattern of a lower-COO matrix (r, c, v)."""
        rows, cols = self.entries[inst_index]
        key = {(int(r), int(c)): e for e, (r, c) in enumerate(zip(rows, cols))}
        out = np.zeros(len(rows))
        for r, c, v in zip(*C):
            out[key[(int(r), int(c))]] += v * (1.0 if r == c else np.sqrt(2.0))
        return out

    def _instances(self, c, b):
        out = []
        oe = om = 0
        for i, t in enumerate(self.templates):
            rows, cols = self.entries[i]
            ce = c[oe:oe + self.nE[i]]
            scale = np.where(rows == cols, 1.0, np.sqrt(2.0))
            C = (rows.astype(np.int32), cols.astype(np.int32), ce / scale)
            inst = type(t)(t.n, t.m, C, t.A, b[om:om + self.m[i]], t.cliques, t.parent)
            out.append(inst)
            oe += self.nE[i]
            om += self.m[i]
        return out

    def __call__(self, c, b):
        return _SolveFn.apply(c, b, self)


class _SolveFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c, b, layer):
        insts = layer._instances(c.detach().cpu().numpy(), b.detach().cpu().numpy())
        s = cdcs.Solver(insts, **layer.settings)
        infos = s.solve()
        bad = [i for i, f in enumerate(infos) if f["status"] != cdcs.SOLVED]
        if bad:
            raise RuntimeError(f"instances {bad} not solved: {[infos[i]['status'] for i in bad]}")
        X = np.concatenate([s.solution(i)[0] for i in range(len(insts))])
        ctx.solver = s
        ctx.layer = layer
        ctx.infos = infos
        return torch.as_tensor(X, dtype=torch.float64, device=c.device)

    @staticmethod
    def backward(ctx, dX):
        layer = ctx.layer
        dXc = dX.detach().to(dtype=torch.float64).contiguous()
        if dXc.is_cuda:
            dc = torch.empty(sum(layer.nE), dtype=torch.float64, device=dXc.device)
            db = torch.empty(sum(layer.m), dtype=torch.float64, device=dXc.device)
            torch.cuda.synchronize()
            it = ctx.solver.adjoint_device(dXc, dc, db, max_iter=layer.adjoint_max_iter, tol=layer.adjoint_tol)
        else:
            dcn, dbn, it = ctx.solver.adjoint(dXc.numpy(), max_iter=layer.adjoint_max_iter, tol=layer.adjoint_tol)
            dc = torch.as_tensor(dcn)
            db = torch.as_tensor(dbn)
        ctx.adjoint_iterations = it
        resid, why = ctx.solver.adjoint_info()
        ctx.solver.close()
        off = [i for i in range(len(resid)) if why[i] != 0]
        if off:
            what = {1: "stalled", 2: "hit the iteration limit"}
            warnings.warn("SDPLayer.backward: the adjoint system of instances "
                          + ", ".join(f"{i} ({what[int(why[i])]}, residual {resid[i]:.1e})" for i in off)
                          + f" is not solved to adjoint_tol = {layer.adjoint_tol:.0e}; their gradients are only "
                          "as accurate as the forward solve", RuntimeWarning)
        return dc, db, None
