"""Differentiable eigenpairs: a torch.autograd.Function over lobpcg_solve (forward)
and lobpcg_adjoint (backward).

forward solves A x = lambda B x for the k smallest pairs with Algorithm 8 on the
GPU and returns (lambda, X) with X^T B X = I; backward maps the adjoints
(lambda_bar, X_bar) of a loss to gradients on the stored values of A (and of
B) with the library's adjoint kernels (first-order perturbation theory: d
lambda_i = x_i^T (dA - lambda_i dB) x_i, eigenvector part by a projected
conjugate-gradient solve).  The gradient of a stored off-diagonal value is the
symmetric one: a_rc and a_cr move together.  The loss must not depend on the
signs of the eigenvectors (they are fixed only up to sign), nor on a rotation
inside a degenerate cluster.

Argument marshalling only: every step runs in the HIP library.
"""

from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
import torch

from . import binding


@dataclasses.dataclass
class CsrPattern:
    """Sparsity pattern of a CSR matrix (device int64 row pointers, int32 columns);
    the values are the differentiable tensor passed beside it."""

    rowptr: torch.Tensor
    colind: torch.Tensor

    @property
    def n(self) -> int:
        return int(self.rowptr.numel() - 1)

    @property
    def nnz(self) -> int:
        return int(self.colind.numel())

    @classmethod
    def from_host(cls, rowptr, colind, device="cuda") -> "CsrPattern":
        return cls(torch.as_tensor(np.ascontiguousarray(rowptr, dtype=np.int64)).to(device),
                   torch.as_tensor(np.ascontiguousarray(colind, dtype=np.int32)).to(device))


def _device_csr(pattern: CsrPattern, values: torch.Tensor) -> dict:
    return {"rowptr": pattern.rowptr, "colind": pattern.colind,
            "values": values.detach().to(torch.float64).contiguous()}


class LobpcgFunction(torch.autograd.Function):
    """(A_values, B_values) -> (lambda, X): the k smallest eigenpairs of (A, B)."""

    @staticmethod
    def forward(ctx, A_values, B_values, A_pattern, B_pattern, k, tol, X0, solver_opts,
                cg_tol):
        if A_values.numel() != A_pattern.nnz:
            raise ValueError("A_values must hold nnz(A) values")
        haveB = B_values is not None
        if haveB and B_values.numel() != B_pattern.nnz:
            raise ValueError("B_values must hold nnz(B) values")
        A = _device_csr(A_pattern, A_values)
        B = _device_csr(B_pattern, B_values) if haveB else None
        s = binding.Solver(A, int(k), B=B, **(solver_opts or {}))
        info = s.solve(float(tol), X0)
        if not info["converged"]:
            raise RuntimeError(f"lobpcg_solve did not converge: {info['status']}, "
                               f"{info['n_converged']} of {k} pairs")
        lam, X, _ = s.eigpairs(int(k))
        ctx.solver = s
        ctx.k = int(k)
        ctx.haveB = haveB
        ctx.cg_tol = float(cg_tol)
        ctx.info = info
        return lam, X

    @staticmethod
    def backward(ctx, lam_bar, X_bar):
        s = ctx.solver
        lb = None if lam_bar is None else lam_bar.detach().to(torch.float64).cpu().numpy()
        xb = None if X_bar is None else X_bar.detach().to(torch.float64).contiguous()
        if ctx.haveB:
            gA, _, gB = s.adjoint(ctx.k, lb, xb, cg_tol=ctx.cg_tol, want_B=True)
        else:
            gA, _ = s.adjoint(ctx.k, lb, xb, cg_tol=ctx.cg_tol)
            gB = None
        need_a, need_b = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        return (gA if need_a else None, gB if need_b else None, None, None, None, None, None,
                None, None)


def eigsh(A_values: torch.Tensor, A_pattern: CsrPattern, k: int,
          B_values: Optional[torch.Tensor] = None, B_pattern: Optional[CsrPattern] = None,
          tol: float = 1e-8, X0=None, cg_tol: float = 1e-12, **solver_opts):
    """The k smallest eigenpairs (lambda, X) of the pencil given by CSR patterns and
    value tensors, differentiable with respect to A_values (and B_values).
    solver_opts go to binding.Solver (precond, precision, block_size, maxit, ...)."""
    return LobpcgFunction.apply(A_values, B_values, A_pattern, B_pattern, k, tol, X0,
                                solver_opts, cg_tol)
