"""torch.autograd wrappers of the reverse sweep (marshalling only).

``rcg(problem, A_vals, P0_vals)`` returns P (values on the pattern) as a
differentiable function of the values of A and of P0; ``loss(problem, P,
A_vals, e, w_energy, w_twogrid)`` the scalar loss
    w_E tr(P^T A P) + w_T ||e - P c||_A^2,  c = (P^T A P)^{-1} P^T A e.
Both run on the device through libemin.so (emin_solve_taped, emin_backward,
emin_loss).  The problem's A and P0 value tensors are the ones the library
reads, so the given values are copied into them first; the pattern, B and
B_c are constants.
"""

from __future__ import annotations

import torch

from . import api


def _load_values(problem: api.Problem, A_vals, P0_vals):
    with torch.no_grad():
        if A_vals is not None and A_vals.data_ptr() != problem.A.vals.data_ptr():
            problem.A.vals.copy_(A_vals)
        if P0_vals is not None and P0_vals.data_ptr() != problem.P0.vals.data_ptr():
            problem.P0.vals.copy_(P0_vals)


class EminRCG(torch.autograd.Function):
    """P = RCG(A, P0) (Alg. 2 then Alg. 3), with its hand-written adjoint."""

    @staticmethod
    def forward(ctx, A_vals, P0_vals, problem):
        _load_values(problem, A_vals, P0_vals)
        P, _, tape = problem.solve_taped()
        ctx.tape = tape  # released with the graph
        return P if P.numel() == problem.nnz else P[: problem.nnz].clone()

    @staticmethod
    def backward(ctx, gP):
        tape = ctx.tape
        p = tape.problem
        g = p.new_values()
        g[: p.nnz].copy_(gP)
        gA, gP0 = tape.backward(g)
        return gA, gP0, None


class EminLoss(torch.autograd.Function):
    """Scalar loss of P and A; both gradients come from the forward call."""

    @staticmethod
    def forward(ctx, P, A_vals, problem, e, w_energy, w_twogrid):
        _load_values(problem, A_vals, None)
        Pf = problem.new_values()
        Pf[: problem.nnz].copy_(P)
        L, gP, gA = problem.loss(Pf, e, w_energy, w_twogrid, grad=True)
        ctx.save_for_backward(gP[: problem.nnz], gA)
        return torch.tensor(L, dtype=torch.float64, device=P.device)

    @staticmethod
    def backward(ctx, gL):
        gP, gA = ctx.saved_tensors
        return gL * gP, gL * gA, None, None, None, None


def rcg(problem: api.Problem, A_vals: torch.Tensor, P0_vals: torch.Tensor) -> torch.Tensor:
    return EminRCG.apply(A_vals, P0_vals, problem)


def loss(problem: api.Problem, P: torch.Tensor, A_vals: torch.Tensor, e=None,
         w_energy: float = 1.0, w_twogrid: float = 0.0) -> torch.Tensor:
    return EminLoss.apply(P, A_vals, problem, e, float(w_energy), float(w_twogrid))
