"""PyTorch autograd binding of the reverse sweep (marshalling only).

``expectations(engine, hamiltonian, alphas, schedule, dtau, n_steps,
observables)`` evolves rho = I through Algorithm 1 with the given term
weights and step, and returns the tensor of <P_j> for the observable strings.
Its backward is the library's reverse sweep (``itpp_backward``): derivatives
with respect to the term weights and to dtau with every gate's kept set held
fixed.  Quantities such as d<H>/dJ, d<H>/dh or d<H>/dbeta then follow from
ordinary autograd on the weights (alpha_ZZ = -J, alpha_X = -h) and on
dtau = beta / N.
"""
from __future__ import annotations

from typing import Sequence, Tuple

import numpy as np
import torch


class _Expectations(torch.autograd.Function):
    @staticmethod
    def forward(ctx, alphas, dtau, engine, hamiltonian, schedule, n_steps, observables, every):
        a = alphas.detach().cpu().double().numpy()
        d = float(dtau.detach().cpu())
        engine.set_hamiltonian(list(hamiltonian), a.tolist())
        engine.set_schedule(list(schedule))
        engine.set_adjoint(int(every))
        engine.evolve(d, int(n_steps))
        vals = [engine.expect([P], [1.0]) for P in observables]
        ctx.engine = engine
        ctx.observables = list(observables)
        return torch.tensor(vals, dtype=torch.float64)

    @staticmethod
    def backward(ctx, grad_out):
        g = grad_out.detach().cpu().double().numpy()
        _, da, dd, _ = ctx.engine.backward(ctx.observables, g.tolist())
        return (torch.from_numpy(np.array(da, dtype=np.float64)), torch.tensor(dd, dtype=torch.float64),
                None, None, None, None, None, None)


def expectations(engine, hamiltonian: Sequence[str], alphas: torch.Tensor, schedule: Sequence[Tuple[int, float]],
                 dtau: torch.Tensor, n_steps: int, observables: Sequence[str], every: int = 10) -> torch.Tensor:
    """<P_j> after n_steps Trotter steps, differentiable in alphas and dtau."""
    return _Expectations.apply(alphas, dtau, engine, tuple(hamiltonian), tuple(schedule), n_steps,
                               tuple(observables), every)
