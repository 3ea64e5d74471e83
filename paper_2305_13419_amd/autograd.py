"""torch.autograd binding of the adjoint: J(inv_lambda2, sigma_n) = |F|^2.

``TwoFluidObjective.apply(inv_lambda2, sigma_n, problem)`` runs the forward
FDTD (checkpointed every ``seg`` steps) through the C ABI and returns the
scalar objective; its backward runs the reverse-time sweep on the GPU and
returns the per-cell gradients (FP64 accumulation, cast to the input dtype).
"""
import math

import torch

from .sim import Simulation


class AdjointProblem:
    """Everything of a run except the two differentiated maps.

    shape, spacing, dt, theta, dtype, pml : as for Simulation
    eps_r : per-cell relative permittivity (fixed)
    fields : initial integer-time (E, H, J) or None for zero fields
    sources : list of dicts for Simulation.add_source
    objective : (comp, box, f0)
    nsteps, seg : run length and checkpoint segment (default about sqrt(nsteps))
    seg2 : inner segment of a three-level schedule (None: two levels)
    """

    def __init__(self, shape, spacing, dt, eps_r, objective, nsteps, seg=None, theta=1.0, dtype=torch.float64,
                 pml=(None, None, None), fields=None, sources=(), device="cuda", seg2=None):
        self.sim = Simulation(shape, spacing, dt, theta, dtype, pml, device=device)
        self.eps_r = self.sim._dev(eps_r)
        self.fields = fields
        self.sources = list(sources)
        for s in self.sources:
            self.sim.add_source(**s)
        self.objective = tuple(objective)
        self.nsteps = int(nsteps)
        self.seg = int(seg) if seg else max(1, int(round(math.sqrt(self.nsteps))))
        self.seg2 = int(seg2) if seg2 else None
        if self.seg2:
            self.ckpt, self.ckpt2, self.snap, self.work = self.sim.adjoint_nested_buffers(self.nsteps, self.seg,
                                                                                         self.seg2)
        else:
            self.ckpt, self.snap, self.work = self.sim.adjoint_buffers(self.nsteps, self.seg)
        self.F = None
        # forward runs made so far: a backward must belong to the latest one, since the checkpoints,
        # F and the maps of the problem are those of its last forward run
        self.generation = 0

    def _reset(self, inv_lambda2, sigma):
        sim = self.sim
        sim.set_materials(self.eps_r, sigma, inv_lambda2)
        if self.fields is None:
            z = [torch.zeros(sim.shape3, dtype=sim.dtype, device=sim.device) for _ in range(3)]
            sim.set_fields(z, z, z)
        else:
            sim.set_fields(*self.fields)

    def forward(self, inv_lambda2, sigma):
        self._reset(inv_lambda2, sigma)
        self.F = self.sim.forward_checkpointed(self.objective, self.nsteps, self.seg, self.ckpt)
        self.generation += 1
        return abs(self.F) ** 2

    def gradient(self):
        if self.seg2:
            return self.sim.adjoint_nested(self.objective, self.nsteps, self.seg, self.seg2, self.ckpt, self.F,
                                           self.ckpt2, self.snap, self.work)
        return self.sim.adjoint(self.objective, self.nsteps, self.seg, self.ckpt, self.F, self.snap, self.work)


class TwoFluidObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, inv_lambda2, sigma, problem):
        J = problem.forward(inv_lambda2.detach(), sigma.detach())
        ctx.problem = problem
        ctx.generation = problem.generation
        ctx.dtypes = (inv_lambda2.dtype, sigma.dtype)
        return torch.tensor(J, dtype=torch.float64, device=inv_lambda2.device)

    @staticmethod
    def backward(ctx, grad_out):
        if ctx.problem.generation != ctx.generation:
            raise RuntimeError("the AdjointProblem ran another forward pass after this one; its checkpoints and "
                               "maps now belong to that run, so this graph's gradient can no longer be formed")
        gl, gs = ctx.problem.gradient()
        g = grad_out.to(torch.float64)
        return (g * gl).to(ctx.dtypes[0]), (g * gs).to(ctx.dtypes[1]), None
