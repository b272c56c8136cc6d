"""Gradient of the band energy with respect to the local potential.

E(V) = sum_{b < n_occ} w_b eps_b(V), the weighted sum of the lowest
eigenvalues of the Hamiltonian of eq. (e5) for the local potential V given
on the FFT grid.  The eigenpairs come from the ParO iterations (MParO I,
Algorithm 2) run to a residual tolerance.  For an eigenpair the derivative
of eps_b with respect to V_j is the expectation of dH/dV_j (Hellmann-
Feynman), and since the potential matrix elements are the grid sums
(1/N) sum_j V_j exp(-2 pi i (n_m - n_n).j / N), N = N1 N2 N3, it is
|psi_b(r_j)|^2 / N with psi_b(r_j) = sum_G c_bG exp(2 pi i n.j / N).  The
backward pass is therefore the device density (paro_density) of the
converged block divided by N.  The error of this gradient is first order in
the eigenvector error, i.e. of the order of the residual tolerance over the
gap to the next band.

Every numerical step runs in libparo's kernels; this module marshals
arguments and wires the result into torch.autograd.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib as L
from .paro import Plan


class BandEnergyProblem:
    """A fixed cell, cutoff and projector set; the local potential is the variable.

    n_occ bands enter the energy with weights w (default 1); n_bands >= n_occ
    bands are iterated (the extra ones speed up convergence of the highest
    occupied band).  The converged block of one call is the starting block of
    the next call (warm start), so that nearby potentials converge in a few
    outer iterations."""

    def __init__(self, cell, ecut, projectors, n_occ, n_bands=None, weights=None, trial=None, n_cg=10,
                 max_outer=200, tol_res=1e-9, device="cuda:0"):
        self.cell = np.asarray(cell, np.float64)
        self.ecut = float(ecut)
        self.projectors = list(projectors)
        self.n_occ = int(n_occ)
        self.n_bands = int(n_bands or n_occ + max(2, n_occ // 4))
        assert self.n_bands >= self.n_occ >= 1
        self.device = torch.device(device)
        w = np.ones(self.n_occ) if weights is None else np.asarray(weights, np.float64)
        assert w.shape == (self.n_occ,)
        self.weights = torch.as_tensor(w, dtype=torch.float64, device=self.device)
        self.trial = trial
        self.n_cg = int(n_cg)
        self.max_outer = int(max_outer)
        self.tol_res = float(tol_res)
        self.last = None  # (psi, plan) of the latest solve

    def solve(self, vloc):
        """Converged (plan, psi, eps, residuals) for the local potential vloc (grid-shaped, float64)."""
        v = np.ascontiguousarray(vloc.detach().to("cpu", torch.float64).numpy())
        plan = Plan(self.cell, self.ecut, v, self.projectors, device=self.device)
        if self.last is not None and self.last[0].shape == (self.n_bands, plan.ng):
            psi = self.last[0].clone()
        elif self.trial is not None:
            psi = torch.as_tensor(np.ascontiguousarray(self.trial), dtype=torch.complex128).to(self.device).clone()
            assert tuple(psi.shape) == (self.n_bands, plan.ng)
        else:
            raise ValueError("BandEnergyProblem: a trial block (n_bands x n_g) is needed for the first solve")
        out = plan.iterate(psi, self.max_outer, self.n_cg, plan.shift_lower_bound(), variant=L.VARIANT_MPARO1,
                           shift_mode=L.SHIFT_ADAPTIVE, n_conv=self.n_occ, tol_res=self.tol_res)
        res = plan.residual_norms(out["psi"], out["hpsi"], out["eps"])
        worst = float(res[: self.n_occ].max().item())
        if not worst <= self.tol_res:
            raise RuntimeError(f"band energy: ParO did not reach |r| <= {self.tol_res:g} in {self.max_outer} "
                               f"outer iterations (max |r| = {worst:.3e})")
        self.last = (out["psi"], plan)
        return plan, out["psi"], out["eps"], res


class _BandEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vloc, problem):
        plan, psi, eps, _ = problem.solve(vloc)
        ctx.plan, ctx.psi, ctx.problem = plan, psi, problem
        ctx.vdevice = vloc.device
        e = (problem.weights * eps[: problem.n_occ]).sum()
        return e.to(vloc.device)

    @staticmethod
    def backward(ctx, grad):
        p = ctx.problem
        rho = ctx.plan.density(ctx.psi[: p.n_occ], p.weights)
        n = float(np.prod(ctx.plan.grid))
        g = rho * (grad.to(rho.device) / n)
        return g.to(ctx.vdevice), None


def band_energy(vloc: torch.Tensor, problem: BandEnergyProblem) -> torch.Tensor:
    """sum_{b < n_occ} w_b eps_b of the Hamiltonian with local potential vloc (N1 x N2 x N3,
    float64, C order); differentiable with respect to vloc (Hellmann-Feynman)."""
    assert vloc.dtype == torch.float64 and vloc.dim() == 3
    return _BandEnergy.apply(vloc, problem)


def potential_gradient(problem: BandEnergyProblem, psi: torch.Tensor, plan: Plan) -> torch.Tensor:
    """d E / d vloc for a converged block psi of plan: rho / (N1 N2 N3) on the device."""
    rho = plan.density(psi[: problem.n_occ], problem.weights)
    return rho / float(np.prod(plan.grid))
