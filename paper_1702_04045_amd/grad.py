"""Gradient of the band energy with respect to the local potential and the
Kleinman-Bylander projectors.

E = sum_{b < n_occ} w_b eps_b, the weighted sum of the lowest eigenvalues of
the Hamiltonian of eq. (e5) for the local potential V given on the FFT grid
and the projectors of Section 2.2.  The eigenpairs come from the ParO
iterations (MParO I, Algorithm 2) run to a residual tolerance.  For an
eigenpair the derivative of eps_b with respect to any parameter of H is the
expectation of dH/d(parameter) (Hellmann-Feynman):
  - V_j: the potential matrix elements are the grid sums
    (1/N) sum_j V_j exp(-2 pi i (n_m - n_n).j / N), N = N1 N2 N3, so
    d eps_b / dV_j = |psi_b(r_j)|^2 / N, psi_b(r_j) = sum_G c_bG exp(2 pi i n.j / N)
    (the device density, paro_density, divided by N);
  - the KB energy d_p and centre R_p of projector p: V_NL = sum_p d_p
    beta_p beta_p^H with beta_p(G) ~ exp(-i G.R_p)
    (paro_projector_gradient).
The error of these gradients is first order in the eigenvector error, i.e.
of the order of the residual tolerance over the gap to the next band.

truncated_band_energy differentiates instead the map of a fixed number K of
ParO outer iterations from a fixed trial block, by reverse mode through
those iterations (paro_truncated_gradient): its gradient is exact for the
truncated map at any K, and tends to the Hellmann-Feynman one as the
iterations converge.

Every numerical step runs in libparo's kernels; this module marshals
arguments and wires the results into torch.autograd.
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

    def projectors_with(self, centers=None, kb=None):
        """The projector list with centres (n_proj x 3) and KB energies (n_proj) replaced."""
        out = [dict(p) for p in self.projectors]
        if centers is not None:
            c = centers.detach().to("cpu", torch.float64).numpy().reshape(len(out), 3)
            for p, r in zip(out, c):
                p["center"] = [float(x) for x in r]
        if kb is not None:
            d = kb.detach().to("cpu", torch.float64).numpy().reshape(len(out))
            for p, x in zip(out, d):
                p["d"] = float(x)
        return out

    def solve(self, vloc, centers=None, kb=None):
        """Converged (plan, psi, eps, residuals) for the local potential vloc (grid-shaped, float64)
        and, optionally, projector centres and KB energies replacing those of the problem."""
        v = np.ascontiguousarray(vloc.detach().to("cpu", torch.float64).numpy())
        plan = Plan(self.cell, self.ecut, v, self.projectors_with(centers, kb), device=self.device)
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
    def forward(ctx, vloc, centers, kb, problem):
        plan, psi, eps, _ = problem.solve(vloc, centers, kb)
        ctx.plan, ctx.psi, ctx.problem = plan, psi, problem
        ctx.devices = (vloc.device, centers.device, kb.device)
        e = (problem.weights * eps[: problem.n_occ]).sum()
        return e.to(vloc.device)

    @staticmethod
    def backward(ctx, grad):
        p = ctx.problem
        psi = ctx.psi[: p.n_occ]
        gv = gr = gd = None
        if ctx.needs_input_grad[0]:
            rho = ctx.plan.density(psi, p.weights)
            gv = (rho * (grad.to(rho.device) / float(np.prod(ctx.plan.grid)))).to(ctx.devices[0])
        if ctx.needs_input_grad[1] or ctx.needs_input_grad[2]:
            dd, dR = ctx.plan.projector_gradient(psi, p.weights)
            g = grad.to(dd.device)
            gr = (dR * g).to(ctx.devices[1])
            gd = (dd * g).to(ctx.devices[2])
        return gv, gr, gd, None


def band_energy(vloc: torch.Tensor, problem: BandEnergyProblem, centers: torch.Tensor = None,
                kb: torch.Tensor = None) -> torch.Tensor:
    """sum_{b < n_occ} w_b eps_b of the Hamiltonian with local potential vloc (N1 x N2 x N3,
    float64, C order), projector centres (n_proj x 3, bohr) and KB energies (n_proj, Ha);
    centers and kb default to the problem's.  Differentiable with respect to all three
    (Hellmann-Feynman)."""
    assert vloc.dtype == torch.float64 and vloc.dim() == 3
    n = len(problem.projectors)
    if centers is None:
        centers = torch.tensor([list(p["center"]) for p in problem.projectors], dtype=torch.float64).reshape(n, 3)
    if kb is None:
        kb = torch.tensor([p["d"] for p in problem.projectors], dtype=torch.float64).reshape(n)
    assert centers.shape == (n, 3) and kb.shape == (n,)
    return _BandEnergy.apply(vloc, centers, kb, problem)


def potential_gradient(problem: BandEnergyProblem, psi: torch.Tensor, plan: Plan) -> torch.Tensor:
    """d E / d vloc for a converged block psi of plan: rho / (N1 N2 N3) on the device."""
    rho = plan.density(psi[: problem.n_occ], problem.weights)
    return rho / float(np.prod(plan.grid))


class TruncatedProblem:
    """The band energy after a fixed number of ParO outer iterations (Algorithm 1,
    fixed shift) from a fixed trial block: E(V, R) = sum_b w_b eps_b^K with
    (eps^0, psi^0) the Rayleigh-Ritz pairs of the trial block and K outer
    iterations of n_cg PCG steps each.  The trial block, the shift and the
    KB energies are constants; the local potential on the grid and the
    projector centres are the variables."""

    def __init__(self, cell, ecut, projectors, trial, n_outer, n_cg, sigma, weights=None, device="cuda:0"):
        self.cell = np.asarray(cell, np.float64)
        self.ecut = float(ecut)
        self.projectors = list(projectors)
        self.device = torch.device(device)
        self.trial = torch.as_tensor(np.ascontiguousarray(trial), dtype=torch.complex128).to(self.device)
        self.n_outer, self.n_cg, self.sigma = int(n_outer), int(n_cg), float(sigma)
        nb = self.trial.shape[0]
        w = np.ones(nb) if weights is None else np.asarray(weights, np.float64)
        assert w.shape == (nb,)
        self.weights = torch.as_tensor(w, dtype=torch.float64, device=self.device)

    def plan(self, vloc, centers=None):
        v = np.ascontiguousarray(vloc.detach().to("cpu", torch.float64).numpy())
        projs = [dict(p) for p in self.projectors]
        if centers is not None:
            c = centers.detach().to("cpu", torch.float64).numpy().reshape(len(projs), 3)
            for p, r in zip(projs, c):
                p["center"] = [float(x) for x in r]
        return Plan(self.cell, self.ecut, v, projs, device=self.device)

    def energy(self, vloc, centers=None):
        """E alone, through paro_iterate (the forward map, for finite differences)."""
        pl = self.plan(vloc, centers)
        out = pl.iterate(self.trial.clone(), self.n_outer, self.n_cg, self.sigma, stats=False)
        return float((self.weights * out["eps"]).sum().item())


class _TruncatedBandEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vloc, centers, problem):
        pl = problem.plan(vloc, centers)
        e, dv, dr = pl.truncated_gradient(problem.trial, problem.n_outer, problem.n_cg, problem.sigma,
                                          problem.weights)
        ctx.save_for_backward(dv, dr)
        ctx.devices = (vloc.device, centers.device)
        return torch.tensor(e, dtype=torch.float64, device=vloc.device)

    @staticmethod
    def backward(ctx, grad):
        dv, dr = ctx.saved_tensors
        g = grad.to(dv.device)
        gv = (dv * g).to(ctx.devices[0]) if ctx.needs_input_grad[0] else None
        gr = (dr * g).to(ctx.devices[1]) if ctx.needs_input_grad[1] else None
        return gv, gr, None


def truncated_band_energy(vloc: torch.Tensor, problem: TruncatedProblem, centers: torch.Tensor = None) -> torch.Tensor:
    """sum_b w_b eps_b after problem.n_outer truncated ParO outer iterations for the local
    potential vloc (N1 x N2 x N3, float64, C order) and projector centres (n_proj x 3, bohr;
    default the problem's).  Differentiable with respect to both by the device reverse-mode
    adjoint of the truncated iterations (paro_truncated_gradient)."""
    assert vloc.dtype == torch.float64 and vloc.dim() == 3
    n = len(problem.projectors)
    if centers is None:
        centers = torch.tensor([list(p["center"]) for p in problem.projectors], dtype=torch.float64).reshape(n, 3)
    assert centers.shape == (n, 3)
    return _TruncatedBandEnergy.apply(vloc, centers, problem)
