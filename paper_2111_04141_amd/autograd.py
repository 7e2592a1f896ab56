"""torch.autograd Functions over a migrid Plan.

Gridding G (records -> grid) and degridding G^H (grid -> records) are the
forward/backward operator pair of the major-cycle residual (Section 1.6:
the residual image is the gridded difference between the measured
visibilities and the degridded model).  Both maps are complex-linear, and
for a complex-linear y = A x PyTorch's backward is grad_x = A^H grad_y
(conjugate Wirtinger convention).  Hence

    Degrid:  vis  = G^H grid   backward: grad_grid = G grad_vis   (gridding)
    Grid:    grid = G vis      backward: grad_vis  = G^H grad_grid (degridding)

Both directions run in the HIP library; the record coordinates (the plan)
are not differentiated.
"""
from __future__ import annotations

import torch


class Degrid(torch.autograd.Function):
    """vis = G^H grid for the records of `plan` (a migrid Plan)."""

    @staticmethod
    def forward(ctx, grid, plan):
        ctx.plan = plan
        return plan.degrid(grid.contiguous())

    @staticmethod
    def backward(ctx, grad_vis):
        return ctx.plan.grid(grad_vis.contiguous()), None


class Grid(torch.autograd.Function):
    """grid = G vis for the records of `plan` (a migrid Plan)."""

    @staticmethod
    def forward(ctx, vis, plan):
        ctx.plan = plan
        return plan.grid(vis.contiguous())

    @staticmethod
    def backward(ctx, grad_grid):
        return ctx.plan.degrid(grad_grid.contiguous()), None


def degrid(grid, plan):
    return Degrid.apply(grid, plan)


def grid(vis, plan):
    return Grid.apply(vis, plan)


def chi2(model_grid, plan, vis_obs, sigma: float):
    """sum |vis_obs - G^H model_grid|^2 / sigma^2 (accumulated in float64)."""
    r = vis_obs - Degrid.apply(model_grid, plan)
    return (r.real.double() ** 2 + r.imag.double() ** 2).sum() / (sigma * sigma)
