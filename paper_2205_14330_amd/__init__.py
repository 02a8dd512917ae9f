"""MI355X-native differentiable point-splat renderer.

Implements the differentiable splat rendering of Zhang et al., "Differentiable
Point-Based Radiance Fields for Efficient View Synthesis" (SIGGRAPH Asia 2022,
Sec. 3.1-3.2) as hand-written HIP kernels for gfx950 behind a C ABI
(include/dpr.h, libdpr.so).  This package is the Python binding: argument
marshalling, torch-allocated workspaces, the autograd form and the serving
loop.  Importing it loads the HIP library and fails loudly if it is absent.
"""
from ._abi import DprError, LIB_PATH, STAGES, load
from .renderer import (Plan, RenderFn, RenderParams, SceneTensors, Workspace, camera_struct, loss_l2_tv, render,
                       render_views)

__all__ = ["DprError", "LIB_PATH", "STAGES", "load", "Plan", "RenderFn", "RenderParams", "SceneTensors", "Workspace",
           "camera_struct", "loss_l2_tv", "render", "render_views"]
