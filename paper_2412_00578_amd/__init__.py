"""MI355X-native Speedy-Splat rasterizer (gfx950 HIP kernels behind a C ABI).

The forward path renders 3D Gaussians with the tile pipeline of Speedy-Splat
(arXiv 2412.00578, Sec. 3.2) and one of three tile assignments: the 3-sigma
square (Eq. radius), SnugBox (Sec. 4.1.1) or AccuTile (Sec. 4.1.2, Alg. 1).
"""
from ._lib import MODES, SplatError, constants, lib  # noqa: F401
from .render import (STAGES, BackwardEvents, BatchFrame, BatchRenderer, Frame,  # noqa: F401
                     Gaussians, Grads, Pairs, RenderOutput, Renderer, StageEvents, backward,
                     pruning_score, render)

__all__ = ["MODES", "SplatError", "constants", "lib", "Frame", "Gaussians", "Pairs",
           "RenderOutput", "Renderer", "StageEvents", "STAGES", "Grads", "backward",
           "pruning_score", "render", "BatchFrame", "BatchRenderer", "BackwardEvents"]
