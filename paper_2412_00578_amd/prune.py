"""Pruning by the efficient pruning score (Speedy-Splat Sec. 4.2).

Soft Pruning (Sec. 4.2.2) removes a large fraction of the Gaussians right
before each opacity reset of the densification phase (80 % at iterations
6000, 9000 and 12000); Hard Pruning (Sec. 4.2.3) removes a constant fraction
every 3000 iterations from iteration 15000 (30 %).  The Gaussians are ranked
by the score of Sec. 4.2.1, the squared gradient of the image with respect
to each Gaussian's projected 2D value, summed over pixels and channels
(``render.pruning_score``) and over the views the caller accumulates.

``prune`` selects the Gaussians to keep on the GPU (``ss_prune_select``: a
radix select on the score bits, ties at the threshold kept by lower index)
and compacts the parameter arrays (``ss_gather_gaussians``); both are
marshalled here only.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from ._lib import check, lib
from .render import Gaussians, _stream


def n_keep(n: int, ratio: float) -> int:
    """Gaussians a prune of the fraction `ratio` keeps: n - floor(ratio n)."""
    out = ctypes.c_int64()
    check(lib().ss_prune_count(int(n), float(ratio), ctypes.byref(out)), "ss_prune_count")
    return int(out.value)


def select(score: torch.Tensor, ratio: float) -> torch.Tensor:
    """Indices (ascending, int32 tensor) of the Gaussians a prune of the
    fraction `ratio` keeps, ranked by `score` [n] float32."""
    score = score.contiguous()
    if score.dtype != torch.float32 or score.dim() != 1:
        raise TypeError("score must be a 1-D float32 tensor")
    n = int(score.numel())
    words = ctypes.c_int64()
    check(lib().ss_prune_tmp_words(n, ctypes.byref(words)), "ss_prune_tmp_words")
    k = n_keep(n, ratio)
    dev = score.device
    tmp = torch.empty(max(int(words.value), 1), dtype=torch.int32, device=dev)
    keep = torch.empty(max(k, 1), dtype=torch.int32, device=dev)
    got = ctypes.c_int64()
    check(lib().ss_prune_select(ctypes.c_void_p(score.data_ptr()), n, float(ratio),
                                ctypes.c_void_p(keep.data_ptr()), ctypes.c_void_p(tmp.data_ptr()),
                                ctypes.byref(got), _stream(dev)), "ss_prune_select")
    assert got.value == k
    return keep[:k]


def gather(g: Gaussians, keep: torch.Tensor) -> Gaussians:
    """The Gaussians of `g` listed in `keep`, in that order (new arrays).  The
    five arrays are gathered as rows of 3, 3, 4, 1 and 3 K floats, so any
    per-Gaussian parameter set with that layout (raw log-scales and logits,
    optimizer moments) compacts the same way."""
    k = int(keep.numel())
    dev = g.device
    out = Gaussians(torch.empty((k, 3), dtype=torch.float32, device=dev),
                    torch.empty((k, 3), dtype=torch.float32, device=dev),
                    torch.empty((k, 4), dtype=torch.float32, device=dev),
                    torch.empty(k, dtype=torch.float32, device=dev),
                    torch.empty((k,) + tuple(g.sh.shape[1:]), dtype=torch.float32, device=dev),
                    g.sh_degree)
    gs, os_ = g.struct(), out.struct()
    check(lib().ss_gather_gaussians(ctypes.byref(gs), ctypes.c_void_p(keep.data_ptr()), k,
                                    ctypes.byref(os_), _stream(dev)), "ss_gather_gaussians")
    return out


def prune(g: Gaussians, score: torch.Tensor, ratio: float):
    """Removes the fraction `ratio` of `g` with the lowest scores.  Returns the
    kept Gaussians and their indices in `g`."""
    if int(score.numel()) != g.n:
        raise ValueError("one score per Gaussian")
    keep = select(score, ratio)
    return gather(g, keep), keep


@dataclass
class Schedule:
    """The pruning schedule of Sec. 4.2.2-4.2.3 over `total` iterations (the
    paper's 30000; shorter runs scale every iteration by total / 30000)."""
    total: int = 30000
    soft_ratio: float = 0.8
    hard_ratio: float = 0.3

    def events(self) -> list:
        """(iteration, ratio, kind) of every prune, in order."""
        f = self.total / 30000.0
        ev = [(int(round(it * f)), self.soft_ratio, "soft") for it in (6000, 9000, 12000)]
        ev += [(int(round(it * f)), self.hard_ratio, "hard")
               for it in range(15000, 30000, 3000)]
        return ev


__all__ = ["n_keep", "select", "gather", "prune", "Schedule"]
