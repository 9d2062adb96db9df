"""Seeded random vectors: sources and the random starts of the adaptive setup.

The paper draws the initial error vectors of its adaptive setup "randomly" and
tests point, Gaussian and Z4 sources.  Here every such vector is produced on the
host from ``numpy.random.default_rng(seed)`` and handed to both the GPU library
and the CPU oracle, so the two see bit-identical random inputs.

Vector layout everywhere: complex128 ``[t][x][dof]`` flattened, with ``dof`` the
per-site degrees of freedom of the level (2 spins on the fine lattice, Nv on a
coarse lattice).  Batches of right-hand sides are ``[nrhs][t][x][dof]``.
"""

from __future__ import annotations

import math
from typing import Sequence

import numpy as np


def gaussian(n: int | tuple, seed: int) -> np.ndarray:
    """Complex Gaussian with Re, Im ~ N(0, 1/2) (unit expected |z|^2)."""
    rng = np.random.default_rng(seed)
    shape = (n,) if isinstance(n, int) else tuple(n)
    z = rng.standard_normal((2,) + shape) * math.sqrt(0.5)
    return (z[0] + 1j * z[1]).astype(np.complex128)


def z2_noise(n: int | tuple, seed: int) -> np.ndarray:
    """Complex Z2 noise (+-1 +- i)/sqrt(2) per component."""
    rng = np.random.default_rng(seed)
    shape = (n,) if isinstance(n, int) else tuple(n)
    s = rng.integers(0, 2, size=(2,) + shape) * 2 - 1
    return ((s[0] + 1j * s[1]) / math.sqrt(2.0)).astype(np.complex128)


def point_source(lx: int, lt: int, x: int = 0, t: int = 0, spin: int = 0) -> np.ndarray:
    """Unit source at one site and spin (the paper's figures use point sources)."""
    v = np.zeros(lx * lt * 2, dtype=np.complex128)
    v[(t * lx + x) * 2 + spin] = 1.0
    return v


def level_shapes(lx: int, lt: int, blocks: Sequence[Sequence[int]], nvs: Sequence[int], split: bool = False):
    """(lx_l, lt_l, dof_l) for every level of a hierarchy; level 0 is the fine lattice.
    A coarse site carries Nv variables, or 2 Nv with chirality-split aggregates."""
    shapes = [(lx, lt, 2)]
    for (bx, bt), nv in zip(blocks, nvs):
        cx, ct, _ = shapes[-1]
        if cx % bx or ct % bt:
            raise ValueError(f"extent {cx}x{ct} not divisible by block {bx}x{bt}")
        shapes.append((cx // bx, ct // bt, nv * (2 if split else 1)))
    return shapes


def setup_randoms(lx: int, lt: int, blocks, nvs, seed: int, split: bool = False):
    """Random starts for the adaptive setup, one array per coarsening.

    For coarsening l (fine side of size n_l = lx_l*lt_l*dof_l) the array has shape
    ``[1 + Nv_l, n_l]``: row 0 starts the smoother calibration, rows 1..Nv_l start
    the Nv_l candidate near-null vectors in order.
    """
    shapes = level_shapes(lx, lt, blocks, nvs, split)
    out = []
    for lvl, nv in enumerate(nvs):
        cx, ct, dof = shapes[lvl]
        out.append(gaussian((1 + nv, cx * ct * dof), seed * 1000 + lvl))
    return out


def gaussian_device(n: int, seed: int, device="cuda", count: int = 1):
    """`count` complex Gaussian vectors (Re, Im ~ N(0, 1/2)) drawn by torch's
    generator on `device` from `seed`: [count, n] complex128.

    For request streams whose right-hand sides are too many to draw on the host;
    the values differ from ``gaussian(n, seed)`` (another generator) but are
    reproducible for a given device type and seed.
    """
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    z = torch.randn((count, n, 2), generator=g, device=device, dtype=torch.float64) * math.sqrt(0.5)
    return torch.view_as_complex(z)
