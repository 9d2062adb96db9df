"""Quenched U(1) gauge fields on a periodic 2D lattice (Results section of the paper).

The paper generates its fields with the Wilson plaquette action and periodic
boundary conditions at beta = 6 and 10 on 128^2.  Those fields are not available,
so seeded Monte Carlo fields with the same action stand in for them.

Conventions
-----------
* ``theta[mu, t, x]`` is the link angle, ``U = exp(i*theta)``; ``mu = 0`` is the x
  direction and ``mu = 1`` the t direction.
* Plaquette angle at site (x, t):
  ``theta_p = theta[0,t,x] + theta[1,t,x+1] - theta[0,t+1,x] - theta[1,t,x]``.
* Boltzmann weight ``exp(+beta * sum_p cos theta_p)``.  With this sign the mean
  plaquette is I1(beta)/I0(beta) and the area-law length ``1/sqrt(-ln(I1/I0))``
  gives 3.30 at beta = 6 and 4.35 at beta = 10, the values the paper quotes; the
  opposite sign would favour anti-aligned plaquettes.

The update is a checkerboard single-hit Metropolis.  Links that share no plaquette
are updated together: x-links on even t rows, then on odd t rows, then t-links on
even x columns, then on odd x columns.  The proposal is ``theta + delta*(2u-1)`` with
``delta = sqrt(2/beta)`` (acceptance about 0.64).  All randomness comes from
``numpy.random.default_rng(seed)`` in a fixed order, so a (L, beta, sweeps, seed)
tuple names one field exactly.
"""

from __future__ import annotations

import math

import numpy as np

TWO_PI = 2.0 * math.pi


def plaquette_angles(theta: np.ndarray) -> np.ndarray:
    """Plaquette angle theta_p[t, x] (unwrapped sum of the four link angles)."""
    th0, th1 = theta[0], theta[1]
    return th0 + np.roll(th1, -1, axis=1) - np.roll(th0, -1, axis=0) - th1


def mean_plaquette(theta: np.ndarray) -> float:
    """<cos theta_p> over all plaquettes."""
    return float(np.mean(np.cos(plaquette_angles(theta))))


def topological_charge(theta: np.ndarray) -> float:
    """Geometric charge Q = (1/2pi) sum_p arg(exp(i theta_p)), arg in (-pi, pi].

    The paper mentions a gauge-invariant topological charge without defining it;
    this is the standard geometric definition.  On a torus it is an integer because
    every link enters two plaquettes with opposite signs.
    """
    p = plaquette_angles(theta)
    wrapped = np.angle(np.exp(1j * p))
    return float(np.sum(wrapped) / TWO_PI)


def links_from_angles(theta: np.ndarray) -> np.ndarray:
    """U[mu, t, x] = exp(i theta) as complex128 (the library's gauge layout)."""
    return np.exp(1j * theta).astype(np.complex128)


def _wrap(a: np.ndarray) -> np.ndarray:
    return (a + math.pi) % TWO_PI - math.pi


def metropolis_u1(lx: int, lt: int, beta: float, sweeps: int, seed: int, cold: bool = False) -> np.ndarray:
    """Return link angles theta[2, lt, lx] after ``sweeps`` Metropolis sweeps from a hot
    start (uniform angles), or from a cold start (all angles 0, topological charge 0,
    which local updates at these couplings practically never change)."""
    if lx % 2 or lt % 2:
        raise ValueError("checkerboard update needs even extents")
    rng = np.random.default_rng(seed)
    theta = rng.uniform(-math.pi, math.pi, size=(2, lt, lx))
    if cold:
        theta[:] = 0.0
    delta = math.sqrt(2.0 / beta) if beta > 0 else math.pi
    for _ in range(sweeps):
        for mu in (0, 1):
            for parity in (0, 1):
                p = plaquette_angles(theta)
                if mu == 0:
                    # x-link at (t, x) enters p[t, x] with + and p[t-1, x] with -.
                    rows = np.arange(parity, lt, 2)
                    p_plus = p[rows, :]
                    p_minus = p[(rows - 1) % lt, :]
                    old = theta[0, rows, :]
                else:
                    # t-link at (t, x) enters p[t, x-1] with + and p[t, x] with -.
                    cols = np.arange(parity, lx, 2)
                    p_plus = p[:, (cols - 1) % lx]
                    p_minus = p[:, cols]
                    old = theta[1][:, cols]
                u = rng.random(old.shape)
                acc = rng.random(old.shape)
                step = delta * (2.0 * u - 1.0)
                ds = beta * (
                    np.cos(p_plus + step)
                    + np.cos(p_minus - step)
                    - np.cos(p_plus)
                    - np.cos(p_minus)
                )
                take = acc < np.exp(np.minimum(ds, 0.0))
                new = np.where(take, _wrap(old + step), old)
                if mu == 0:
                    theta[0, rows, :] = new
                else:
                    theta[1][:, cols] = new
    return theta


def string_length(beta: float) -> float:
    """Correlation length l from the area law W ~ exp(-Area / l^2).

    In 2D U(1) a Wilson loop of area a is (I1(beta)/I0(beta))^a exactly, so
    l = 1 / sqrt(-ln(I1/I0)).
    """
    from scipy.special import i0, i1

    return 1.0 / math.sqrt(-math.log(i1(beta) / i0(beta)))


def metropolis_u1_device(lx: int, lt: int, beta: float, sweeps: int, seed: int, count: int = 1,
                         device="cuda"):
    """`count` fields of link angles [count, 2, lt, lx] from the same checkerboard
    Metropolis as metropolis_u1 (hot start, the same update order and proposal width),
    run with torch on `device` for request streams over many large fields.  The random
    numbers come from torch's generator seeded with `seed`, so the fields differ from
    metropolis_u1's for the same seed but are reproducible for a device type and seed."""
    import torch

    if lx % 2 or lt % 2:
        raise ValueError("checkerboard update needs even extents")
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    f64 = torch.float64
    theta = (torch.rand((count, 2, lt, lx), generator=g, device=device, dtype=f64) * 2.0 - 1.0) * math.pi
    delta = math.sqrt(2.0 / beta) if beta > 0 else math.pi

    def plaq(th):
        return th[:, 0] + torch.roll(th[:, 1], -1, dims=2) - torch.roll(th[:, 0], -1, dims=1) - th[:, 1]

    for _ in range(sweeps):
        for mu in (0, 1):
            for parity in (0, 1):
                p = plaq(theta)
                if mu == 0:  # x-link at (t, x): + in p[t, x], - in p[t-1, x]
                    p_plus = p[:, parity::2, :]
                    p_minus = torch.roll(p, 1, dims=1)[:, parity::2, :]
                    old = theta[:, 0, parity::2, :]
                else:  # t-link at (t, x): + in p[t, x-1], - in p[t, x]
                    p_plus = torch.roll(p, 1, dims=2)[:, :, parity::2]
                    p_minus = p[:, :, parity::2]
                    old = theta[:, 1, :, parity::2]
                u = torch.rand(old.shape, generator=g, device=device, dtype=f64)
                acc = torch.rand(old.shape, generator=g, device=device, dtype=f64)
                step = delta * (2.0 * u - 1.0)
                ds = beta * (torch.cos(p_plus + step) + torch.cos(p_minus - step) - torch.cos(p_plus)
                             - torch.cos(p_minus))
                take = acc < torch.exp(torch.clamp(ds, max=0.0))
                new = torch.where(take, torch.remainder(old + step + math.pi, TWO_PI) - math.pi, old)
                if mu == 0:
                    theta[:, 0, parity::2, :] = new
                else:
                    theta[:, 1, :, parity::2] = new
    return theta
