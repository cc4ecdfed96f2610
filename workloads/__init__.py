"""Seeded synthetic workloads (problem parameters and random inputs only).

This module holds no arithmetic of the method: it only states the problem
parameters of the benchmark configurations and draws the random inputs (per-cell
mu fields, the batch of independent problems).  Both the oracle and the GPU path
consume the same arrays, so no cross-implementation random number generator is
needed.

Configurations (all on axis-aligned unit boxes, kappa = 1, incident plane wave
E^inc = pol * exp(-i w d.x) on the x = 0 side, impedance on every other side):
  c1  2D 16^2 quads, degree 0, w = 10, single domain
  c2  2D 256^2 quads, degree 2, w = 50, 4x4 subdomains
  c3  3D 32^3 hexes, degree 1, mu ~ U[1,2] per cell (seed 3), w = 20, 2x2x2 subdomains
  c4  256 independent 2D problems: m in {32,64,96,128}, degree in {0,1,2},
      w ~ U[5,60], incidence angle theta ~ U[0, pi/2) (seed 4, drawn per problem in
      the order m, p, w, theta); d = (cos t, sin t), pol = (-sin t, cos t); 32 members
      sampled for member-by-member comparison (seed 7)
  c5  2D 128^2 quads, degree 1, w = 30, mu = clip(1 + 3 f, 1, 4) with f a
      standardised Gaussian random field (seed 5, correlation length 0.1);
      target box [0.7,0.9]^2; 32 finite-difference cells (seed 6)
  block  the block benchmark of Sec. 4.1: unit square, a centre square of refractive
      index 1.516 (eps = 1.516^2) in air (eps = 1); centre [0.25, 0.75]^2 (the paper gives
      no size), degree 1, mesh m^2, single domain, swept over w in {5, 10, 20, 40, 80}
"""
import math

import numpy as np


def _base(dim, n, p, omega, **kw):
    d = dict(dim=dim, n=tuple(n) + (1,) * (3 - len(n)), p=p, omega=float(omega), kappa=1.0,
             mu=None, inc_faces=1, inc_dir=(1.0, 0.0, 0.0), inc_pol=(0.0, 1.0, 0.0),
             lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), subdomains=(1, 1, 1), eps=None)
    d.update(kw)
    return d


def c1():
    return _base(2, (16, 16), 0, 10.0)


def c2(m=256, sub=4):
    return _base(2, (m, m), 2, 50.0, subdomains=(sub, sub, 1))


def mu_uniform(n_cells, seed=3):
    return np.random.default_rng(seed).uniform(1.0, 2.0, n_cells)


def c3(m=32, sub=2):
    return _base(3, (m, m, m), 1, 20.0, mu=mu_uniform(m ** 3), subdomains=(sub, sub, sub))


def c4_draws(count=256, seed=4):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        m = int(rng.choice([32, 64, 96, 128]))
        p = int(rng.integers(0, 3))
        w = float(rng.uniform(5.0, 60.0))
        th = float(rng.uniform(0.0, math.pi / 2))
        out.append((m, p, w, th))
    return out


def c4(count=256, seed=4, scale=1):
    """List of problem dicts; scale > 1 divides every mesh size (small test variants)."""
    probs = []
    for m, p, w, th in c4_draws(count, seed):
        mm = max(2, m // scale)
        probs.append(_base(2, (mm, mm), p, w, inc_dir=(math.cos(th), math.sin(th), 0.0),
                           inc_pol=(-math.sin(th), math.cos(th), 0.0)))
    return probs


def c4_sample(count=32, total=256, seed=7):
    """Seeded sample of member indices of the uneven batch (compared member by member with
    the oracle's LU at full size)."""
    return np.sort(np.random.default_rng(seed).choice(total, size=count, replace=False))


def grf(m, seed=5, corr=0.1):
    """Standardised periodic Gaussian random field on the m x m cell-centre grid."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((m, m))
    x = (np.arange(m) + 0.5) / m
    dx = np.abs(x - x[0])                 # periodic distance to the first cell centre
    dx = np.minimum(dx, 1.0 - dx)
    r2 = dx[:, None] ** 2 + dx[None, :] ** 2
    k = np.exp(-r2 / (2 * corr ** 2))
    f = np.real(np.fft.ifft2(np.fft.fft2(w) * np.fft.fft2(k)))
    f = (f - f.mean()) / f.std()
    return f


def mu_grf(m=128, seed=5):
    """mu = clip(1 + 3 f, 1, 4), row-major with x fastest (index j*m + i)."""
    f = grf(m, seed)
    return np.clip(1.0 + 3.0 * f, 1.0, 4.0).ravel()


def c5(m=128):
    return _base(2, (m, m), 1, 30.0, mu=mu_grf(m))


C5_TARGET = ((0.7, 0.7, 0.0), (0.9, 0.9, 1.0))


def fd_cells(n_cells, count=32, seed=6):
    return np.sort(np.random.default_rng(seed).choice(n_cells, size=count, replace=False))


BLOCK_OMEGAS = (5.0, 10.0, 20.0, 40.0, 80.0)


def eps_block(m, n_center=1.516, lo=0.25, hi=0.75):
    """eps per cell of an m x m unit square (x fastest): n_center^2 where the cell centre lies
    in [lo, hi]^2, 1 elsewhere."""
    c = (np.arange(m) + 0.5) / m
    inside = (c >= lo) & (c <= hi)
    e = np.where(inside[:, None] & inside[None, :], n_center ** 2, 1.0)  # [j, i]
    return e.ravel()


def block(m=128, omega=20.0, p=1):
    return _base(2, (m, m), p, omega, eps=eps_block(m))
