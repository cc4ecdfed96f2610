"""Closed-form solutions used to pin the oracle (not part of the method).

Waveguide variant of eq. (1): Gamma^inc = {x=0} u {y=0} u {y=1} (and z-sides in 3D),
Gamma^inf = {x=1}, mu = kappa = 1, E^inc = (0, exp(-i w x)[, 0]).  The exact field
E = E^inc satisfies the equation and the first-order impedance condition at
x = 1 exactly (normal incidence), and its tangential trace on the y-, z-sides is
the Dirichlet data itself.

For the lowest order in 2D the discrete field is exactly (0, u_h(x)), with u_h the
continuous piecewise-linear Galerkin solution of u'' + w^2 u = 0, u(0) = 1,
u'(1) = -i w u(1).  Its nodal values solve a three-term recurrence whose
solutions are exp(+-i theta j) with the linear-element dispersion relation
    cos(theta) = (6 - 2 (w h)^2) / (6 + (w h)^2),
and the two amplitudes follow from u_0 = 1 and the discrete impedance row.  The
degree-0 DoF of a vertical edge at x_j is the circulation h * u_j.
"""
import numpy as np

WAVEGUIDE_INC_2D = 0b1101    # x=0, y=0, y=1
WAVEGUIDE_INC_3D = 0b111101  # x=0, y=0, y=1, z=0, z=1


def plane_wave(dim, omega):
    def exact(x):
        ph = np.exp(-1j * omega * x[:, 0])
        E = np.zeros((x.shape[0], dim), dtype=np.complex128)
        E[:, 1] = ph
        if dim == 2:
            C = (-1j * omega * ph)[:, None]
        else:
            C = np.zeros((x.shape[0], 3), dtype=np.complex128)
            C[:, 2] = -1j * omega * ph
        return E, C

    return exact


def waveguide_p0_nodal(nx, omega, kappa=1.0):
    """Nodal values u_0..u_nx of the exact 1D discrete (P1) solution."""
    h = 1.0 / nx
    wh = omega * h
    c = (6.0 - 2.0 * wh ** 2) / (6.0 + wh ** 2)
    theta = np.arccos(c)
    j = np.arange(nx + 1)
    ep = np.exp(-1j * theta * j)   # outgoing-type branch
    em = np.exp(1j * theta * j)
    # boundary row at x = 1:  (u_N - u_{N-1})/h - w^2 h/6 (2u_N + u_{N-1}) + i k w u_N = 0
    def brow(v):
        return (v[-1] - v[-2]) / h - omega ** 2 * h / 6.0 * (2 * v[-1] + v[-2]) + 1j * kappa * omega * v[-1]
    Mx = np.array([[ep[0], em[0]], [brow(ep), brow(em)]])
    a, b = np.linalg.solve(Mx, np.array([1.0, 0.0]))
    return a * ep + b * em
