"""FP64 oracle of the paper's linear-wave example (TEST INFRASTRUCTURE ONLY).

Nothing in the product library imports this module; only the tests, the
smoke check and the benchmark's CPU-baseline leg do.  It shares no code with
the HIP path.

What it follows (section "An Example of Orthotope Machine Data-Flow Graph"):
the wave equation f_tt = c^2 f_xx written as f_t = g, g_t = c^2 f_xx on a
periodic line of n cells, advanced by the paper's discrete scheme (its
equations for f^{n+1} and g^{n+1}):

    f^{n+1}[i] = f^n[i] + dt g^n[i]
    g^{n+1}[i] = g^n[i] + (c^2 dt / dx^2) (f^{n+1}[i+1] + f^{n+1}[i-1] - 2 f^{n+1}[i])

and the discrete energy after each step, in the form the paper's source
listing computes (the printed equation squares c^2 and drops the 1/2; the
listing's form is the one whose continuum limit is the conserved energy):

    E^{n+1} = sum_i (1/2) (c^2 ((f^{n+1}[i+1] - f^{n+1}[i-1]) / (2 dx))^2
                           + ((g^n[i] + g^{n+1}[i]) / 2)^2) dx

The paper's runs use c = 3.43 on 0 <= x < 2 pi, dt = dx / c, f = sin x,
g = cos 3x, n = 8 ... 3072.
"""
from __future__ import annotations

import numpy as np


def step(f: np.ndarray, g: np.ndarray, c, dx, dt):
    """One step; returns (f^{n+1}, g^{n+1}, E^{n+1}).  FP64 arrays, or object
    arrays of exact numbers (fractions.Fraction, with c, dx, dt exact too):
    only +, -, * and / by integers and those numbers are used."""
    f = np.asarray(f)
    g = np.asarray(g)
    n = f.shape[0]
    right = (np.arange(n) + 1) % n   # index of cell i+1 (periodic)
    left = (np.arange(n) - 1) % n    # index of cell i-1
    f1 = f + dt * g
    g1 = g + (c * c * dt / (dx * dx)) * (f1[right] + f1[left] - 2 * f1)
    dfdx = (f1[right] - f1[left]) / (2 * dx)
    e = (c * c * dfdx * dfdx + ((g + g1) / 2) ** 2) * dx / 2
    return f1, g1, np.sum(e)


def advance(f, g, c: float, dx: float, dt: float, steps: int):
    """`steps` steps; returns (f, g, energies) with energies[k] = E after step k+1."""
    energies = []
    for _ in range(steps):
        f, g, e = step(f, g, c, dx, dt)
        energies.append(e)
    return f, g, np.array(energies)


def paper_initial(n: int, length: float = 2.0 * np.pi):
    """f = sin x, g = cos 3x at x_i = i dx, dx = length / n."""
    x = np.arange(n) * (length / n)
    return np.sin(x), np.cos(3.0 * x)
