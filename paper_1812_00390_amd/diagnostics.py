"""Flow diagnostics of the paper's cylinder cases (Sections 3.3-3.4) built on
the library's wall force.

  force_coefficients  C_d, C_l = F / (rho_inf U^2 D / 2) from fvlbm_wall_force
  pressure_coefficient C_p = (p - p_inf) / (rho_inf U^2 / 2), p = rho/3 per wall face
  strouhal            St = f D / U from the dominant frequency of a lift history

The force and the wall pressure are computed on the GPU (FP64 reductions of the
stored state); this module only scales them and analyses time series on the host.
"""
from __future__ import annotations

import numpy as np


def force_coefficients(force, rho_inf: float, u_inf: float, diameter: float):
    """(C_d, C_l) of a force per unit depth (Fx along the free stream, Fy across it)."""
    q = 0.5 * rho_inf * u_inf * u_inf * diameter
    return float(force[0]) / q, float(force[1]) / q


def pressure_coefficient(face_p, rho_inf: float, u_inf: float):
    """C_p of wall-face pressures p = rho/3 against p_inf = rho_inf/3."""
    return (np.asarray(face_p, dtype=float) - rho_inf / 3.0) / (0.5 * rho_inf * u_inf * u_inf)


def strouhal(t, cl, diameter: float, u_inf: float, discard: float = 0.0) -> float:
    """St = f D / U, f the dominant frequency of cl(t) (uniform samples), located by
    the largest periodogram bin of the mean-removed, Hann-windowed series, refined by
    a parabola through the peak bin and its neighbours.  The first `discard` fraction
    of the history (the start-up) is dropped."""
    t = np.asarray(t, dtype=float)
    cl = np.asarray(cl, dtype=float)
    k0 = int(discard * len(t))
    t, cl = t[k0:], cl[k0:]
    if len(t) < 8:
        raise ValueError("too few samples for a frequency")
    dt = float(np.mean(np.diff(t)))
    x = (cl - cl.mean()) * np.hanning(len(cl))
    spec = np.abs(np.fft.rfft(x)) ** 2
    spec[0] = 0.0
    k = int(np.argmax(spec))
    delta = 0.0
    if 0 < k < len(spec) - 1:
        a, b, c = np.log(spec[k - 1] + 1e-300), np.log(spec[k] + 1e-300), np.log(spec[k + 1] + 1e-300)
        den = a - 2 * b + c
        if den != 0:
            delta = 0.5 * (a - c) / den
    f = (k + delta) / (len(cl) * dt)
    return f * diameter / u_inf
