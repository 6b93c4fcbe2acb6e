"""Host-side scaling and time-series analysis of the flow diagnostics."""
import numpy as np
import pytest

from paper_1812_00390_amd import diagnostics as D


def test_force_and_pressure_coefficients():
    cd, cl = D.force_coefficients([0.0134, -0.002], rho_inf=1.0, u_inf=0.1, diameter=1.0)
    assert cd == pytest.approx(2.68) and cl == pytest.approx(-0.4)
    cp = D.pressure_coefficient([1 / 3 + 0.005, 1 / 3], rho_inf=1.0, u_inf=0.1)
    assert cp == pytest.approx([1.0, 0.0])


@pytest.mark.parametrize("st", [0.164, 0.2, 0.25])
def test_strouhal_of_a_sinusoid(st):
    U, Dm = 0.1, 1.0
    f = st * U / Dm
    t = np.arange(0, 40 / f, 0.37)
    cl = 0.3 * np.sin(2 * np.pi * f * t + 0.4) + 0.05 * np.sin(2 * np.pi * 3 * f * t) + 0.01
    assert D.strouhal(t, cl, Dm, U) == pytest.approx(st, rel=2e-3)


def test_strouhal_ignores_the_startup():
    U, Dm, f = 0.1, 1.0, 0.0165
    t = np.arange(0, 60 / f, 1.0)
    cl = np.where(t < 20 / f, 0.5 * np.exp(-t * 1e-3), 0.2 * np.sin(2 * np.pi * f * t))
    assert D.strouhal(t, cl, Dm, U, discard=0.4) == pytest.approx(f * Dm / U, rel=3e-3)
