"""Small parameter sets shared by the oracle pin tests and the parity tests."""
import numpy as np


def theta(range_=0.1, nu=0.5, sigma2=1.0, tau2=0.1, ratio=1.0, angle=0.0):
    return dict(range=range_, nu=nu, sigma2=sigma2, tau2=tau2, aniso_ratio=ratio, aniso_angle=angle)


def grid(n1, n2):
    return (n1, n2, 1.0 / n1, 1.0 / n2)
