"""Detector response: antenna patterns and time delays (plain FP64).

The paper projects each template onto the network through antenna patterns
and a time delay (Sec. III.D, heterodyne paragraph; Sec. IV.A).  Conventions:
source direction s = (cos dec cos phi, cos dec sin phi, sin dec) with
phi = ra - gmst; polarisation frame X = -cos(psi) m + sin(psi) n,
Y = sin(psi) m + cos(psi) n with m = (-sin phi, cos phi, 0) and
n = (-sin dec cos phi, -sin dec sin phi, cos dec);
F+ = X.D.X - Y.D.Y, Fx = X.D.Y + Y.D.X; delay dt = -s.r / c.
"""
from __future__ import annotations

import math

import numpy as np

C_SI = 299792458.0


def source_frame(ra: float, dec: float, gmst: float = 0.0):
    phi = ra - gmst
    s = np.array([math.cos(dec) * math.cos(phi), math.cos(dec) * math.sin(phi), math.sin(dec)])
    m = np.array([-math.sin(phi), math.cos(phi), 0.0])
    n = np.array([-math.sin(dec) * math.cos(phi), -math.sin(dec) * math.sin(phi), math.cos(dec)])
    return s, m, n


def antenna_pattern(tensor: np.ndarray, ra: float, dec: float, psi: float, gmst: float = 0.0):
    """(F+, Fx) of one detector with tensor ``tensor`` [3, 3]."""
    _, m, n = source_frame(ra, dec, gmst)
    x = -math.cos(psi) * m + math.sin(psi) * n
    y = math.sin(psi) * m + math.cos(psi) * n
    fp = x @ tensor @ x - y @ tensor @ y
    fx = x @ tensor @ y + y @ tensor @ x
    return float(fp), float(fx)


def time_delay(pos: np.ndarray, ra: float, dec: float, gmst: float = 0.0) -> float:
    """Arrival time at ``pos`` (m) minus arrival time at the geocentre (s)."""
    s, _, _ = source_frame(ra, dec, gmst)
    return -float(s @ pos) / C_SI
