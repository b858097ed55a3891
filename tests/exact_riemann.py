"""Exact solution of the 1D Riemann problem for the shallow water equations
over a flat bed (wet states on both sides; each of the two waves a shock or
a rarefaction), and Ritter's dam break onto a dry bed.  Textbook material
(two-wave structure, Newton iteration on the middle depth), used by the
tests as ground truth."""
import math

import numpy as np

G = 9.81


def _wave_function(h, hK):
    """Velocity change across a wave from depth hK to depth h, and its derivative."""
    cK = math.sqrt(G * hK)
    if h <= hK:  # rarefaction
        c = math.sqrt(G * h)
        return 2.0 * (c - cK), G / c
    gk = math.sqrt(0.5 * G * (h + hK) / (h * hK))  # shock
    return (h - hK) * gk, gk - G * (h - hK) / (4.0 * gk * h * h)


def exact_riemann(hL, uL, hR, uR, xi):
    """Depth and velocity of the exact solution at x/t = xi."""
    h = 0.5 * (hL + hR)
    for _ in range(100):
        fL, dL = _wave_function(h, hL)
        fR, dR = _wave_function(h, hR)
        step = (fL + fR + uR - uL) / (dL + dR)
        h = max(h - step, 1e-12)
        if abs(step) < 1e-15 * h:
            break
    fL, _ = _wave_function(h, hL)
    fR, _ = _wave_function(h, hR)
    hs, us = h, 0.5 * (uL + uR) + 0.5 * (fR - fL)
    cL, cR, cs = math.sqrt(G * hL), math.sqrt(G * hR), math.sqrt(G * hs)
    out_h, out_u = np.empty_like(xi), np.empty_like(xi)
    for k, x in enumerate(xi):
        if x <= us:  # left of the contact: left wave
            if hs > hL:  # shock
                sL = uL - cL * math.sqrt(0.5 * hs * (hs + hL)) / hL
                out_h[k], out_u[k] = (hL, uL) if x < sL else (hs, us)
            elif x < uL - cL:
                out_h[k], out_u[k] = hL, uL
            elif x > us - cs:
                out_h[k], out_u[k] = hs, us
            else:
                c = (uL + 2.0 * cL - x) / 3.0
                out_h[k], out_u[k] = c * c / G, x + c
        else:
            if hs > hR:
                sR = uR + cR * math.sqrt(0.5 * hs * (hs + hR)) / hR
                out_h[k], out_u[k] = (hR, uR) if x > sR else (hs, us)
            elif x > uR + cR:
                out_h[k], out_u[k] = hR, uR
            elif x < us + cs:
                out_h[k], out_u[k] = hs, us
            else:
                c = (x - uR + 2.0 * cR) / 3.0
                out_h[k], out_u[k] = c * c / G, x - c
    return out_h, out_u, hs, us



def ritter(h0, xi, g=G):
    """Dam break of depth h0 at rest onto a dry bed: depth and velocity at x/t = xi."""
    c0 = math.sqrt(g * h0)
    xi = np.asarray(xi, dtype=np.float64)
    h = np.where(xi <= -c0, h0, np.where(xi >= 2 * c0, 0.0, (2 * c0 - xi) ** 2 / (9 * g)))
    u = np.where((xi > -c0) & (xi < 2 * c0), 2.0 * (c0 + xi) / 3.0, 0.0)
    return h, u
