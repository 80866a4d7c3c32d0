"""Closed-form quantities used to pin the oracle.

Ray geometry here is built from the stated conventions with vector algebra
(explicit source, detector centre and detector axes), not from the oracle's
code; the line integrals are exact integrals of the continuous phantoms.

Unit-ball profiles, for a line at distance s from the centre:
  uniform density 1:     integral = 2 sqrt(1 - s^2)
  smooth (1 - rho^2)^2:  integral = (16/15) (1 - s^2)^(5/2)
An ellipse/ellipsoid x = c + R S u (u in the unit ball) maps a unit-speed
world line o + t d to u0 + t e with e = S^-1 R^T d, so the world integral is
the unit-ball integral along the line through u0 with direction e/|e|,
divided by |e|.
"""

import math
import numpy as np
from scipy.special import dawsn


def uniform_angles(kind, n_views):
    span = math.pi if kind == 0 else 2.0 * math.pi
    return np.array([(span * p) / n_views for p in range(n_views)])


def angles_of(g):
    return uniform_angles(g.kind, g.n_views) if g.angles is None else np.asarray(g.angles, float)


def rays_2d(g):
    """Unit-speed rays (origin, direction) of a 2D parallel geometry,
    arrays of shape (P, nu, 2)."""
    th = angles_of(g)
    s = (np.arange(g.nu) - 0.5 * (g.nu - 1)) * g.du
    n = np.stack([np.cos(th), np.sin(th)], axis=-1)          # (P, 2)
    d = np.stack([-np.sin(th), np.cos(th)], axis=-1)
    o = s[None, :, None] * n[:, None, :]
    return o, np.broadcast_to(d[:, None, :], o.shape)


def cone_frame(g, theta):
    src = np.array([g.sod * math.cos(theta), g.sod * math.sin(theta), 0.0])
    cen = src - g.sdd * np.array([math.cos(theta), math.sin(theta), 0.0])
    eu = np.array([-math.sin(theta), math.cos(theta), 0.0])
    ev = np.array([0.0, 0.0, 1.0])
    return src, cen, eu, ev


def rays_3d(g):
    """Unit-speed rays of a cone geometry, arrays (P, nv, nu, 3)."""
    th = angles_of(g)
    u = (np.arange(g.nu) - 0.5 * (g.nu - 1)) * g.du
    v = (np.arange(g.nv) - 0.5 * (g.nv - 1)) * g.dv
    O = np.zeros((g.n_views, g.nv, g.nu, 3))
    D = np.zeros_like(O)
    for p, t in enumerate(th):
        src, cen, eu, ev = cone_frame(g, t)
        pix = cen[None, None, :] + u[None, :, None] * eu + v[:, None, None] * ev
        r = pix - src
        O[p] = src
        D[p] = r / np.linalg.norm(r, axis=-1, keepdims=True)
    return O, D


def _unit_ball_integral(u0, e, profile):
    en = np.linalg.norm(e, axis=-1)
    eh = e / en[..., None]
    proj = (u0 * eh).sum(-1)
    s2 = np.maximum((u0 * u0).sum(-1) - proj * proj, 0.0)
    inside = s2 < 1.0
    one = np.where(inside, 1.0 - s2, 0.0)
    if profile == "uniform":
        val = 2.0 * np.sqrt(one)
    else:
        val = (16.0 / 15.0) * one ** 2.5
    return val / en


def ellipse_line_integrals(ells, O, D, profile="uniform"):
    out = np.zeros(O.shape[:-1])
    for el in ells:
        c, s_ = math.cos(el["phi"]), math.sin(el["phi"])
        Rt = np.array([[c, s_], [-s_, c]])
        Sinv = np.array([1.0 / el["a"], 1.0 / el["b"]])
        u0 = ((O - np.array([el["cx"], el["cy"]])) @ Rt.T) * Sinv
        e = (D @ Rt.T) * Sinv
        out += el["rho"] * _unit_ball_integral(u0, e, profile)
    return out


def ellipsoid_line_integrals(ells, O, D, profile="uniform"):
    out = np.zeros(O.shape[:-1])
    for el in ells:
        Rt = el["R"].T
        Sinv = 1.0 / el["semi"]
        u0 = ((O - el["centre"]) @ Rt.T) * Sinv
        e = (D @ Rt.T) * Sinv
        out += el["rho"] * _unit_ball_integral(u0, e, profile)
    return out


def ramp_filtered_gaussian(x, sigma):
    """Continuous ramp filter (|k| in cycles per unit length) applied to
    exp(-x^2 / (2 sigma^2)):
      R g(x) = 2 sigma sqrt(2 pi) * int_0^inf k exp(-a k^2) cos(b k) dk,
      a = 2 pi^2 sigma^2, b = 2 pi x,
    and int_0^inf k exp(-a k^2) cos(b k) dk = (1 - (b/sqrt a) D(b/(2 sqrt a))) / (2a)
    with D Dawson's integral."""
    a = 2.0 * math.pi ** 2 * sigma ** 2
    b = 2.0 * math.pi * np.asarray(x, float)
    inner = (1.0 - (b / math.sqrt(a)) * dawsn(b / (2.0 * math.sqrt(a)))) / (2.0 * a)
    return 2.0 * sigma * math.sqrt(2.0 * math.pi) * inner
