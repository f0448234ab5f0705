"""Closed-form potentials that pin the oracle independently of its own code.

All of them follow from one-dimensional Gaussian integrals (the kernel is a
product over axes, Section 2):

* sigma = 1 on B, free space (Eq. (gkernel)):
      u(x) = prod_a sqrt(pi*delta)/2 [erf((1/2 - x_a)/sqrt(delta)) + erf((1/2 + x_a)/sqrt(delta))]
* sigma = 1, periodic kernel (Eq. (gper_kernel)): u = (pi*delta)^(d/2).
* one Gaussian blob a*exp(-|y-c|^2/w^2) restricted to B, free space:
  completing the square with s^2 = w^2 delta/(w^2+delta) and
  mu = (w^2 x + delta c)/(w^2+delta) gives, per axis,
      exp(-(x-c)^2/(delta+w^2)) * s sqrt(pi)/2 [erf((1/2-mu)/s) + erf((1/2+mu)/s)].
* a periodized blob with the periodic kernel: the integral over B of a
  periodic density against G_p equals the integral over R^d against G, so per
  axis  s sqrt(pi) * sum_j exp(-(x - c - j)^2/(delta+w^2)).
* the sin/cos density of Eq. (sigmap) is an eigenfunction of the periodic
  transform (Fourier form, Eq. (gp:fourier)):
      u = (pi*delta)^(d/2) exp(-d pi^2 delta nu^2) sigma_p(x).
"""

from __future__ import annotations

import math

import numpy as np
from scipy.special import erf


def const_free(x: np.ndarray, delta: float) -> np.ndarray:
    sd = math.sqrt(delta)
    f = 0.5 * math.sqrt(math.pi * delta) * (erf((0.5 - x) / sd) + erf((0.5 + x) / sd))
    return np.prod(f, axis=-1)


def const_periodic(x: np.ndarray, delta: float) -> np.ndarray:
    d = x.shape[-1]
    return np.full(x.shape[:-1], (math.pi * delta) ** (d / 2))


def blob_free(x: np.ndarray, delta: float, c, w: float, a: float) -> np.ndarray:
    w2 = w * w
    s = math.sqrt(w2 * delta / (w2 + delta))
    mu = (w2 * x + delta * np.asarray(c)) / (w2 + delta)
    f = (np.exp(-(x - c) ** 2 / (delta + w2)) * 0.5 * s * math.sqrt(math.pi)
         * (erf((0.5 - mu) / s) + erf((0.5 + mu) / s)))
    return a * np.prod(f, axis=-1)


def gaussian_sum_free(x, delta, dens) -> np.ndarray:
    out = np.zeros(x.shape[:-1])
    for c, w, a in zip(dens.centers, dens.widths, dens.amps):
        out += blob_free(x, delta, c, w, a)
    return out


def blob_periodized(x: np.ndarray, delta: float, c, w: float, a: float,
                    nimg: int = 3) -> np.ndarray:
    w2 = w * w
    s = math.sqrt(w2 * delta / (w2 + delta))
    f = np.zeros(x.shape)
    for j in range(-nimg, nimg + 1):
        f += np.exp(-(x - np.asarray(c) - j) ** 2 / (delta + w2))
    return a * np.prod(s * math.sqrt(math.pi) * f, axis=-1)


def gaussian_sum_periodized(x, delta, dens) -> np.ndarray:
    out = np.zeros(x.shape[:-1])
    for c, w, a in zip(dens.centers, dens.widths, dens.amps):
        out += blob_periodized(x, delta, c, w, a)
    return out


def sincos_periodic(x: np.ndarray, delta: float, nu: int) -> np.ndarray:
    d = x.shape[-1]
    sig = np.ones(x.shape[:-1])
    for a in range(d):
        f = np.sin if a % 2 == 0 else np.cos
        sig = sig * f(2 * math.pi * nu * x[..., a])
    return (math.pi * delta) ** (d / 2) * math.exp(-d * math.pi ** 2 * delta * nu ** 2) * sig


def rel_l2(a, b) -> float:
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def max_rel(a, b) -> float:
    """max |a - b| over max |b|: the pointwise companion of rel_l2."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
