"""Integrands for per-pixel integro-approximation, in FP64 (Sec. 2.5 and Sec. 3 use
light-transport integrands; the paper's test-function advice in Sec. 2.6 motivates
these synthetic stand-ins with closed-form integrals).

Genz product (per pixel p, d = 8, parameters u_0..u_7 centres, a_0..a_7 widths):
  f_p(x) = exp(-sum_{j<4} a_j^2 (x_j - u_j)^2) * cos(2 pi u_4 + sum_{j=4..7} a_j x_j)
  envelope_p(x) = exp(-sum_{j<4} a_j^2 (x_j - u_j)^2)   (the bound |f_p| <= envelope_p)

Gaussian lobes (shared theta; L lobes in d dimensions; per-pixel offset delta_p):
  theta = [centres c (L x d), log-widths l (L x d), weights w (L)]
  G_k(y) = exp(-1/2 sum_j ((y_j - c_kj) e^{-l_kj})^2),   f(y) = sum_k w_k G_k(y),
  evaluated at y = x + delta_p (no wrap-around).
  df/dw_k = G_k,   df/dc_kj = w_k G_k r_kj / sigma_kj,   df/dl_kj = w_k G_k r_kj^2,
  with sigma_kj = e^{l_kj} and r_kj = (y_j - c_kj) / sigma_kj.
"""

import math

import numpy as np
from scipy.special import erf


def genz(x, pp):
    """(f, envelope) for points x [8][n] (float64) and per-sample params pp [n][16] (float64)."""
    u = pp[:, :8].T
    a = pp[:, 8:].T
    e = np.zeros(x.shape[1])
    for j in range(4):
        e += a[j] ** 2 * (x[j] - u[j]) ** 2
    phase = 2.0 * math.pi * u[4]
    for j in range(4, 8):
        phase += a[j] * x[j]
    env = np.exp(-e)
    return env * np.cos(phase), env


def genz_integral(pp):
    """Closed-form integral of f_p over [0,1)^8 for one pixel's params pp [16]."""
    u = np.asarray(pp[:8], dtype=np.float64)
    a = np.asarray(pp[8:], dtype=np.float64)
    gauss = 1.0
    for j in range(4):
        gauss *= math.sqrt(math.pi) / (2.0 * a[j]) * (erf(a[j] * (1.0 - u[j])) + erf(a[j] * u[j]))
    z = complex(math.cos(2 * math.pi * u[4]), math.sin(2 * math.pi * u[4]))
    for j in range(4, 8):
        z *= (complex(math.cos(a[j]), math.sin(a[j])) - 1.0) / complex(0.0, a[j])
    return gauss * z.real


def split_theta(theta, num_lobes, dim):
    """(centres [L][d], log-widths [L][d], weights [L]) views of theta (float64)."""
    L, d = num_lobes, dim
    th = np.asarray(theta, dtype=np.float64)
    return th[: L * d].reshape(L, d), th[L * d: 2 * L * d].reshape(L, d), th[2 * L * d: 2 * L * d + L]


def lobes(y, theta, num_lobes, dim):
    """f(y) for points y [d][n] (float64)."""
    c, ell, w = split_theta(theta, num_lobes, dim)
    f = np.zeros(y.shape[1])
    for k in range(num_lobes):
        q = np.zeros(y.shape[1])
        for j in range(dim):
            r = (y[j] - c[k, j]) / math.exp(ell[k, j])
            q += r * r
        f += w[k] * np.exp(-0.5 * q)
    return f


def lobes_weighted_gradient(y, scale, theta, num_lobes, dim):
    """sum_n scale_n * d f(y_n) / d theta, float64 [L*(2d+1)]."""
    c, ell, w = split_theta(theta, num_lobes, dim)
    L, d = num_lobes, dim
    gc = np.zeros((L, d))
    gl = np.zeros((L, d))
    gw = np.zeros(L)
    for k in range(L):
        sig = np.exp(ell[k])
        r = (y - c[k][:, None]) / sig[:, None]           # [d][n]
        G = np.exp(-0.5 * np.sum(r * r, axis=0))         # [n]
        sG = scale * G
        gw[k] = math.fsum(sG)
        for j in range(d):
            gc[k, j] = math.fsum(w[k] * sG * r[j] / sig[j])
            gl[k, j] = math.fsum(w[k] * sG * r[j] * r[j])
    return np.concatenate([gc.ravel(), gl.ravel(), gw])


def lobes_weighted_gradient_abs(y, scale, theta, num_lobes, dim):
    """sum_n |scale_n| * |d f(y_n) / d theta| per parameter, float64 [L*(2d+1)]: the size of the
    terms a gradient sum adds up, which bounds its rounding error (a test tolerance, not part of
    the method)."""
    c, ell, w = split_theta(theta, num_lobes, dim)
    L, d = num_lobes, dim
    gc = np.zeros((L, d))
    gl = np.zeros((L, d))
    gw = np.zeros(L)
    a = np.abs(scale)
    for k in range(L):
        sig = np.exp(ell[k])
        r = (y - c[k][:, None]) / sig[:, None]
        G = np.exp(-0.5 * np.sum(r * r, axis=0))
        sG = a * G
        gw[k] = math.fsum(sG)
        for j in range(d):
            gc[k, j] = math.fsum(np.abs(w[k] * sG * r[j] / sig[j]))
            gl[k, j] = math.fsum(np.abs(w[k] * sG * r[j] * r[j]))
    return np.concatenate([gc.ravel(), gl.ravel(), gw])


def lobes_box_integral(delta, theta, num_lobes, dim):
    """Closed-form integral over x in [0,1)^d of f(x + delta) for one offset vector delta [d]."""
    c, ell, w = split_theta(theta, num_lobes, dim)
    total = 0.0
    for k in range(num_lobes):
        prod = 1.0
        for j in range(dim):
            sig = math.exp(ell[k, j])
            lo = (delta[j] - c[k, j]) / (sig * math.sqrt(2.0))
            hi = (1.0 + delta[j] - c[k, j]) / (sig * math.sqrt(2.0))
            prod *= sig * math.sqrt(math.pi / 2.0) * (erf(hi) - erf(lo))
        total += w[k] * prod
    return total
