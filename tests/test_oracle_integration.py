"""Pins for the oracle's integrands, per-pixel estimator and gradients.

The integrands are synthetic stand-ins for light transport (Sec. 2.6 recommends test
functions with analytic integrals); they are pinned by closed forms, by adaptive
quadrature from scipy, by QMC convergence and by central finite differences.
"""

import math

import numpy as np
import pytest
from scipy import integrate

from oracle import digital, estimator, integrands
from synth import counts_uniform, genz_params, lobe_params, perturb, sobol_direction_init


def _sampler(s, flags, seed=9):
    return {"kind": "sobol", "s": s, "table": digital.sobol_matrices(s, sobol_direction_init(s, 0)),
            "seed": seed, "flags": flags}


def test_genz_closed_form_factors_match_quadrature():
    pp = genz_params(3, 4)[2].astype(np.float64)
    u, a = pp[:8], pp[8:]
    gauss = 1.0
    for j in range(4):
        gauss *= integrate.quad(lambda t: math.exp(-a[j] ** 2 * (t - u[j]) ** 2), 0, 1,
                                epsabs=1e-14, epsrel=1e-12, limit=200)[0]
    # oscillatory factor: integrate cos(phase) over [0,1)^4 as the real part of a product
    z = complex(math.cos(2 * math.pi * u[4]), math.sin(2 * math.pi * u[4]))
    for j in range(4, 8):
        re = integrate.quad(lambda t: math.cos(a[j] * t), 0, 1, limit=200)[0]
        im = integrate.quad(lambda t: math.sin(a[j] * t), 0, 1, limit=200)[0]
        z *= complex(re, im)
    assert integrands.genz_integral(pp) == pytest.approx(gauss * z.real, rel=1e-9, abs=1e-13)


def test_genz_peak_value_and_envelope():
    pp = genz_params(1, 4).astype(np.float64)
    x = np.zeros((8, 1))
    x[:4, 0] = pp[0, :4]
    x[4:, 0] = 0.0
    f, env = integrands.genz(x, pp)
    assert env[0] == 1.0
    assert f[0] == pytest.approx(math.cos(2 * math.pi * pp[0, 4]), rel=1e-15)


def test_genz_estimator_converges_to_closed_form():
    # Moderate widths so that 2^14 unscrambled Sobol' points resolve the integrand.
    pp = genz_params(4, 4).astype(np.float64)
    pp[:, 8:] = 1.0 + 0.25 * (pp[:, 8:] - 2.0) / 18.0 * 4.0
    integrand = {"kind": "genz", "d": 8, "pixel_params": pp.astype(np.float32)}
    n = 1 << 14
    r = estimator.integrate_pixels(_sampler(8, 0), integrand, np.full(4, n, np.uint32), range(4))
    for p in range(4):
        exact = integrands.genz_integral(pp[p].astype(np.float32).astype(np.float64))
        assert abs(r["mean"][p] - exact) < 2e-4, (p, r["mean"][p], exact)


def test_lobes_box_integral_matches_quadrature():
    theta = lobe_params(2, 2, 6).astype(np.float64)
    delta = np.array([0.1, -0.2])
    c, ell, w = integrands.split_theta(theta, 2, 2)
    num = 0.0
    for k in range(2):
        prod = 1.0
        for j in range(2):
            prod *= integrate.quad(lambda t: math.exp(-0.5 * ((t + delta[j] - c[k, j]) / math.exp(ell[k, j])) ** 2),
                                   0, 1, epsabs=1e-14)[0]
        num += w[k] * prod
    assert integrands.lobes_box_integral(delta, theta, 2, 2) == pytest.approx(num, rel=1e-10)


def test_lobes_estimator_converges_to_box_integral():
    # Widened lobes (sigma x 2.5) so that 2^14 points resolve them in 8 dimensions.
    L, d = 4, 8
    theta = lobe_params(L, d, 6)
    theta[L * d:2 * L * d] += np.float32(math.log(2.5))
    integrand = {"kind": "lobes", "d": d, "num_lobes": L, "params": theta, "pixel_seed": 3}
    counts = np.full(3, 1 << 14, np.uint32)
    r = estimator.integrate_pixels(_sampler(d, estimator.PIXEL_NUS | estimator.PIXEL_SHIFT), integrand,
                                   counts, range(3))
    for p in range(3):
        delta = estimator.pixel_offsets(3, np.array([p]), d)[:, 0].astype(np.float64)
        exact = integrands.lobes_box_integral(delta, theta.astype(np.float64), L, d)
        assert abs(r["mean"][p] - exact) < 2e-3 * exact, (p, r["mean"][p], exact)


def test_scrambled_estimates_are_unbiased():
    # RQMC (Sec. 2.5.2): independent per-pixel scrambles give estimates centred on the
    # integral.  64 pixels x 256 samples of one Genz integrand with moderate widths.
    pp1 = genz_params(1, 4).astype(np.float64)[0]
    pp1[8:] = 1.5
    P = 64
    pp = np.tile(pp1.astype(np.float32), (P, 1))
    integrand = {"kind": "genz", "d": 8, "pixel_params": pp}
    r = estimator.integrate_pixels(_sampler(8, estimator.PIXEL_NUS | estimator.PIXEL_SHIFT), integrand,
                                   counts_uniform(P, 1, 256), range(P))
    exact = integrands.genz_integral(pp1.astype(np.float32).astype(np.float64))
    m = r["mean"]
    assert abs(np.mean(m) - exact) < 4 * np.std(m) / math.sqrt(P) + 1e-12
    assert np.std(m) > 0.0


def test_lobe_gradient_matches_central_differences():
    L, d = 3, 4
    theta = lobe_params(L, d, 6)
    integrand = {"kind": "lobes", "d": d, "num_lobes": L, "params": theta, "pixel_seed": 1}
    sampler = _sampler(d, estimator.PIXEL_NUS | estimator.PIXEL_SHIFT)
    counts = np.array([4, 16, 1, 32, 8, 2], dtype=np.uint32)
    pixels = np.arange(6)
    tgt_int = dict(integrand, params=perturb(theta, 7))
    target = estimator.integrate_pixels(sampler, tgt_int, counts, pixels)["mean"]
    loss, g, _ = estimator.loss_and_gradient(sampler, integrand, counts, pixels, target)
    idx = list(range(theta.size))
    fd = estimator.finite_difference(sampler, integrand, counts, pixels, target, idx, rel_step=1e-5)
    scale = np.max(np.abs(fd))
    assert np.all(np.abs(g - fd) <= 1e-6 * np.maximum(np.abs(fd), 1e-3 * scale)), np.abs(g - fd).max()


def test_lobe_weight_gradient_homogeneity():
    # f is linear in the weights, so sum_k w_k df/dw_k = f at every sample.
    L, d = 5, 3
    theta = lobe_params(L, d, 6).astype(np.float64)
    y = np.random.default_rng(0).random((d, 50))
    f = integrands.lobes(y, theta, L, d)
    for n in range(3):
        g = integrands.lobes_weighted_gradient(y[:, n:n + 1], np.ones(1), theta, L, d)
        gw = g[2 * L * d:]
        assert math.fsum(gw * theta[2 * L * d:]) == pytest.approx(f[n], rel=1e-13)


def test_windows_add_up_to_the_full_estimate():
    integrand = {"kind": "genz", "d": 8, "pixel_params": genz_params(5, 4)}
    sampler = _sampler(8, estimator.PIXEL_NUS | estimator.PIXEL_SHIFT)
    counts = np.array([1, 7, 64, 100, 256], dtype=np.uint32)
    full = estimator.integrate_pixels(sampler, integrand, counts, range(5))["sum"]
    a = estimator.integrate_pixels(sampler, integrand, counts, range(5), 0, 50)["sum"]
    b = estimator.integrate_pixels(sampler, integrand, counts, range(5), 50, 2 ** 32)["sum"]
    assert np.allclose(a + b, full, rtol=1e-14, atol=1e-300)


def test_unscrambled_coordinate_mean_is_exact():
    # The first 2^m points of every dimension are exactly {k / 2^m}, so the mean of x_j
    # over them is (2^m - 1) / 2^(m+1) for the unscrambled sequence.
    sampler = _sampler(8, 0)
    for m in (0, 3, 8):
        n = 1 << m
        x = estimator.pixel_samples_f32(sampler, np.zeros(n, np.int64), np.arange(n))
        for j in range(8):
            assert math.fsum(x[j].astype(np.float64)) / n == (n - 1) / (2.0 * n)


def test_gradient_term_sizes_bound_the_gradient():
    """The term sizes used to bound rounding error dominate the gradient they describe, and
    equal it where every term has the same sign (a target far below every estimate makes all
    dL/dI_p positive, and the weight derivatives G are positive)."""
    from oracle import estimator
    from synth import counts_uniform, lobe_params

    W, H, L, d = 6, 3, 4, 3
    counts = counts_uniform(W, H, 16)
    theta = lobe_params(L, d, 6)
    sp = {"kind": "sobol", "s": d, "table": digital.sobol_matrices(d, sobol_direction_init(d, 0)), "seed": 3,
          "flags": estimator.PIXEL_NUS | estimator.PIXEL_SHIFT}
    ig = {"kind": "lobes", "d": d, "num_lobes": L, "params": theta, "pixel_seed": 9}
    rng = np.random.default_rng(1)
    target = rng.uniform(0, 1, W * H)
    _, g, means = estimator.loss_and_gradient(sp, ig, counts, range(W * H), target)
    sizes = estimator.l2_gradient_term_sizes(sp, ig, counts, range(W * H), target)
    assert np.all(sizes >= np.abs(g) * (1 - 1e-12))
    low = np.full(W * H, -100.0)
    _, g2, m2 = estimator.loss_and_gradient(sp, ig, counts, range(W * H), low)
    s2 = estimator.l2_gradient_term_sizes(sp, ig, counts, range(W * H), low)
    # weights: all terms positive; the sizes add |I_p| to |I_p - T_p|
    ratio = (np.abs(m2 - low) + np.abs(m2)) / np.abs(m2 - low)
    gw, sw = g2[2 * L * d:], s2[2 * L * d:]
    assert np.all(sw <= gw * ratio.max() * (1 + 1e-12)) and np.all(sw >= gw * ratio.min() * (1 - 1e-12))
